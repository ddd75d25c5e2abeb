"""The C ABI library (no GPU needed): it loads, exports every symbol its
header declares, and rejects bad arguments before any device work."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rfim.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rfim_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree(rfim_mod):
    assert declared_symbols() == sorted(rfim_mod.EXPORTS)


def test_library_exports_every_declared_symbol(rfim_mod):
    lib = rfim_mod.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_library_has_gfx950_code():
    so = os.path.join(ROOT, "paper_1508_06268_amd", "librfim.so")
    assert b"gfx950" in open(so, "rb").read()


@pytest.mark.parametrize("L,R,J,h,temps,fields,msg", [
    (3, 2, 1.0, 1.0, [1.0, 2.0], None, "even"),
    (2050, 2, 1.0, 1.0, [1.0, 2.0], None, "even"),
    (4, 0, 1.0, 1.0, [], None, "R must be"),
    (4, 2, 1.0, 1.0, [2.0, 1.0], None, "ascending"),
    (4, 2, 1.0, 1.0, [-1.0, 1.0], None, "> 0"),
    (4, 2, np.inf, 1.0, [1.0, 2.0], None, "finite"),
    (4, 2, 1.0, 1.0, [1.0, 2.0], "nan", "finite"),
])
def test_create_rejects_bad_arguments(rfim_mod, L, R, J, h, temps, fields, msg):
    from paper_1508_06268_amd import rfim as B
    n = L ** 3 if L <= 64 else 8
    f = np.ones(n, dtype=np.float32)
    if fields == "nan":
        f[3] = np.nan
    T = np.asarray(temps + [0.0] * 0, dtype=np.float64)
    handle = B.rfim_create(L, R, J, h, f, T if T.size else np.zeros(1), 0)
    assert not handle
    assert msg in B.last_error()


def test_null_handle_calls_fail_cleanly(rfim_mod):
    lib = rfim_mod.load_library()
    assert lib.rfim_sweep(None, 1, 1) == -1
    assert lib.rfim_energies(None, None) == -1
    lib.rfim_destroy(None)


def test_null_handle_getters_and_setters_fail_cleanly(rfim_mod):
    lib = rfim_mod.load_library()
    assert lib.rfim_set_concurrency(None, 0) == -1
    assert lib.rfim_get_concurrency(None) == -1
    assert lib.rfim_set_launch_shape(None, 0, 4, 128) == -1
    assert lib.rfim_num_replicas(None) == -1
    assert lib.rfim_set_measure(None, 1) == -1
    assert lib.rfim_fourier(None, None) == -1
    assert b"NULL" in lib.rfim_last_error()
