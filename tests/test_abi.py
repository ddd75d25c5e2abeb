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


def test_pool_job_calls_reject_bad_arguments(rfim_mod):
    """rfim_pool_admit_job, rfim_pool_poll and rfim_pool_result validate
    their arguments before any device work."""
    import ctypes as C

    from paper_1508_06268_amd import rfim as B

    lib = rfim_mod.load_library()
    job = B.rfim_job_t()
    assert lib.rfim_pool_admit_job(None, C.byref(job)) == -1
    assert lib.rfim_pool_poll(None, None, 0) == -1
    res = B.rfim_result_t()
    assert lib.rfim_pool_result(None, 0, C.byref(res)) == -1
    assert b"no such pool slot" in lib.rfim_last_error()


def test_null_handle_getters_and_setters_fail_cleanly(rfim_mod):
    lib = rfim_mod.load_library()
    assert lib.rfim_set_concurrency(None, 0) == -1
    assert lib.rfim_get_concurrency(None) == -1
    assert lib.rfim_set_launch_shape(None, 0, 4, 128) == -1
    assert lib.rfim_num_replicas(None) == -1
    assert lib.rfim_set_measure(None, 1) == -1
    assert lib.rfim_fourier(None, None) == -1
    assert lib.rfim_batch_set_group_bytes(None, 0) == -1
    assert lib.rfim_batch_get_group_bytes(None) == -1
    assert b"NULL" in lib.rfim_last_error()


@pytest.mark.parametrize("L,R,R_cap,kind", [(8, 16, 0, "b"), (32, 64, 0, "g"), (64, 128, 192, "b"),
                                            (64, 128, 192, "g"), (24, 5, 9, "b")])
def test_pool_bytes_needed_accounts_every_buffer(rfim_mod, L, R, R_cap, kind):
    """The device bytes a realization reserves (host arithmetic, no GPU):
    at least its spins (R_cap L^3 bytes) and fields (L^3 bytes, or two FP32
    copies for continuous fields), whole 256-byte pieces, growing with R_cap;
    invalid parameters give 0."""
    from paper_1508_06268_amd import workloads as W

    f = W.bimodal_fields(L, [0, 1]) if kind == "b" else W.gaussian_fields(L, [0, 1])
    Rc = R_cap or R
    w = W.Realization(L=L, R=R, J=1.0, h=1.0, fields=f, temps=W.linear_temps(R, 1.0, 5.0), seed=0,
                      sweeps=0, every=10, R_cap=R_cap)
    need = rfim_mod.Pool.bytes_needed(w)
    N = L ** 3
    assert need >= Rc * N + (N if kind == "b" else 8 * N)
    if L in (64, 128, 256):
        # the bit arrays a bit-storage class adds (spin bits, and the field bits
        # or the reordered FP32 field copy) are reserved whatever the class shape
        assert need >= Rc * N * 9 // 8 + (N + N // 8 if kind == "b" else 12 * N)
    assert need % 256 == 0
    bigger = W.Realization(L=L, R=R, J=1.0, h=1.0, fields=f, temps=W.linear_temps(R, 1.0, 5.0), seed=0,
                           sweeps=0, every=10, R_cap=Rc + 8)
    assert rfim_mod.Pool.bytes_needed(bigger) >= need + 8 * N
    bad = W.Realization(L=L, R=R, J=1.0, h=1.0, fields=f, temps=W.linear_temps(R, 5.0, 1.0), seed=0,
                        sweeps=0, every=10, R_cap=R_cap)
    assert rfim_mod.Pool.bytes_needed(bad) == 0


@pytest.mark.parametrize("L,R,J,ptr,code,msg", [
    (7, 4, 1.0, 16, -1, "even"),
    (8, 0, 1.0, 16, -1, "R must be"),
    (8, (1 << 18) + 1, 1.0, 16, -5, "fixed partial array"),
    (8, 4, 1.0, 0, -1, "NULL"),
    (8, 4, float("nan"), 16, -1, "finite"),
])
def test_noalloc_energies_reject_bad_arguments(rfim_mod, L, R, J, ptr, code, msg):
    """Validation happens before any device work (no GPU needed)."""
    from paper_1508_06268_amd import rfim as B
    lib = rfim_mod.load_library()
    assert lib.rfim_energies_noalloc(L, R, J, 1.0, ptr, ptr, ptr, None) == code
    assert msg in B.last_error()
