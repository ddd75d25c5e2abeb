"""Pins of the oracle's Philox4x32-10 against what fixes it from outside:
the published known-answer vectors and an independent implementation (the
Philox engine header shipped with PyTorch, compiled only here)."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_published_known_answer_vectors(oracle_mod):
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        out = oracle_mod.philox4x32_10(v[0:4], v[4:6])
        assert out.tolist() == v[6:10]


_KAT_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
extern "C" void torch_philox(const unsigned* ctr, const unsigned* key, unsigned* out, int n) {
  for (int q = 0; q < n; ++q) {
    uint64_t seed = (uint64_t)key[2*q] | ((uint64_t)key[2*q+1] << 32);
    uint64_t sub = (uint64_t)ctr[4*q+2] | ((uint64_t)ctr[4*q+3] << 32);
    uint64_t off = (uint64_t)ctr[4*q] | ((uint64_t)ctr[4*q+1] << 32);
    at::philox_engine e(seed, sub, off);
    for (int w = 0; w < 4; ++w) out[4*q+w] = e();
  }
}
"""


@pytest.fixture(scope="module")
def torch_philox():
    torch = pytest.importorskip("torch")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("PyTorch Philox header not available")
    d = tempfile.mkdtemp(prefix="philox_kat_")
    src = os.path.join(d, "k.cpp")
    so = os.path.join(d, "k.so")
    open(src, "w").write(_KAT_SRC)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-shared", "-fPIC", "-I" + inc, src, "-o", so])
    lib = C.CDLL(so)
    lib.torch_philox.argtypes = [C.c_void_p] * 3 + [C.c_int]
    return lib


def test_matches_independent_implementation(oracle_mod, torch_philox):
    rng = np.random.default_rng(123)
    n = 4000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    # include the counter shapes the method uses: small word 0, tag in word 3
    ctr[: n // 2, 0] %= 4096
    ctr[: n // 2, 3] = (2 << 28) | (ctr[: n // 2, 3] % 256)
    ref = np.zeros((n, 4), dtype=np.uint32)
    torch_philox.torch_philox(ctr.ctypes.data, key.ctypes.data, ref.ctypes.data, n)
    mine = np.array([oracle_mod.philox4x32_10(ctr[q], key[q]) for q in range(n)])
    assert np.array_equal(mine, ref)


def test_output_bits_balanced(oracle_mod):
    # every output bit is 1 about half the time over consecutive counters
    outs = np.array([oracle_mod.philox4x32_10([q, 7, 3, (2 << 28)], [0, 0]) for q in range(4096)])
    bits = np.unpackbits(outs.view(np.uint8)).reshape(-1, 8 * 16).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(4096))
