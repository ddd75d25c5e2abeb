"""Closed-form and textbook limits that pin the oracle's sweep:
J = 0 (independent spins, <s_i> = tanh(beta h h_i)), T -> 0 (deterministic
checkerboard quench, compared with a numpy implementation), and h = 0 (the
3D Ising model, whose Binder cumulants for two sizes cross near
T_c = 4.5115)."""
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W
from helpers import batch_means_sem, quench_numpy


@pytest.mark.parametrize("kind", ["bimodal", "gauss"])
def test_independent_spins_at_zero_coupling(oracle_mod, kind):
    L = 4
    f = W.bimodal_fields(L, [1, 1]) if kind == "bimodal" else W.gaussian_fields(L, [1, 1])
    h = 0.8
    temps = np.array([0.7, 1.5, 3.0])
    o = oracle_mod.Oracle(L, 3, 0.0, h, f, temps, seed=5)
    o.sweep(50, 0)
    n = 20000
    q = np.zeros((n, 3))
    fd = f.astype(np.float64)
    for step in range(n):
        o.sweep(1, 0)
        s = o.spins().astype(np.float64)          # no exchange: replica r = slot r
        q[step] = (s * fd).mean(axis=1)
    for t, T in enumerate(temps):
        want = float((fd * np.tanh(h * fd / T)).mean())
        sem = batch_means_sem(q[:, t])
        assert abs(q[:, t].mean() - want) <= 4.5 * sem, (t, q[:, t].mean(), want, sem)


@pytest.mark.parametrize("L,J,h,kind", [
    (2, 1.0, 1.0, "bimodal"),
    (4, 1.0, 1.0, "bimodal"),
    (6, 1.0, 2.0, "bimodal"),      # Delta E = 0 ties occur: always accepted
    (4, 1.0, 1.5, "gauss"),
    (8, 0.5, 1.0, "gauss"),
])
def test_zero_temperature_quench_matches_numpy(oracle_mod, L, J, h, kind):
    f = W.bimodal_fields(L, [2, L]) if kind == "bimodal" else W.gaussian_fields(L, [2, L])
    o = oracle_mod.Oracle(L, 2, J, h, f, np.array([1e-6, 2e-6]), seed=3)
    s0 = o.spins()
    o.sweep(6, 0)
    s6 = o.spins()
    for r in range(2):
        assert np.array_equal(s6[r], quench_numpy(s0[r], f, L, J, h, 6))


def _binder(L, temps, sweeps, seed):
    from oracle.oracle import Oracle
    f = np.zeros(L ** 3, dtype=np.float32)
    o = Oracle(L, len(temps), 1.0, 0.0, f, temps, seed=seed, field_kind=1)
    o.sweep(sweeps // 5, 1)
    m2 = np.zeros(len(temps))
    m4 = np.zeros(len(temps))
    for _ in range(sweeps):
        o.sweep(1, 1)
        m = o.magnetizations().astype(np.float64) / L ** 3
        m2 += m * m
        m4 += m ** 4
    m2 /= sweeps
    m4 /= sweeps
    return 1.0 - m4 / (3.0 * m2 * m2)


@pytest.mark.slow
def test_ising_binder_crossing(oracle_mod):
    temps = np.array([4.20, 4.35, 4.45, 4.52, 4.58, 4.68, 4.85])
    u8 = _binder(8, temps, 40000, 1)
    u16 = _binder(16, temps, 12000, 2)
    d = u16 - u8
    assert d[0] > 0 and d[-1] < 0, d
    sign_change = [q for q in range(len(d) - 1) if d[q] > 0 >= d[q + 1]]
    assert sign_change, d
    q = sign_change[0]
    Tc = temps[q] + (temps[q + 1] - temps[q]) * d[q] / (d[q] - d[q + 1])
    assert 4.42 <= Tc <= 4.62, (Tc, d)


def test_oracle_rejects_lattices_it_cannot_hold(oracle_mod):
    """The oracle accepts even L up to 512 (its neighbour table needs 24 L^3
    bytes); larger L are refused before anything is read or allocated."""
    import ctypes as C

    lib = oracle_mod.lib()
    f = np.ones(8, dtype=np.float32)
    T = np.array([1.0])
    for L in (514, 1024):
        h = lib.orc_create(L, 1, 1.0, 1.0, f.ctypes.data_as(C.c_void_p), T.ctypes.data_as(C.c_void_p),
                           0, 0, -1, 0)
        assert not h
        assert b"2..512" in lib.orc_last_error()
