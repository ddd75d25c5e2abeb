"""Acceptance thresholds of the oracle pinned against 50-digit arithmetic:
thr = floor(exp(-beta*dE) * 2^32), dE = 2(J a + h b) for a = s_i n_i,
b = s_i h_i (Metropolis rule with the energy of Eq. 1)."""
import mpmath
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W

mpmath.mp.dps = 50


@pytest.mark.parametrize("J,h,temps", [
    (1.0, 1.0, W.linear_temps(16, 1.5, 5.0)),
    (1.0, 2.25, W.linear_temps(128, 1.0, 6.0)),
    (1.0, 2.0, W.geometric_temps(64, 1.0, 6.0)),
    (0.7, 0.3, np.array([0.05, 0.5, 2.0, 40.0])),
    (-1.0, 1.5, np.array([0.8, 3.0])),
])
def test_thresholds_match_high_precision(oracle_mod, J, h, temps):
    L = 2
    f = np.array([1, -1, 1, 1, -1, -1, 1, -1], dtype=np.float32)
    o = oracle_mod.Oracle(L, len(temps), J, h, f, temps)
    thr, always = o.thresholds()
    near = 0
    for cls in range(14):
        k, fb = cls >> 1, cls & 1
        dE = 2 * (mpmath.mpf(J) * (2 * k - 6) + mpmath.mpf(h) * (2 * fb - 1))
        assert bool(always[cls]) == (dE <= 0)
        if dE <= 0:
            continue
        for t, T in enumerate(temps):
            beta = mpmath.mpf(1.0 / float(T))       # the oracle's FP64 beta
            exact = mpmath.exp(-beta * dE) * mpmath.mpf(2) ** 32
            want = int(mpmath.floor(exact))
            want = min(want, 2 ** 32 - 1)
            frac = exact - mpmath.floor(exact)
            if exact >= 1 and min(frac, 1 - frac) < mpmath.mpf(10) ** -4:
                near += 1
                assert abs(int(thr[t, cls]) - want) <= 1
            else:
                assert int(thr[t, cls]) == want, (t, cls)
    assert near <= 2


def test_extreme_temperatures(oracle_mod):
    f = np.ones(8, dtype=np.float32)
    o = oracle_mod.Oracle(2, 2, 1.0, 1.0, f, np.array([1e-6, 1e12]))
    thr, always = o.thresholds()
    up = ~always
    assert np.all(thr[0, up] == 0)              # T -> 0: no uphill move
    assert np.all(thr[1, up] == 2 ** 32 - 1)    # T -> inf: clamped at 2^32 - 1
