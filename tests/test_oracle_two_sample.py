"""The two-sample statistic of the continuous-field parity test, checked on
the oracle alone (no GPU): the stored oracle statistics
(tests/golden/gaussian_two_sample.json, written by make_gaussian_stats.py
from the oracle) must be the oracle's, the statistic must reject oracle runs
whose inverse temperatures are scaled by 1.01, and must accept a second
independent set of oracle seeds at the same temperatures."""
import json
import os

import numpy as np
import pytest

from two_sample import compare, from_json

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "gaussian_two_sample.json")


def _load():
    return json.load(open(FIXTURE))


def _set(d, name):
    s = d["sets"][name]
    return from_json(s["E"]), from_json(s["absM"])


def test_rejects_beta_scaled_by_one_percent():
    d = _load()
    a, b = _set(d, "l32_null"), _set(d, "l32_beta")
    reject, pmin, thr, tmax = compare(a[0], a[1], b[0], b[1])
    print("beta x 1.01: p_min %.3g (threshold %.3g), max |t| %.1f" % (pmin, thr, tmax))
    assert reject
    assert tmax > 10.0          # not a marginal rejection


def test_accepts_independent_oracle_seeds():
    d = _load()
    a, c = _set(d, "l32_null"), _set(d, "l32_null2")
    reject, pmin, thr, tmax = compare(a[0], a[1], c[0], c[1])
    print("oracle vs oracle: p_min %.3g (threshold %.3g), max |t| %.2f" % (pmin, thr, tmax))
    assert not reject


def test_statistic_on_planted_shifts():
    """Synthetic summaries: a shift of 6 standard errors in one slot of one
    observable is rejected; a shift of 2 standard errors everywhere is not
    (the family is read at three sigma with the Bonferroni correction)."""
    rng = np.random.default_rng(7)
    R, n = 64, 32
    x = rng.normal(0.0, 1.0, size=(n, R))
    y = rng.normal(0.0, 1.0, size=(n, R))
    from two_sample import summary

    sx, sy = summary(x), summary(y)
    se = np.sqrt(sx["var"] / n + sy["var"] / n)
    shifted = dict(sy, mean=sy["mean"].copy())
    shifted["mean"][17] += 6.0 * se[17] + (sx["mean"][17] - sy["mean"][17])
    assert compare(sx, sx, shifted, sy)[0]
    mild = dict(sy, mean=sx["mean"] + 2.0 * se)
    assert not compare(sx, sx, mild, sy)[0]


@pytest.mark.slow
def test_fixture_is_the_oracles():
    """The first seed of the L=64 set, recomputed now, equals its stored
    time averages (guards the fixture against a stale oracle)."""
    import sys

    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_gaussian_stats as M

    d = _load()
    s = d["sets"]["l64_null"]
    E, Mabs = M.oracle_run((s["case"], s["seed0"], s["beta_scale"]))
    assert np.allclose(E, s["first_seed"]["E"], rtol=0, atol=1e-9)
    assert np.array_equal(np.asarray(Mabs), np.asarray(s["first_seed"]["absM"]))
