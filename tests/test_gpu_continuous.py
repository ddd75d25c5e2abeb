"""Continuous (Gaussian) fields: the device evaluates dE and exp(-beta dE)
in FP32, so rare decisions may differ from the oracle's FP64.  (i) From
identical states, fewer than 1e-6 of the flip decisions of one sweep may
differ; (ii) 32 GPU seeds and 32 disjoint oracle seeds agree per slot in
their time-averaged energy and |M| (two-sample test at three sigma over the
family of slots)."""
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W
from parity_util import make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["bits", "bytes"])
def test_one_sweep_decision_mismatch_rate(rfim_mod, oracle_mod, storage):
    L, R = 64, 40
    f = W.gaussian_fields(L, [0, 1])
    T = W.geometric_temps(R, 1.0, 6.0)
    g, o = make_pair(rfim_mod, oracle_mod, L, R, 1.0, 2.0, f, T, seed=0)
    g.set_spin_storage(rfim_mod.rfim.SPINS_BITS if storage == "bits" else rfim_mod.rfim.SPINS_BYTES)
    total = 0
    mism = 0
    for rep in range(3):
        s = W.random_spins(R, L, [21, rep]) if rep else g.spins()
        g.set_spins(s)
        o.set_spins(s)
        g.sweep(1, 0)
        o.sweep(1, 0)
        total += R * L ** 3
        mism += int((g.spins() != o.spins()).sum())
    print("continuous-field decisions %d in %s, mismatches %d" % (total, storage, mism))
    assert total >= 10 ** 7
    assert mism / total < 1e-6


def test_energies_consistent_with_oracle_components(rfim_mod, oracle_mod):
    L, R = 16, 8
    f = W.gaussian_fields(L, [22, 0])
    T = W.geometric_temps(R, 1.0, 6.0)
    g, o = make_pair(rfim_mod, oracle_mod, L, R, 1.0, 2.0, f, T, seed=1)
    s = W.random_spins(R, L, [22, 1])
    g.set_spins(s)
    o.set_spins(s)
    gb, gf, gm = g.components()
    ob, of, om = o.components()
    assert np.array_equal(gb, ob) and np.array_equal(gm, om)
    assert np.allclose(gf, of, rtol=1e-12, atol=1e-9)


def _gpu_time_averages(rfim_mod, case, seeds, concurrency=0, shape=None, storage=None):
    """Per-seed time averages of E and |M| by slot over the measurement
    window of a case (same protocol as the oracle fixture: burn sweeps with
    an exchange every 10, then one sample after every exchange step of the
    window, accumulated on the device)."""
    import make_gaussian_stats as M

    c = M.CASES[case]
    f, T = M.case_inputs(case)
    E, A = [], []
    for seed in seeds:
        g = rfim_mod.Rfim(c["L"], c["R"], c["J"], c["h"], f, T, seed=seed)
        if shape is not None:
            g.set_launch_shape(*shape)
        if storage is not None:
            g.set_spin_storage(storage)
        if concurrency:
            g.set_concurrency(concurrency)
        g.sweep(c["burn"], c["every"])
        g.reset_observables()
        g.sweep(c["meas"], c["every"])
        o = g.observables()
        assert np.all(o[:, 0] == c["meas"] // c["every"])
        E.append(o[:, 1] / o[:, 0])
        A.append(o[:, 3] / o[:, 0])
        g.close()
    return np.array(E), np.array(A)


@pytest.mark.parametrize("case,set_name,concurrency,shape,storage", [
    ("l32", "l32_null", 0, None, None),            # L=32, R=64: the default slab shape
    ("l32", "l32_null", 0, (1, 4, 1024), None),    # the LDS-resident shape
    ("l64", "l64_null", 2, None, 1),               # L=64, R=8: bit sweep, half-sweeps on two streams
    ("l64", "l64_null", 2, None, 0),               # the same in byte storage (streaming kernel)
])
def test_statistics_over_seeds(rfim_mod, case, set_name, concurrency, shape, storage):
    """32 GPU seeds against 32 disjoint oracle seeds (stored statistics from
    tests/golden/make_gaussian_stats.py): per slot, Welch's t on the
    time-averaged energy and |M|; the family of 2R comparisons must pass at
    three sigma with the Bonferroni correction (no slot may fall outside).
    The statistic's power is shown on the CPU (test_oracle_two_sample.py:
    oracle runs with beta scaled by 1.01 are rejected)."""
    import json
    import os

    from two_sample import compare, from_json, summary

    here = os.path.dirname(os.path.abspath(__file__))
    d = json.load(open(os.path.join(here, "golden", "gaussian_two_sample.json")))
    ref = d["sets"][set_name]
    E, A = _gpu_time_averages(rfim_mod, case, range(1000, 1000 + d["nseeds"]), concurrency, shape, storage)
    reject, pmin, thr, tmax = compare(summary(E), summary(A), from_json(ref["E"]), from_json(ref["absM"]))
    print("%s: GPU vs oracle seeds, p_min %.3g (threshold %.3g), max |t| %.2f" % (case, pmin, thr, tmax))
    assert not reject, (pmin, thr, tmax)
