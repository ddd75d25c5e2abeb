"""Adaptive temperature insertion (Sec. 4): after a trial run the pair
rates go into a min-heap and the lowest-rate intervals (below the
threshold, within the caps) get a new temperature at their midpoint; the
new replica starts from a copy of the colder neighbour.  The expected
insertions are recomputed here from an identical trial run with a sort,
not a heap."""
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W


def _pair(oracle_mod, temps, L=4, seed=2, R_cap=0):
    f = W.bimodal_fields(L, [6, L])
    mk = lambda: oracle_mod.Oracle(L, len(temps), 1.0, 1.0, f, temps, seed=seed, R_cap=R_cap)
    return mk(), mk()


@pytest.mark.parametrize("a_max,theta,R_cap", [(2, 0.2, 12), (5, 0.5, 12), (3, 1.1, 8), (4, 0.0, 12)])
def test_one_trial_matches_sorted_rule(oracle_mod, a_max, theta, R_cap):
    temps = np.array([1.0, 1.1, 1.2, 2.6, 2.7, 4.5, 4.6])
    o, clone = _pair(oracle_mod, temps, R_cap=R_cap)
    S, every = 300, 1
    clone.reset_exchange_stats()
    clone.sweep(S, every)
    att, acc = clone.exchange_stats()
    spins_after = clone.spins()
    perm_after = clone.perm()
    rates = [(acc[p] / att[p], p) for p in range(len(temps) - 1) if att[p] > 0]
    picks = []
    for rate, p in sorted(rates):
        if not rate < theta or len(picks) >= a_max or len(temps) + len(picks) >= R_cap:
            break
        picks.append(p)
    R_new = o.adapt_temps(1, S, every, theta, a_max, R_cap)
    assert R_new == len(temps) + len(picks)
    T_new = o.temps()
    want_T = np.sort(np.concatenate([temps, [(temps[p] + temps[p + 1]) / 2 for p in picks]]))
    assert np.array_equal(T_new, want_T)
    perm = o.perm()
    s = o.spins()
    for q, p in enumerate(picks):
        new_id = len(temps) + q
        slot = int(np.flatnonzero(perm == new_id)[0])
        assert T_new[slot] == (temps[p] + temps[p + 1]) / 2
        assert np.array_equal(s[new_id], spins_after[perm_after[p]])
    # old replicas keep their temperatures and configurations
    for t_old in range(len(temps)):
        rid = perm_after[t_old]
        slot = int(np.flatnonzero(perm == rid)[0])
        assert T_new[slot] == temps[t_old]
        assert np.array_equal(s[rid], spins_after[rid])
    att2, acc2 = o.exchange_stats()
    assert not att2.any() and not acc2.any()


def test_insertion_raises_minimum_rate(oracle_mod):
    # Sec. 6: inserting at the lowest-rate intervals lifts the minimum rate.
    temps = np.array([1.0, 1.5, 2.5, 3.5, 5.0])
    o, _ = _pair(oracle_mod, temps, L=6, R_cap=16)
    o.reset_exchange_stats()
    o.sweep(2000, 1)
    att, acc = o.exchange_stats()
    before = (acc / att).min()
    o.adapt_temps(3, 2000, 1, 0.3, 2, 16)
    o.reset_exchange_stats()
    o.sweep(4000, 1)
    att, acc = o.exchange_stats()
    assert (acc / att).min() > before


def test_caps(oracle_mod):
    temps = np.array([1.0, 3.0, 5.0, 7.0])
    o, _ = _pair(oracle_mod, temps, R_cap=6)
    assert o.adapt_temps(5, 100, 1, 2.0, 10, 6) == 6
    with pytest.raises(RuntimeError):
        o.adapt_temps(1, 10, 1, 0.5, 1, 7)      # beyond the capacity given at create
