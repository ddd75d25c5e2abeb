"""Brute-force pins at L=2 (N=8, 256 states): the sweep + exchange chain of
the oracle samples the Boltzmann distribution of Eq. 1 at every temperature
slot, and the exchange step accepts with min(1, e^Delta) (Eq. 2 read with
the Hukushima-Nemoto sign)."""
import itertools

import numpy as np
import pytest

from helpers import batch_means_sem, energy_numpy

L = 2
N = 8


def enumerate_states(fields, J, h):
    states = np.array(list(itertools.product([-1, 1], repeat=N)), dtype=np.int8)
    E = np.array([energy_numpy(s, fields, L, J, h)[0] for s in states])
    M = states.astype(np.int64).sum(axis=1)
    return states, E, M


def boltzmann(E, T):
    w = np.exp(-(E - E.min()) / T)
    return w / w.sum()


@pytest.mark.parametrize("kind", ["bimodal", "gauss"])
def test_chain_matches_enumeration(oracle_mod, kind):
    if kind == "bimodal":
        f = np.array([1, -1, -1, 1, 1, 1, -1, 1], dtype=np.float32)
        J, h = 1.0, 1.0
    else:
        f = np.random.default_rng(11).standard_normal(N).astype(np.float32)
        J, h = 1.0, 1.3
    temps = np.array([1.0, 1.8, 3.0, 5.0])
    R = len(temps)
    _, Es, Ms = enumerate_states(f, J, h)
    o = oracle_mod.Oracle(L, R, J, h, f, temps, seed=77)
    o.sweep(200, 1)
    n = 100_000
    E = np.zeros((n, R))
    M = np.zeros((n, R))
    for q in range(n):
        o.sweep(1, 1)
        E[q] = o.energies()
        M[q] = o.magnetizations()
    for t, T in enumerate(temps):
        p = boltzmann(Es, T)
        for series, exact_vals in ((E[:, t], Es), (M[:, t], Ms), (np.abs(M[:, t]), np.abs(Ms))):
            want = float((p * exact_vals).sum())
            got = series.mean()
            sem = batch_means_sem(series)
            assert abs(got - want) <= 4.5 * sem + 1e-12, (t, got, want, sem)
        # energy histogram: each level's frequency within 4.5 sigma
        levels = np.unique(np.round(Es, 9))
        for lev in levels:
            pw = float(p[np.isclose(Es, lev)].sum())
            ind = np.isclose(E[:, t], lev).astype(np.float64)
            sem = batch_means_sem(ind)
            assert abs(ind.mean() - pw) <= 4.5 * sem + 2e-3, (t, lev, ind.mean(), pw)


def _two_levels(fields, J, h):
    states, Es, _ = enumerate_states(fields, J, h)
    lo = int(np.argmin(Es))
    gap = np.unique(np.round(Es - Es[lo], 9))[1]
    hi = int(np.flatnonzero(np.isclose(Es - Es[lo], gap))[0])
    return states[lo], states[hi], float(Es[hi] - Es[lo])


def test_exchange_acceptance_is_min_one_exp_delta(oracle_mod):
    f = np.array([1, -1, -1, 1, 1, 1, -1, 1], dtype=np.float32)
    J, h = 1.0, 1.0
    cold_state, hot_state, dE = _two_levels(f, J, h)
    b_hot = 0.5
    b_cold = b_hot + 1.2 / dE
    temps = np.array([1.0 / b_cold, 1.0 / b_hot])
    o = oracle_mod.Oracle(L, 2, J, h, f, temps)
    o.set_spins(np.stack([cold_state, hot_state]))
    E = o.energies()
    beta = 1.0 / temps
    delta = (beta[1] - beta[0]) * (E[1] - E[0])     # low energy already cold
    assert abs(delta + 1.2) < 1e-9
    n = 20000
    acc = 0
    for q in range(n):
        o.set_perm([0, 1])
        o.set_counters(0, 2 * q)
        o.exchange_once()
        acc += int(o.perm()[0] == 1)
    p = np.exp(delta)
    assert abs(acc / n - p) <= 4.5 * np.sqrt(p * (1 - p) / n)
    # the reverse order (low energy at the hot slot): Delta > 0, always taken
    for q in range(200):
        o.set_perm([1, 0])
        o.set_counters(0, 2 * q)
        o.exchange_once()
        assert o.perm().tolist() == [0, 1]


def test_exchange_odd_even_alternation(oracle_mod):
    f = np.ones(N, dtype=np.float32)
    temps = np.linspace(1.0, 3.0, 5)
    o = oracle_mod.Oracle(L, 5, 1.0, 1.0, f, temps)
    for k in range(6):
        o.reset_exchange_stats()
        o.set_counters(0, k)
        o.exchange_once()
        att, _ = o.exchange_stats()
        want = np.array([1 if p % 2 == k % 2 else 0 for p in range(4)], dtype=np.uint64)
        assert np.array_equal(att, want)
        assert o.counters()[1] == k + 1
