"""Exact stationarity of one oracle sweep at L=2 (N=8, 256 states).

Within a half-sweep the sites of one colour have no neighbour of their own
colour, so their flips are independent given the other colour: the
half-sweep is a product of per-site flips and its 256 x 256 transition
matrix can be written out.  Each per-site flip probability is the fraction
of 32-bit words for which the oracle's own decision function (the one its
sweep calls) flips the site.  Metropolis with these probabilities leaves
the Boltzmann distribution of Eq. 1 invariant up to the 2^-32 rounding of
the bound, so pi P = pi must hold to ~1e-9 -- a dropped field term, a wrong
sign or a wrong neighbour in the oracle's Delta E breaks it by orders of
magnitude.  Brute force on the whole state space, no sampling."""
import itertools

import numpy as np
import pytest

from helpers import energy_numpy

L, N = 2, 8
STATES = np.array(list(itertools.product([-1, 1], repeat=N)), dtype=np.int8)
COLOUR = np.array([((i % L) + (i // L) % L + i // (L * L)) % 2 for i in range(N)])


def _flip_prob(o, i):
    """Fraction of the 2^32 words for which the oracle's own decision
    (orc_accept, the function its sweep calls) flips site i of replica 0.
    Its rules accept exactly the words below a bound, so a binary search
    over u finds the bound."""
    if o.accept(0, i, 0xFFFFFFFF):
        return 1.0
    lo, hi = 0, 0xFFFFFFFF          # accept(lo - 1) holds, accept(hi) does not
    while lo < hi:
        mid = (lo + hi) // 2
        if o.accept(0, i, mid):
            lo = mid + 1
        else:
            hi = mid
    return lo / 2.0 ** 32


def _flip_probs(o):
    """p[state, site]: probability that the oracle flips `site` when it is
    visited in `state` (neighbours as in `state`)."""
    p = np.zeros((len(STATES), N))
    for q, s in enumerate(STATES):
        o.set_spins(s.reshape(1, N))
        for i in range(N):
            p[q, i] = _flip_prob(o, i)
    return p


def _half_sweep_matrix(p, colour):
    idx = {tuple(s): q for q, s in enumerate(STATES)}
    sites = [i for i in range(N) if COLOUR[i] == colour]
    P = np.zeros((len(STATES), len(STATES)))
    for q, s in enumerate(STATES):
        for flips in itertools.product([0, 1], repeat=len(sites)):
            t = s.copy()
            w = 1.0
            for i, fl in zip(sites, flips):
                w *= p[q, i] if fl else 1.0 - p[q, i]
                if fl:
                    t[i] = -t[i]
            P[q, idx[tuple(t)]] += w
    return P


@pytest.mark.parametrize("kind,J,h,T", [
    ("bimodal", 1.0, 1.0, 1.3),
    ("bimodal", 1.0, 2.25, 3.0),
    ("bimodal", 0.7, 0.4, 0.9),
    ("gauss", 1.0, 1.3, 1.7),
    ("gauss", 1.0, 2.0, 4.5),
])
def test_sweep_leaves_boltzmann_invariant(oracle_mod, kind, J, h, T):
    rng = np.random.default_rng(17)
    if kind == "bimodal":
        f = np.where(rng.random(N) < 0.5, -1.0, 1.0).astype(np.float32)
    else:
        f = rng.standard_normal(N).astype(np.float32)
    o = oracle_mod.Oracle(L, 1, J, h, f, [T], seed=3)
    beta = 1.0 / T
    p = _flip_probs(o)
    P = _half_sweep_matrix(p, 0) @ _half_sweep_matrix(p, 1)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
    E = np.array([energy_numpy(s, f, L, J, h)[0] for s in STATES])
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    resid = np.abs(pi @ P - pi).max() / pi.max()
    assert resid < 1e-8, resid
    # the same matrix is far from stationary for a neighbouring temperature
    pi2 = np.exp(-(beta * 1.1) * (E - E.min()))
    pi2 /= pi2.sum()
    assert np.abs(pi2 @ P - pi2).max() / pi2.max() > 1e-4
