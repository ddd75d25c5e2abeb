"""Pins of the oracle's double-checkerboard order with multi-hit updates
(Sec. 3.2, Sec. 5.2): tiles in a coarse checkerboard, the tiles of coarse
colour 0 then 1 per sweep, `hits` local two-colour sweeps per tile visit.

* J = 0: sites do not interact, so the order of updates cannot matter and
  only the random words do; `hits` local sweeps of sweep t use the words of
  plain sweeps t hits ... t hits + hits - 1, so n tile sweeps must equal
  hits * n plain sweeps bit for bit.  Pins the counter mapping.
* T -> 0: the dynamics is deterministic; an independent numpy formulation
  of the tile order (coarse colour, hit, fine colour) must give the same
  spins.  Pins the order: coarse colours, frozen neighbours, hit count.
* L = 2 with 1x1x1 tiles: each phase (one coarse colour, `hits` updates
  per site) leaves the Boltzmann distribution of Eq. 1 invariant, exactly
  (transition matrix from the oracle's decision function), and the chain
  with exchanges samples it (brute-force enumeration)."""
import itertools

import numpy as np
import pytest

from helpers import batch_means_sem, energy_numpy, quench_numpy, tile_quench_numpy
from paper_1508_06268_amd import workloads as W


def _fields(kind, L, key):
    return W.bimodal_fields(L, key) if kind == "bimodal" else W.gaussian_fields(L, key)


@pytest.mark.parametrize("kind", ["bimodal", "gauss"])
@pytest.mark.parametrize("L,tiles,hits", [(4, (2, 2, 2), 1), (4, (2, 1, 2), 3), (8, (4, 2, 2), 2),
                                          (8, (2, 4, 1), 1), (16, (8, 4, 2), 3)])
def test_zero_coupling_tiles_equal_plain_sweeps(oracle_mod, kind, L, tiles, hits):
    f = _fields(kind, L, [61, L])
    T = np.array([0.8, 1.7, 3.9])
    a = oracle_mod.Oracle(L, 3, 0.0, 1.3, f, T, seed=12)
    b = oracle_mod.Oracle(L, 3, 0.0, 1.3, f, T, seed=12)
    a.set_update_order(1, tiles, hits)
    a.sweep(3, 0)
    b.sweep(3 * hits, 0)
    assert np.array_equal(a.spins(), b.spins())
    assert a.counters() == (3, 0) and b.counters() == (3 * hits, 0)


@pytest.mark.parametrize("kind", ["bimodal", "gauss"])
@pytest.mark.parametrize("L,J,h,tiles,hits", [
    (4, 1.0, 1.0, (2, 2, 2), 1),
    (4, 1.0, 2.0, (1, 2, 2), 2),      # Delta E = 0 ties with bimodal fields
    (8, 1.0, 1.5, (4, 2, 2), 3),
    (8, 0.5, 1.0, (2, 4, 2), 1),
    (8, 1.0, 0.6, (8 // 2, 4, 4), 4),
])
def test_zero_temperature_tile_quench_matches_numpy(oracle_mod, kind, L, J, h, tiles, hits):
    f = _fields(kind, L, [62, L])
    o = oracle_mod.Oracle(L, 2, J, h, f, np.array([1e-6, 2e-6]), seed=5)
    o.set_update_order(1, tiles, hits)
    s0 = o.spins()
    o.sweep(4, 0)
    s4 = o.spins()
    for r in range(2):
        assert np.array_equal(s4[r], tile_quench_numpy(s0[r], f, L, J, h, tiles, hits, 4))


def test_tile_quench_is_not_the_plain_quench(oracle_mod):
    """The quench pin above can tell the two orders apart: on these inputs
    the tile order ends in other states than the plain checkerboard."""
    seen = 0
    for L, tiles, hits in [(4, (2, 2, 2), 1), (8, (4, 2, 2), 3), (8, (2, 4, 2), 1)]:
        f = _fields("bimodal", L, [62, L])
        s0 = W.random_spins(1, L, [63, L])[0]
        a = tile_quench_numpy(s0, f, L, 1.0, 1.0, tiles, hits, 4)
        b = quench_numpy(s0, f, L, 1.0, 1.0, 4)
        seen += int(not np.array_equal(a, b))
    assert seen >= 2


L2, N2 = 2, 8
STATES = np.array(list(itertools.product([-1, 1], repeat=N2)), dtype=np.int8)
COLOUR2 = np.array([((i % 2) + (i // 2) % 2 + i // 4) % 2 for i in range(N2)])


def _flip_prob(o, state, i):
    """Fraction of the 2^32 words for which the oracle's decision function
    flips site i of `state` (a bound: binary search over u)."""
    o.set_spins(state.reshape(1, N2))
    if o.accept(0, i, 0xFFFFFFFF):
        return 1.0
    lo, hi = 0, 0xFFFFFFFF
    while lo < hi:
        mid = (lo + hi) // 2
        if o.accept(0, i, mid):
            lo = mid + 1
        else:
            hi = mid
    return lo / 2.0 ** 32


def _site_update_matrix(o, i):
    idx = {tuple(s): q for q, s in enumerate(STATES)}
    P = np.zeros((len(STATES), len(STATES)))
    for q, s in enumerate(STATES):
        p = _flip_prob(o, s, i)
        t = s.copy()
        t[i] = -t[i]
        P[q, idx[tuple(t)]] += p
        P[q, q] += 1.0 - p
    return P


@pytest.mark.parametrize("kind,J,h,T,hits", [("bimodal", 1.0, 1.0, 1.3, 2), ("gauss", 1.0, 1.3, 1.7, 3),
                                             ("bimodal", 0.7, 2.0, 3.0, 5)])
def test_tile_phase_leaves_boltzmann_invariant(oracle_mod, kind, J, h, T, hits):
    """L = 2, tiles of one site: the phase of coarse colour a updates each
    site of colour a `hits` times in a row (its neighbours, of the other
    colour, frozen).  The phase's transition matrix, a product of per-site
    Metropolis matrices to the power `hits`, keeps pi invariant."""
    rng = np.random.default_rng(19)
    f = (np.where(rng.random(N2) < 0.5, -1.0, 1.0) if kind == "bimodal" else rng.standard_normal(N2)).astype(np.float32)
    o = oracle_mod.Oracle(L2, 1, J, h, f, [T], seed=3)
    o.set_update_order(1, (1, 1, 1), hits)
    E = np.array([energy_numpy(s, f, L2, J, h)[0] for s in STATES])
    pi = np.exp(-(E - E.min()) / T)
    pi /= pi.sum()
    for a in (0, 1):
        P = np.eye(len(STATES))
        for i in range(N2):
            if COLOUR2[i] == a:
                P = P @ np.linalg.matrix_power(_site_update_matrix(o, i), hits)
        assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
        assert np.abs(pi @ P - pi).max() / pi.max() < 1e-8


@pytest.mark.parametrize("kind,hits", [("bimodal", 2), ("gauss", 3)])
def test_tile_chain_matches_enumeration(oracle_mod, kind, hits):
    """The oracle's own tile-order chain with exchanges at L = 2 samples the
    Boltzmann distribution of every slot (mean E, M, |M| within 4.5 batch
    standard errors of the enumerated values)."""
    if kind == "bimodal":
        f = np.array([1, -1, -1, 1, 1, 1, -1, 1], dtype=np.float32)
        J, h = 1.0, 1.0
    else:
        f = np.random.default_rng(11).standard_normal(N2).astype(np.float32)
        J, h = 1.0, 1.3
    temps = np.array([1.0, 1.8, 3.0, 5.0])
    R = len(temps)
    Es = np.array([energy_numpy(s, f, L2, J, h)[0] for s in STATES])
    Ms = STATES.astype(np.int64).sum(axis=1)
    o = oracle_mod.Oracle(L2, R, J, h, f, temps, seed=78)
    o.set_update_order(1, (1, 1, 1), hits)
    o.sweep(200, 1)
    n = 60_000
    E = np.zeros((n, R))
    M = np.zeros((n, R))
    for q in range(n):
        o.sweep(1, 1)
        E[q] = o.energies()
        M[q] = o.magnetizations()
    for t, T in enumerate(temps):
        p = np.exp(-(Es - Es.min()) / T)
        p /= p.sum()
        for series, exact in ((E[:, t], Es), (M[:, t], Ms), (np.abs(M[:, t]), np.abs(Ms))):
            want = float((p * exact).sum())
            sem = batch_means_sem(series)
            assert abs(series.mean() - want) <= 4.5 * sem + 1e-12, (t, series.mean(), want, sem)


@pytest.mark.parametrize("tiles,hits,msg", [((3, 2, 2), 1, "even number"), ((8, 2, 2), 1, "even number"),
                                            ((2, 2, 2), 0, "hits")])
def test_tile_order_rejects_bad_arguments(oracle_mod, tiles, hits, msg):
    L = 8
    o = oracle_mod.Oracle(L, 1, 1.0, 1.0, _fields("bimodal", L, [1, 1]), [2.0], seed=1)
    with pytest.raises(RuntimeError, match=msg):
        o.set_update_order(1, tiles, hits)


def test_tile_order_sweep_counter_limit(oracle_mod):
    L = 4
    o = oracle_mod.Oracle(L, 1, 1.0, 1.0, _fields("bimodal", L, [1, 2]), [2.0], seed=1)
    o.set_update_order(1, (2, 2, 2), 1024)
    o.set_counters((1 << 21) - 1, 0)
    o.sweep(1, 0)                       # (t + 1) * hits = 2^31: allowed
    with pytest.raises(RuntimeError, match="hits"):
        o.sweep(1, 0)
