"""GPU parity of the double-checkerboard order with multi-hit updates
(Sec. 3.2, Sec. 5.2; rfim_set_update_order) against the oracle's tile
order: +-1 fields bit for bit (spins, permutation, counters, exchange
statistics, energies) over several tile shapes and hit counts, calls split
anywhere; continuous fields from identical states, decision mismatches
below 1e-6."""
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W
from parity_util import assert_same_state, make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,R,tiles,hits", [
    (16, 4, (8, 8, 8), 1),
    (16, 3, (8, 8, 8), 3),
    (32, 4, (16, 8, 8), 2),
    (32, 3, (8, 8, 8), 5),
    (32, 3, (16, 4, 8), 1),
    (64, 3, (32, 8, 8), 4),
    (64, 2, (32, 4, 16), 2),
])
def test_tile_order_matches_oracle(rfim_mod, oracle_mod, L, R, tiles, hits):
    f = W.bimodal_fields(L, [71, L])
    T = W.linear_temps(R, 2.0, 2.0 + 0.002 * (R - 1) * 64 / L)
    g, o = make_pair(rfim_mod, oracle_mod, L, R, 1.0, 1.5, f, T, seed=hits)
    g.set_update_order(rfim_mod.rfim.ORDER_TILES, tiles, hits)
    o.set_update_order(1, tiles, hits)
    assert g.update_order() == (1, tiles, hits)
    g.sweep(3, 2)           # calls split inside an exchange interval
    g.sweep(3, 2)
    o.sweep(6, 2)
    assert_same_state(g, o, "tiles %s hits %d" % (tiles, hits))
    assert g.exchange_stats()[1].sum() > 0          # exchanges were accepted
    g.close()
    o.close()


def test_tile_order_then_plain_order_continue_the_chain(rfim_mod, oracle_mod):
    """Switching orders mid-run (and the adaptive insertion in tile order)
    keeps the handle on the oracle's chain."""
    L, R = 32, 4
    f = W.bimodal_fields(L, [72, 0])
    T = W.linear_temps(R, 2.0, 2.3)
    g, o = make_pair(rfim_mod, oracle_mod, L, R, 1.0, 1.0, f, T, seed=4, R_cap=6)
    for order, tiles, hits in [(1, (16, 8, 8), 2), (0, (0, 0, 0), 1), (1, (8, 8, 8), 1)]:
        g.set_update_order(order, tiles, hits)
        o.set_update_order(order, tiles, hits)
        g.sweep(4, 2)
        o.sweep(4, 2)
    g.adapt_temps(1, 4, 2, 0.99, 2, 6)
    o.adapt_temps(1, 4, 2, 0.99, 2, 6)
    assert g.R == o.R > R
    assert_same_state(g, o, "mixed orders")
    g.close()
    o.close()


def test_tile_order_continuous_fields_decisions(rfim_mod, oracle_mod):
    """Continuous fields: from identical states one tile sweep (hits 1 and
    2) on the GPU and in the oracle; the spins that end up different are at
    most a few per million decisions."""
    L, R = 64, 8
    f = W.gaussian_fields(L, [73, 0])
    T = W.geometric_temps(R, 1.0, 6.0)
    total = mism = 0
    for hits, tiles in ((1, (32, 8, 8)), (2, (16, 8, 8))):
        g, o = make_pair(rfim_mod, oracle_mod, L, R, 1.0, 2.0, f, T, seed=hits)
        s = W.random_spins(R, L, [74, hits])
        g.set_spins(s)
        o.set_spins(s)
        g.set_update_order(1, tiles, hits)
        o.set_update_order(1, tiles, hits)
        g.sweep(1, 0)
        o.sweep(1, 0)
        total += R * L ** 3 * hits
        mism += int((g.spins() != o.spins()).sum())
        g.close()
        o.close()
    print("tile order, continuous fields: %d decisions, %d spins differ" % (total, mism))
    assert mism / total < 1e-6


def test_tile_order_zero_coupling_equals_plain_sweeps(rfim_mod):
    """J = 0: n tile sweeps with `hits` = 3 equal 3n plain sweeps (same
    words, no interactions), on the GPU alone."""
    L, R = 32, 3
    f = W.gaussian_fields(L, [75, 0])
    T = W.linear_temps(R, 1.0, 3.0)
    a = rfim_mod.Rfim(L, R, 0.0, 1.2, f, T, seed=8)
    b = rfim_mod.Rfim(L, R, 0.0, 1.2, f, T, seed=8)
    a.set_update_order(1, (16, 8, 8), 3)
    a.sweep(4, 0)
    b.sweep(12, 0)
    assert np.array_equal(a.spins(), b.spins())
    a.close()
    b.close()


@pytest.mark.parametrize("L,tiles,hits", [(8, (8, 8, 8), 1), (32, (32, 8, 8), 1), (32, (8, 2, 2), 1),
                                          (32, (12, 8, 8), 1), (32, (16, 8, 8), 0)])
def test_tile_order_rejects_invalid_shapes(rfim_mod, L, tiles, hits):
    f = W.bimodal_fields(L, [76, 0])
    g = rfim_mod.Rfim(L, 2, 1.0, 1.0, f, W.linear_temps(2, 1.0, 2.0), seed=1)
    with pytest.raises(rfim_mod.rfim.RfimError, match="not valid"):
        g.set_update_order(1, tiles, hits)
    assert g.update_order() == (0, (0, 0, 0), 1)
    g.close()


def test_tile_order_sweep_counter_limit(rfim_mod):
    L = 16
    g = rfim_mod.Rfim(L, 1, 1.0, 1.0, W.bimodal_fields(L, [77, 0]), [2.0], seed=1)
    g.set_update_order(1, (8, 8, 8), 1024)
    g.set_counters((1 << 21) - 1, 0)
    g.sweep(1, 0)                       # (t + 1) * hits = 2^31: allowed
    with pytest.raises(rfim_mod.rfim.RfimError, match="2\\^31"):
        g.sweep(1, 0)
    g.close()
