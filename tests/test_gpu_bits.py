"""GPU parity of one-bit-per-spin storage (rfim_set_spin_storage): the bit
sweep takes the same decisions with the same random words, so +-1 fields
follow the oracle's chain bit for bit (spins, permutation, counters,
exchange statistics, energies) and continuous fields follow the byte
sweep's chain (same FP32 decisions; energies to FP64 rounding, another
summation order)."""
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W
from parity_util import assert_same_state, make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,R,concurrency", [(64, 6, 1), (64, 64, 0), (128, 3, 2), (64, 5, 2)])
def test_bits_match_oracle(rfim_mod, oracle_mod, L, R, concurrency):
    f = W.bimodal_fields(L, [81, L])
    T = W.linear_temps(R, 2.0, 2.0 + 0.001 * (R - 1) * 64 / L) if R < 16 else W.linear_temps(R, 1.0, 6.0)
    g, o = make_pair(rfim_mod, oracle_mod, L, R, 1.0, 1.5, f, T, seed=R)
    g.set_concurrency(concurrency)
    g.set_spin_storage(rfim_mod.rfim.SPINS_BITS)
    assert g.spin_storage() == rfim_mod.rfim.SPINS_BITS
    g.sweep(3, 2)           # split inside an exchange interval
    g.sweep(4, 2)
    o.sweep(7, 2)
    assert_same_state(g, o, "bits L=%d R=%d" % (L, R))
    assert g.exchange_stats()[1].sum() > 0
    g.close()
    o.close()


def test_bits_adaptive_insertion_and_storage_switches(rfim_mod, oracle_mod):
    """Insertion in bit storage (the new replica copies its colder
    neighbour's bits), spins written and read in bit storage, and switching
    storage mid-run keep the oracle's chain."""
    L, R = 64, 4
    f = W.bimodal_fields(L, [82, 0])
    T = W.linear_temps(R, 2.0, 2.1)      # spaced so that some pair rates fall below the threshold
    g, o = make_pair(rfim_mod, oracle_mod, L, R, 1.0, 1.0, f, T, seed=5, R_cap=7)
    g.set_spin_storage(1)
    g.sweep(4, 2)
    o.sweep(4, 2)
    s = W.random_spins(R, L, [83, 0])
    g.set_spins(s)
    o.set_spins(s)
    g.adapt_temps(1, 4, 2, 0.999, 3, 7)
    o.adapt_temps(1, 4, 2, 0.999, 3, 7)
    assert g.R == o.R > R
    assert_same_state(g, o, "after insertion in bit storage")
    g.set_spin_storage(0)
    g.sweep(2, 2)
    o.sweep(2, 2)
    g.set_spin_storage(1)
    g.sweep(3, 2)
    o.sweep(3, 2)
    assert_same_state(g, o, "after storage switches")
    g.close()
    o.close()


@pytest.mark.parametrize("L,R", [(64, 8), (128, 4), (256, 2)])
def test_bits_continuous_fields_equal_byte_sweep(rfim_mod, L, R):
    """Continuous fields: the bit sweep and the byte sweep take the same FP32
    decisions on the same words, so their chains agree exactly (energies
    to FP64 rounding)."""
    f = W.gaussian_fields(L, [84, L])
    T = W.geometric_temps(R, 1.0, 6.0)
    a = rfim_mod.Rfim(L, R, 1.0, 2.0, f, T, seed=3)
    b = rfim_mod.Rfim(L, R, 1.0, 2.0, f, T, seed=3)
    a.set_spin_storage(rfim_mod.rfim.SPINS_BYTES)      # L = 64..256 start in bits
    b.set_spin_storage(rfim_mod.rfim.SPINS_BITS)
    assert a.spin_storage() == rfim_mod.rfim.SPINS_BYTES
    a.sweep(6, 3)
    b.sweep(6, 3)
    assert np.array_equal(a.spins(), b.spins())
    assert np.array_equal(a.perm(), b.perm())
    assert np.allclose(a.energies(), b.energies(), rtol=1e-12, atol=1e-9)
    a.close()
    b.close()


def test_bits_l256_equal_byte_sweep(rfim_mod):
    """+-1 fields at L = 256 (four words per row): the bit chain equals the
    byte chain, which the oracle pins at smaller L."""
    L, R = 256, 2
    f = W.bimodal_fields(L, [85, 0])
    T = np.array([2.0, 2.00001])
    a = rfim_mod.Rfim(L, R, 1.0, 1.0, f, T, seed=9)
    b = rfim_mod.Rfim(L, R, 1.0, 1.0, f, T, seed=9)
    a.set_spin_storage(rfim_mod.rfim.SPINS_BYTES)      # +-1 fields at L = 256 start in bits
    b.set_spin_storage(rfim_mod.rfim.SPINS_BITS)
    assert a.spin_storage() == rfim_mod.rfim.SPINS_BYTES
    a.sweep(4, 2)
    b.sweep(4, 2)
    assert np.array_equal(a.spins(), b.spins())
    assert np.array_equal(a.perm(), b.perm())
    assert np.array_equal(a.energies(), b.energies())
    assert np.array_equal(a.exchange_stats()[1], b.exchange_stats()[1])
    a.close()
    b.close()


@pytest.mark.parametrize("L", [32, 48])
def test_bits_refuse_unsupported_sizes(rfim_mod, L):
    g = rfim_mod.Rfim(L, 2, 1.0, 1.0, W.bimodal_fields(L, [86, L]), [1.0, 2.0], seed=1)
    with pytest.raises(rfim_mod.rfim.RfimError, match="L = 64, 128 or 256"):
        g.set_spin_storage(1)
    assert g.spin_storage() == 0
    g.close()


def test_default_storage_and_switches_to_bytes(rfim_mod):
    """Both field kinds start in bits at L = 64..256 and in bytes at other
    L; a launch shape, the Fourier measurement or the tile order switch a
    handle to bytes."""
    B = rfim_mod.rfim
    for L, kind, want in ((64, "b", 1), (128, "b", 1), (64, "g", 1), (128, "g", 1), (32, "b", 0), (32, "g", 0)):
        f = W.bimodal_fields(L, [88, L]) if kind == "b" else W.gaussian_fields(L, [88, L])
        g = rfim_mod.Rfim(L, 2, 1.0, 1.0, f, [1.0, 2.0], seed=1)
        assert g.spin_storage() == want, (L, kind)
        g.close()
    L = 64
    f = W.bimodal_fields(L, [87, 0])
    for switch in ("shape", "measure", "tiles"):
        g = rfim_mod.Rfim(L, 2, 1.0, 1.0, f, [1.0, 2.0], seed=1)
        assert g.spin_storage() == B.SPINS_BITS
        if switch == "shape":
            g.set_launch_shape(0, 4, 128)
        elif switch == "measure":
            g.set_measure(rfim_mod.MEASURE_FOURIER)
        else:
            g.set_update_order(B.ORDER_TILES, (32, 8, 8), 2)
        assert g.spin_storage() == B.SPINS_BYTES, switch
        if switch != "shape":       # bits refuse the measurement and the tile order
            with pytest.raises(B.RfimError):
                g.set_spin_storage(B.SPINS_BITS)
        g.close()


@pytest.mark.parametrize("storage", ["bits", "bytes"])
def test_zero_word_on_a_never_class_at_l64(rfim_mod, oracle_mod, storage):
    """The zero word of seed 4320 (sweep 153, colour 0, replica 0,
    sublattice index 205; the counter does not depend on L) lands at L=64 on
    site 410 while it sits in a class whose bound is 0 at T = 0.05 (dE = 2):
    the bit sweep and the byte sweep must both refuse it, as the oracle
    does.  The state is compared right after sweep 153."""
    L, seed, t, c, r, j = 64, 4320, 153, 0, 0, 205
    i = 2 * j                                   # the colour-0 site of the pair (x + y + z even)
    assert ((i % L) + (i // L) % L + i // (L * L)) % 2 == c
    f = W.bimodal_fields(L, [7, L, 0])
    T = np.array([0.05, 0.06, 0.07, 0.08])
    o = oracle_mod.Oracle(L, 4, 1.0, 1.0, f, T, seed=seed)
    o.sweep(t, 10)
    w = oracle_mod.philox4x32_10([j >> 2, 2 * t + c, r, 2 << 28], [seed & 0xFFFFFFFF, seed >> 32])
    assert w[j & 3] == 0
    assert o.flip_delta(r, i) > 0 and not o.accept(r, i, 0)
    o.sweep(1, 10)
    g = rfim_mod.Rfim(L, 4, 1.0, 1.0, f, T, seed=seed)
    if storage == "bytes":
        g.set_spin_storage(rfim_mod.rfim.SPINS_BYTES)
    assert g.spin_storage() == (rfim_mod.rfim.SPINS_BITS if storage == "bits" else rfim_mod.rfim.SPINS_BYTES)
    g.sweep(t + 1, 10)
    assert_same_state(g, o, "L=64 zero word, %s" % storage)
    g.close()
    o.close()
