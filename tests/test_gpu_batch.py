"""Batched realizations: one launch per (L, field kind) class and a captured
HIP graph per exchange interval.  Each item must reproduce the same
realization run alone, bit for bit (both field kinds), and the +-1 items
must match the oracle."""
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W
from parity_util import assert_same_state

pytestmark = pytest.mark.gpu


def _mix():
    out = []
    specs = [(8, 16, "b"), (16, 8, "g"), (32, 6, "b"), (8, 5, "g"), (16, 12, "b"), (64, 3, "b"),
             (32, 4, "g"), (8, 16, "b")]
    for rho, (L, R, kind) in enumerate(specs):
        f = W.bimodal_fields(L, [30, rho]) if kind == "b" else W.gaussian_fields(L, [30, rho])
        out.append(W.Realization(L=L, R=R, J=1.0, h=1.0 + 0.2 * rho, fields=f,
                                 temps=W.geometric_temps(R, 1.0, 6.0), seed=11, realization=rho,
                                 sweeps=0, every=10))
    return out


def _alone(rfim_mod, w, n, every):
    g = rfim_mod.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization)
    g.sweep(n, every)
    return g


def test_batch_items_equal_single_runs(rfim_mod):
    mix = _mix()
    b = rfim_mod.Batch(mix)
    assert len(b) == len(mix)
    for n, every in ((35, 10), (7, 10), (18, 10)):   # graph replays and ragged segments
        b.sweep(n, every)
    b.synchronize()
    for q, w in enumerate(mix):
        g = _alone(rfim_mod, w, 60, 10)
        it = b.item(q)
        assert np.array_equal(it.spins(), g.spins()), q
        assert np.array_equal(it.perm(), g.perm()), q
        assert it.counters() == g.counters() == (60, 6)
        assert np.array_equal(it.energies(), g.energies()), q
        ga, gc = g.exchange_stats()
        ia, ic = it.exchange_stats()
        assert np.array_equal(ga, ia) and np.array_equal(gc, ic)
        g.close()
    b.close()


def test_batch_bimodal_items_match_oracle(rfim_mod, oracle_mod):
    mix = [w for w in _mix() if w.fields.min() == -1.0 and np.all(np.abs(w.fields) == 1.0)]
    b = rfim_mod.Batch(mix)
    b.sweep(40, 10)
    b.synchronize()
    for q, w in enumerate(mix):
        o = oracle_mod.Oracle(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization)
        o.sweep(40, 10)
        assert_same_state(b.item(q), o, "batch item %d (L=%d)" % (q, w.L))
    b.close()


def test_batch_shapes_do_not_change_results(rfim_mod):
    mix = _mix()
    ref = rfim_mod.Batch(mix)
    ref.sweep(30, 10)
    ref.synchronize()
    alt = rfim_mod.Batch(mix)
    alt.set_shape(8, 0, 0, 1, 64)
    alt.set_shape(16, 1, 0, 2, 128)
    alt.set_shape(32, 0, 1, 4, 1024)
    alt.set_shape(32, 1, 0, 4, 256)
    alt.set_shape(64, 0, 0, 2, 256)
    alt.sweep(30, 10)
    alt.synchronize()
    for q in range(len(mix)):
        assert np.array_equal(ref.item(q).spins(), alt.item(q).spins()), q
        assert np.array_equal(ref.item(q).perm(), alt.item(q).perm()), q
    ref.close()
    alt.close()


def test_batch_items_refuse_standalone_sweeps(rfim_mod):
    b = rfim_mod.Batch(_mix()[:2])
    with pytest.raises(rfim_mod.RfimError):
        b.item(0).sweep(1, 0)
    with pytest.raises(rfim_mod.RfimError):
        b.item(1).adapt_temps(1, 10, 5, 0.5, 1, 20)
    b.close()


def test_every_graph_replay_matches_eager(rfim_mod):
    """The captured interval graph is replayed several times with eager work
    and synchronizations in between; after every replay each item equals the
    same realization advanced eagerly (no graph) one interval at a time."""
    mix = _mix()[:4]
    b = rfim_mod.Batch(mix)
    singles = [rfim_mod.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization)
               for w in mix]
    for rep in range(4):
        b.sweep(10, 10)                       # one graph replay
        b.synchronize()
        for q, g in enumerate(singles):
            g.sweep(10, 10)                   # eager launches
            it = b.item(q)
            assert np.array_equal(it.spins(), g.spins()), (rep, q)
            assert np.array_equal(it.perm(), g.perm()), (rep, q)
            assert np.array_equal(it.energies(), g.energies()), (rep, q)
        if rep == 1:
            b.sweep(3, 10)                    # an eager ragged segment between replays
            b.sweep(7, 10)
            for g in singles:
                g.sweep(10, 10)
    for g in singles:
        g.close()
    b.close()


def test_batch_items_measure_fourier_like_single_runs(rfim_mod):
    """A batch item with the Fourier measurement on gets the same samples as
    the same realization run alone (graph-replayed intervals included)."""
    mix = _mix()[:4]
    b = rfim_mod.Batch(mix)
    b.item(1).set_measure(rfim_mod.MEASURE_FOURIER)
    b.item(2).set_measure(rfim_mod.MEASURE_FOURIER)
    b.sweep(40, 10)
    b.synchronize()
    for q in (1, 2):
        w = mix[q]
        g = rfim_mod.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization)
        g.set_measure(rfim_mod.MEASURE_FOURIER)
        g.sweep(40, 10)
        assert np.array_equal(b.item(q).fourier(), g.fourier()), q
        g.close()
    assert not b.item(0).fourier().any()
    # switched on after the interval graph was captured: the next interval
    # measures it (the graph is captured again)
    b.item(0).set_measure(rfim_mod.MEASURE_FOURIER)
    b.sweep(10, 10)
    w = mix[0]
    g = rfim_mod.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization)
    g.sweep(40, 10)
    g.set_measure(rfim_mod.MEASURE_FOURIER)
    g.sweep(10, 10)
    got = b.item(0).fourier()
    assert np.all(got[:, 0] == 1.0)
    assert np.array_equal(got, g.fourier())
    g.close()
    b.close()


@pytest.mark.parametrize("shape", [(0, 1, 64), (0, 2, 64)])
def test_batch_class_without_fused_energy_matches_single_runs(rfim_mod, oracle_mod, shape):
    """An L=128 class whose streaming shape has more than 1024 workgroups per
    replica: its sweep kernels do not write energy partials, and the batch
    runs the separate energy kernel for its items before the exchange step.
    Items must equal the same realizations run alone (and the oracle for
    +-1 fields), with accepted exchanges in the run: at 2M sites per replica
    the energies of neighbouring replicas differ by thousands, so the ladder
    is spaced by 2e-5 in T for |dbeta dE| to stay well below one."""
    specs = []
    for rho, kind in enumerate(("b", "g", "b")):
        L, R = 128, 3
        f = W.bimodal_fields(L, [31, rho]) if kind == "b" else W.gaussian_fields(L, [31, rho])
        specs.append(W.Realization(L=L, R=R, J=1.0, h=1.0, fields=f, temps=np.array([2.0, 2.00002, 2.00004]),
                                   seed=12, realization=rho, sweeps=0, every=2))
    b = rfim_mod.Batch(specs)
    b.set_shape(128, 0, *shape)
    b.set_shape(128, 1, *shape)
    b.sweep(6, 2)
    b.synchronize()
    accepted = 0
    for q, w in enumerate(specs):
        g = rfim_mod.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization)
        g.set_launch_shape(*shape)
        g.sweep(6, 2)
        it = b.item(q)
        assert np.array_equal(it.spins(), g.spins()), q
        assert np.array_equal(it.perm(), g.perm()), q
        assert np.array_equal(it.energies(), g.energies()), q
        accepted += int(it.exchange_stats()[1].sum())
        if q % 2 == 0:
            o = oracle_mod.Oracle(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization)
            o.sweep(6, 2)
            assert_same_state(it, o, "non-fused batch item %d" % q)
            o.close()
        g.close()
    assert accepted > 0
    b.close()


def test_large_streaming_class_in_groups_equals_single_runs(rfim_mod):
    """A streaming class larger than twice the group budget runs as two lanes
    of groups of consecutive items, each group all sweeps of an interval
    before the next on its stream: 7 realizations of L=64, R=128 (32 MiB of
    byte spins each) form groups of 3, 3 and 1, the lanes [3] and [3, 1].
    Every item equals the same realization run alone, both field kinds,
    with accepted exchanges.  (Byte shapes set here: classes at L=64 start
    in bit storage.)"""
    specs = []
    for rho in range(7):
        L, R = 64, 128
        f = W.bimodal_fields(L, [33, rho]) if rho % 2 == 0 else W.gaussian_fields(L, [33, rho])
        specs.append(W.Realization(L=L, R=R, J=1.0, h=1.0, fields=f,
                                   temps=W.linear_temps(R, 4.0, 4.0 + 0.0002 * (R - 1)), seed=13,
                                   realization=rho, sweeps=0, every=3))
    B = rfim_mod.rfim
    b = rfim_mod.Batch(specs)
    for kind in (B.FIELDS_BIMODAL, B.FIELDS_CONTINUOUS):
        b.set_shape(64, kind, 0, 4, 128)
    assert b.group_bytes() == 96 << 20
    b.sweep(3, 3)            # graph capture or eager, whichever the batch takes
    b.sweep(6, 3)
    b.synchronize()
    flat = rfim_mod.Batch(specs)
    for kind in (B.FIELDS_BIMODAL, B.FIELDS_CONTINUOUS):
        flat.set_shape(64, kind, 0, 4, 128)
    flat.set_group_bytes(0)  # no temporal blocking: every half-sweep over the whole class
    flat.sweep(9, 3)
    flat.synchronize()
    with pytest.raises(rfim_mod.rfim.RfimError):
        flat.set_group_bytes(1000)
    accepted = 0
    for q, w in enumerate(specs):
        g = rfim_mod.Rfim(w.L, w.R, w.J, w.h, w.fields, w.temps, seed=w.seed, realization=w.realization)
        g.sweep(9, 3)
        it = b.item(q)
        assert np.array_equal(it.spins(), g.spins()), q
        assert np.array_equal(it.perm(), g.perm()), q
        assert np.allclose(it.energies(), g.energies(), rtol=1e-12, atol=1e-9), q
        assert np.array_equal(flat.item(q).spins(), g.spins()), q
        accepted += int(it.exchange_stats()[1].sum())
        g.close()
    assert accepted > 0
    b.close()
    flat.close()


def _l64_mix(Rs, tag):
    """L=64 items of both field kinds with the given replica counts, and one
    small L=16 item beside them."""
    out = []
    for rho, (R, kind) in enumerate([(R, "b") for R in Rs] + [(R, "g") for R in Rs] + [(8, "g")]):
        L = 16 if rho == 2 * len(Rs) else 64
        f = W.bimodal_fields(L, [tag, rho]) if kind == "b" else W.gaussian_fields(L, [tag, rho])
        out.append(W.Realization(L=L, R=R, J=1.0, h=1.5 + 0.25 * rho, fields=f,
                                 temps=W.geometric_temps(R, 1.0, 6.0), seed=13, realization=rho,
                                 sweeps=0, every=10))
    return out


@pytest.mark.parametrize("Rs", [(4, 6), (128,), (128, 96)])
def test_bit_storage_class_equals_single_runs(rfim_mod, Rs):
    """A class in bit storage (MODE_BITS): its items are swept item by item
    on one lane, or on two lanes (one item's replica halves for Rs = (128,),
    the items themselves for (128, 96)).  Each item equals the same
    realization run alone, bit for bit, also after the class goes back to a
    byte shape."""
    B = rfim_mod.rfim
    mix = _l64_mix(Rs, 31)
    b = rfim_mod.Batch(mix)
    for kind in (B.FIELDS_BIMODAL, B.FIELDS_CONTINUOUS):
        b.set_shape(64, kind, rfim_mod.MODE_BITS, 0, 0)
    for q, w in enumerate(mix):
        it = b.item(q)
        want = (B.SPINS_BITS, (rfim_mod.MODE_BITS, 0, 0)) if w.L == 64 else (B.SPINS_BYTES, it.launch_shape())
        assert (it.spin_storage(), it.launch_shape()) == want, q
    for n, every in ((25, 10), (7, 10), (8, 10)):       # graph replays and ragged segments
        b.sweep(n, every)
    b.synchronize()
    singles = []
    for q, w in enumerate(mix):
        g = _alone(rfim_mod, w, 40, 10)
        it = b.item(q)
        assert np.array_equal(it.spins(), g.spins()), q
        assert np.array_equal(it.perm(), g.perm()), q
        assert it.counters() == g.counters() == (40, 4)
        assert np.array_equal(it.energies(), g.energies()), q      # both in bit storage at L=64
        assert np.array_equal(it.exchange_stats()[1], g.exchange_stats()[1]), q
        singles.append(g)
    for kind in (B.FIELDS_BIMODAL, B.FIELDS_CONTINUOUS):
        b.set_shape(64, kind, 0, 4, 128)
    b.sweep(10, 10)
    b.synchronize()
    for q, (w, g) in enumerate(zip(mix, singles)):
        it = b.item(q)
        if w.L == 64:
            assert (it.spin_storage(), it.launch_shape()) == (B.SPINS_BYTES, (0, 4, 128)), q
        g.sweep(10, 10)
        assert np.array_equal(it.spins(), g.spins()), q
        assert np.array_equal(it.perm(), g.perm()), q
        assert np.allclose(it.energies(), g.energies(), rtol=1e-12, atol=1e-9), q
        g.close()
    b.close()


def test_bit_storage_class_shape_checks(rfim_mod):
    """Bit storage needs L = 64, 128 or 256 and the shape (MODE_BITS, 0, 0);
    its items refuse the Fourier measurement and a storage switch of their
    own (the class shape decides)."""
    B = rfim_mod.rfim
    mix = _l64_mix((2,), 32)
    b = rfim_mod.Batch(mix)
    # the default: bit storage at L=64, the resident shape at L=16
    assert [b.item(q).spin_storage() for q in range(3)] == [B.SPINS_BITS, B.SPINS_BITS, B.SPINS_BYTES]
    assert b.item(1).launch_shape() == (rfim_mod.MODE_BITS, 0, 0)
    b.set_shape(64, B.FIELDS_BIMODAL, 0, 4, 128)
    assert b.item(0).spin_storage() == B.SPINS_BYTES
    with pytest.raises(B.RfimError):
        b.set_shape(16, B.FIELDS_CONTINUOUS, rfim_mod.MODE_BITS, 0, 0)
    with pytest.raises(B.RfimError):
        b.set_shape(64, B.FIELDS_BIMODAL, rfim_mod.MODE_BITS, 4, 128)
    b.set_shape(64, B.FIELDS_BIMODAL, rfim_mod.MODE_BITS, 0, 0)
    it = b.item(0)
    with pytest.raises(B.RfimError):
        it.set_measure(rfim_mod.MEASURE_FOURIER)
    with pytest.raises(B.RfimError):
        it.set_spin_storage(B.SPINS_BYTES)
    assert it.spin_storage() == B.SPINS_BITS
    b.sweep(10, 10)
    b.synchronize()
    g = _alone(rfim_mod, mix[0], 10, 10)
    assert np.array_equal(it.spins(), g.spins())
    g.close()
    b.close()
