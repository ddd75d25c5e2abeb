"""GPU parity of the slab shapes (modes 2..4: nw slabs per replica, mode - 1
sweeps per launch with the halo recomputed): the plain order's chain, so +-1
fields follow the oracle bit for bit and continuous fields follow the other
shapes' chain (same FP32 decisions; energies to FP64 rounding)."""
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W
from parity_util import assert_same_state, make_pair

pytestmark = pytest.mark.gpu

CASES = [(16, 4, (2, 4, 256)), (16, 3, (3, 2, 128)), (16, 3, (4, 8, 512)), (32, 4, (3, 4, 512)),
         (32, 3, (2, 8, 1024)), (32, 3, (4, 2, 1024)), (32, 2, (4, 4, 1024)), (32, 5, (3, 4, 1024))]


@pytest.mark.parametrize("L,R,shape", CASES)
def test_slabs_match_oracle(rfim_mod, oracle_mod, L, R, shape):
    f = W.bimodal_fields(L, [91, L])
    T = W.linear_temps(R, 2.0, 2.0 + 0.002 * (R - 1) * (64 / L) ** 1.5)
    g, o = make_pair(rfim_mod, oracle_mod, L, R, 1.0, 1.5, f, T, seed=shape[0] + 10 * shape[1], R_cap=R + 2)
    g.set_launch_shape(*shape)
    assert g.launch_shape() == shape
    g.sweep(4, 3)           # intervals of 3 sweeps: launches of mode - 1 sweeps end ragged
    g.sweep(5, 3)
    o.sweep(9, 3)
    assert_same_state(g, o, "slabs L=%d shape %s" % (L, shape))
    assert g.exchange_stats()[1].sum() > 0
    g.adapt_temps(1, 3, 3, 0.999, 2, R + 2)
    o.adapt_temps(1, 3, 3, 0.999, 2, R + 2)
    g.sweep(3, 3)
    o.sweep(3, 3)
    assert_same_state(g, o, "slabs L=%d shape %s after insertion" % (L, shape))
    g.close()
    o.close()


@pytest.mark.parametrize("L,R,shape", [(32, 8, (3, 4, 1024)), (16, 6, (2, 4, 512)), (32, 3, (2, 2, 1024)),
                                       (32, 4, (4, 4, 1024))])
def test_slabs_continuous_fields_equal_default_shape(rfim_mod, L, R, shape):
    f = W.gaussian_fields(L, [92, L])
    T = W.geometric_temps(R, 1.0, 6.0)
    a = rfim_mod.Rfim(L, R, 1.0, 2.0, f, T, seed=4)
    b = rfim_mod.Rfim(L, R, 1.0, 2.0, f, T, seed=4)
    b.set_launch_shape(*shape)
    a.sweep(10, 5)
    b.sweep(10, 5)
    assert np.array_equal(a.spins(), b.spins())
    assert np.array_equal(a.perm(), b.perm())
    assert np.allclose(a.energies(), b.energies(), rtol=1e-12, atol=1e-9)
    a.close()
    b.close()


def test_slab_shapes_validated(rfim_mod):
    L = 32
    f = W.bimodal_fields(L, [93, 0])
    g = rfim_mod.Rfim(L, 2, 1.0, 1.0, f, [1.0, 2.0], seed=1)
    # 16 slabs of 2 planes; 1 slab; workgroup of 64; 4 sweeps per launch;
    # more than two positions per thread
    for bad in [(2, 16, 256), (4, 1, 256), (2, 4, 64), (5, 4, 256), (3, 4, 256)]:
        with pytest.raises(rfim_mod.rfim.RfimError, match="not valid"):
            g.set_launch_shape(*bad)
    g.close()
    g = rfim_mod.Rfim(64, 2, 1.0, 1.0, W.bimodal_fields(64, [93, 1]), [1.0, 2.0], seed=1)
    with pytest.raises(rfim_mod.rfim.RfimError, match="not valid"):
        g.set_launch_shape(2, 8, 1024)        # slabs are for L = 16 and 32
    g.close()
    spec = W.Realization(L=L, R=2, J=1.0, h=1.0, fields=f, temps=np.array([1.0, 2.0]), seed=1, realization=0,
                         sweeps=0, every=1)
    b = rfim_mod.Batch([spec])
    with pytest.raises(rfim_mod.rfim.RfimError, match="single realizations"):
        b.set_shape(L, 0, 2, 4, 256)
    b.close()


def test_slabs_fourier_measurement_reads_the_current_buffer(rfim_mod):
    """The slab launches alternate two spin buffers; the per-exchange Fourier
    measurement must read the one that holds the current configuration."""
    L, R = 32, 4
    f = W.bimodal_fields(L, [94, 0])
    T = W.linear_temps(R, 3.0, 5.0)
    a = rfim_mod.Rfim(L, R, 1.0, 1.0, f, T, seed=6)
    b = rfim_mod.Rfim(L, R, 1.0, 1.0, f, T, seed=6)
    b.set_launch_shape(2, 4, 1024)          # one sweep per launch: a swap per sweep
    for h in (a, b):
        h.set_measure(rfim_mod.rfim.MEASURE_FOURIER)
        h.sweep(7, 7)                       # odd number of launches before the step
        h.sweep(6, 3)
    assert np.array_equal(a.spins(), b.spins())
    assert np.array_equal(a.fourier(), b.fourier())
    a.close()
    b.close()
