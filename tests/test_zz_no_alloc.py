"""rfim_energies_noalloc, the entry point for callers that cannot allocate,
against rfim_energies on the same configurations, through the C ABI: two
calls in a row on one stream, the second with a smaller input; +-1 fields
bit for bit, Gaussian fields to FP64 rounding (another summation order)."""
import numpy as np
import pytest

from paper_1508_06268_amd import workloads as W

pytestmark = pytest.mark.gpu

J, H = 1.0, 1.5


def _reference(rfim_mod, L, R, kind, key, sweeps):
    """Spins by replica id after `sweeps` sweeps with exchanges, and their
    energies from rfim_energies (by slot) put in replica order."""
    f = W.bimodal_fields(L, key) if kind == "b" else W.gaussian_fields(L, key)
    T = W.geometric_temps(R, 1.0, 6.0) if R > 1 else np.array([2.5])
    g = rfim_mod.Rfim(L, R, J, H, f, T, seed=key[1] + 3)
    g.sweep(sweeps, 5)
    s, E, t2r = g.spins(), g.energies(), g.perm()
    g.close()
    assert sorted(t2r) == list(range(R))
    by_replica = np.empty(R)
    by_replica[t2r] = E
    return f, s, by_replica


def _run_two(rfim_mod, cases):
    import torch

    lib = rfim_mod.load_library()
    stream = torch.cuda.Stream()
    refs, outs, keep = [], [], []
    for (L, R, kind, key, sweeps) in cases:
        f, s, E = _reference(rfim_mod, L, R, kind, key, sweeps)
        ds = torch.from_numpy(np.ascontiguousarray(s, dtype=np.int8)).cuda()
        df = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()
        dE = torch.full((R,), np.nan, dtype=torch.float64, device="cuda")
        keep += [ds, df]
        refs.append(E)
        outs.append(dE)
    torch.cuda.synchronize()
    # both calls queued back to back on one stream, then one synchronization
    for (L, R, _, _, _), ds, df, dE in zip(cases, keep[0::2], keep[1::2], outs):
        rc = lib.rfim_energies_noalloc(L, R, J, H, ds.data_ptr(), df.data_ptr(), dE.data_ptr(), stream.cuda_stream)
        assert rc == 0, rfim_mod.rfim.last_error()
    stream.synchronize()
    return refs, [o.cpu().numpy() for o in outs]


def test_noalloc_energies_equal_rfim_energies_bimodal(rfim_mod):
    refs, got = _run_two(rfim_mod, [(32, 24, "b", [41, 0], 30), (12, 7, "b", [41, 1], 20)])
    for E, G in zip(refs, got):
        assert np.array_equal(G, E), (G, E)


def test_noalloc_energies_match_rfim_energies_gaussian(rfim_mod):
    refs, got = _run_two(rfim_mod, [(16, 9, "g", [42, 0], 25), (6, 3, "g", [42, 1], 10)])
    for E, G in zip(refs, got):
        assert np.allclose(G, E, rtol=1e-12, atol=1e-9), (G, E)
