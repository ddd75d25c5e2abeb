"""The oracle's use of its random stream, replayed decision by decision
from the (separately pinned) Philox block function: initial spins, the
per-site sweep word, and the strict "u32 < threshold" acceptance boundary.
These conventions are the project's own (the paper names no generator); the
HIP path must reproduce them bit for bit."""
import math

import numpy as np

from paper_1508_06268_amd import workloads as W
from helpers import lattice, colour_mask

TAG_INIT, TAG_SWEEP = 1, 2


def _words(oracle_mod, seed, c0, c1, c2, tag, rho=0):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    return oracle_mod.philox4x32_10([c0, c1, c2, (tag << 28) | rho], key)


def test_initial_spins_follow_init_stream(oracle_mod):
    L, R, seed, rho = 4, 3, 0x123456789ABCDEF, 5
    f = W.bimodal_fields(L, [0, 0])
    o = oracle_mod.Oracle(L, R, 1.0, 1.0, f, [1.0, 2.0, 3.0], seed=seed, realization=rho)
    s = o.spins()
    for r in range(R):
        for i in range(L ** 3):
            w = _words(oracle_mod, seed, i >> 2, 0, r, TAG_INIT, rho)[i & 3]
            assert s[r, i] == (1 if w >= 2 ** 31 else -1)
    big = oracle_mod.Oracle(16, 1, 1.0, 1.0, W.bimodal_fields(16, [0, 1]), [1.0])
    m = big.spins().astype(np.float64).mean()
    assert abs(m) < 5 / np.sqrt(16 ** 3)


def _site_class(s_lat, f_lat, z, y, x):
    L = s_lat.shape[0]
    si = s_lat[z, y, x]
    n = (s_lat[z, y, (x + 1) % L] + s_lat[z, y, (x - 1) % L] + s_lat[z, (y + 1) % L, x]
         + s_lat[z, (y - 1) % L, x] + s_lat[(z + 1) % L, y, x] + s_lat[(z - 1) % L, y, x])
    k = (si * n + 6) // 2
    fb = 1 if si * f_lat[z, y, x] > 0 else 0
    return 2 * k + fb


def test_sweep_replay_and_strict_boundary(oracle_mod):
    """Replay colour-0 decisions of sweep 0 from the words, with one
    temperature tuned so that the threshold of one site equals its word
    exactly: "<" must reject it, and one step up must accept it."""
    L, seed = 4, 42
    f = W.bimodal_fields(L, [5, 5])
    J, h = 1.0, 1.0
    base = oracle_mod.Oracle(L, 1, J, h, f, [3.0], seed=seed)
    s0 = base.spins()[0]
    s_lat, f_lat = lattice(s0, L), lattice(f, L)
    col = colour_mask(L)
    # first colour-0 site whose move is uphill
    target = None
    for j in range(L ** 3 // 2):
        i0 = 2 * j
        z, y, x = i0 // (L * L), (i0 // L) % L, i0 % L
        i = i0 if col[z, y, x] == 0 else i0 + 1
        z, y, x = i // (L * L), (i // L) % L, i % L
        cls = _site_class(s_lat, f_lat, z, y, x)
        dE = 2 * (J * (2 * (cls >> 1) - 6) + h * (2 * (cls & 1) - 1))
        if dE > 0:
            target = (j, i, cls, dE)
            break
    j, i, cls, dE = target
    u = int(_words(oracle_mod, seed, j >> 2, 0, 0, TAG_SWEEP)[j & 3])
    for offset, flips in ((0, False), (1, True)):
        want_thr = u + offset
        T = -dE / math.log((want_thr + 0.5) / 2 ** 32)
        o = oracle_mod.Oracle(L, 1, J, h, f, [T], seed=seed)
        thr, _ = o.thresholds()
        assert int(thr[0, cls]) == want_thr
        o.sweep(1, 0)
        after = o.spins()[0]
        # colour-0 sites decided on the initial state: replay every one
        thr_row = thr[0]
        for jj in range(L ** 3 // 2):
            i0 = 2 * jj
            zz, yy, xx = i0 // (L * L), (i0 // L) % L, i0 % L
            ii = i0 if col[zz, yy, xx] == 0 else i0 + 1
            zz, yy, xx = ii // (L * L), (ii // L) % L, ii % L
            c = _site_class(s_lat, f_lat, zz, yy, xx)
            dd = 2 * (J * (2 * (c >> 1) - 6) + h * (2 * (c & 1) - 1))
            w = int(_words(oracle_mod, seed, jj >> 2, 0, 0, TAG_SWEEP)[jj & 3])
            acc = dd <= 0 or w < int(thr_row[c])
            # a colour-0 site is not touched again by the colour-1 half-sweep
            assert (after[ii] != s0[ii]) == acc, (jj, ii)
        assert (after[i] != s0[i]) == flips


ZERO_WORD_CASES = [(8, 4320, 153, 0, 0, 205), (6, 8188, 225, 0, 2, 2)]


def test_zero_words_land_on_never_classes(oracle_mod):
    """The seeds the GPU never-class test uses: the sweep word of (t, c, r,
    j) is 0, and at the frozen temperatures that site's move is uphill with
    threshold 0, so "u < threshold" refuses it even for u = 0."""
    for L, seed, t, c, r, j in ZERO_WORD_CASES:
        assert int(_words(oracle_mod, seed, j >> 2, 2 * t + c, r, TAG_SWEEP)[j & 3]) == 0
        f = W.bimodal_fields(L, [7, L, 0])
        o = oracle_mod.Oracle(L, 4, 1.0, 1.0, f, [0.05, 0.06, 0.07, 0.08], seed=seed)
        o.sweep(t, 10)
        i0 = 2 * j
        z, y, x = i0 // (L * L), (i0 // L) % L, i0 % L
        i = i0 if (x + y + z) % 2 == c else i0 + 1
        before = o.spins()[r, i]
        dE = o.flip_delta(r, i)
        assert dE > 0
        thr, always = o.thresholds()
        slot = int(np.argwhere(o.perm() == r)[0, 0])
        s_lat, f_lat = lattice(o.spins()[r], L), lattice(f, L)
        cls = _site_class(s_lat, f_lat, i // (L * L), (i // L) % L, i % L)
        assert not always[cls] and int(thr[slot, cls]) == 0
        o.sweep(1, 10)
        assert o.spins()[r, i] == before
