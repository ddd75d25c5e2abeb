"""Autotuner helpers (CPU): the paper's halo-minimising block (Sec. 3.2,
Eq. 4-5) and the candidate shape lists."""
import math

from paper_1508_06268_amd import autotune


def test_paper_block_shape():
    # V = 2 * 1024 spins, 32-wide warps: x = y = sqrt(V / w) = 8, so the box is
    # 32 x 8 x 8 spins and, with two spins per thread, B_opt = (32, 4, 8)
    w, y, x = autotune.halo_optimal_block(2 * 1024, 32)
    assert (w, y, x) == (32, 8, 8)
    assert (w, y // 2, x) == (32, 4, 8)
    # it is the minimum of the surface at fixed volume
    s_opt = autotune.halo_surface(32, 8, 8)
    for xx in (2, 4, 16, 32):
        yy = 2048 / (32 * xx)
        assert autotune.halo_surface(32, xx, yy) >= s_opt


def test_wave64_analogue_is_not_integral():
    # for 64-wide waves the continuous optimum sqrt(2048 / 64) is not an integer
    assert abs(math.sqrt(2048 / 64) - 5.657) < 1e-3


def test_candidate_shapes():
    for L in (8, 16, 32, 64, 128):
        shapes = autotune.candidate_shapes(L)
        assert shapes, L
        # bit storage is a candidate exactly where it is valid, tried first
        assert ((autotune.MODE_BITS, 0, 0) in shapes) == (L in (64, 128)), L
        if L >= 64:
            assert shapes[0] == (autotune.MODE_BITS, 0, 0)
        for mode, nw, wg in shapes:
            if mode == autotune.MODE_BITS:
                assert (nw, wg) == (0, 0)
                continue
            assert nw in (1, 2, 4, 8) and 4 * nw <= L // 2
            assert mode in (0, 1)
            if mode == 1:
                assert L <= 32
            else:
                chunks = L ** 3 // 8 // nw
                assert chunks % wg == 0 or chunks < wg
        assert len(set(shapes)) == len(shapes)
    assert not any(m == 1 for m, _, _ in autotune.candidate_shapes(64))
