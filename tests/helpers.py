"""Independent plain-numpy formulations used to pin the oracle.  They are
written from the paper's definitions (Eq. 1 and Eq. 3) with array rolls,
not from the oracle's loops."""
import numpy as np


def lattice(s, L):
    """Natural site order i = x + L*(y + L*z) -> array indexed [z, y, x]."""
    return np.asarray(s).reshape(L, L, L)


def energy_numpy(s, fields, L, J, h):
    a = lattice(s, L).astype(np.int64)
    bonds = sum(int((a * np.roll(a, -1, axis=ax)).sum()) for ax in range(3))
    f = lattice(fields, L).astype(np.float64)
    return -J * bonds - h * float((f * a).sum()), bonds


def colour_mask(L):
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    return (x + y + z) % 2


def quench_numpy(s, fields, L, J, h, sweeps):
    """Zero-temperature checkerboard dynamics: colour 0 then colour 1, a spin
    flips iff its flip does not raise the energy (Delta E <= 0)."""
    a = lattice(s, L).astype(np.float64).copy()
    f = lattice(fields, L).astype(np.float64)
    col = colour_mask(L)
    for _ in range(sweeps):
        for c in (0, 1):
            n = sum(np.roll(a, d, axis=ax) for ax in range(3) for d in (1, -1))
            dE = 2.0 * a * (J * n + h * f)
            flip = (col == c) & (dE <= 0)
            a[flip] = -a[flip]
    return a.reshape(-1).astype(np.int8)


def batch_means_sem(x, nb=50):
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // nb
    b = x[: m * nb].reshape(nb, m).mean(axis=1)
    return b.std(ddof=1) / np.sqrt(nb)


def tile_colour_mask(L, tiles):
    """Coarse colour (X + Y + Z) mod 2 of the tile of each site, tiles of
    tx * ty * tz sites, array indexed [z, y, x]."""
    tx, ty, tz = tiles
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    return (x // tx + y // ty + z // tz) % 2


def tile_quench_numpy(s, fields, L, J, h, tiles, hits, sweeps):
    """Zero-temperature double-checkerboard dynamics: per sweep the tiles of
    coarse colour 0, then those of colour 1; a visited tile runs `hits`
    local sweeps (fine colour 0 then 1) in which a spin flips iff its flip
    does not raise the energy.  Tiles of one coarse colour share no face,
    so all of them are updated at once."""
    a = lattice(s, L).astype(np.float64).copy()
    f = lattice(fields, L).astype(np.float64)
    col = colour_mask(L)
    tcol = tile_colour_mask(L, tiles)
    for _ in range(sweeps):
        for coarse in (0, 1):
            for _ in range(hits):
                for c in (0, 1):
                    n = sum(np.roll(a, d, axis=ax) for ax in range(3) for d in (1, -1))
                    dE = 2.0 * a * (J * n + h * f)
                    flip = (tcol == coarse) & (col == c) & (dE <= 0)
                    a[flip] = -a[flip]
    return a.reshape(-1).astype(np.int8)
