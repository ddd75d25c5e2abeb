"""Host-side estimators of the paper's observables (Eq. 11-13) from
per-slot sums, checked on sums built from known samples."""
import numpy as np
import pytest

from paper_1508_06268_amd import observables as ob


def _sums(E, M):
    E = np.asarray(E, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    return np.array([len(E), E.sum(), (E * E).sum(), np.abs(M).sum(), (M * M).sum(), (M ** 4).sum()])


def test_thermal_from_samples():
    rng = np.random.default_rng(0)
    N = 512
    E = rng.normal(-800, 20, size=(3, 1000))
    M = rng.integers(-N, N, size=(3, 1000))
    obs = np.stack([_sums(E[t], M[t]) for t in range(3)])
    T = np.array([1.0, 2.0, 3.0])
    th = ob.thermal(obs, T, N)
    assert np.allclose(th["E"], E.mean(axis=1) / N)
    assert np.allclose(th["C"], E.var(axis=1) / (N * T * T))
    assert np.allclose(th["absm"], np.abs(M).mean(axis=1) / N)


def test_binder_limits():
    # fully ordered: M = +-N always -> g = 1; Gaussian M -> g = 0
    N = 1000
    T = np.array([1.0])
    ordered = ob.thermal(np.stack([_sums(np.zeros(100), np.full(100, N))]), T, N)
    gauss = np.random.default_rng(1).normal(0, 30, 200000)
    disordered = ob.thermal(np.stack([_sums(np.zeros(gauss.size), gauss)]), T, N)
    assert ob.disorder_average([ordered])["g"][0] == pytest.approx(1.0)
    assert abs(ob.disorder_average([disordered])["g"][0]) < 0.02


def test_crossing():
    T = np.array([1.0, 2.0, 3.0, 4.0])
    assert ob.crossing(T, [4, 3, 2, 1], [1, 2, 3, 4]) == pytest.approx(2.5)
    assert ob.crossing(T, [1, 1, 1, 1], [0, 0, 0, 0]) is None


def test_correlation_length_of_an_ornstein_zernike_form():
    """With chi(k) = chi0 / (1 + xi^2 4 sin^2(k/2)), <M^2>/N = chi0 and
    <F> = chi(2 pi / L) give back xi; xi_paper lacks the 2 sin(pi/L)."""
    L = 16
    N = L ** 3
    xi = np.array([0.5, 2.0, 5.0])
    chi0 = np.array([3.0, 40.0, 400.0])
    F = chi0 / (1.0 + xi ** 2 * 4 * np.sin(np.pi / L) ** 2)
    n = 1000.0
    obs = np.zeros((3, 6))
    obs[:, 0] = n
    obs[:, 4] = n * chi0 * N          # sum of M^2
    obs[:, 5] = n * (chi0 * N) ** 2   # any positive M^4
    fo = np.stack([np.full(3, n), n * F], axis=1)
    th = ob.thermal(obs, np.array([1.0, 2.0, 3.0]), N, fourier=fo)
    assert np.allclose(th["xi"], xi)
    assert np.allclose(th["xi_paper"], xi * 2 * np.sin(np.pi / L))
    avg = ob.disorder_average([th, th])
    assert np.allclose(avg["xi"], xi)
