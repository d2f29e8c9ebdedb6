"""Pins of the oracle's transform conventions (CPU only)."""
import numpy as np
import pytest

from oracle import spectral as sp


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 6, 6), (10, 10, 10), (12, 12, 12), (6, 8, 10), (7, 14, 8), (14, 7, 14)])
def test_rfft3_matches_brute_force_dft(shape):
    rng = np.random.default_rng(1)
    u = rng.standard_normal(shape)
    ref = sp.brute_rdft3(u)
    got = sp.rfft3(u)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.sqrt(np.sum(u * u)) * np.sqrt(u.size)


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 10, 8), (14, 7, 14)])
def test_irfft3_matches_brute_force_inverse(shape):
    rng = np.random.default_rng(2)
    u = rng.standard_normal(shape)
    U = sp.rfft3(u)
    back = sp.brute_irdft3(U, shape)
    assert np.max(np.abs(back - u)) <= 1e-13
    assert np.max(np.abs(sp.irfft3(U, shape) - u)) <= 1e-14


def test_odd_size_15_matches_brute_force():
    rng = np.random.default_rng(3)
    u = rng.standard_normal((15, 15, 15))
    U = sp.rfft3(u)
    # brute force along each axis (separable definition), cheaper than the full matrix
    def dft(n, half=False):
        k = np.arange(n // 2 + 1 if half else n)[:, None]
        return np.exp(-2j * np.pi * k * np.arange(n)[None, :] / n)
    ref = np.einsum("az,by,cx,zyx->abc", dft(15), dft(15), dft(15, True), u)
    assert np.max(np.abs(U - ref)) <= 1e-13 * np.sqrt(np.sum(u * u)) * np.sqrt(u.size)


@pytest.mark.parametrize("m", [(1, 0, 0), (0, 3, 0), (2, 1, 5), (4, 4, 4), (0, 0, 4)])
def test_single_cosine_lands_in_its_bins(m):
    n = 8
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    u = np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / n)
    U = sp.rfft3(u)
    mask = np.zeros(U.shape, bool)
    for sgn in (1, -1):
        kx, ky, kz = (sgn * m[0]) % n, (sgn * m[1]) % n, (sgn * m[2]) % n
        if kx <= n // 2:
            mask[kz, ky, kx] = True
    assert np.max(np.abs(U[~mask])) <= 1e-12
    # amplitude: N^3/2 per bin, N^3 if the mode is its own conjugate
    vals = np.abs(U[mask])
    self_conj = all((2 * q) % n == 0 for q in m)
    expect = n ** 3 if self_conj else n ** 3 / 2
    assert np.allclose(vals, expect, rtol=1e-13)


def test_parseval_with_multiplicity():
    rng = np.random.default_rng(4)
    shape = (8, 12, 10)
    u = rng.standard_normal(shape)
    U = sp.rfft3(u)
    lhs = np.sum(u * u)
    rhs = np.sum(sp.multiplicity(shape) * np.abs(U) ** 2) / np.prod(shape)
    assert abs(lhs - rhs) <= 1e-12 * lhs


@pytest.mark.parametrize("m", [(1, 0, 0), (2, 3, 1), (0, 0, 4)])
def test_spectral_laplacian_and_biharmonic_eigenvalues(m):
    n, dx = 16, 0.7
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    arg = 2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / n
    u = np.sin(arg + 0.3)
    k2 = sum((2 * np.pi * q / (n * dx)) ** 2 for q in m)
    lap = sp.irfft3(-sp.ksq(u.shape, dx) * sp.rfft3(u), u.shape)
    bih = sp.irfft3(sp.ksq(u.shape, dx) ** 2 * sp.rfft3(u), u.shape)
    assert np.max(np.abs(lap + k2 * u)) <= 1e-12 * max(1.0, k2)
    assert np.max(np.abs(bih - k2 * k2 * u)) <= 1e-12 * max(1.0, k2 * k2)


def test_wavevector_layout():
    kz, ky, kx = sp.wavevectors((8, 6, 10), dx=2.0)
    assert kx.shape == (1, 1, 6) and ky.shape == (1, 6, 1) and kz.shape == (8, 1, 1)
    assert np.isclose(kx[0, 0, 5], 2 * np.pi * 5 / 20)
    assert np.isclose(ky[0, 5, 0], -2 * np.pi * 1 / 12)
    mult = sp.multiplicity((8, 6, 10))
    assert mult[0, 0, 0] == 1 and mult[0, 0, 5] == 1 and np.all(mult[0, 0, 1:5] == 2)


def test_single_coefficient_by_definition_matches_brute_force():
    rng = np.random.default_rng(11)
    u = rng.standard_normal((6, 10, 12))
    X = sp.brute_rdft3(u)
    for m in [(0, 0, 0), (1, 2, 3), (5, 9, 6), (3, 0, 1)]:
        want = X[m[0], m[1], m[2]]
        assert abs(sp.dft_coefficient(u, m) - want) <= 1e-12 * np.abs(X).max()
