"""Grid, wavevectors and the real 3D DFT used by the oracle (FP64).

Follows the paper's pseudospectral discretisation (Methods, "MEUMAPPS C++ and
the MEUMAPPS-SS application": fields are moved by FFT between real space and
reciprocal space, where the time integration is done).

Conventions
-----------
* Arrays are ``[z][y][x]`` (x fastest); the half spectrum keeps
  ``kx = 0 .. nx/2``: shape ``(nz, ny, nx//2 + 1)``.
* Forward transform is unnormalised, ``u~(k) = sum_r u(r) exp(-i k.r)``;
  the inverse carries ``1/(nx ny nz)`` (the ``numpy.fft.rfftn/irfftn`` pair).
* Integer mode numbers ``m`` follow ``fftfreq``; ``k_i = 2 pi m_i / (N_i dx)``.

Pinned by: brute-force DFT on tiny grids (``brute_rdft3``), a single Fourier
mode landing in its own bins, Parseval and round trip (tests/test_oracle_spectral.py).
"""
from __future__ import annotations

import numpy as np

_BACKEND = {"name": "numpy", "workers": 1}


def set_fft_backend(name="numpy", workers=1):
    """Select the FFT library: ``numpy`` (pocketfft, one thread) or ``scipy``."""
    if name not in ("numpy", "scipy"):
        raise ValueError(name)
    _BACKEND["name"] = name
    _BACKEND["workers"] = int(workers)


def fft_backend():
    return dict(_BACKEND)


def rfft3(u):
    """Forward real 3D DFT over the last three axes (unnormalised)."""
    if _BACKEND["name"] == "scipy":
        import scipy.fft as sfft
        return sfft.rfftn(u, axes=(-3, -2, -1), workers=_BACKEND["workers"])
    return np.fft.rfftn(u, axes=(-3, -2, -1))


def irfft3(U, shape):
    """Inverse of :func:`rfft3` with ``1/N^3`` scaling; ``shape`` = (nz, ny, nx)."""
    if _BACKEND["name"] == "scipy":
        import scipy.fft as sfft
        return sfft.irfftn(U, s=shape, axes=(-3, -2, -1), workers=_BACKEND["workers"])
    return np.fft.irfftn(U, s=shape, axes=(-3, -2, -1))


def mode_numbers(n):
    """Integer mode numbers of a full axis of length ``n`` (fftfreq order)."""
    return np.fft.fftfreq(n, d=1.0 / n)


def half_mode_numbers(n):
    """Integer mode numbers kept on the halved x axis: 0 .. n//2."""
    return np.arange(n // 2 + 1, dtype=float)


def wavevectors(shape, dx=1.0):
    """Return ``(kz, ky, kx)`` broadcastable over the half spectrum."""
    nz, ny, nx = shape
    kz = 2.0 * np.pi * mode_numbers(nz) / (nz * dx)
    ky = 2.0 * np.pi * mode_numbers(ny) / (ny * dx)
    kx = 2.0 * np.pi * half_mode_numbers(nx) / (nx * dx)
    return kz[:, None, None], ky[None, :, None], kx[None, None, :]


def ksq(shape, dx=1.0):
    """``|k|^2`` on the half spectrum."""
    kz, ky, kx = wavevectors(shape, dx)
    return kz * kz + ky * ky + kx * kx


def multiplicity(shape):
    """How many full-spectrum modes each half-spectrum entry stands for (1 or 2)."""
    nx = shape[2]
    m = np.full((1, 1, nx // 2 + 1), 2.0)
    m[..., 0] = 1.0
    if nx % 2 == 0:
        m[..., nx // 2] = 1.0
    return m


def brute_rdft3(u):
    """Forward real 3D DFT straight from the definition (tiny grids only).

    Builds the full ``exp(-i k.r)`` matrix over every (k, r) pair and keeps the
    half spectrum; O(N^6) work, intended for N <= 12.
    """
    nz, ny, nx = u.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.stack([z.ravel() / nz, y.ravel() / ny, x.ravel() / nx], axis=1)
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx // 2 + 1), indexing="ij")
    k = np.stack([kz.ravel(), ky.ravel(), kx.ravel()], axis=1).astype(float)
    phase = np.exp(-2j * np.pi * (k @ r.T))
    return (phase @ u.ravel()).reshape(nz, ny, nx // 2 + 1)


def brute_irdft3(U, shape):
    """Inverse of :func:`brute_rdft3` from the definition (tiny grids only).

    Rebuilds the full spectrum by Hermitian symmetry, then sums
    ``(1/N^3) sum_k U(k) exp(+i k.r)`` and keeps the real part.
    """
    nz, ny, nx = shape
    full = np.zeros((nz, ny, nx), complex)
    nxh = nx // 2 + 1
    full[:, :, :nxh] = U
    for kx in range(nxh, nx):
        for ky in range(ny):
            for kz in range(nz):
                full[kz, ky, kx] = np.conj(U[(-kz) % nz, (-ky) % ny, nx - kx])
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.stack([z.ravel() / nz, y.ravel() / ny, x.ravel() / nx], axis=1)
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    k = np.stack([kz.ravel(), ky.ravel(), kx.ravel()], axis=1).astype(float)
    phase = np.exp(2j * np.pi * (r @ k.T))
    return (phase @ full.ravel()).real.reshape(shape) / (nz * ny * nx)


def dft_coefficient(u, m):
    """One coefficient of the unnormalised forward transform by its definition,
    X(m) = sum_r u(r) exp(-2 pi i (m_z z / N_z + m_y y / N_y + m_x x / N_x)),
    summed axis by axis (x first), for a real field u[z][y][x] and an integer
    mode m = (m_z, m_y, m_x).  O(N^3) per coefficient."""
    nz, ny, nx = u.shape
    ex = np.exp(-2j * np.pi * m[2] * np.arange(nx) / nx)
    ey = np.exp(-2j * np.pi * m[1] * np.arange(ny) / ny)
    ez = np.exp(-2j * np.pi * m[0] * np.arange(nz) / nz)
    return complex(ez @ ((u @ ex) @ ey))
