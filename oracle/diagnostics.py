"""Mass, free energy and precipitate volume fraction of a reciprocal-space state (FP64).

* mass: mean composition, the k = 0 coefficient over N^3 (the CH equation is in
  divergence form, Eq. x_gov, so this is conserved);
* free energy: the discrete total free energy (Eq. 1 with the stand-in
  model's f, isotropic gradient terms and the elastic energy at mechanical
  equilibrium), the Lyapunov functional of the gradient flow
  (Eqs. x_gov, phi_gov);
* volume fraction: the mean of ``H = sum_v h(eta_v)``, plus a threshold
  variant (fraction of points with ``max_v eta_v > 0.5``).

Pinned by tests/test_oracle_model.py (energy against an explicit displacement
solve in real space; RHS against finite differences of this energy),
tests/test_oracle_ark.py (monotone decrease under IMEX Euler) and
tests/test_oracle_diagnostics.py (volume fraction: uniform fields against h
worked by hand, disjoint boxes counted by hand, a smooth field's closed-form
mean; the threshold variant's counts; mass as the mean of c).
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp


def mass(y_hat, shape):
    return float(y_hat[0, 0, 0, 0].real / np.prod(shape))


def volume_fraction(model, y_hat):
    u = sp.irfft3(y_hat, model.shape)
    H = sum(model.h(u[1 + v]) for v in range(3))
    vf = float(np.mean(H))
    vf_thr = float(np.mean(np.max(u[1:4], axis=0) > 0.5))
    return vf, vf_thr


def elastic_energy(model, theta_hat):
    """``E_el = 1/(2 N^3) sum_k m(k) sum_vw B_vw Re(theta~_v conj theta~_w)`` plus the mean-strain terms."""
    B = model.B()
    prod = np.einsum("vw...,v...,w...->...", B, theta_hat, np.conj(theta_hat)).real
    E = 0.5 * float(np.sum(model.mult * prod)) / model.N3
    if model.mean_strain_mode == 0:
        eb = np.diag(model.eps_bar)
        C = model.C
        # 1/2 N^3 (eps_bar : C : eps_bar) - eps_bar : C : sum_v eps*_v theta~_v(0)
        E += 0.5 * model.N3 * float(np.einsum("ij,ijkl,kl->", eb, C, eb))
        t0 = theta_hat[:, 0, 0, 0].real
        E -= float(np.einsum("ij,ijkl,vkl,v->", eb, C, model.eps, t0))
    return E * model.dx ** 3


def free_energy(model, y_hat):
    """Total discrete free energy F of the state (grid volume element dx^3)."""
    u = sp.irfft3(y_hat, model.shape)
    c, eta = u[0], u[1:4]
    dV = model.dx ** 3
    F = float(np.sum(model.f_bulk(c, eta))) * dV
    k2m = model.k2 * model.mult
    F += 0.5 * model.kappa_c * float(np.sum(k2m * np.abs(y_hat[0]) ** 2)) / model.N3 * dV
    for v in range(3):
        F += 0.5 * model.kappa_eta * float(np.sum(k2m * np.abs(y_hat[1 + v]) ** 2)) / model.N3 * dV
    theta = np.stack([model.h(eta[v]) for v in range(3)])
    F += elastic_energy(model, sp.rfft3(theta))
    return F
