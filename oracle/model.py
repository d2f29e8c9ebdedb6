"""Free-energy terms, Khachaturyan elasticity and the ImEx-split RHS (FP64 oracle).

What is computed (Methods, "Phase-field model formulation", restricted to the
dimensionless stand-in model with one homogeneous stiffness tensor):

* interpolation ``h(eta) = eta^3 (6 eta^2 - 15 eta + 10)`` (equation for h);
* bulk free energy ``f = W (c-c_m)^2 (1-H) + W (c-c_p)^2 H + w sum_v eta_v^2 (1-eta_v)^2``
  with ``H = sum_v h(eta_v)`` (the interpolated chemical energy, Eq. f_ch, with
  parabolic single-phase energies, Eq. f_ch_p, and a per-variant double well);
* gradient energy with isotropic kappa (Eq. f_b, scalar kappa);
* elastic energy with per-variant eigenstrain and homogeneous cubic stiffness
  (Eqs. for f_el, epsilon_el; mechanical equilibrium Eq. u_gov solved exactly
  per wavevector, which is the homogeneous-modulus case of the iterative
  solver the paper uses);
* Cahn-Hilliard evolution of c (Eq. x_gov) and Allen-Cahn evolution of eta
  (Eq. phi_gov), written in reciprocal space and split into a stiff linear
  implicit part and a nonlinear explicit part (Eqs. composition, order).

Readings of the paper used here (where it is silent or garbled):
* implicit CH symbol ``-M k^2 (a_c + kappa_c k^2)`` with ``a_c = 2W`` (split
  B, default) or 0 (split A); implicit AC symbol ``-L kappa_eta k^2``;
* mean strain either prescribed (``eps_bar``, default 0) or stress-free.

Pinned by tests/test_oracle_model.py: values and finite-difference derivatives
of the pointwise terms; Omega * Omega^-1 = I; an explicit displacement solve
(numpy.linalg.solve per mode) giving the same elastic potential and energy;
the isotropic dilatational closed form; the cube-axis closed form; cubic
symmetry; the whole RHS against a brute-force DFT evaluation and against
finite differences of the discrete free energy.
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp


class Model:
    """Dimensionless KKS-style stand-in model on a periodic ``(nz, ny, nx)`` grid."""

    def __init__(self, shape, params):
        p = dict(params)
        self.shape = tuple(int(s) for s in shape)
        self.dx = float(p.get("dx", 1.0))
        for key in ("W", "w", "kappa_c", "kappa_eta", "M", "L", "c_m", "c_p",
                    "C11", "C12", "C44"):
            setattr(self, key, float(p[key]))
        self.eps_diag = np.array(p["eps_star"], dtype=float)          # [v][i]
        self.eps_bar = np.array(p.get("eps_bar", [0.0, 0.0, 0.0]), dtype=float)
        self.mean_strain_mode = int(p.get("mean_strain_mode", 0))
        self.implicit_bulk_c = int(p.get("implicit_bulk_c", 1))
        self.a_c = 2.0 * self.W if self.implicit_bulk_c else 0.0

        self.C = stiffness_tensor(self.C11, self.C12, self.C44)
        self.eps = np.zeros((3, 3, 3))
        for v in range(3):
            self.eps[v] = np.diag(self.eps_diag[v])
        self.sig = np.einsum("ijkl,vkl->vij", self.C, self.eps)         # sigma*_v = C : eps*_v

        self.k2 = sp.ksq(self.shape, self.dx)
        self.mult = sp.multiplicity(self.shape)
        self.N3 = float(np.prod(self.shape))
        self._B = None

    # ---- pointwise terms -------------------------------------------------
    @staticmethod
    def h(eta):
        return eta ** 3 * (6.0 * eta * eta - 15.0 * eta + 10.0)

    @staticmethod
    def dh(eta):
        return 30.0 * eta * eta * (1.0 - eta) ** 2

    def f_bulk(self, c, eta):
        """Pointwise bulk free-energy density f(c, eta_1..3)."""
        H = sum(self.h(eta[v]) for v in range(3))
        dw = sum(eta[v] ** 2 * (1.0 - eta[v]) ** 2 for v in range(3))
        return (self.W * (c - self.c_m) ** 2 * (1.0 - H)
                + self.W * (c - self.c_p) ** 2 * H + self.w * dw)

    def dfdc(self, c, eta):
        H = sum(self.h(eta[v]) for v in range(3))
        return 2.0 * self.W * (c - self.c_m) * (1.0 - H) + 2.0 * self.W * (c - self.c_p) * H

    def chi(self, c):
        """``W[(c-c_p)^2 - (c-c_m)^2]``: the factor multiplying h'(eta_v) in df/deta_v."""
        return self.W * ((c - self.c_p) ** 2 - (c - self.c_m) ** 2)

    def dgdw(self, eta):
        """Derivative of the double well ``w eta^2 (1-eta)^2``."""
        return 2.0 * self.w * eta * (1.0 - eta) * (1.0 - 2.0 * eta)

    def dfdeta(self, c, eta, v):
        return self.dh(eta[v]) * self.chi(c) + self.dgdw(eta[v])

    # ---- elasticity ------------------------------------------------------
    def unit_normals(self):
        """Unit wavevector directions n = k/|k| on the half spectrum (0 at k = 0)."""
        kz, ky, kx = sp.wavevectors(self.shape, self.dx)
        kk = np.broadcast_arrays(kx, ky, kz)
        kvec = np.stack([a.astype(float) for a in kk], axis=-1)       # (..., 3) as (x, y, z)
        norm = np.sqrt(np.sum(kvec * kvec, axis=-1, keepdims=True))
        with np.errstate(invalid="ignore", divide="ignore"):
            n = np.where(norm > 0, kvec / np.where(norm > 0, norm, 1.0), 0.0)
        return n

    def B(self):
        """Khachaturyan kernel ``B_vw(n)`` on the half spectrum, shape (3, 3, nz, ny, nxh).

        ``B_vw = eps*_v : C : eps*_w - (sigma*_v n) . Omega(n) . (sigma*_w n)``
        for k != 0 with ``Omega^-1_ik = C_ijkl n_j n_l``; at k = 0 it is
        ``eps*_v : C : eps*_w`` (prescribed mean strain) or 0 (stress-free).
        """
        if self._B is not None:
            return self._B
        n = self.unit_normals()
        self_term = np.einsum("vij,ijkl,wkl->vw", self.eps, self.C, self.eps)
        om_inv = np.einsum("ijkl,...j,...l->...ik", self.C, n, n)
        kzero = np.all(n == 0.0, axis=-1)
        om_inv[kzero] = np.eye(3)
        om = np.linalg.inv(om_inv)
        sn = np.einsum("vij,...j->...vi", self.sig, n)                # (sigma*_v n)_i
        red = np.einsum("...vi,...ik,...wk->...vw", sn, om, sn)
        B = self_term[None, None, None] - red
        B[kzero] = self_term if self.mean_strain_mode == 0 else 0.0
        self._B = np.moveaxis(B, (-2, -1), (0, 1)).copy()
        return self._B

    def homogeneous_potential(self):
        """Constant ``-eps*_v : C : eps_bar`` added to e_v for a prescribed mean strain."""
        if self.mean_strain_mode != 0:
            return np.zeros(3)
        eb = np.diag(self.eps_bar)
        return -np.einsum("vij,ijkl,kl->v", self.eps, self.C, eb)

    def elastic_potential(self, theta_hat):
        """Real-space ``e_v = IFFT(sum_w B_vw theta~_w) + homogeneous term``."""
        B = self.B()
        e_hat = np.einsum("vw...,w...->v...", B, theta_hat)
        e = sp.irfft3(e_hat, self.shape)
        return e + self.homogeneous_potential()[:, None, None, None]

    # ---- ImEx split RHS (reciprocal space) --------------------------------
    def implicit_symbol(self):
        """Diagonal stiff linear operator L(k) for (c, eta_1, eta_2, eta_3)."""
        k2 = self.k2
        Lc = -self.M * k2 * (self.a_c + self.kappa_c * k2)
        Le = -self.L * self.kappa_eta * k2
        return np.stack([Lc, Le, Le, Le])

    def f_implicit(self, y_hat):
        return self.implicit_symbol() * y_hat

    def f_explicit(self, y_hat):
        """Nonlinear explicit part for (c, eta_1..3), shape (4, nz, ny, nxh)."""
        u = sp.irfft3(y_hat, self.shape)
        c, eta = u[0], u[1:4]
        theta = np.stack([self.h(eta[v]) for v in range(3)])
        theta_hat = sp.rfft3(theta)
        e = self.elastic_potential(theta_hat)
        out = np.empty_like(y_hat)
        k2 = self.k2
        mu_hat = sp.rfft3(self.dfdc(c, eta))
        out[0] = -self.M * k2 * (mu_hat - self.a_c * y_hat[0])
        chi = self.chi(c)
        for v in range(3):
            g = self.dh(eta[v]) * (chi + e[v]) + self.dgdw(eta[v])
            out[1 + v] = -self.L * sp.rfft3(g)
        return out

    def rhs(self, y_hat):
        return self.f_implicit(y_hat), self.f_explicit(y_hat)


def stiffness_tensor(C11, C12, C44):
    """Cubic stiffness ``C_ijkl = C12 d_ij d_kl + C44 (d_ik d_jl + d_il d_jk) + (C11-C12-2C44) d_ijkl``."""
    d = np.eye(3)
    C = (C12 * np.einsum("ij,kl->ijkl", d, d)
         + C44 * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))
    aniso = C11 - C12 - 2.0 * C44
    for i in range(3):
        C[i, i, i, i] += aniso
    return C


def to_kspace(c, eta):
    """Stack real fields (c, eta_1..3) and transform: state vector in reciprocal space."""
    return sp.rfft3(np.concatenate([c[None], eta], axis=0))


def to_real(y_hat, shape):
    u = sp.irfft3(y_hat, shape)
    return u[0], u[1:4]
