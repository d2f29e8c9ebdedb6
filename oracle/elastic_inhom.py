"""Inhomogeneous elasticity: Reuss-averaged stiffness and the Hu-Chen
iteration for mechanical equilibrium (FP64 oracle; test infrastructure).

What is computed (Methods, "Phase-field model formulation": Eq. u_gov and the
Reuss average of the phases' stiffness beneath it; Methods, "MEUMAPPS C++ and
the MEUMAPPS-SS application": the iterative approach of Hu and Chen for the
nonlinear mechanical equilibrium; Results, "Improved performance via time
integration approach": its tight (1e-16) and loose (1e-6) tolerances):

* local compliance S(r) = H(r) S_p + (1 - H(r)) S_m with H = sum_v h(eta_v),
  local stiffness C(r) = S(r)^-1 (the Reuss average; every variant shares the
  precipitate stiffness C_p here, cubic in the grid axes);
* stress sigma = C(r) (eps_bar + eps_u - eps*(r)), eps*(r) = sum_v h(eta_v)
  eps*_v, eps_u the symmetric gradient of a periodic displacement;
* equilibrium div sigma = 0 solved by the Hu-Chen iteration with a
  homogeneous reference stiffness C0 (the mean of C_m and C_p) and
  dC(r) = C(r) - C0:  tau = C0 eps* - dC (eps_bar + eps_u - eps*), then
  eps_u <- Gamma0 tau, where Gamma0 solves div(C0 eps_u) = div tau per
  wavevector:  eps~_ij = (n_j p_i + n_i p_j) / 2,  p = Omega0(n) tau~ n,
  Omega0(n)^-1_ik = C0_ijkl n_j n_l, n along the wavevector with its Nyquist
  components zeroed (eps~ = 0 where nothing is left, k = 0 included).  The start
  (iteration 0) drops dC: with C_p = C_m it is the exact Khachaturyan
  solution.  Updates stop when the largest change of a strain component is
  at most el_tol, or after el_max_iter updates;
* elastic driving force (the derivative of the elastic energy at
  equilibrium):  d f_el / d eta_v = h'(eta_v) [ -sigma : eps*_v
  - 1/2 sigma : (S_p - S_m) : sigma ];
* elastic energy  sum_r 1/2 sigma : (eps_bar + eps_u - eps*) dV.

Readings (the paper gives neither the precipitate stiffness nor the
iteration's details): the precipitate stiffness is a parameter (C11p, C12p,
C44p); C0 = (C_m + C_p) / 2; the mean strain is prescribed (eps_bar); the
iteration starts from the homogeneous-C0 solution at every evaluation; the
change is measured on the tensor strain components; the strain is the
symmetric spectral gradient of a real periodic displacement with the Nyquist
component of each derivative set to zero (so the discrete problem is a
minimisation over real fields; the shear parts of the Green operator are odd
in a Nyquist component and would otherwise break Hermitian symmetry).  On
grids without Nyquist modes (odd sizes) equal stiffnesses give exactly the
homogeneous model.

Pinned by tests/test_oracle_inhom.py: the limits H = 0 / 1 and C S = I of the
Reuss stiffness; with C_p = C_m the driving force of the homogeneous model;
the converged strain against an independent dense solve of the discrete
equilibrium on an 8^3 grid; the equilibrium residual k_j sigma~_ij = 0 at
every k != 0; the driving force against finite differences of the elastic
energy at equilibrium; the free energy non-increasing under IMEX Euler.
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp
from .model import Model, stiffness_tensor

# Voigt order of the symmetric tensor components
VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def cubic_voigt(C11, C12, C44):
    """6 x 6 Voigt stiffness of a cubic crystal in its axes (engineering shear strains)."""
    C = np.zeros((6, 6))
    C[:3, :3] = C12
    for i in range(3):
        C[i, i] = C11
        C[3 + i, 3 + i] = C44
    return C


def strain_to_voigt(e):
    """Tensor strain components (..., 3, 3) -> Voigt vector with engineering shears (..., 6)."""
    out = np.stack([e[..., i, j] for i, j in VOIGT], axis=-1)
    out[..., 3:] *= 2.0
    return out


def stress_to_tensor(s):
    """Voigt stress (..., 6) -> symmetric tensor (..., 3, 3)."""
    t = np.zeros(s.shape[:-1] + (3, 3))
    for a, (i, j) in enumerate(VOIGT):
        t[..., i, j] = s[..., a]
        t[..., j, i] = s[..., a]
    return t


class InhomModel(Model):
    """The stand-in model with a Reuss-averaged stiffness between the matrix
    (C11, C12, C44) and the precipitate (C11p, C12p, C44p)."""

    def __init__(self, shape, params):
        super().__init__(shape, params)
        p = dict(params)
        if self.mean_strain_mode != 0:
            raise ValueError("the inhomogeneous model takes a prescribed mean strain")
        self.Cp = (float(p["C11p"]), float(p["C12p"]), float(p["C44p"]))
        self.el_tol = float(p.get("el_tol", 1e-16))
        self.el_max_iter = int(p.get("el_max_iter", 50))
        self.Cm_v = cubic_voigt(self.C11, self.C12, self.C44)
        self.Cp_v = cubic_voigt(*self.Cp)
        self.Sm_v = np.linalg.inv(self.Cm_v)
        self.Sp_v = np.linalg.inv(self.Cp_v)
        self.C0_v = 0.5 * (self.Cm_v + self.Cp_v)
        C0 = [0.5 * (a + b) for a, b in zip((self.C11, self.C12, self.C44), self.Cp)]
        self.C0_t = stiffness_tensor(*C0)
        self.last_iterations = 0
        self._om0 = None

    # ---- local stiffness -----------------------------------------------------
    def local_stiffness(self, H):
        """C(r) = (H S_p + (1 - H) S_m)^-1 as Voigt matrices, shape H.shape + (6, 6)."""
        S = H[..., None, None] * self.Sp_v + (1.0 - H)[..., None, None] * self.Sm_v
        return np.linalg.inv(S)

    def eigenstrain_voigt(self, theta):
        """eps*(r) = sum_v theta_v eps*_v as Voigt vectors (..., 6)."""
        e = np.zeros(theta.shape[1:] + (6,))
        for v in range(3):
            for i in range(3):
                e[..., i] += theta[v] * self.eps_diag[v, i]
        return e

    # ---- the homogeneous-reference Green operator -------------------------------
    def derivative_normals(self):
        """Unit vectors along the derivative wavevector: k with every Nyquist
        component (|m_i| = N_i / 2, even N_i) set to zero, the usual convention
        for an odd spectral derivative of a real field (0 where nothing is left)."""
        kz, ky, kx = sp.wavevectors(self.shape, self.dx)
        nz, ny, nx = self.shape
        kz = np.where(np.abs(sp.mode_numbers(nz))[:, None, None] * 2 == nz, 0.0, kz)
        ky = np.where(np.abs(sp.mode_numbers(ny))[None, :, None] * 2 == ny, 0.0, ky)
        kx = np.where(sp.half_mode_numbers(nx)[None, None, :] * 2 == nx, 0.0, kx)
        kk = np.broadcast_arrays(kx, ky, kz)
        kvec = np.stack([a.astype(float) for a in kk], axis=-1)
        norm = np.sqrt(np.sum(kvec * kvec, axis=-1, keepdims=True))
        with np.errstate(invalid="ignore", divide="ignore"):
            return np.where(norm > 0, kvec / np.where(norm > 0, norm, 1.0), 0.0)

    def omega0(self):
        """Omega0(n) = (C0_ijkl n_j n_l)^-1 along the derivative normals (identity where n = 0)."""
        if self._om0 is None:
            n = self.derivative_normals()
            g = np.einsum("ijkl,...j,...l->...ik", self.C0_t, n, n)
            kzero = np.all(n == 0.0, axis=-1)
            g[kzero] = np.eye(3)
            self._om0 = (np.linalg.inv(g), n, kzero)
        return self._om0

    def gamma0(self, tau_voigt):
        """Strain (Voigt, engineering shears) solving div(C0 eps) = div(tau) for
        the real stress-like field tau (Voigt (..., 6)); zero mean."""
        om, n, kzero = self.omega0()
        tau_t = stress_to_tensor(tau_voigt)                     # (nz, ny, nx, 3, 3)
        tau_hat = sp.rfft3(np.moveaxis(tau_t, (-2, -1), (0, 1)))  # (3, 3, nz, ny, nxh)
        tau_hat = np.moveaxis(tau_hat, (0, 1), (-2, -1))
        p = np.einsum("...ik,...kl,...l->...i", om, tau_hat, n)
        e_hat = 0.5 * (n[..., None, :] * p[..., :, None] + n[..., :, None] * p[..., None, :])
        e_hat[kzero] = 0.0
        e = sp.irfft3(np.moveaxis(e_hat, (-2, -1), (0, 1)), self.shape)
        return strain_to_voigt(np.moveaxis(e, (0, 1), (-2, -1)))

    # ---- Hu-Chen iteration --------------------------------------------------------
    def solve_strain(self, theta):
        """Periodic strain eps_u (Voigt) at mechanical equilibrium for theta_v = h(eta_v)."""
        H = theta.sum(axis=0)
        C = self.local_stiffness(H)
        dC = C - self.C0_v
        es = self.eigenstrain_voigt(theta)
        eb = np.zeros(6)
        eb[:3] = self.eps_bar
        c0es = es @ self.C0_v.T
        eu = self.gamma0(c0es)
        it = 0
        while it < self.el_max_iter:
            tau = c0es - np.einsum("...ij,...j->...i", dC, eb + eu - es)
            new = self.gamma0(tau)
            # largest change of a tensor component (Voigt shears carry a factor 2)
            d = np.abs(new - eu)
            d[..., 3:] *= 0.5
            eu = new
            it += 1
            if float(d.max()) <= self.el_tol:
                break
        self.last_iterations = it
        return eu, C, es, eb

    def stress(self, theta):
        eu, C, es, eb = self.solve_strain(theta)
        sig = np.einsum("...ij,...j->...i", C, eb + eu - es)
        return sig, eu, es, eb

    def elastic_force(self, theta):
        """e_v(r) = -sigma : eps*_v - 1/2 sigma : (S_p - S_m) : sigma, v = 1..3 (the
        driving force divided by h'(eta_v))."""
        sig, _, _, _ = self.stress(theta)
        dS = self.Sp_v - self.Sm_v
        quad = np.einsum("...i,ij,...j->...", sig, dS, sig)
        out = np.empty_like(theta)
        for v in range(3):
            out[v] = -np.einsum("...i,i->...", sig[..., :3], self.eps_diag[v]) - 0.5 * quad
        return out

    def f_explicit(self, y_hat):
        """Nonlinear explicit part with the inhomogeneous elastic force."""
        u = sp.irfft3(y_hat, self.shape)
        c, eta = u[0], u[1:4]
        theta = np.stack([self.h(eta[v]) for v in range(3)])
        e = self.elastic_force(theta)
        out = np.empty_like(y_hat)
        k2 = self.k2
        mu_hat = sp.rfft3(self.dfdc(c, eta))
        out[0] = -self.M * k2 * (mu_hat - self.a_c * y_hat[0])
        chi = self.chi(c)
        for v in range(3):
            g = self.dh(eta[v]) * (chi + e[v]) + self.dgdw(eta[v])
            out[1 + v] = -self.L * sp.rfft3(g)
        return out

    # ---- energy -------------------------------------------------------------------
    def elastic_energy_real(self, theta):
        sig, eu, es, eb = self.stress(theta)
        return 0.5 * float(np.sum(np.einsum("...i,...i->...", sig, eb + eu - es))) * self.dx ** 3

    def free_energy(self, y_hat):
        """Total discrete free energy with the elastic energy at the converged strain."""
        u = sp.irfft3(y_hat, self.shape)
        c, eta = u[0], u[1:4]
        dV = self.dx ** 3
        F = float(np.sum(self.f_bulk(c, eta))) * dV
        k2m = self.k2 * self.mult
        F += 0.5 * self.kappa_c * float(np.sum(k2m * np.abs(y_hat[0]) ** 2)) / self.N3 * dV
        for v in range(3):
            F += 0.5 * self.kappa_eta * float(np.sum(k2m * np.abs(y_hat[1 + v]) ** 2)) / self.N3 * dV
        theta = np.stack([self.h(eta[v]) for v in range(3)])
        return F + self.elastic_energy_real(theta)
