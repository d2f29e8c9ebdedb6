"""Pins of the oracle's model terms, elasticity and split RHS (CPU only)."""
import numpy as np
import pytest

import pfinputs
from oracle import diagnostics as dg
from oracle import model as om
from oracle import spectral as sp


def _rand_state(shape, seed=0, eta_scale=1.0):
    rng = np.random.default_rng(seed)
    c = 0.16 + 0.05 * rng.standard_normal(shape)
    eta = eta_scale * rng.uniform(0.0, 1.0, size=(3,) + shape)
    return c, eta


# ---- pointwise terms ---------------------------------------------------
def test_interpolation_function_values():
    h, dh = om.Model.h, om.Model.dh
    assert h(0.0) == 0.0 and h(1.0) == 1.0 and h(0.5) == 0.5
    assert dh(0.0) == 0.0 and dh(1.0) == 0.0
    x = np.linspace(-0.3, 1.3, 41)
    d = 1e-6
    fd = (h(x + d) - h(x - d)) / (2 * d)
    assert np.max(np.abs(fd - dh(x))) < 1e-8


def test_bulk_derivatives_match_finite_differences(params):
    m = om.Model((4, 4, 4), params)
    rng = np.random.default_rng(5)
    c = rng.uniform(-0.1, 0.4, 50)
    eta = rng.uniform(-0.2, 1.2, (3, 50))
    d = 1e-6
    fd_c = (m.f_bulk(c + d, eta) - m.f_bulk(c - d, eta)) / (2 * d)
    assert np.max(np.abs(fd_c - m.dfdc(c, eta))) < 1e-8
    for v in range(3):
        ep, em = eta.copy(), eta.copy()
        ep[v] += d
        em[v] -= d
        fd = (m.f_bulk(c, ep) - m.f_bulk(c, em)) / (2 * d)
        assert np.max(np.abs(fd - m.dfdeta(c, eta, v))) < 1e-8


# ---- stiffness and elasticity -------------------------------------------
def test_stiffness_tensor_components(params):
    C = om.stiffness_tensor(250.0, 150.0, 120.0)
    assert C[0, 0, 0, 0] == 250 and C[1, 1, 2, 2] == 150 and C[0, 1, 0, 1] == 120
    assert C[0, 1, 1, 0] == 120 and C[0, 0, 0, 1] == 0
    assert np.allclose(C, C.transpose(1, 0, 2, 3)) and np.allclose(C, C.transpose(2, 3, 0, 1))


def test_omega_inverse_closed_form(params):
    m = om.Model((6, 6, 6), params)
    n = m.unit_normals().reshape(-1, 3)
    n = n[np.any(n != 0, axis=1)]
    C11, C12, C44 = m.C11, m.C12, m.C44
    closed = (C44 * np.eye(3)[None] + (C12 + C44) * n[:, :, None] * n[:, None, :]
              + (C11 - C12 - 2 * C44) * np.einsum("ai,ik->aik", n * n, np.eye(3)))
    contr = np.einsum("ijkl,aj,al->aik", m.C, n, n)
    assert np.max(np.abs(closed - contr)) < 1e-12


def _explicit_elastic_solution(m, theta, eps_bar):
    """Mechanical equilibrium solved per wavevector with numpy.linalg.solve.

    Returns real-space stress and strain fields (3, 3, nz, ny, nx) for the
    eigenstrain field sum_v theta_v eps*_v with mean strain eps_bar.
    """
    shape = m.shape
    eps0 = np.einsum("vij,v...->ij...", m.eps, theta)          # eigenstrain field
    sig0_hat = sp.rfft3(np.einsum("ijkl,kl...->ij...", m.C, eps0))
    kz, ky, kx = sp.wavevectors(shape, m.dx)
    kk = np.broadcast_arrays(kx, ky, kz)
    k = np.stack(kk, axis=0).astype(float)                    # (3, ...) as (x, y, z)
    A = np.einsum("ijkl,j...,l...->...ik", m.C, k, k)          # acoustic tensor
    rhs = -1j * np.einsum("ij...,j...->...i", sig0_hat, k)     # -i k_j sigma0~_ij
    zero = np.all(k == 0, axis=0)
    A[zero] = np.eye(3)
    rhs[zero] = 0
    u_hat = np.linalg.solve(A, rhs[..., None])[..., 0]         # (..., 3)
    # strain of u: sym(i k u)
    grad = 1j * np.einsum("i...,...j->ij...", k, u_hat)
    eps_u_hat = 0.5 * (grad + grad.transpose(1, 0, *range(2, grad.ndim)))
    eps_u = sp.irfft3(eps_u_hat, shape)
    strain = eps_u + np.asarray(eps_bar)[:, :, None, None, None] - eps0
    stress = np.einsum("ijkl,kl...->ij...", m.C, strain)
    return stress, strain, k, sp.rfft3(stress)


@pytest.mark.parametrize("mode", [0, 1])
def test_elastic_potential_matches_explicit_displacement_solve(params, mode):
    p = dict(params)
    p["mean_strain_mode"] = mode
    if mode == 0:
        p["eps_bar"] = [0.003, -0.002, 0.001]
    shape = (8, 6, 10)
    m = om.Model(shape, p)
    rng = np.random.default_rng(7)
    theta = rng.uniform(0, 1, size=(3,) + shape)
    # Nyquist planes carry no real-space derivative, so a real-space
    # displacement cannot represent them: compare on band-limited fields.
    th = sp.rfft3(theta)
    th[:, shape[0] // 2] = 0
    th[:, :, shape[1] // 2] = 0
    th[:, :, :, shape[2] // 2] = 0
    theta = sp.irfft3(th, shape)
    if mode == 0:
        eps_bar = np.diag(m.eps_bar)
    else:  # stress-free: the mean strain relaxes to the mean eigenstrain
        eps_bar = np.einsum("vij,v->ij", m.eps, theta.mean(axis=(1, 2, 3)))
    stress, strain, k, stress_hat = _explicit_elastic_solution(m, theta, eps_bar)
    # equilibrium: k_j sigma~_ij = 0 for every k
    resid = np.einsum("ij...,j...->i...", stress_hat, k)
    assert np.max(np.abs(resid)) < 1e-10 * np.max(np.abs(stress_hat))
    # driving potential: e_v = -sigma : eps*_v
    e_ref = -np.einsum("ij...,vij->v...", stress, m.eps)
    e = m.elastic_potential(sp.rfft3(theta))
    assert np.max(np.abs(e - e_ref)) < 1e-12 * np.max(np.abs(e_ref)) + 1e-15
    # energy: 1/2 sum_r eps_el : C : eps_el
    E_ref = 0.5 * np.sum(np.einsum("ij...,ij...->...", stress, strain))
    E = dg.elastic_energy(m, sp.rfft3(theta))
    assert abs(E - E_ref) < 1e-11 * abs(E_ref)


def test_isotropic_dilatational_closed_form():
    lam, mu, e0 = 100.0, 60.0, 0.01
    p = pfinputs.default_params()
    p.update(C11=lam + 2 * mu, C12=lam, C44=mu,
             eps_star=[[e0, e0, e0]] * 3)
    m = om.Model((8, 8, 8), p)
    B = m.B()
    K = lam + 2 * mu / 3
    expect = 12 * K * mu * e0 ** 2 / (lam + 2 * mu)
    Bk = B[0, 0].copy()
    Bk[0, 0, 0] = expect
    assert np.max(np.abs(Bk - expect)) < 1e-14 * expect * 100


def test_cube_axis_closed_form(params):
    m = om.Model((8, 8, 8), params)
    B = m.B()
    # mode along x: kx index 1, ky = kz = 0  -> Omega = diag(1/C11, 1/C44, 1/C44)
    s = np.einsum("vij->vi", m.sig)  # diagonal of sigma*_v
    self_term = np.einsum("vij,ijkl,wkl->vw", m.eps, m.C, m.eps)
    expect = self_term - np.outer(s[:, 0], s[:, 0]) / m.C11
    assert np.max(np.abs(B[:, :, 0, 0, 1] - expect)) < 1e-14 * np.max(np.abs(expect)) * 10
    # along z
    expect_z = self_term - np.outer(s[:, 2], s[:, 2]) / m.C11
    assert np.max(np.abs(B[:, :, 1, 0, 0] - expect_z)) < 1e-13


def test_cubic_symmetry_swaps_variants(params):
    n = 8
    m = om.Model((n, n, n), params)
    B = m.B()
    perm = [1, 0, 2]  # x <-> y swaps variants 1 <-> 2
    for (mx, my, mz) in [(1, 2, 3), (3, 1, 0), (2, 2, 1), (4, 1, 2)]:
        a = B[:, :, mz % n, my % n, mx]
        b = B[:, :, mz % n, mx % n, my]
        assert np.max(np.abs(a - b[np.ix_(perm, perm)])) < 1e-13


def test_nyquist_sign_invariance(params):
    """Flipping the sign of one wavevector component leaves B unchanged (cubic C, diagonal eigenstrain)."""
    n = 8
    m = om.Model((n, n, n), params)
    B = m.B()
    for (mx, my, mz) in [(1, 2, 3), (3, 1, 2), (4, 3, 1)]:
        assert np.max(np.abs(B[:, :, mz, my, mx] - B[:, :, (-mz) % n, my, mx])) < 1e-14
        assert np.max(np.abs(B[:, :, mz, my, mx] - B[:, :, mz, (-my) % n, mx])) < 1e-14


# ---- whole RHS ------------------------------------------------------------
def test_rhs_with_brute_force_dft(params, monkeypatch):
    shape = (6, 6, 8)
    c, eta = _rand_state(shape, seed=11)
    m = om.Model(shape, params)
    y = om.to_kspace(c, eta)
    FI, FE = m.rhs(y)

    def brute_f(u):
        u = np.asarray(u)
        if u.ndim == 3:
            return sp.brute_rdft3(u)
        return np.stack([brute_f(a) for a in u])

    def brute_i(U, s):
        U = np.asarray(U)
        if U.ndim == 3:
            return sp.brute_irdft3(U, s)
        return np.stack([brute_i(a, s) for a in U])

    monkeypatch.setattr(sp, "rfft3", brute_f)
    monkeypatch.setattr(sp, "irfft3", brute_i)
    m2 = om.Model(shape, params)
    FI2, FE2 = m2.rhs(brute_f(np.concatenate([c[None], eta])))
    for a, b in ((FI, FI2), (FE, FE2)):
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def test_rhs_translation_equivariance(params):
    shape = (8, 8, 8)
    c, eta = _rand_state(shape, seed=12)
    m = om.Model(shape, params)
    FI, FE = m.rhs(om.to_kspace(c, eta))
    s = (2, -3, 5)
    c2 = np.roll(c, s, axis=(0, 1, 2))
    eta2 = np.roll(eta, s, axis=(1, 2, 3))
    FI2, FE2 = m.rhs(om.to_kspace(c2, eta2))
    r1 = sp.irfft3(FI + FE, shape)
    r2 = sp.irfft3(FI2 + FE2, shape)
    assert np.max(np.abs(np.roll(r1, s, axis=(1, 2, 3)) - r2)) < 1e-12 * np.max(np.abs(r1))


@pytest.mark.parametrize("split,mode", [(1, 0), (0, 0), (1, 1)])
def test_rhs_is_gradient_flow_of_discrete_energy(params, split, mode):
    """Total RHS equals -L dF/deta (AC) and div M grad dF/dc (CH), dF by finite differences."""
    p = dict(params)
    p["implicit_bulk_c"] = split
    p["mean_strain_mode"] = mode
    if mode == 0:
        p["eps_bar"] = [0.002, 0.0, -0.001]
    shape = (4, 4, 6)
    c, eta = _rand_state(shape, seed=13)
    m = om.Model(shape, p)
    y = om.to_kspace(c, eta)
    FI, FE = m.rhs(y)
    total = sp.irfft3(FI + FE, shape)

    def energy(cc, ee):
        return dg.free_energy(m, om.to_kspace(cc, ee))

    d = 1e-5
    mu = np.zeros(shape)
    dFe = np.zeros((3,) + shape)
    for idx in np.ndindex(shape):
        cp, cm = c.copy(), c.copy()
        cp[idx] += d
        cm[idx] -= d
        mu[idx] = (energy(cp, eta) - energy(cm, eta)) / (2 * d)
        for v in range(3):
            ep, em = eta.copy(), eta.copy()
            ep[(v,) + idx] += d
            em[(v,) + idx] -= d
            dFe[(v,) + idx] = (energy(c, ep) - energy(c, em)) / (2 * d)
    dV = m.dx ** 3
    ch = sp.irfft3(-m.M * m.k2 * sp.rfft3(mu / dV), shape)
    scale_c = np.max(np.abs(ch))
    assert np.max(np.abs(total[0] - ch)) < 1e-6 * scale_c
    for v in range(3):
        ac = -m.L * dFe[v] / dV
        assert np.max(np.abs(total[1 + v] - ac)) < 1e-6 * np.max(np.abs(ac))


def test_mass_mode_untouched(params):
    shape = (8, 8, 8)
    c, eta = _rand_state(shape, seed=14)
    m = om.Model(shape, params)
    FI, FE = m.rhs(om.to_kspace(c, eta))
    assert FI[0, 0, 0, 0] == 0 and FE[0, 0, 0, 0] == 0
