"""Pins of the inhomogeneous-elasticity oracle (CPU only): the Reuss stiffness,
the homogeneous limit, an independent dense solve of the discrete
equilibrium, the equilibrium residual, the driving force against finite
differences of the elastic energy, energy decrease under IMEX Euler."""
import numpy as np
import pytest

import pfinputs
from oracle import ark
from oracle import elastic_inhom as ei
from oracle import model as om
from oracle import spectral as sp


def _params(scale=1.6, **over):
    p = pfinputs.default_params()
    p.update(C11p=scale * p["C11"], C12p=scale * p["C12"], C44p=scale * p["C44"], el_tol=1e-15,
             el_max_iter=400)
    p.update(over)
    return p


def _state(n, seed, smooth=True):
    """Seeded nuclei, smoothed by a Gaussian filter in k-space so every field varies."""
    c, eta, _ = pfinputs.seeded_nuclei(n, seed, c0=0.16, n_nuclei=max(2, n // 6), radius=(2, 3), d_min=4.0)
    if smooth:
        k2 = sp.ksq((n, n, n))
        eta = sp.irfft3(sp.rfft3(eta) * np.exp(-0.5 * k2), (n, n, n))
    return c, eta


def test_reuss_stiffness_limits_and_closed_form():
    m = ei.InhomModel((4, 4, 4), _params(1.6))
    C = m.local_stiffness(np.array([0.0, 1.0, 0.5]))
    assert np.allclose(C[0], m.Cm_v, rtol=1e-14, atol=1e-10)
    assert np.allclose(C[1], m.Cp_v, rtol=1e-14, atol=1e-10)
    S = 0.5 * (m.Sm_v + m.Sp_v)
    assert np.allclose(C[2] @ S, np.eye(6), atol=1e-13)

    # cubic closed forms: S11 = (C11 + C12) / ((C11 - C12)(C11 + 2 C12)),
    # S12 = -C12 / ((C11 - C12)(C11 + 2 C12)), S44 = 1 / C44, and back
    def comp(c11, c12, c44):
        d = (c11 - c12) * (c11 + 2 * c12)
        return (c11 + c12) / d, -c12 / d, 1.0 / c44

    sm = comp(250.0, 150.0, 120.0)
    spp = comp(400.0, 240.0, 192.0)
    s11, s12, s44 = [0.5 * (a + b) for a, b in zip(sm, spp)]
    d = (s11 - s12) * (s11 + 2 * s12)
    assert C[2][0, 0] == pytest.approx((s11 + s12) / d, rel=1e-13)
    assert C[2][0, 1] == pytest.approx(-s12 / d, rel=1e-13)
    assert C[2][3, 3] == pytest.approx(1.0 / s44, rel=1e-13)


@pytest.mark.parametrize("eps_bar", [[0.0, 0.0, 0.0], [0.002, -0.001, 0.0015]])
def test_equal_stiffness_gives_the_homogeneous_model(eps_bar):
    """C_p = C_m: the Hu-Chen start is the exact Khachaturyan solution.  On a
    grid without Nyquist modes (odd sizes) the explicit right-hand side equals
    the homogeneous model's; on an even grid the elastic force agrees at every
    mode without a Nyquist component (the derivative convention differs only
    there)."""
    prm = _params(1.0, eps_bar=eps_bar)
    shape = (15, 9, 11)
    rng = np.random.default_rng(3)
    c = 0.16 + 0.01 * rng.standard_normal(shape)
    eta = np.clip(sp.irfft3(sp.rfft3(rng.uniform(0, 1, (3,) + shape)) * np.exp(-0.3 * sp.ksq(shape)), shape),
                  0, 1)
    y = om.to_kspace(c, eta)
    a = ei.InhomModel(shape, prm).f_explicit(y)
    b = om.Model(shape, prm).f_explicit(y)
    for f in range(4):
        assert np.linalg.norm(a[f] - b[f]) <= 1e-12 * np.linalg.norm(b[f]), f
    n = 16
    c, eta = _state(n, 3)
    mi, mh = ei.InhomModel((n, n, n), prm), om.Model((n, n, n), prm)
    theta = np.stack([mh.h(eta[v]) for v in range(3)])
    ei_hat = sp.rfft3(mi.elastic_force(theta))
    eh_hat = sp.rfft3(mh.elastic_potential(sp.rfft3(theta)))
    keep = np.ones(ei_hat.shape[1:], bool)
    keep[n // 2] = False
    keep[:, n // 2] = False
    keep[:, :, n // 2] = False
    assert np.max(np.abs(ei_hat[:, keep] - eh_hat[:, keep])) <= 1e-12 * np.max(np.abs(eh_hat))
    assert np.max(np.abs(ei_hat[:, ~keep] - eh_hat[:, ~keep])) > 1e-8 * np.max(np.abs(eh_hat))


def _compatible_direct_solve(m, theta):
    """Independent solve of the discrete equilibrium (no reference medium, no
    iteration): the strain is parametrised as eps~(k) = sym(n (x) w(k)) with n
    along the derivative wavevector (compatible, periodic) and w is found by
    least squares from the 2 x 3 x (number of modes) real equations
    n_j sigma~_ij(k) = 0, with sigma = C(r)(eps_bar + eps_u - eps*) and C(r)
    the Reuss stiffness."""
    shape = m.shape
    H = theta.sum(axis=0)
    C = m.local_stiffness(H)
    es = m.eigenstrain_voigt(theta)
    eb = np.zeros(6)
    eb[:3] = m.eps_bar
    n = m.derivative_normals()
    modes = [idx for idx in np.ndindex(n.shape[:3]) if np.any(n[idx] != 0.0)]

    def strain_of(w):            # w: dict mode -> complex 3-vector
        e_hat = np.zeros((3, 3) + n.shape[:3], complex)
        for idx, wv in w.items():
            nv = n[idx]
            e_hat[(slice(None), slice(None)) + idx] = 0.5 * (np.outer(wv, nv) + np.outer(nv, wv))
        e = sp.irfft3(e_hat, shape)
        return ei.strain_to_voigt(np.moveaxis(e, (0, 1), (-2, -1)))

    def residual(eu, with_source):
        sig = np.einsum("...ij,...j->...i", C, eu + (eb - es if with_source else 0.0))
        s_hat = np.moveaxis(sp.rfft3(np.moveaxis(ei.stress_to_tensor(sig), (-2, -1), (0, 1))), (0, 1), (-2, -1))
        r = np.einsum("...ij,...j->...i", s_hat, n)
        out = np.concatenate([r[idx] for idx in modes])
        return np.concatenate([out.real, out.imag])

    cols = []
    for q, idx in enumerate(modes):
        for comp in range(3):
            for part in (1.0, 1j):
                wv = np.zeros(3, complex)
                wv[comp] = part
                cols.append(residual(strain_of({idx: wv}), False))
    A = np.stack(cols, axis=1)
    b = -residual(np.zeros(H.shape + (6,)), True)
    sol = np.linalg.lstsq(A, b, rcond=None)[0]
    w = {}
    for q, idx in enumerate(modes):
        w[idx] = np.array([sol[6 * q + 2 * comp] + 1j * sol[6 * q + 2 * comp + 1] for comp in range(3)])
    return strain_of(w)


def test_converged_strain_matches_an_independent_dense_solve():
    n = 8
    m = ei.InhomModel((n, n, n), _params(1.6, eps_bar=[0.001, 0.0, -0.0005]))
    c, eta = _state(n, 5)
    theta = np.stack([m.h(eta[v]) for v in range(3)])
    eu, _, _, _ = m.solve_strain(theta)
    assert m.last_iterations > 5
    ref = _compatible_direct_solve(m, theta)
    assert np.linalg.norm(eu - ref) <= 1e-10 * np.linalg.norm(ref)
    # the homogeneous-reference start alone is not the answer
    m0 = ei.InhomModel((n, n, n), _params(1.6, eps_bar=[0.001, 0.0, -0.0005], el_max_iter=0))
    e0, _, _, _ = m0.solve_strain(theta)
    assert np.linalg.norm(e0 - ref) > 1e-3 * np.linalg.norm(ref)


def test_equilibrium_residual_vanishes():
    n = 16
    m = ei.InhomModel((n, n, n), _params(0.7))
    c, eta = _state(n, 8)
    theta = np.stack([m.h(eta[v]) for v in range(3)])
    sig, _, _, _ = m.stress(theta)
    s_hat = np.moveaxis(sp.rfft3(np.moveaxis(ei.stress_to_tensor(sig), (-2, -1), (0, 1))), (0, 1), (-2, -1))
    r = np.einsum("...ij,...j->...i", s_hat, m.derivative_normals())
    assert np.max(np.abs(r)) <= 1e-11 * np.max(np.abs(s_hat))


def test_driving_force_is_the_energy_derivative():
    """Central differences of the elastic energy at equilibrium (re-solved for
    each perturbation) against h'(eta_v) e_v at the perturbed point."""
    n = 8
    m = ei.InhomModel((n, n, n), _params(1.6, eps_bar=[0.001, 0.0, 0.0], dx=0.9))
    # three disjoint balls, one per variant, smoothed (precipitates never overlap,
    # so H stays within [0, 1] and the Reuss compliance stays positive)
    shape = (n, n, n)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    eta = np.zeros((3,) + shape)
    for v, ctr in enumerate(((1.5, 1.5, 1.5), (5.5, 1.5, 5.5), (3.5, 5.5, 3.0))):
        eta[v][(x - ctr[0]) ** 2 + (y - ctr[1]) ** 2 + (z - ctr[2]) ** 2 <= 1.8 ** 2] = 1.0
    eta = sp.irfft3(sp.rfft3(eta) * np.exp(-0.4 * sp.ksq(shape)), shape)
    theta = np.stack([m.h(eta[v]) for v in range(3)])
    assert 0.0 <= theta.sum(axis=0).min() and theta.sum(axis=0).max() <= 1.0
    e = m.elastic_force(theta)
    dV = m.dx ** 3
    delta = 1e-4
    # per variant, the point where eta_v is closest to 1/2 (h' well away from 0)
    picks = [(v, np.unravel_index(np.argmin(np.abs(eta[v] - 0.5)), eta[v].shape)) for v in range(3)
             if np.max(eta[v]) > 0.3]
    assert len(picks) == 3
    for v, idx in picks:
        def energy(shift):
            et = eta.copy()
            et[(v,) + idx] += shift
            th = np.stack([m.h(et[w]) for w in range(3)])
            return m.elastic_energy_real(th)
        fd = (energy(delta) - energy(-delta)) / (2 * delta * dV)
        an = m.dh(eta[(v,) + idx]) * e[(v,) + idx]
        assert fd == pytest.approx(an, rel=1e-6, abs=1e-9 * max(abs(an), 1.0)), (v, idx, fd, an)


def test_free_energy_decreases_under_imex_euler():
    n = 16
    m = ei.InhomModel((n, n, n), _params(1.5, el_tol=1e-12))
    c, eta, _ = pfinputs.seeded_nuclei(n, 21, c0=0.16, n_nuclei=2, radius=3, d_min=8.0)
    y = om.to_kspace(c, eta)
    L = m.implicit_symbol()
    F = [m.free_energy(y)]
    for _ in range(15):
        y, _, _ = ark.ark_step(y, 0.05, ark.imex_euler(), m.f_explicit, L)
        F.append(m.free_energy(y))
    for k in range(15):
        assert F[k + 1] <= F[k] + 1e-12 * abs(F[k]), (k, F[k], F[k + 1])
    assert F[-1] < F[0]


def test_tolerance_sets_the_iteration_count():
    n = 16
    c, eta = _state(n, 13)
    its = {}
    for tol in (1e-6, 1e-10, 1e-15):
        m = ei.InhomModel((n, n, n), _params(1.6, el_tol=tol))
        theta = np.stack([m.h(eta[v]) for v in range(3)])
        m.solve_strain(theta)
        its[tol] = m.last_iterations
    assert 1 <= its[1e-6] < its[1e-10] < its[1e-15] < 400
