"""Inhomogeneous elasticity on the GPU (Reuss-averaged stiffness, Hu-Chen
iteration) against the FP64 oracle: the explicit right-hand side with a fixed
number of updates and with a tolerance, equal stiffnesses, ARK4 steps, the
free energy, energy decrease, and the tight / loose tolerances' iteration
counts (Methods, "Phase-field model formulation": Eq. u_gov and the Reuss
stiffness; Results, "Improved performance via time integration approach":
the elasticity tolerances)."""
import sys

import numpy as np
import pytest

import pfinputs
from oracle import ark as oark
from oracle import elastic_inhom as ei
from oracle import model as om
from oracle import spectral as osp

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    return _t


def _prm(scale=1.5, tol=1e-12, max_iter=200, **over):
    p = pfinputs.default_params()
    p.update(C11p=scale * p["C11"], C12p=scale * p["C12"], C44p=scale * p["C44"], el_tol=tol, el_max_iter=max_iter)
    p.update(over)
    return p


def _smooth_state(shape, seed, n_nuclei, steps=2):
    """Seeded nuclei advanced by a few oracle IMEX Euler steps of the homogeneous
    model: smooth fields, non-overlapping precipitates."""
    nz, ny, nx = shape
    n = max(shape)
    c, eta, _ = pfinputs.seeded_nuclei(n, seed, c0=0.16, n_nuclei=n_nuclei, radius=(2, 4), d_min=9.0)
    c, eta = c[:nz, :ny, :nx], eta[:, :nz, :ny, :nx]
    m = om.Model(shape, pfinputs.default_params())
    y = om.to_kspace(c, eta)
    for _ in range(steps):
        y, _, _ = oark.ark_step(y, 0.05, oark.imex_euler(), m.f_explicit, m.implicit_symbol())
    return y


def _solver(shape, prm, **kw):
    from paper_2609_36100_amd import Solver
    n = shape if isinstance(shape, int) else (shape[2], shape[1], shape[0])
    return Solver(n, prm, **kw)


CASES = [((16, 16, 16), 1.5, 0.0, 3), ((16, 16, 16), 0.6, 1e-12, 200), ((32, 32, 32), 1.5, 1e-12, 200),
         ((16, 24, 32), 1.8, 1e-11, 200), ((32, 32, 32), 1.0, 1e-12, 200)]


@pytest.mark.parametrize("shape,scale,tol,max_iter", CASES)
def test_rhs_matches_oracle(torch, shape, scale, tol, max_iter):
    _say("inhom rhs", shape, scale, tol, max_iter)
    prm = _prm(scale, tol, max_iter, eps_bar=[0.001, -0.0005, 0.0])
    y = _smooth_state(shape, 300 + shape[0], n_nuclei=4)
    m = ei.InhomModel(shape, prm)
    FI, FE = m.rhs(y)
    its = m.last_iterations
    with _solver(shape, prm) as s:
        fI, fE = s.rhs(s.kspace_from_numpy(y))
        gI, gE = s.kspace_to_numpy(fI), s.kspace_to_numpy(fE)
        st = s.stats()
    print("iterations", its, st["el_last"], flush=True)
    assert st["el_last"] == its
    for f in range(4):
        assert _rel(gI[f], FI[f]) < TOL, f
        assert _rel(gE[f], FE[f]) < TOL, (f, _rel(gE[f], FE[f]))


def test_rhs_at_128_matches_oracle(torch):
    """128^3, a fixed number of updates (the oracle's dense per-point Voigt
    inverses take about a minute here)."""
    shape = (128, 128, 128)
    _say("inhom rhs 128^3")
    prm = _prm(1.5, 0.0, 4)
    y = _smooth_state(shape, 777, n_nuclei=30, steps=1)
    m = ei.InhomModel(shape, prm)
    FE = m.f_explicit(y)
    with _solver(shape, prm) as s:
        fI, fE = s.rhs(s.kspace_from_numpy(y))
        gE = s.kspace_to_numpy(fE)
        assert s.stats()["el_last"] == 4
    for f in range(4):
        assert _rel(gE[f], FE[f]) < TOL, (f, _rel(gE[f], FE[f]))


def test_ark4_steps_match_oracle(torch):
    _say("inhom ark4 steps 32^3")
    n = 32
    prm = _prm(1.5, 1e-12, 200)
    y = _smooth_state((n, n, n), 55, n_nuclei=4)
    m = ei.InhomModel((n, n, n), prm)
    tab = oark.ark436l2sa()
    with _solver(n, prm, method="ark436l", dt0=0.05) as s:
        s.set_state_hat(s.kspace_from_numpy(y))
        for _ in range(2):
            y, lte, _ = oark.ark_step(y, 0.05, tab, m.f_explicit, m.implicit_symbol())
            acc, err, _ = s.step(0.05)
            assert acc
        g = s.kspace_to_numpy(s.get_state_hat())
        st = s.stats()
    assert st["el_iterations"] > 12 * 1
    for f in range(4):
        assert _rel(g[f], y[f]) < TOL, f


def test_free_energy_matches_oracle_and_decreases(torch):
    _say("inhom free energy 32^3")
    n = 32
    prm = _prm(1.5, 1e-12, 200)
    y = _smooth_state((n, n, n), 66, n_nuclei=4)
    m = ei.InhomModel((n, n, n), prm)
    F0 = m.free_energy(y)
    Fs = []
    with _solver(n, prm, method="imex_euler", dt0=0.05) as s:
        s.set_state_hat(s.kspace_from_numpy(y))
        Fs.append(s.free_energy())
        for _ in range(10):
            acc, _, _ = s.step(0.05)
            assert acc
            Fs.append(s.free_energy())
    assert abs(Fs[0] - F0) <= 1e-10 * abs(F0)
    for k in range(10):
        assert Fs[k + 1] <= Fs[k] + 1e-12 * abs(Fs[k]), (k, Fs[k], Fs[k + 1])


def test_tight_and_loose_tolerances(torch):
    """The paper's two elasticity tolerances: 1e-6 stops after few updates,
    1e-16 runs to the round-off floor (capped); both against the oracle's
    counts."""
    _say("inhom tolerances")
    n = 32
    y = _smooth_state((n, n, n), 88, n_nuclei=4)
    counts = {}
    for tol in (1e-6, 1e-16):
        prm = _prm(1.5, tol, 60)
        m = ei.InhomModel((n, n, n), prm)
        FE = m.f_explicit(y)
        with _solver(n, prm) as s:
            _, fE = s.rhs(s.kspace_from_numpy(y))
            counts[tol] = (s.stats()["el_last"], m.last_iterations)
            g = s.kspace_to_numpy(fE)
        for f in range(4):
            assert _rel(g[f], FE[f]) < 1e-9, (tol, f)
    print("updates (gpu, oracle)", counts, flush=True)
    assert counts[1e-6][0] == counts[1e-6][1]
    assert 1 <= counts[1e-6][0] < counts[1e-16][0] <= 60
