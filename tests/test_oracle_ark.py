"""Pins of the oracle's ImEx-ARK integrators, WRMS and invariants (CPU only)."""
import itertools
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import pfinputs
from oracle import ark
from oracle import diagnostics as dg
from oracle import model as om
from oracle import spectral as sp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden_table():
    vals = {}
    with open(os.path.join(GOLDEN, "ark436l2sa.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, i, j, v = line.split()
            vals[(name, int(i), int(j))] = Fr(v)
    return vals


def test_table_equals_published_coefficients():
    g = _load_golden_table()
    t = ark.ark436l2sa()
    s = t.s
    for i in range(s):
        assert t.c_q[i] == g[("c", i + 1, 0)]
        assert t.b_q[i] == g[("b", i + 1, 0)]
        assert t.bt_q[i] == g[("bt", i + 1, 0)]
        for j in range(s):
            assert Fr(t.AE_q[i][j]) == g.get(("AE", i + 1, j + 1), Fr(0))
            assert Fr(t.AI_q[i][j]) == g.get(("AI", i + 1, j + 1), Fr(0))


def _order_conditions(A_list, b, c, order):
    """Residuals of the additive RK order conditions up to ``order`` (exact rationals).

    Every matrix slot independently takes each of the tables in ``A_list``.
    """
    s = len(b)
    res = []
    sb = sum(b)
    res.append(sb - 1)
    if order >= 2:
        res.append(sum(b[i] * c[i] for i in range(s)) - Fr(1, 2))
    if order >= 3:
        res.append(sum(b[i] * c[i] ** 2 for i in range(s)) - Fr(1, 3))
        for A in A_list:
            res.append(sum(b[i] * A[i][j] * c[j] for i in range(s) for j in range(s)) - Fr(1, 6))
    if order >= 4:
        res.append(sum(b[i] * c[i] ** 3 for i in range(s)) - Fr(1, 4))
        for A in A_list:
            res.append(sum(b[i] * c[i] * A[i][j] * c[j] for i in range(s) for j in range(s)) - Fr(1, 8))
            res.append(sum(b[i] * A[i][j] * c[j] ** 2 for i in range(s) for j in range(s)) - Fr(1, 12))
        for A1, A2 in itertools.product(A_list, A_list):
            res.append(sum(b[i] * A1[i][j] * A2[j][k] * c[k]
                           for i in range(s) for j in range(s) for k in range(s)) - Fr(1, 24))
    return res


def test_ark436_order_conditions_exact():
    t = ark.ark436l2sa()
    AE = [[Fr(x) for x in r] for r in t.AE_q]
    AI = [[Fr(x) for x in r] for r in t.AI_q]
    for A in (AE, AI):
        for i in range(t.s):
            # published explicit rows are rationals accurate to ~1e-25
            assert abs(float(sum(A[i]) - t.c_q[i])) < 1e-20
    res = _order_conditions([AE, AI], t.b_q, t.c_q, 4)
    assert len(res) == 14
    assert max(abs(float(r)) for r in res) < 1e-26
    res3 = _order_conditions([AE, AI], t.bt_q, t.c_q, 3)
    assert len(res3) == 5
    assert max(abs(float(r)) for r in res3) < 1e-26
    # the embedding is genuinely third order: some fourth-order condition fails
    res4 = _order_conditions([AE, AI], t.bt_q, t.c_q, 4)
    assert max(abs(float(r)) for r in res4) > 1e-6


def test_ark2_order_conditions_exact_in_q_sqrt2():
    """ARK2's entries are exact in Q(sqrt 2): row sums, second order for both
    halves and their coupling, first-order embedding, stiff accuracy."""
    t = ark.ark2()
    for A in (t.AE_q, t.AI_q):
        for i in range(t.s):
            assert sum(A[i]) == t.c_q[i]
    res = _order_conditions([t.AE_q, t.AI_q], t.b_q, t.c_q, 2)
    assert all(r == 0 for r in res)
    assert _order_conditions([t.AE_q, t.AI_q], t.bt_q, t.c_q, 1) == [0]
    assert _order_conditions([t.AE_q, t.AI_q], t.bt_q, t.c_q, 2)[1] != 0   # genuinely first order
    assert any(r != 0 for r in _order_conditions([t.AE_q, t.AI_q], t.b_q, t.c_q, 3))
    assert list(t.AI_q[-1]) == list(t.b_q)                                  # stiffly accurate
    g = t.AI_q[1][1]
    assert all(t.AI_q[i][i] == g for i in range(1, t.s)) and t.AI_q[0][0] == 0
    assert g * g - 2 * g + ark.QS2(Fr(1, 2)) == 0    # gamma = 1 - 1/sqrt 2 solves g^2 - 2g + 1/2 = 0


def test_ark324_order_conditions_exact():
    t = ark.ark324l2sa()
    for A in (t.AE_q, t.AI_q):
        for i in range(t.s):
            assert abs(float(sum(A[i]) - t.c_q[i])) < 1e-20
    res = _order_conditions([t.AE_q, t.AI_q], t.b_q, t.c_q, 3)
    assert len(res) == 5
    assert max(abs(float(r)) for r in res) < 1e-25
    res2 = _order_conditions([t.AE_q, t.AI_q], t.bt_q, t.c_q, 2)
    assert max(abs(float(r)) for r in res2) < 1e-25
    assert max(abs(float(r)) for r in _order_conditions([t.AE_q, t.AI_q], t.bt_q, t.c_q, 3)) > 1e-4
    assert max(abs(float(r)) for r in _order_conditions([t.AE_q, t.AI_q], t.b_q, t.c_q, 4)) > 1e-4
    assert list(t.AI_q[-1]) == list(t.b_q)
    assert all(t.AI_q[i][i] == t.AI_q[1][1] for i in range(1, t.s))


def test_imex_euler_order_conditions():
    t = ark.imex_euler()
    assert _order_conditions([t.AE_q], t.b_q, t.c_q, 1) == [0]
    assert _order_conditions([t.AI_q], t.bI_q, t.c_q, 1) == [0]
    # and it is not second order in either half
    assert _order_conditions([t.AE_q], t.b_q, t.c_q, 2)[1] != 0
    assert _order_conditions([t.AI_q], t.bI_q, t.c_q, 2)[1] != 0


@pytest.mark.parametrize("table", ["imex_euler", "ark2", "ark324l", "ark436l"])
@pytest.mark.parametrize("lam", [(-3.0, -0.5), (-50.0, 0.2), (-0.1, -1.5), (0.4, -0.3)])
def test_stability_function_on_scalar_problem(table, lam):
    t = ark.TABLES[table]()
    lI, lE = lam
    dt = 0.37
    y0 = np.array([1.3])
    y1, _, _ = ark.ark_step(y0, dt, t, lambda y: lE * y, np.array([lI]))
    zI, zE = dt * lI, dt * lE
    M = np.eye(t.s) - zI * t.AI - zE * t.AE
    R = 1.0 + (zI * t.bI + zE * t.b) @ np.linalg.solve(M, np.ones(t.s))
    assert abs(y1[0] - R * y0[0]) <= 1e-14 * abs(R * y0[0]) + 1e-15


def test_imex_euler_ark_form_equals_direct_formula(params):
    spec, c, eta = pfinputs.config("small32", n=16)
    m = om.Model((16, 16, 16), params)
    y = om.to_kspace(c, eta)
    t = ark.imex_euler()
    L = m.implicit_symbol()
    y_ark, _, nexp = ark.ark_step(y, 0.05, t, m.f_explicit, L)
    y_dir = ark.imex_euler_direct(y, 0.05, m.f_explicit, L)
    assert nexp == 1
    u1 = sp.irfft3(y_ark, m.shape)
    u2 = sp.irfft3(y_dir, m.shape)
    assert np.max(np.abs(u1 - u2)) < 1e-15


def test_rhs_evaluations_per_step_match_paper(params):
    counts = {}
    with open(os.path.join(GOLDEN, "rhs_per_step.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                counts[k] = int(v)
    m = om.Model((8, 8, 8), params)
    c, eta, _ = pfinputs.seeded_nuclei(8, 3, n_nuclei=1, radius=2)
    y = om.to_kspace(c, eta)
    for name, expect in counts.items():
        _, _, n = ark.ark_step(y, 0.01, ark.TABLES[name](), m.f_explicit, m.implicit_symbol())
        assert n == expect


def test_wrms_hand_vectors():
    assert ark.wrms([3.0, 4.0], np.array([1.0, 1.0])) == pytest.approx(np.sqrt(12.5), rel=1e-15)
    w = ark.wrms_weights(np.array([2.0, -1.0, 0.0]), rtol=0.5, atol=0.25)
    assert np.allclose(w, [1 / 1.25, 1 / 0.75, 1 / 0.25], rtol=1e-15)
    v = np.array([0.1, 0.2, -0.3])
    assert ark.wrms(v, w) == pytest.approx(np.sqrt(np.mean((v * w) ** 2)), rel=1e-15)


def test_kspace_wrms_equals_realspace_rms_for_uniform_weights():
    rng = np.random.default_rng(8)
    shape = (8, 6, 10)
    e = rng.standard_normal((4,) + shape)
    E = sp.rfft3(e)
    atol = 1e-3
    got = ark.wrms_kspace(E, np.zeros_like(E), 0.0, atol, sp.multiplicity(shape), np.prod(shape))
    ref = ark.wrms(e.ravel(), np.full(e.size, 1 / atol))
    assert got == pytest.approx(ref, rel=1e-13)


def test_wrms_kspace_relative_tolerance_single_mode():
    """k-space WRMS with rtol > 0, worked by hand on one Fourier mode.

    Error and previous state live in eta_1 only: e(r) = a cos(2 pi x / 8) and
    y(r) = b cos(2 pi x / 8) on an 8^3 grid.  A cosine of amplitude A puts
    A N^3 / 2 into the half-spectrum bin kx = 1 (and nothing elsewhere), so
    the unitary coefficients are E = a sqrt(N^3) / 2 and Y = b sqrt(N^3) / 2;
    the bin stands for two full-spectrum modes (kx = +-1).  With the reading's
    weight w = 1 / (rtol |Y| + atol) and vector length 4 N^3:
    WRMS^2 = 2 (E w)^2 / (4 N^3)."""
    n3 = 512.0
    a, b, rtol, atol = 1e-3, 0.5, 1e-2, 1e-4
    x = np.arange(8.0)
    shape = (8, 8, 8)
    e = np.zeros((4,) + shape)
    y = np.zeros((4,) + shape)
    e[1] = a * np.cos(2 * np.pi * x / 8)[None, None, :]
    y[1] = b * np.cos(2 * np.pi * x / 8)[None, None, :]
    E_hat, Y_hat = sp.rfft3(e), sp.rfft3(y)
    # hand values: sqrt(512) / 2 = 8 sqrt(2)
    E = a * 8 * np.sqrt(2.0)
    Y = b * 8 * np.sqrt(2.0)
    w = 1.0 / (rtol * Y + atol)
    expect = np.sqrt(2 * (E * w) ** 2 / (4 * n3))
    got = ark.wrms_kspace(E_hat, Y_hat, rtol, atol, sp.multiplicity(shape), n3)
    assert got == pytest.approx(expect, rel=1e-13)
    # a slip of one factor sqrt(N^3) in the weight's state term changes it by orders of magnitude
    assert abs(got - np.sqrt(2 * (E / (rtol * Y * np.sqrt(n3) + atol)) ** 2 / (4 * n3))) > 0.5 * got


def test_wrms_real_space_hand_values_and_parseval():
    """norm_space = 1: constant error alpha in c only, constant state beta in
    every field: WRMS = sqrt(((alpha / (rtol beta + atol))^2 N^3) / (4 N^3));
    with rtol = 0 it equals the k-space norm (Parseval)."""
    shape = (6, 8, 10)
    alpha, beta, rtol, atol = 2e-4, 0.3, 1e-3, 1e-5
    e = np.zeros((4,) + shape)
    e[0] = alpha
    y = np.full((4,) + shape, beta)
    got = ark.wrms_real(sp.rfft3(e), sp.rfft3(y), rtol, atol, shape)
    assert got == pytest.approx(0.5 * alpha / (rtol * beta + atol), rel=1e-12)
    rng = np.random.default_rng(3)
    e = rng.standard_normal((4,) + shape)
    y = rng.standard_normal((4,) + shape)
    E, Y = sp.rfft3(e), sp.rfft3(y)
    k = ark.wrms_kspace(E, Y, 0.0, 1e-3, sp.multiplicity(shape), np.prod(shape))
    r = ark.wrms_real(E, Y, 0.0, 1e-3, shape)
    assert r == pytest.approx(k, rel=1e-13)


def test_controller_rules():
    assert ark.controller(1.0, 0.0, 3) == 5.0
    assert ark.controller(1.0, 1e9, 3) == pytest.approx(0.2)
    assert ark.controller(2.0, 1.0, 3) == pytest.approx(1.8)
    assert ark.controller(1.0, 0.5, 3, after_reject=True) == 1.0
    assert ark.controller(1.0, np.inf, 3) == 0.25


def test_mass_conserved_bitwise_and_energy_decreases(params):
    for mode in (0, 1):
        p = dict(params)
        p["mean_strain_mode"] = mode
        spec, c, eta = pfinputs.config("small32")
        m = om.Model((32, 32, 32), p)
        y = om.to_kspace(c, eta)
        t = ark.imex_euler()
        L = m.implicit_symbol()
        c0 = y[0, 0, 0, 0]
        F_prev = dg.free_energy(m, y)
        for step in range(spec["steps"]):
            y, _, _ = ark.ark_step(y, spec["dt"], t, m.f_explicit, L)
            assert y[0, 0, 0, 0] == c0
            F = dg.free_energy(m, y)
            assert F <= F_prev + 1e-12 * abs(F_prev), (mode, step, F, F_prev)
            F_prev = F
        cm = sp.irfft3(y, m.shape)[0].mean()
        assert abs(cm - c.mean()) < 1e-12


@pytest.mark.parametrize("split", [1, 0])
@pytest.mark.parametrize("W", [1.0, -1.0])
@pytest.mark.parametrize("table", ["imex_euler", "ark2", "ark324l", "ark436l"])
def test_linearised_cahn_hilliard_amplification(params, split, W, table):
    """eta = 0 is invariant and the c equation is exactly linear: per-mode amplification R."""
    p = dict(params)
    p["W"] = W
    p["implicit_bulk_c"] = split
    n = 16
    c, eta = pfinputs.single_mode(n, m=(1, 2, 0), amp=1e-3, c0=0.16)
    m = om.Model((n, n, n), p)
    y = om.to_kspace(c, eta)
    t = ark.TABLES[table]()
    dt = 0.01
    y1, _, _ = ark.ark_step(y, dt, t, m.f_explicit, m.implicit_symbol())
    assert np.max(np.abs(y1[1:])) == 0.0
    k2 = (2 * np.pi / n) ** 2 * 5
    lam_I = -m.M * k2 * (m.a_c + m.kappa_c * k2)
    lam_E = -m.M * k2 * (2 * W - m.a_c)
    zI, zE = dt * lam_I, dt * lam_E
    R = 1 + (zI * t.bI + zE * t.b) @ np.linalg.solve(np.eye(t.s) - zI * t.AI - zE * t.AE, np.ones(t.s))
    idx = (2, 1)  # (ky, kx) = (2, 1) at kz = 0
    amp = y1[0, 0, idx[0], idx[1]] / y[0, 0, idx[0], idx[1]]
    assert abs(amp - R) < 1e-13
    sigma = lam_I + lam_E
    if W < 0:
        assert sigma > 0  # genuine spinodal growth for k^2 < 2/kappa_c
    # continuous-time growth rate reached to O(dt^p)
    assert abs(amp.real - np.exp(sigma * dt)) < 10 * (abs(sigma) * dt) ** (t.order + 1)


def _order_slope(errs, dts):
    return np.polyfit(np.log(dts), np.log(errs), 1)[0]


def test_observed_order_linear_single_mode(params):
    p = dict(params)
    p["implicit_bulk_c"] = 0   # split A: the bulk term is explicit so both halves act
    n = 16
    c, eta = pfinputs.single_mode(n, m=(1, 0, 0), amp=1e-3)
    m = om.Model((n, n, n), p)
    y0 = om.to_kspace(c, eta)
    k2 = (2 * np.pi / n) ** 2
    sigma = -m.M * k2 * (2 * m.W + m.kappa_c * k2)
    T = 2.0
    for table, dts, lo, hi in (("imex_euler", [0.2, 0.1, 0.05, 0.025], 0.9, 1.1),
                               ("ark2", [0.1, 0.05, 0.025, 0.0125], 1.8, 2.3),
                               ("ark324l", [0.4, 0.2, 0.1, 0.05], 2.8, 3.4),
                               ("ark436l", [0.4, 0.2, 0.1, 0.05], 3.7, 4.6)):
        errs = []
        for dt in dts:
            integ = ark.Integrator(m, table=table, adaptive=False, dt0=dt)
            y, _ = integ.advance(y0.copy(), 0.0, T)
            errs.append(abs(y[0, 0, 0, 1] - y0[0, 0, 0, 1] * np.exp(sigma * T)))
        s = _order_slope(errs, dts)
        assert lo <= s <= hi, (table, s, errs)


@pytest.mark.slow
def test_observed_order_nonlinear_self_convergence(params):
    n = 16
    spec, c, eta = pfinputs.config("small32", n=n)
    m = om.Model((n, n, n), params)
    y = om.to_kspace(c, eta)
    t = ark.imex_euler()
    L = m.implicit_symbol()
    for _ in range(20):   # smooth the sharp initial nuclei
        y, _, _ = ark.ark_step(y, 0.05, t, m.f_explicit, L)
    T = 2.0
    for table, dts, lo, hi in (("imex_euler", [0.05, 0.025, 0.0125, 0.00625], 0.9, 1.1),
                               ("ark2", [0.2, 0.1, 0.05, 0.025], 1.8, 2.3),
                               ("ark324l", [0.4, 0.2, 0.1, 0.05], 2.7, 3.4),
                               ("ark436l", [0.4, 0.2, 0.1, 0.05], 3.6, 4.4)):
        ref_int = ark.Integrator(m, table=table, dt0=dts[-1] / 16)
        yref, _ = ref_int.advance(y.copy(), 0.0, T)
        uref = sp.irfft3(yref, m.shape)
        errs = []
        for dt in dts:
            integ = ark.Integrator(m, table=table, dt0=dt)
            yy, _ = integ.advance(y.copy(), 0.0, T)
            errs.append(np.sqrt(np.mean((sp.irfft3(yy, m.shape) - uref) ** 2)))
        s = _order_slope(errs, dts)
        assert lo <= s <= hi, (table, s, errs)


def test_no_growth_after_a_rejection_in_the_loop(params):
    """Time-loop level: an accepted attempt that follows a rejected one
    proposes no larger step (Hairer-Norsett-Wanner facmax = 1); an accepted
    attempt after an accepted one may grow; a rejected attempt shrinks by the
    controller factor max(0.2, 0.9 err^(-1/4))."""
    n = 16
    spec, c, eta = pfinputs.config("small32", n=n)
    m = om.Model((n, n, n), params)
    y = om.to_kspace(c, eta)
    integ = ark.Integrator(m, table="ark436l", adaptive=True, dt0=5.0, rtol=1e-6, atol=1e-9)
    integ.advance(y, 0.0, 6.0)
    log = integ.stats["log"]
    after_reject = [i for i in range(1, len(log)) if log[i][3] and not log[i - 1][3]]
    after_accept = [i for i in range(1, len(log)) if log[i][3] and log[i - 1][3]]
    assert after_reject and after_accept
    for i in after_reject:
        t, dt, err, ok, nxt = log[i]
        assert nxt <= dt, (i, dt, nxt)
        # the cap is what binds here: the plain factor would have grown the step
        if err < (0.9) ** 4:
            assert nxt == dt
    assert any(log[i][4] > log[i][1] for i in after_accept)
    for t, dt, err, ok, nxt in log:
        if not ok:
            assert nxt == pytest.approx(dt * max(0.2, 0.9 * err ** -0.25), rel=1e-15)
    # every step right after a reject/accept pair: dt_k = the proposal made at k-1
    for i in range(1, len(log)):
        prev_next = log[i - 1][4]
        t, dt, err, ok, nxt = log[i]
        assert dt == pytest.approx(min(prev_next, 6.0 - t), rel=1e-15)


def test_adaptive_loop_reaches_final_time_and_rejects(params):
    n = 16
    spec, c, eta = pfinputs.config("small32", n=n)
    m = om.Model((n, n, n), params)
    y = om.to_kspace(c, eta)
    integ = ark.Integrator(m, table="ark436l", adaptive=True, dt0=5.0, rtol=1e-6, atol=1e-9)
    y1, t1 = integ.advance(y, 0.0, 3.0)
    assert t1 == pytest.approx(3.0, abs=1e-12)
    assert integ.stats["rejects"] >= 1            # dt0 = 5 is far too large
    assert all(e <= 1.0 for e in integ.stats["errs"])
    assert integ.stats["n_rhs"] == 6 * integ.stats["attempts"]
    assert y1[0, 0, 0, 0] == y[0, 0, 0, 0]
