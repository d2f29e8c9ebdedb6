"""Adaptive step control on the GPU against the FP64 oracle's time loop:
every attempt (step size, WRMS error, accept / reject, next proposal) with
rejections in the sequence, so the no-growth rule after a rejection is
exercised; the real-space WRMS option; resuming an ensemble advance; the
ensemble's per-member device controller against the oracle.

Step control follows Methods, "Time integration" (embedded error, WRMS test,
reject and recompute, accept and propose), with the elementary I-controller
of the reading the oracle documents."""
import sys

import numpy as np
import pytest

import pfinputs
from oracle import ark as oark
from oracle import model as om

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


def _attempts_match(log, s, t_final, err_rel=1e-6):
    """Drive pf_ark_step with the GPU's own proposals and compare each attempt
    with the oracle's log entry.  Returns False (no assertion) if an oracle
    error lies so close to 1 that round-off may flip the decision."""
    t = 0.0
    dt = log[0][1]
    for i, (t_o, dt_o, err_o, ok_o, nxt_o) in enumerate(log):
        if abs(err_o - 1.0) < 1e-6:
            return False
        dt = min(dt, t_final - t)
        assert dt == pytest.approx(dt_o, rel=1e-12), (i, dt, dt_o)
        acc, err, nxt = s.step(dt)
        assert acc == ok_o, (i, err, err_o)
        # relative agreement, with an absolute floor far below the acceptance
        # threshold 1 for the tiny error of a step clipped to land on t_final
        assert abs(err - err_o) <= err_rel * err_o + 1e-12, (i, err, err_o)
        assert nxt == pytest.approx(nxt_o, rel=1e-9), (i, nxt, nxt_o)
        if acc:
            t += dt
        dt = nxt
    return True


@pytest.mark.parametrize("method,dt0,rtol,atol,tf", [("ark436l", 5.0, 1e-6, 1e-9, 0.1),
                                                     ("ark324l", 2.0, 1e-5, 1e-8, 0.1)])
def test_attempt_sequence_with_rejections_matches_oracle(torch, params, method, dt0, rtol, atol, tf):
    from paper_2609_36100_amd import Solver
    _say("attempt log", method, dt0)
    n = 32
    spec, c, eta = pfinputs.config("small32", n=n)
    m = om.Model((n, n, n), params)
    integ = oark.Integrator(m, table=method, adaptive=True, dt0=dt0, rtol=rtol, atol=atol)
    yref, _ = integ.advance(om.to_kspace(c, eta), 0.0, tf)
    log = integ.stats["log"]
    rej_then_acc = [i for i in range(1, len(log)) if log[i][3] and not log[i - 1][3]]
    assert rej_then_acc, "the sequence must contain a rejection followed by an acceptance"
    with Solver(n, params, method=method, adaptive=True, dt0=dt0, rtol=rtol, atol=atol) as s:
        s.set_state(c, eta)
        if _attempts_match(log, s, tf):
            assert _rel(s.kspace_to_numpy(s.get_state_hat()), yref) < TOL
    # the library's own loop makes the same decisions
    with Solver(n, params, method=method, adaptive=True, dt0=dt0, rtol=rtol, atol=atol) as s:
        s.set_state(c, eta)
        st = s.advance(tf)
        assert st["steps"] == integ.stats["steps"] and st["rejects"] == integ.stats["rejects"]
        assert st["dt_next"] == pytest.approx(log[-1][4], rel=1e-9)


def test_real_space_norm_matches_oracle(torch, params):
    """norm_space = 1: WRMS over the real-space fields, weights from the
    previous state point by point.  Replayed dt sequence (error per step), then
    the library's own decisions."""
    from paper_2609_36100_amd import Solver
    _say("norm_space 1")
    n = 32
    spec, c, eta = pfinputs.config("small32", n=n)
    m = om.Model((n, n, n), params)
    integ = oark.Integrator(m, table="ark436l", adaptive=True, dt0=1.0, rtol=1e-4, atol=1e-7, norm_space=1)
    yref, _ = integ.advance(om.to_kspace(c, eta), 0.0, 2.0)
    log = integ.stats["log"]
    # the two norms differ on this state (so the option is really taken)
    y0 = om.to_kspace(c, eta)
    _, lte, _ = oark.ark_step(y0, 0.1, oark.ark436l2sa(), m.f_explicit, m.implicit_symbol())
    ek = oark.wrms_kspace(lte, y0, 1e-4, 1e-7, m.mult, m.N3)
    er = oark.wrms_real(lte, y0, 1e-4, 1e-7, m.shape)
    assert abs(ek - er) > 0.1 * er
    with Solver(n, params, method="ark436l", adaptive=True, dt0=1.0, rtol=1e-4, atol=1e-7, norm_space=1) as s:
        s.set_state(c, eta)
        if _attempts_match(log, s, 2.0):
            assert _rel(s.kspace_to_numpy(s.get_state_hat()), yref) < TOL
    for prec in ("fp64", "mixed"):
        with Solver(n, params, method="ark436l", adaptive=True, dt0=1.0, rtol=1e-4, atol=1e-7, norm_space=1,
                    precision=prec) as s:
            s.set_state(c, eta)
            st = s.advance(2.0)
            if prec == "fp64":
                assert st["steps"] == integ.stats["steps"] and st["rejects"] == integ.stats["rejects"]
            assert abs(st["t"] - 2.0) < 1e-12


def _members(sizes, seed0):
    out = []
    for i, n in enumerate(sizes):
        c, eta, _ = pfinputs.seeded_nuclei(n, seed0 + i, c0=0.15 + 0.01 * i, n_nuclei=3 + i, radius=(2, 5),
                                           d_min=8.0)
        out.append((n, c, eta))
    return out


def test_ensemble_advance_resumes_from_the_proposed_step(torch, params):
    """Adaptive two-member ensemble advanced to t1 and then to t2 takes the same
    steps as single-grid contexts advanced to t1 and then t2 (the proposal is
    kept across calls, not the clipped last step)."""
    from paper_2609_36100_amd import Ensemble, Solver
    _say("ensemble resume")
    mem = _members([32, 48], 610)
    kw = dict(adaptive=True, dt0=0.05, rtol=1e-6, atol=1e-9)
    t1, t2 = 0.37, 1.0
    with Ensemble([dict(n=n, model=params, **kw) for n, _, _ in mem]) as E:
        for m, (n, c, eta) in enumerate(mem):
            E.set_state(m, c, eta)
        s1 = E.advance(t1)
        s2 = E.advance(t2)
        for m, (n, c, eta) in enumerate(mem):
            assert s2[m]["steps"] > s1[m]["steps"]
            assert s1[m]["dt_next"] > 0 and s2[m]["dt_next"] > 0
            with Solver(n, params, **kw) as s:
                s.set_state(c, eta)
                a = s.advance(t1)
                b = s.advance(t2)
                assert (s1[m]["steps"], s1[m]["rejects"]) == (a["steps"], a["rejects"])
                assert (s2[m]["steps"], s2[m]["rejects"]) == (b["steps"], b["rejects"]), (m, s2[m], b)
                assert s2[m]["dt_next"] == pytest.approx(b["dt_next"], rel=1e-12)
                g = s.kspace_to_numpy(s.get_state_hat())
            assert _rel(E.get_state_hat(m), g) < TOL
            assert abs(s2[m]["t"] - t2) < 1e-12


def test_ensemble_device_controller_matches_oracle(torch, params):
    """Mixed 32^3 / 48^3 ensemble, adaptive ARK4 with rejections (large dt0):
    each member's accepted steps, rejections, final proposal and state against
    the oracle's time loop."""
    from paper_2609_36100_amd import Ensemble
    _say("ensemble controller vs oracle")
    mem = _members([32, 48, 32], 720)
    kw = dict(adaptive=True, dt0=2.0, rtol=1e-6, atol=1e-9)
    tf = 0.06
    with Ensemble([dict(n=n, model=params, **kw) for n, _, _ in mem]) as E:
        for m, (n, c, eta) in enumerate(mem):
            E.set_state(m, c, eta)
        st = E.advance(tf)
        for m, (n, c, eta) in enumerate(mem):
            mdl = om.Model((n, n, n), params)
            integ = oark.Integrator(mdl, table="ark436l", adaptive=True, dt0=2.0, rtol=1e-6, atol=1e-9)
            yref, _ = integ.advance(om.to_kspace(c, eta), 0.0, tf)
            assert integ.stats["rejects"] >= 1
            if any(abs(e[2] - 1.0) < 1e-6 for e in integ.stats["log"]):
                continue
            assert st[m]["steps"] == integ.stats["steps"], m
            assert st[m]["rejects"] == integ.stats["rejects"], m
            assert st[m]["dt_next"] == pytest.approx(integ.stats["log"][-1][4], rel=1e-9)
            assert _rel(E.get_state_hat(m), yref) < TOL, m
