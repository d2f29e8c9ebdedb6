"""Batched ensemble (one launch per pass for all members, device-side step
control, hipGraph replay) against independent single-grid runs and the oracle."""
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
    assert _t.cuda.is_available()
    return _t


def _members(sizes, seed0=500):
    out = []
    for i, n in enumerate(sizes):
        c, eta, _ = pfinputs.seeded_nuclei(n, seed0 + i, c0=0.15 + 0.01 * i, n_nuclei=3 + i, radius=(2, 5),
                                           d_min=8.0)
        out.append((n, c, eta))
    return out


@pytest.mark.parametrize("block_threads", [128, 256])
def test_fixed_step_ensemble_matches_oracle(torch, params, block_threads):
    from paper_2609_36100_amd import Ensemble
    _say("ensemble fixed", block_threads)
    mem = _members([32, 48, 64])
    with Ensemble([dict(n=n, model=params, adaptive=False, dt0=0.1) for n, _, _ in mem]) as E:
        for k in range(7):
            E.set_tuning(k, block_threads)
        for m, (n, c, eta) in enumerate(mem):
            E.set_state(m, c, eta)
        st = E.advance([0.3, 0.2, 0.3])
        for m, (n, c, eta) in enumerate(mem):
            mdl = om.Model((n, n, n), params)
            y = om.to_kspace(c, eta)
            for _ in range(int(round([0.3, 0.2, 0.3][m] / 0.1))):
                y, _, _ = oark.ark_step(y, 0.1, oark.ark436l2sa(), mdl.f_explicit, mdl.implicit_symbol())
            g = E.get_state_hat(m)
            assert _rel(g, y) < TOL, (m, _rel(g, y))
            assert st[m]["steps"] == [3, 2, 3][m] and st[m]["n_rhs"] == 6 * st[m]["steps"]


def test_large_members_match_oracle(torch, params):
    """The 96^3 and 128^3 members (the largest sizes of the 64-member workload,
    whose batched tiles differ most from the small members') against the oracle:
    two fixed ARK4 steps each, FP64 at 1e-10 and the mixed form at its stated
    1e-5 bound."""
    from paper_2609_36100_amd import Ensemble
    _say("ensemble 96^3 + 128^3 vs oracle")
    mem = _members([96, 128], seed0=880)
    refs = []
    for n, c, eta in mem:
        mdl = om.Model((n, n, n), params)
        y = om.to_kspace(c, eta)
        for _ in range(2):
            y, _, _ = oark.ark_step(y, 0.1, oark.ark436l2sa(), mdl.f_explicit, mdl.implicit_symbol())
        refs.append(y)
    for prec, tol in (("fp64", TOL), ("mixed", 1e-5)):
        with Ensemble([dict(n=n, model=params, adaptive=False, dt0=0.1, precision=prec) for n, _, _ in mem]) as E:
            for m, (n, c, eta) in enumerate(mem):
                E.set_state(m, c, eta)
            st = E.advance(0.2)
            for m in range(2):
                assert st[m]["steps"] == 2
                g = E.get_state_hat(m)
                for f in range(4):
                    r = _rel(g[f], refs[m][f])
                    assert r < tol, (prec, m, f, r)


@pytest.mark.parametrize("method,nrhs", [("ark2", 3), ("ark324l", 4)])
def test_fixed_step_ensemble_lower_order_pairs(torch, params, method, nrhs):
    """Batched members with the second- and third-order pairs match the oracle."""
    from paper_2609_36100_amd import Ensemble
    _say("ensemble fixed", method)
    mem = _members([32, 48])
    with Ensemble([dict(n=n, model=params, adaptive=False, dt0=0.1, method=method) for n, _, _ in mem]) as E:
        for m, (n, c, eta) in enumerate(mem):
            E.set_state(m, c, eta)
        st = E.advance([0.3, 0.2])
        for m, (n, c, eta) in enumerate(mem):
            mdl = om.Model((n, n, n), params)
            y = om.to_kspace(c, eta)
            for _ in range([3, 2][m]):
                y, _, _ = oark.ark_step(y, 0.1, oark.TABLES[method](), mdl.f_explicit, mdl.implicit_symbol())
            assert _rel(E.get_state_hat(m), y) < TOL, m
            assert st[m]["steps"] == [3, 2][m] and st[m]["n_rhs"] == nrhs * st[m]["steps"]


def test_adaptive_ensemble_matches_single_runs(torch, params):
    from paper_2609_36100_amd import Ensemble, Solver
    _say("ensemble adaptive")
    mem = _members([64, 32, 96, 48, 128, 64])
    tf = [2.0, 1.5, 1.0, 2.5, 0.5, 1.0]
    kw = dict(adaptive=True, dt0=0.5, rtol=1e-6, atol=1e-9)
    with Ensemble([dict(n=n, model=params, **kw) for n, _, _ in mem]) as E:
        for m, (n, c, eta) in enumerate(mem):
            E.set_state(m, c, eta)
        E.autotune(1)
        st = E.advance(tf)
        for m, (n, c, eta) in enumerate(mem):
            with Solver(n, params, method="ark436l", **kw) as s:
                s.set_state(c, eta)
                ref = s.advance(tf[m])
                g_ref = s.kspace_to_numpy(s.get_state_hat())
            g = E.get_state_hat(m)
            assert abs(st[m]["t"] - tf[m]) < 1e-12
            assert st[m]["steps"] == ref["steps"] and st[m]["rejects"] == ref["rejects"], (m, st[m], ref)
            assert _rel(g, g_ref) < TOL, (m, _rel(g, g_ref))


def test_full_64_member_workload_matches_single_runs(torch, params):
    """The ensemble workload at its full size (64 seeded members of sizes 48,
    64, 96 and 128, adaptive ARK4(3)6L, tuned block sizes) over the first
    stretch of the run (t = 0.3, every member dissolving its sharp nuclei):
    each member's accepted and rejected steps and state against the same
    member on the single-grid path."""
    from paper_2609_36100_amd import Ensemble, Solver
    _say("ensemble 64 members")
    mem = pfinputs.ensemble_members(64)
    kw = dict(adaptive=True, dt0=0.01, rtol=1e-6, atol=1e-9)
    tf = 0.3
    with Ensemble([dict(n=m["n"], model=params, **kw) for m in mem]) as E:
        for i, m in enumerate(mem):
            E.set_state(i, m["c"], m["eta"])
        E.autotune(1)
        st = E.advance([tf] * len(mem))
        for i, m in enumerate(mem):
            with Solver(m["n"], params, method="ark436l", **kw) as s:
                s.set_state(m["c"], m["eta"])
                ref = s.advance(tf)
                g_ref = s.kspace_to_numpy(s.get_state_hat())
            g = E.get_state_hat(i)
            assert abs(st[i]["t"] - tf) < 1e-12
            assert st[i]["steps"] == ref["steps"] and st[i]["rejects"] == ref["rejects"], (i, st[i], ref)
            assert _rel(g, g_ref) < TOL, (i, _rel(g, g_ref))


def test_mixed_ensemble_error_bound(torch, params):
    from paper_2609_36100_amd import Ensemble
    _say("ensemble mixed")
    mem = _members([48, 64])
    with Ensemble([dict(n=n, model=params, adaptive=False, dt0=0.1, precision="mixed") for n, _, _ in mem]) as E:
        for m, (n, c, eta) in enumerate(mem):
            E.set_state(m, c, eta)
        E.advance(0.3)
        for m, (n, c, eta) in enumerate(mem):
            mdl = om.Model((n, n, n), params)
            y = om.to_kspace(c, eta)
            for _ in range(3):
                y, _, _ = oark.ark_step(y, 0.1, oark.ark436l2sa(), mdl.f_explicit, mdl.implicit_symbol())
            g = E.get_state_hat(m)
            errs = [_rel(g[f], y[f]) for f in range(4) if np.linalg.norm(y[f]) > 0]
            print("mixed ensemble member", m, errs, flush=True)
            assert max(errs) < 1e-5


def test_ensemble_rejects_unsupported_size(torch, params):
    from paper_2609_36100_amd import Ensemble, PFError
    with pytest.raises(PFError):
        Ensemble([dict(n=40, model=params)])
