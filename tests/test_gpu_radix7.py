"""Grids with a factor 7 (the paper's 168^3, 336^3 and 504^3 runs): radix-7
butterflies in the line FFTs, radix-6 line ends for 504 = 6 * 84 and the
tile-width cap that keeps those work-groups within 1024 threads, against the
FP64 CPU oracle on identical seeded inputs.

Tolerances as for the other grids: 1e-13 for transforms alone, relative L2
1e-10 per field for right-hand sides and steps.
"""
import sys

import numpy as np
import pytest

import pfinputs
from oracle import ark as oark
from oracle import model as om
from oracle import spectral as osp

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    return _t


def _solver(shape, prm, **kw):
    from paper_2609_36100_amd import Solver
    n = shape if isinstance(shape, int) else (shape[2], shape[1], shape[0])
    return Solver(n, prm, **kw)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _rand_fields(shape, seed):
    rng = np.random.default_rng(seed)
    c = 0.16 + 0.05 * rng.standard_normal(shape)
    eta = rng.uniform(0, 1, (3,) + shape)
    return c, eta


# (nz, ny, nx): 504 along each axis in turn (x lines are 252-point complex
# transforms after the real-to-complex packing), and mixed factor-7 boxes
FFT_SHAPES = [(56, 56, 56), (8, 16, 504), (16, 504, 8), (504, 8, 16), (168, 336, 56), (336, 56, 168)]


@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_fft3d_factor7_forward_inverse(torch, params, shape):
    _say("fft3d radix 7", shape)
    rng = np.random.default_rng(7)
    u = rng.standard_normal((2,) + shape)
    ref = osp.rfft3(u)
    with _solver(shape, params) as s:
        src = torch.from_numpy(u).cuda()
        dst = s.kspace_empty(2)
        s.fft3d(-1, 2, src, dst)
        assert _rel(s.kspace_to_numpy(dst), ref) < 1e-13
        back = torch.empty_like(src)
        s.fft3d(+1, 2, dst, back)
        assert _rel(back.cpu().numpy(), u) < 1e-13


RHS_SHAPES = [(56, 56, 56), (504, 24, 16), (24, 168, 56), (168, 56, 336)]


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("shape", RHS_SHAPES)
def test_rhs_factor7_matches_oracle(torch, params, shape, variant):
    _say("rhs radix 7", shape, "variant", variant)
    c, eta = _rand_fields(shape, seed=sum(shape))
    n = min(shape)
    c2, eta2, _ = pfinputs.seeded_nuclei(n, 5, n_nuclei=2, radius=2, d_min=4)
    sel = eta2.max(axis=0) > 0
    c[:n, :n, :n] = np.where(sel, c2, c[:n, :n, :n])
    eta[:, :n, :n, :n] = np.where(sel, eta2, eta[:, :n, :n, :n])
    m = om.Model(shape, params)
    y = om.to_kspace(c, eta)
    FI, FE = m.rhs(y)
    with _solver(shape, params) as s:
        for k in range(4):
            s.set_tuning(k, variant)
        fI, fE = s.rhs(s.kspace_from_numpy(y))
        gI, gE = s.kspace_to_numpy(fI), s.kspace_to_numpy(fE)
    for f in range(4):
        assert _rel(gI[f], FI[f]) < TOL, ("FI", f, _rel(gI[f], FI[f]))
        assert _rel(gE[f], FE[f]) < TOL, ("FE", f, _rel(gE[f], FE[f]))


def test_ark4_fixed_steps_56(torch, params):
    _say("ark4 fixed 56^3")
    n, dt, steps = 56, 0.1, 2
    spec, c, eta = pfinputs.config("small32", n=n)
    m = om.Model((n, n, n), params)
    y = om.to_kspace(c, eta)
    t = oark.ark436l2sa()
    L = m.implicit_symbol()
    with _solver(n, params, method="ark436l", dt0=dt) as s:
        s.set_state(c, eta)
        s.autotune(1)
        for _ in range(steps):
            y_old = y
            y, lte, _ = oark.ark_step(y, dt, t, m.f_explicit, L)
            err_ref = oark.wrms_kspace(lte, y_old, 1e-6, 1e-9, m.mult, m.N3)
            acc, err, _ = s.step(dt)
            assert acc
            assert abs(err - err_ref) <= 1e-8 * err_ref, (err, err_ref)
        g = s.kspace_to_numpy(s.get_state_hat())
        for f in range(4):
            assert _rel(g[f], y[f]) < TOL, (f, _rel(g[f], y[f]))


def test_mixed_precision_rhs_factor7(torch, params):
    """The precision form on a factor-7 grid: the implicit part stays FP64
    (1e-10), the explicit part within the stated 1e-4 per field."""
    _say("mixed rhs 56^3")
    n = 56
    spec, c, eta = pfinputs.config("twin64", n=n)
    m = om.Model((n, n, n), params)
    y = om.to_kspace(c, eta)
    for _ in range(20):   # diffuse the sharp nuclei (oracle IMEX Euler)
        y, _, _ = oark.ark_step(y, 0.05, oark.imex_euler(), m.f_explicit, m.implicit_symbol())
    FI, FE = m.rhs(y)
    with _solver(n, params, precision="mixed") as s:
        fI, fE = s.rhs(s.kspace_from_numpy(y))
        gI, gE = s.kspace_to_numpy(fI), s.kspace_to_numpy(fE)
    for f in range(4):
        assert _rel(gI[f], FI[f]) < TOL
        if np.linalg.norm(FE[f]) > 0:
            assert _rel(gE[f], FE[f]) < 1e-4, (f, _rel(gE[f], FE[f]))
        else:
            assert float(np.max(np.abs(gE[f]))) < 1e-4


@pytest.mark.parametrize("variant", [0, 1])
def test_mixed_precision_rhs_504_lines(torch, params, variant):
    """The precision form with 504-point z lines (radix-6 line ends in every
    column pass, the elastic one included) in both tile variants: the implicit
    part within 1e-10, the explicit part within the stated 1e-4 per field."""
    shape = (504, 24, 16)
    _say("mixed rhs", shape, "variant", variant)
    c, eta = _rand_fields(shape, seed=77)
    m = om.Model(shape, params)
    y = om.to_kspace(c, eta)
    for _ in range(5):   # smooth the random fields (oracle IMEX Euler)
        y, _, _ = oark.ark_step(y, 0.05, oark.imex_euler(), m.f_explicit, m.implicit_symbol())
    FI, FE = m.rhs(y)
    with _solver(shape, params, precision="mixed") as s:
        for k in range(4):
            s.set_tuning(k, variant)
        fI, fE = s.rhs(s.kspace_from_numpy(y))
        gI, gE = s.kspace_to_numpy(fI), s.kspace_to_numpy(fE)
    for f in range(4):
        assert _rel(gI[f], FI[f]) < TOL, ("FI", f, _rel(gI[f], FI[f]))
        assert _rel(gE[f], FE[f]) < 1e-4, ("FE", f, _rel(gE[f], FE[f]))


@pytest.mark.parametrize("shape,precision,expect", [
    ((64, 64, 64), "fp64", dict(colfft=8, stage_invz=8, zpass_elastic=4, zpass_fwd_ac=8)),
    ((64, 64, 64), "mixed", dict(colfft=8, stage_invz=8, zpass_elastic=8, zpass_fwd_ac=8)),
    ((504, 24, 16), "fp64", dict(colfft=6, stage_invz=6, zpass_elastic=6, zpass_fwd_ac=6)),
    ((504, 24, 16), "mixed", dict(colfft=6, stage_invz=6, zpass_elastic=6, zpass_fwd_ac=6)),
    ((56, 56, 56), "fp64", dict(colfft=2, stage_invz=2, zpass_elastic=2, zpass_fwd_ac=2)),
])
def test_tuning_reports_the_z_line_end_radix(torch, params, shape, precision, expect):
    """pf_tuning_get reports the first (= last) radix of the z-line plan each
    column-pass kind runs: radix-8 ends where 64 divides the length (radix 4
    for the FP64 elastic pass, which holds three fields per thread), radix-6
    ends at 504 = 6 * 84 in every kind, radix 2 at 56."""
    _say("tuning end radix", shape, precision)
    with _solver(shape, params, precision=precision) as s:
        got = {k: v["end_radix"] for k, v in s.tuning().items()}
    assert got == expect, got


def _band_limited_state(n):
    """Cosines with wavevector components 0 or +-1 (units of 2 pi / L): every
    product the right-hand side forms (degree <= 9 in the fields) stays below
    9 per component, so on any grid with N >= 20 the pointwise terms are exact
    and the spectrum is the same."""
    i = np.arange(n) * (2 * np.pi / n)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    c = 0.16 + 0.05 * np.cos(x + y + z) + 0.02 * np.sin(x - z)
    eta = np.stack([0.45 + 0.2 * np.cos(x - y),
                    0.3 + 0.1 * np.sin(y + z) + 0.05 * np.cos(x),
                    0.2 + 0.15 * np.cos(z)])
    return c, eta


def test_fft3d_504_sampled_coefficients(torch, params):
    """The 3D transform at the paper's 504^3 grid with tuned tile plans: sampled
    coefficients against the oracle's one-coefficient DFT by definition, and
    the round trip over the whole field."""
    _say("fft3d 504^3 sampled")
    n = 504
    rng = np.random.default_rng(22)
    u = rng.standard_normal((1, n, n, n))
    modes = [(0, 0, 0), (1, 0, 0), (0, 7, 3), (251, 1, 252), (300, 503, 17), (252, 252, 252), (5, 400, 100)]
    want = [osp.dft_coefficient(u[0], m) for m in modes]
    with _solver(n, params, method="imex_euler", dt0=0.05) as s:
        s.set_state(u[0], np.zeros((3, n, n, n)))
        s.autotune(1)
        src = torch.from_numpy(u).cuda()
        dst = s.kspace_empty(1)
        s.fft3d(-1, 1, src, dst)
        rms = float(torch.linalg.vector_norm(dst[..., : n // 2 + 1])) / (n * n * (n // 2 + 1)) ** 0.5
        for m, w in zip(modes, want):
            got = complex(dst[0, m[0], m[1], m[2]].item())
            assert abs(got - w) <= 1e-12 * 27 * rms, (m, got, w)
        back = torch.empty_like(src)
        s.fft3d(+1, 1, dst, back)
        err = float(torch.linalg.vector_norm(back - src) / torch.linalg.vector_norm(src))
        assert err < 1e-13, err


def test_rhs_at_504_matches_oracle_on_a_band_limited_state(torch, params):
    """pf_rhs at 504^3 with tuned tile plans against the oracle on 28^3 with dx
    scaled by 18 (the same box and wavevectors): in-band modes agree after
    division by N^3; modes the 28^3 grid cannot hold are round-off (1e-12 of
    the state, 1e-8 of the explicit derivative, whose high-k round-off is
    amplified by k^2)."""
    _say("rhs 504^3 band-limited")
    big, small = 504, 28
    p_small = dict(params)
    p_small["dx"] = params.get("dx", 1.0) * big / small
    c, eta = _band_limited_state(small)
    m = om.Model((small,) * 3, p_small)
    Y = om.to_kspace(c, eta)
    FI, FE = m.rhs(Y)
    cb, eb = _band_limited_state(big)
    with _solver(big, params, method="imex_euler", dt0=0.05) as s:
        s.set_state(cb, eb)
        s.autotune(1)
        fI, fE = s.rhs(s.get_state_hat())
        del cb, eb
        idx = np.concatenate([np.arange(0, small // 2 + 1), np.arange(big - small // 2 + 1, big)])
        it = torch.from_numpy(idx).cuda()
        y_hat = s.get_state_hat()
        for name, g, ref, out_tol in (("y", y_hat, Y, 1e-12), ("fI", fI, FI, None), ("fE", fE, FE, 1e-8)):
            sub = g.index_select(1, it).index_select(2, it)[..., : small // 2 + 1]
            sub_np = sub.cpu().numpy() / float(big) ** 3
            ref_n = ref / float(small) ** 3
            for f in range(4):
                rel = _rel(sub_np[f], ref_n[f])
                assert rel < 1e-10, (name, f, rel)
            if out_tol is None:
                continue
            sel = torch.zeros(big, dtype=torch.bool, device="cuda")
            sel[it] = True
            band = sel[:, None, None] & sel[None, :, None] & \
                (torch.arange(big // 2 + 1, device="cuda") < small // 2 + 1)[None, None, :]
            outside = torch.where(band, torch.zeros((), dtype=g.dtype, device="cuda"), g[..., : big // 2 + 1])
            rest = float(torch.linalg.vector_norm(outside))
            tot = float(torch.linalg.vector_norm(sub))
            del outside, band
            assert rest <= out_tol * tot, (name, rest, tot)
