"""FNO surrogate kernels (BF16 MFMA, FP32 accumulate) against the FP64 oracle:
forward output at 3e-2 relative L2 and every parameter gradient at 1e-2
(BF16 activations and weights carry ~4e-3 relative rounding per value; on
zero-mean inputs the gradients measure 4e-5 to 2e-3, the imaginary spectral
weights 6.3e-3 to 7.9e-3)."""
import sys

import numpy as np
import pytest

from oracle import fno as of

pytestmark = pytest.mark.gpu
BOUND = 3e-2
GRAD_BOUND = 1e-2


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _flat(net, p):
    return np.concatenate([p[k].ravel() for k in net.param_shapes()]).astype(np.float32)


def _unflat(net, v):
    out, o = {}, 0
    for k, s in net.param_shapes().items():
        sz = int(np.prod(s))
        out[k] = v[o:o + sz].reshape(s)
        o += sz
    return out


@pytest.mark.parametrize("n,w,m,L,h", [(8, 4, 2, 2, 8), (16, 8, 4, 2, 16), (32, 32, 12, 4, 128)])
def test_fno_forward_and_gradients_match_oracle(n, w, m, L, h):
    import torch
    from paper_2609_36100_amd import FNO
    _say("fno", n, w, m, L, h)
    net = of.FNO(n, width=w, modes=m, layers=L, hidden=h)
    p = net.init_params(seed=7)
    rng = np.random.default_rng(8)
    for k in p:
        if k.startswith("b") or k.startswith("c"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    # bf16-representable parameters and inputs so both sides start from the same values
    to_bf = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    p = {k: to_bf(v) for k, v in p.items()}
    # zero-mean inputs: with a large mean the k = 0 mode dominates every
    # spectral weight's gradient (and the imaginary part's gradient is zero
    # there), so a check through the norm would mostly see one mode
    x = rng.uniform(-1, 1, (n, n, n, 4))
    x = to_bf(x - x.mean(axis=(0, 1, 2)))
    tgt = rng.standard_normal((n, n, n, 4)) * 0.5
    out, tape = net.forward(p, x, keep=True)
    loss, dout = of.mse_loss(out, tgt)
    g = net.backward(p, tape, dout)
    with FNO(n, width=w, modes=m, layers=L, hidden=h) as f:
        f.set_params(_flat(net, p))
        xt = torch.from_numpy(np.ascontiguousarray(np.moveaxis(x, -1, 0))).float().cuda()
        yt = xt + torch.from_numpy(np.ascontiguousarray(np.moveaxis(tgt, -1, 0))).float().cuda()
        gout = f.forward(xt).cpu().numpy().reshape(n, n, n, 4)
        rel_out = np.linalg.norm(gout - out) / np.linalg.norm(out)
        f.zero_grad()
        gl = f.grad(xt, yt)
        gg = _unflat(net, f.get_grad().astype(np.float64))
    print("forward rel", rel_out, "loss", gl, loss, flush=True)
    assert rel_out < BOUND
    assert abs(gl - loss) < BOUND * loss
    worst = {}
    for k in g:
        r = np.linalg.norm(gg[k] - g[k]) / max(np.linalg.norm(g[k]), 1e-30)
        worst[k] = r
    print("grad rel", {k: "%.2e" % v for k, v in worst.items()}, flush=True)
    for k, r in worst.items():
        assert r < GRAD_BOUND, (k, r)
    # The spectral weights without the k = 0 mode: there the biases give v a
    # non-zero mean, so R_re's gradient is dominated by that one mode while
    # R_im has none (R_im S(0) is imaginary and drops out of the real
    # inverse); away from it both gradients have the same size and the same
    # bound holds for each.
    for k in g:
        if k.startswith("R"):
            a, b = gg[k].copy(), g[k].copy()
            a[0, 0, 0], b[0, 0, 0] = 0.0, 0.0
            r = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            print("grad rel without k = 0", k, "%.2e" % r, flush=True)
            assert r < GRAD_BOUND, (k, r)


def test_fno_forward_at_128_matches_oracle():
    """The surrogate's own configuration at its full size (128^3, width 32, 12
    modes, 4 layers, hidden 128): forward output and loss against the FP64
    oracle (about a minute of oracle time; the gradients are checked on the
    smaller grids above with the same kernels)."""
    import torch
    from paper_2609_36100_amd import FNO
    n, w, m, L, h = 128, 32, 12, 4, 128
    _say("fno forward", n, w, m, L, h)
    net = of.FNO(n, width=w, modes=m, layers=L, hidden=h)
    p = net.init_params(seed=17)
    rng = np.random.default_rng(18)
    for k in p:
        if k.startswith("b") or k.startswith("c"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    to_bf = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    p = {k: to_bf(v) for k, v in p.items()}
    x = to_bf(rng.uniform(0, 1, (n, n, n, 4)))
    tgt = rng.standard_normal((n, n, n, 4)) * 0.5
    out = net.forward(p, x)
    loss, _ = of.mse_loss(out, tgt)
    with FNO(n, width=w, modes=m, layers=L, hidden=h) as f:
        f.set_params(_flat(net, p))
        xt = torch.from_numpy(np.ascontiguousarray(np.moveaxis(x, -1, 0))).float().cuda()
        yt = xt + torch.from_numpy(np.ascontiguousarray(np.moveaxis(tgt, -1, 0))).float().cuda()
        gout = f.forward(xt).cpu().numpy().reshape(n, n, n, 4)
        f.zero_grad()
        gl = f.grad(xt, yt)
    rel_out = np.linalg.norm(gout - out) / np.linalg.norm(out)
    print("forward rel", rel_out, "loss", gl, loss, flush=True)
    assert rel_out < BOUND
    assert abs(gl - loss) < BOUND * loss


def test_fno_input_normalisation_matches_oracle():
    """The network sees (x - shift) / scale rounded to bf16: the oracle fed that
    input gives the same output and gradients; the loss target stays (y - x)."""
    import torch
    from paper_2609_36100_amd import FNO, PFError
    _say("fno input normalisation")
    n, w, m, L, h = 16, 8, 4, 2, 16
    net = of.FNO(n, width=w, modes=m, layers=L, hidden=h)
    p = net.init_params(seed=3)
    to_bf = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    p = {k: to_bf(v) for k, v in p.items()}
    rng = np.random.default_rng(4)
    shift = np.array([0.16, 0.1, 0.2, 0.05], np.float32)
    scale = np.array([0.004, 0.3, 0.25, 0.1], np.float32)
    raw = (shift + scale * rng.standard_normal((n, n, n, 4))).astype(np.float32)
    xn = (torch.from_numpy(raw) - torch.from_numpy(shift)) * (torch.tensor(1.0, dtype=torch.float32)
                                                               / torch.from_numpy(scale))
    x = xn.to(torch.bfloat16).to(torch.float64).numpy()
    tgt = rng.standard_normal((n, n, n, 4)) * 0.5
    out, tape = net.forward(p, x, keep=True)
    loss, dout = of.mse_loss(out, tgt)
    g = net.backward(p, tape, dout)
    with FNO(n, width=w, modes=m, layers=L, hidden=h) as f:
        f.set_params(_flat(net, p))
        f.set_input_norm(shift, scale)
        xt = torch.from_numpy(np.ascontiguousarray(np.moveaxis(raw, -1, 0))).cuda()
        yt = xt + torch.from_numpy(np.ascontiguousarray(np.moveaxis(tgt, -1, 0))).float().cuda()
        gout = f.forward(xt).cpu().numpy().reshape(n, n, n, 4)
        f.zero_grad()
        gl = f.grad(xt, yt)
        gg = _unflat(net, f.get_grad().astype(np.float64))
        with pytest.raises(PFError):
            f.set_input_norm(shift, np.zeros(4, np.float32))
    rel_out = np.linalg.norm(gout - out) / np.linalg.norm(out)
    print("forward rel", rel_out, flush=True)
    assert rel_out < BOUND
    assert abs(gl - loss) < BOUND * loss
    for k in g:
        r = np.linalg.norm(gg[k] - g[k]) / max(np.linalg.norm(g[k]), 1e-30)
        assert r < BOUND, (k, r)


def test_fno_adam_reduces_loss():
    import torch
    from paper_2609_36100_amd import FNO
    _say("fno adam")
    n, w, m, L, h = 16, 8, 4, 2, 16
    net = of.FNO(n, width=w, modes=m, layers=L, hidden=h)
    p = net.init_params(seed=1)
    rng = np.random.default_rng(2)
    x = torch.from_numpy(rng.uniform(0, 1, (4, n, n, n)).astype(np.float32)).cuda()
    y = x + 0.1 * torch.sin(3 * x)
    with FNO(n, width=w, modes=m, layers=L, hidden=h) as f:
        f.set_params(_flat(net, p))
        losses = []
        for it in range(60):
            f.zero_grad()
            losses.append(f.grad(x, y))
            f.adam_step(3e-3)
    print("losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.2 * losses[0]


def test_train_step_equals_the_separate_calls():
    """pf_fno_train_step (zero the gradient, loss and backward per pair, one
    Adam step with the batch mean) gives exactly what the separate calls give."""
    import torch
    from paper_2609_36100_amd import FNO
    _say("fno train_step composite")
    n, w, m, L, h = 16, 8, 4, 2, 16
    net = of.FNO(n, width=w, modes=m, layers=L, hidden=h)
    theta = _flat(net, net.init_params(seed=21))
    rng = np.random.default_rng(22)
    x = torch.from_numpy(rng.uniform(-1, 1, (3, 4, n, n, n)).astype(np.float32)).cuda()
    y = x + 0.1 * torch.from_numpy(rng.standard_normal((3, 4, n, n, n)).astype(np.float32)).cuda()
    with FNO(n, width=w, modes=m, layers=L, hidden=h) as a, FNO(n, width=w, modes=m, layers=L, hidden=h) as b:
        a.set_params(theta)
        b.set_params(theta)
        for it in range(2):
            la = a.train_step(x, y, 1e-3)
            b.zero_grad()
            lb = [b.grad(x[i], y[i]) for i in range(3)]
            b.adam_step(1e-3, grad_scale=1.0 / 3)
            assert la == pytest.approx(float(np.float32(np.mean(lb))), rel=1e-6)
        assert np.array_equal(a.get_params(), b.get_params())
        assert not np.array_equal(a.get_params(), theta)


def test_load_float32_and_bfloat16_weights():
    """pf_fno_load takes the flat vector as float32 or as bfloat16 bit patterns
    (widened exactly); other sizes are refused."""
    import torch
    from paper_2609_36100_amd import FNO, PFError
    _say("fno load")
    n, w, m, L, h = 8, 4, 2, 2, 8
    net = of.FNO(n, width=w, modes=m, layers=L, hidden=h)
    theta = _flat(net, net.init_params(seed=5))
    bf = torch.from_numpy(theta).to(torch.bfloat16)
    bits = bf.view(torch.int16).numpy().view(np.uint16)
    widened = bf.to(torch.float32).numpy()
    with FNO(n, width=w, modes=m, layers=L, hidden=h) as f:
        f.load(theta)
        assert np.array_equal(f.get_params(), theta)
        f.load(bits)
        assert np.array_equal(f.get_params(), widened)
        with pytest.raises(PFError):
            f.load(theta[:-1])


def test_work_accounting_counts_the_network():
    """pf_fno_work: one advance is 5 truncated-DFT GEMMs (the inverse x stage
    carried by the channel-mixing GEMM at n = 32), one channel-mixing GEMM
    and one per-mode mixing per layer plus lift and the two projection
    GEMMs; their flops are those of the network's shapes (x stage 4 m w n^3,
    y 16 m^2 w n^2, z 32 m^3 w n each way per layer; channel mixing 2 P K N
    with the input padded to 8 channels; mixing 8 w^2 per retained mode), and
    accounting off counts nothing."""
    import torch
    from paper_2609_36100_amd import FNO
    _say("fno work accounting")
    n, w, m, L, h = 32, 8, 4, 2, 16
    P = n ** 3
    net = of.FNO(n, width=w, modes=m, layers=L, hidden=h)
    rng = np.random.default_rng(3)
    u = torch.from_numpy(rng.uniform(0, 1, (4, n, n, n))).cuda()
    v = torch.empty_like(u)
    with FNO(n, width=w, modes=m, layers=L, hidden=h) as f:
        f.set_params(_flat(net, net.init_params(seed=4)))
        f.work(1)
        f.apply(u, v)
        wk = f.work(0)
        f.apply(u, v)
        assert all(x["launches"] == 0 for x in f.work(-1).values())
    # with n % 32 == 0 the inverse x stage rides on the layer's channel-mixing GEMM
    x_inv = L * 4 * m * w * n ** 3
    assert wk["lm_gemm"]["launches"] == 5 * L
    assert wk["cm_gemm"]["launches"] == L + 3
    assert wk["mix"]["launches"] == L
    assert wk["lm_gemm"]["flops"] == L * 2 * (4 * m * w * n ** 3 + 16 * m * m * w * n * n + 32 * m ** 3 * w * n) - x_inv
    assert wk["cm_gemm"]["flops"] == 2 * P * (8 * w + L * w * w + w * h + h * 4) + x_inv
    assert wk["mix"]["flops"] == L * 8 * (4 * m ** 3) * w * w
    # every GEMM reads its activations at least once: the channel-mixing bytes
    # cover the BF16 inputs of lift, the layers and both projections
    assert wk["cm_gemm"]["bytes"] > 2 * P * (8 + L * w + w + h)
