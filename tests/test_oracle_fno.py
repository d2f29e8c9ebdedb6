"""Pins of the oracle FNO: the explicit-DFT spectral convolution equals its
rfftn / irfftn definition; every gradient equals central finite differences."""
import numpy as np
import pytest

from oracle import fno as of


def test_gelu_exact_and_derivative():
    x = np.linspace(-5, 5, 101)
    from scipy.stats import norm
    assert np.max(np.abs(of.gelu(x) - x * norm.cdf(x))) < 1e-14
    d = 1e-6
    fd = (of.gelu(x + d) - of.gelu(x - d)) / (2 * d)
    assert np.max(np.abs(fd - of.gelu_grad(x))) < 1e-8


@pytest.mark.parametrize("n,m,w", [(8, 2, 3), (12, 3, 2)])
def test_spectral_conv_matches_fft_definition(n, m, w):
    net = of.FNO(n, width=w, modes=m, layers=1)
    rng = np.random.default_rng(0)
    v = rng.standard_normal((n, n, n, w))
    R = rng.standard_normal((2 * m, 2 * m, m, w, w)) + 1j * rng.standard_normal((2 * m, 2 * m, m, w, w))
    S = net.spec_fwd(v)
    T = np.einsum("ijkab,ijka->ijkb", R, S)
    got = net.spec_inv(T)
    ref = of.spectral_conv_fft(v, R, m)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_spectral_adjoints():
    n, m, w = 8, 2, 3
    net = of.FNO(n, width=w, modes=m)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((n, n, n, w))
    G = rng.standard_normal((2 * m, 2 * m, m, w)) + 1j * rng.standard_normal((2 * m, 2 * m, m, w))
    # <spec_fwd v, G>_R = <v, spec_fwd_T G>
    lhs = np.sum((net.spec_fwd(v) * np.conj(G)).real)
    rhs = np.sum(v * net.spec_fwd_T(G))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    g = rng.standard_normal((n, n, n, w))
    T = G
    lhs = np.sum(net.spec_inv(T) * g)
    rhs = np.sum((T * np.conj(net.spec_inv_T(g))).real)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_gradients_match_finite_differences():
    n, m, w = 8, 2, 4
    net = of.FNO(n, width=w, modes=m, layers=2, hidden=6)
    p = net.init_params(seed=3)
    for k in p:  # non-zero biases so every term is exercised
        if k.startswith("b") or k.startswith("c"):
            p[k] = np.random.default_rng(4).standard_normal(p[k].shape) * 0.1
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, (n, n, n, 4))
    target = rng.standard_normal((n, n, n, 4)) * 0.1
    out, tape = net.forward(p, x, keep=True)
    loss, dout = of.mse_loss(out, target)
    g = net.backward(p, tape, dout)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(4, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            lp, _ = of.mse_loss(net.forward(p, x), target)
            flat[i] = old - eps
            lm, _ = of.mse_loss(net.forward(p, x), target)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3 * abs(loss)), (k, i, fd, an)
