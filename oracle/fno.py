"""Fourier neural operator surrogate: FP64 forward and backward (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper has no learned component; the surrogate is the learned form built
beside the method: a classic Fourier neural operator mapping the state
(c, eta_1..3) on an n^3 grid to the increment of the state a fixed time later.

Architecture (width w, retained modes m per axis, L spectral layers):
  v0 = x W_lift + b_lift                                  (pointwise 4 -> w)
  v_{l+1} = act_l( K_l v_l + v_l W_l + b_l ),  l = 0..L-1  (act = GELU except the last layer)
  K_l v   = irfftn( R_l . truncate( rfftn(v) ) )          (per retained mode a w x w complex matrix)
  out = GELU(v_L P1 + c1) P2 + c2                          (pointwise w -> 4w -> 4)
Retained modes: kx in [0, m), ky, kz in {0..m-1} U {n-m..n-1} (the four
low-frequency corners of the half spectrum).  GELU is the exact
x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.

The spectral convolution is written here with explicit truncated DFT
matrices (einsum), so the backward pass is the transpose of each real linear
map; tests/test_oracle_fno.py pins the forward against the rfftn / irfftn
definition above and the gradients against central finite differences.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def mode_lists(n, m):
    """(kx list, ky/kz list) of retained integer modes."""
    kx = np.arange(m)
    kyz = np.concatenate([np.arange(m), np.arange(n - m, n)])
    return kx, kyz


def dft_mats(n, m):
    """Real truncated DFT matrices.

    Forward x (real -> complex, kx < m):  A[kx] = sum_x v[x] exp(-2 pi i kx x / n)
    Forward y/z (complex, k in kyz).  Inverse x (complex -> real) with the
    half-spectrum weights (1 for kx = 0, 2 otherwise, real part of kx = 0 only)
    and the full 1/n^3 normalisation folded into the x inverse.
    """
    kx, kyz = mode_lists(n, m)
    r = np.arange(n)
    ax = 2 * np.pi * np.outer(kx, r) / n       # (m, n)
    ay = 2 * np.pi * np.outer(kyz, r) / n      # (2m, n)
    Fx = np.exp(-1j * ax)                      # forward x
    Fy = np.exp(-1j * ay)                      # forward y / z
    wx = np.where(kx == 0, 1.0, 2.0)
    Gx = (wx[:, None] * np.exp(1j * ax)) / n ** 3   # inverse x weights (take real part)
    Gy = np.exp(1j * ay)                       # inverse y / z
    return Fx, Fy, Gx, Gy


class FNO:
    """FP64 FNO with explicit parameters (dict of arrays)."""

    def __init__(self, n, width=32, modes=12, layers=4, cin=4, cout=4, hidden=None):
        self.n, self.w, self.m, self.L = n, width, modes, layers
        self.cin, self.cout = cin, cout
        self.h = hidden if hidden is not None else 4 * width
        self.Fx, self.Fy, self.Gx, self.Gy = dft_mats(n, modes)

    def param_shapes(self):
        w, m, h = self.w, self.m, self.h
        shp = {"W_lift": (self.cin, w), "b_lift": (w,)}
        for l in range(self.L):
            shp["R%d_re" % l] = (2 * m, 2 * m, m, w, w)   # [kz][ky][kx][in][out]
            shp["R%d_im" % l] = (2 * m, 2 * m, m, w, w)
            shp["W%d" % l] = (w, w)
            shp["b%d" % l] = (w,)
        shp.update({"P1": (w, h), "c1": (h,), "P2": (h, self.cout), "c2": (self.cout,)})
        return shp

    def init_params(self, seed=0):
        """Seeded initialisation (scaled normal / uniform spectral weights)."""
        rng = np.random.default_rng(seed)
        p = {}
        for k, s in self.param_shapes().items():
            if k.startswith("R"):
                p[k] = rng.uniform(-1.0, 1.0, s) / (self.w * self.w)
            elif k.startswith("b") or k.startswith("c"):
                p[k] = np.zeros(s)
            else:
                p[k] = rng.standard_normal(s) / math.sqrt(s[0])
        return p

    # -- spectral convolution (explicit truncated DFTs) ------------------------
    def spec_fwd(self, v):
        """v (z, y, x, c) real -> S (kz, ky, kx, c) complex."""
        a = np.einsum("kx,zyxc->zykc", self.Fx, v)
        b = np.einsum("jy,zykc->zjkc", self.Fy, a)
        return np.einsum("iz,zjkc->ijkc", self.Fy, b)

    def spec_inv(self, T):
        """T (kz, ky, kx, c) complex -> real (z, y, x, c)."""
        b = np.einsum("iz,ijkc->zjkc", self.Gy, T)
        a = np.einsum("jy,zjkc->zykc", self.Gy, b)
        return np.einsum("kx,zykc->zyxc", self.Gx, a).real

    def spec_inv_T(self, g):
        """Adjoint (as a real linear map) of spec_inv: real (z,y,x,c) -> complex cotangent."""
        a = np.einsum("kx,zyxc->zykc", np.conj(self.Gx), g)
        b = np.einsum("jy,zykc->zjkc", np.conj(self.Gy), a)
        return np.einsum("iz,zjkc->ijkc", np.conj(self.Gy), b)

    def spec_fwd_T(self, G):
        """Adjoint of spec_fwd: complex cotangent (kz,ky,kx,c) -> real (z,y,x,c)."""
        b = np.einsum("iz,ijkc->zjkc", np.conj(self.Fy), G)
        a = np.einsum("jy,zjkc->zykc", np.conj(self.Fy), b)
        return np.einsum("kx,zykc->zyxc", np.conj(self.Fx), a).real

    # -- network --------------------------------------------------------------
    def forward(self, p, x, keep=False):
        """x (z, y, x, cin) -> out (z, y, x, cout); keep=True also returns the tape."""
        tape = {}
        v = x @ p["W_lift"] + p["b_lift"]
        tape["x"] = x
        for l in range(self.L):
            tape["v%d" % l] = v
            S = self.spec_fwd(v)
            R = p["R%d_re" % l] + 1j * p["R%d_im" % l]
            T = np.einsum("ijkab,ijka->ijkb", R, S)
            tape["S%d" % l] = S
            pre = self.spec_inv(T) + v @ p["W%d" % l] + p["b%d" % l]
            tape["pre%d" % l] = pre
            v = gelu(pre) if l < self.L - 1 else pre
        tape["vL"] = v
        hpre = v @ p["P1"] + p["c1"]
        tape["hpre"] = hpre
        out = gelu(hpre) @ p["P2"] + p["c2"]
        return (out, tape) if keep else out

    def backward(self, p, tape, dout):
        """Gradients of sum(dout * out) with respect to every parameter."""
        g = {}
        hpre = tape["hpre"]
        hact = gelu(hpre)
        g["P2"] = np.einsum("zyxh,zyxo->ho", hact, dout)
        g["c2"] = dout.sum(axis=(0, 1, 2))
        dh = (dout @ p["P2"].T) * gelu_grad(hpre)
        vL = tape["vL"]
        g["P1"] = np.einsum("zyxc,zyxh->ch", vL, dh)
        g["c1"] = dh.sum(axis=(0, 1, 2))
        dv = dh @ p["P1"].T
        for l in reversed(range(self.L)):
            pre = tape["pre%d" % l]
            dpre = dv * gelu_grad(pre) if l < self.L - 1 else dv
            v = tape["v%d" % l]
            g["W%d" % l] = np.einsum("zyxa,zyxb->ab", v, dpre)
            g["b%d" % l] = dpre.sum(axis=(0, 1, 2))
            dT = self.spec_inv_T(dpre)                       # cotangent of T (as Re + i Im)
            S = tape["S%d" % l]
            # T = R S (complex, per mode): real-parameter gradients
            g["R%d_re" % l] = (np.einsum("ijka,ijkb->ijkab", S.real, dT.real)
                               + np.einsum("ijka,ijkb->ijkab", S.imag, dT.imag))
            g["R%d_im" % l] = (np.einsum("ijka,ijkb->ijkab", S.real, dT.imag)
                               - np.einsum("ijka,ijkb->ijkab", S.imag, dT.real))
            Rr, Ri = p["R%d_re" % l], p["R%d_im" % l]
            dS = (np.einsum("ijkab,ijkb->ijka", Rr, dT.real) + np.einsum("ijkab,ijkb->ijka", Ri, dT.imag)
                  + 1j * (np.einsum("ijkab,ijkb->ijka", Rr, dT.imag)
                          - np.einsum("ijkab,ijkb->ijka", Ri, dT.real)))
            dv = dpre @ p["W%d" % l].T + self.spec_fwd_T(dS)
        x = tape["x"]
        g["W_lift"] = np.einsum("zyxc,zyxw->cw", x, dv)
        g["b_lift"] = dv.sum(axis=(0, 1, 2))
        return g


def spectral_conv_fft(v, R, m):
    """The spectral convolution by its definition: rfftn, keep the corner modes, multiply, irfftn."""
    n = v.shape[0]
    V = np.fft.rfftn(v, axes=(0, 1, 2))
    out = np.zeros(V.shape[:3] + (R.shape[-1],), complex)
    kyz = np.concatenate([np.arange(m), np.arange(n - m, n)])
    for i, kz in enumerate(kyz):
        for j, ky in enumerate(kyz):
            for kx in range(m):
                out[kz, ky, kx] = V[kz, ky, kx] @ R[i, j, kx]
    return np.fft.irfftn(out, s=(n, n, n), axes=(0, 1, 2))


def mse_loss(pred, target):
    d = pred - target
    return float(np.mean(d * d)), 2.0 * d / d.size
