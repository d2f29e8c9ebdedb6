"""Learned surrogate beside the plain method: training data, training, and the
checked surrogate advance.

* :func:`reference_dt` -- the mean accepted step of adaptive ARK4(3)6L on a
  training run; the surrogate's interval is ``delta = 10 * dt_ref``.
* :func:`generate_snapshots` -- plain adaptive ARK4(3)6L (libpf) from seeded
  initial conditions, the real-space state kept every ``delta``; consecutive
  snapshots are the training pairs (state, state delta later).
* :func:`train` -- Adam on the MSE of the per-channel-scaled increments
  (libpf BF16 MFMA forward/backward kernels).
* :func:`validate` -- relative L2 error of c after one surrogate advance
  against the stored plain-solver snapshot.
* :func:`checked_advance` -- the surrogate advance with periodic plain checks
  and fallback (``pf_fno_advance``).

Arithmetic runs in libpf; torch only holds device buffers and, once, the
per-channel spread of the training increments.
"""
from __future__ import annotations

import time

import numpy as np

import pfinputs

from . import FNO, FnoStats, Solver, rel_l2

ARK4 = "ark436l"


def _torch():
    import torch
    return torch


def reference_dt(n=128, run=0, t_end=10.0, rtol=1e-6, atol=1e-9, base_seed=3000, nuclei=(10, 80)):
    """Mean accepted adaptive ARK4(3)6L step over [0, t_end] of one training run."""
    ic = pfinputs.surrogate_run(run, n, base_seed, nuclei)
    with Solver(n, None, method=ARK4, adaptive=True, dt0=0.01, rtol=rtol, atol=atol) as s:
        s.set_state(ic["c"], ic["eta"])
        st = s.advance(t_end)
    return t_end / st["steps"], st


def generate_snapshots(n=128, runs=40, snapshots=50, delta=0.5, rtol=1e-6, atol=1e-9, base_seed=3000,
                       nuclei=(10, 80), log=None):
    """float32 device tensor (runs, snapshots + 1, 4, n, n, n): the plain solver's state every delta."""
    torch = _torch()
    out = torch.empty((runs, snapshots + 1, 4, n, n, n), dtype=torch.float32, device="cuda")
    u = torch.empty((4, n, n, n), dtype=torch.float64, device="cuda")
    steps = 0
    for r in range(runs):
        ic = pfinputs.surrogate_run(r, n, base_seed, nuclei)
        with Solver(n, None, method=ARK4, adaptive=True, dt0=0.01, rtol=rtol, atol=atol) as s:
            s.set_state(ic["c"], ic["eta"])
            out[r, 0] = s.get_state_device(u).float()
            for i in range(1, snapshots + 1):
                st = s.advance(i * delta)
                out[r, i] = s.get_state_device(u).float()
            steps += st["steps"]
        if log:
            log("snapshots: run %d/%d (%d plain steps so far)" % (r + 1, runs, steps))
    return out, steps


def increment_scale(snaps, train_runs):
    """Per-channel RMS of the snapshot increments over the training runs."""
    acc = np.zeros(4)
    cnt = 0
    for r in range(train_runs):
        d = (snaps[r, 1:] - snaps[r, :-1]).double()
        acc += (d * d).sum(dim=(0, 2, 3, 4)).cpu().numpy()
        cnt += d.shape[0] * d[0, 0].numel()
    return np.maximum(np.sqrt(acc / cnt), 1e-12)


def state_norm(snaps, train_runs):
    """Per-channel mean and standard deviation of the training states (the
    network's input normalisation, so that bf16 resolves the deviations)."""
    s1 = np.zeros(4)
    s2 = np.zeros(4)
    cnt = 0
    for r in range(train_runs):
        d = snaps[r].double()
        s1 += d.sum(dim=(0, 2, 3, 4)).cpu().numpy()
        s2 += (d * d).sum(dim=(0, 2, 3, 4)).cpu().numpy()
        cnt += d.shape[0] * d[0, 0].numel()
    mean = s1 / cnt
    std = np.sqrt(np.maximum(s2 / cnt - mean * mean, 0.0))
    return mean, np.maximum(std, 1e-6)


def param_shapes(width, modes, layers, hidden, cin=4, cout=4):
    """(name, shape) of every parameter block in the flat libpf order."""
    m2 = 2 * modes
    shp = [("W_lift", (cin, width)), ("b_lift", (width,))]
    for l in range(layers):
        shp += [("R%d_re" % l, (m2, m2, modes, width, width)), ("R%d_im" % l, (m2, m2, modes, width, width)),
                ("W%d" % l, (width, width)), ("b%d" % l, (width,))]
    shp += [("P1", (width, hidden)), ("c1", (hidden,)), ("P2", (hidden, cout)), ("c2", (cout,))]
    return shp


def init_params(width, modes, layers, hidden, cin=4, cout=4, seed=0):
    """Seeded initial parameters: spectral weights U(-1, 1) / width^2, dense
    weights N(0, 1) / sqrt(fan-in), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shp in param_shapes(width, modes, layers, hidden, cin, cout):
        if name.startswith("R"):
            parts.append(rng.uniform(-1.0, 1.0, shp) / (width * width))
        elif name[0] in "bc":
            parts.append(np.zeros(shp))
        else:
            parts.append(rng.standard_normal(shp) / np.sqrt(shp[0]))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def make_fno(n=128, width=32, modes=12, layers=4, hidden=128, seed=0, scale=None, norm=None):
    """FNO with seeded parameters, output scale (per channel) and input
    normalisation ((mean, std) per channel)."""
    f = FNO(n, width=width, modes=modes, layers=layers, hidden=hidden)
    f.set_params(init_params(width, modes, layers, hidden, seed=seed))
    if scale is not None:
        f.set_scale(scale)
    if norm is not None:
        f.set_input_norm(norm[0], norm[1])
    return f


def train(fno, snaps, train_runs, epochs=4, lr=1e-3, lr_final=None, batch=4, seed=0, log=None,
          time_limit=None):
    """Adam on the MSE of the scaled increments; cosine learning-rate decay to
    lr_final (default lr / 10).  Returns the per-epoch mean losses."""
    ns = snaps.shape[1] - 1
    pairs = [(r, k) for r in range(train_runs) for k in range(ns)]
    rng = np.random.Generator(np.random.PCG64(seed))
    lr_final = lr / 10 if lr_final is None else lr_final
    nb = (len(pairs) + batch - 1) // batch
    total = epochs * nb
    it = 0
    hist = []
    t_start = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tot = 0.0
        t0 = time.perf_counter()
        for i0 in range(0, len(order), batch):
            fno.zero_grad()
            idx = order[i0:i0 + batch]
            for j in idx:
                r, k = pairs[j]
                tot += fno.grad(snaps[r, k], snaps[r, k + 1])
            a = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * it / max(total - 1, 1)))
            fno.adam_step(float(a), grad_scale=1.0 / len(idx))
            it += 1
        hist.append(tot / len(pairs))
        if log:
            log("epoch %d: loss %.4e (%.1f s)" % (ep, hist[-1], time.perf_counter() - t0))
        if time_limit is not None and time.perf_counter() - t_start > time_limit:
            break
    return hist


def validate(fno, snaps, runs):
    """Scores one surrogate advance against the stored plain-solver snapshots.

    Returns (err, keep, inc): per pair the relative L2 error of c and the same
    for the no-change guess, and per channel the relative L2 error of the
    predicted increment over all the pairs."""
    torch = _torch()
    n = snaps.shape[-1]
    u = torch.empty((4, n, n, n), dtype=torch.float64, device="cuda")
    nxt = torch.empty_like(u)
    ref = torch.empty_like(u)
    err, keep = [], []
    num = np.zeros(4)
    den = np.zeros(4)
    for r in runs:
        for k in range(snaps.shape[1] - 1):
            u.copy_(snaps[r, k])
            ref.copy_(snaps[r, k + 1])
            fno.apply(u, nxt)
            err.append(rel_l2(nxt[0], ref[0]))
            keep.append(rel_l2(u[0], ref[0]))
            num += ((nxt - ref) ** 2).sum(dim=(1, 2, 3)).cpu().numpy()
            den += ((u - ref) ** 2).sum(dim=(1, 2, 3)).cpu().numpy()
    return np.array(err), np.array(keep), np.sqrt(num / np.maximum(den, 1e-300))


def checked_advance(fno, plain, u, t_final, delta, check_every=5, tol=1e-3, stats=None):
    """Advance u (device float64 (4, n, n, n), in place) to t_final with the checked
    surrogate; returns the FnoStats."""
    n_adv = int(round(t_final / delta))
    assert abs(n_adv * delta - t_final) < 1e-9 * max(1.0, t_final), "t_final must be a multiple of delta"
    return fno.advance(plain, u, n_adv, delta, check_every, tol, stats if stats is not None else FnoStats())
