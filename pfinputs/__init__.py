"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This module only draws random numbers and paints initial fields; it holds none
of the phase-field method's arithmetic (no free energy, no transforms, no time
integration).  Both the product path and the oracle consume the arrays it
returns, so they start from bit-identical inputs.

Field layout: C order ``[z][y][x]`` (x fastest), float64.  ``eta`` is stacked
``[3][z][y][x]`` for the three orientation variants.

Initial conditions follow the paper's description of seeded precipitate
nuclei (pseudorandom positions and orientation variants at a fixed number
density; Results, "Improved performance via GPU acceleration") and its
two-particle geometry (Results, "Improved performance via time integration
approach"), restated on the dimensionless model in grid units.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "default_params",
    "seeded_nuclei",
    "two_particle",
    "single_mode",
    "config",
    "ensemble_members",
]

# Matrix / precipitate reference compositions and model constants of the
# dimensionless stand-in model (values only).
def default_params() -> dict:
    """Model constants of the dimensionless stand-in model (values, no arithmetic)."""
    return dict(
        dx=1.0,
        W=1.0, w=1.0, kappa_c=1.0, kappa_eta=1.0, M=1.0, L=1.0,
        c_m=0.02, c_p=0.25,
        C11=250.0, C12=150.0, C44=120.0,
        # diagonal eigenstrain of variant v: 0.0286 along axis v, 0.0067 on the others
        eps_star=[[0.0286, 0.0067, 0.0067],
                  [0.0067, 0.0286, 0.0067],
                  [0.0067, 0.0067, 0.0286]],
        eps_bar=[0.0, 0.0, 0.0],
        mean_strain_mode=0,      # 0: prescribed mean strain (eps_bar), 1: stress-free
        implicit_bulk_c=1,       # 1: 2W k^2 bulk term implicit (split B), 0: split A
    )


def _periodic_dist2(a, b, n):
    d = np.abs(np.asarray(a, float) - np.asarray(b, float))
    d = np.minimum(d, n - d)
    return float(np.sum(d * d))


def seeded_nuclei(n, seed, c0=0.16, n_nuclei=4, radius=3, d_min=8.0,
                  noise=0.005, c_in=0.25, max_attempts=100000, rng=None):
    """Matrix with uniform noise plus sharp spherical nuclei of random variant.

    Draw order from ``numpy.random.Generator(PCG64(seed))``: the noise field
    ``U(-noise, noise)`` in C order, then per nucleus attempt: centre
    ``U[0, n)^3`` (x, y, z), radius (integer, uniform in ``[lo, hi]`` when
    ``radius`` is a pair), variant in {1, 2, 3}.  A centre closer than
    ``d_min`` (periodic minimum image) to an accepted centre is rejected.
    Points with periodic distance ``<= R`` to a centre get ``eta_v = 1``, the
    other order parameters 0 and ``c = c_in``; later nuclei overwrite earlier.
    Returns ``(c, eta, nuclei)`` with ``nuclei`` a list of (x, y, z, R, v).
    """
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    c = c0 + rng.uniform(-noise, noise, size=(n, n, n))
    eta = np.zeros((3, n, n, n))
    nuclei = []
    attempts = 0
    while len(nuclei) < n_nuclei and attempts < max_attempts:
        attempts += 1
        ctr = rng.uniform(0.0, n, size=3)
        if isinstance(radius, (tuple, list)):
            r = int(rng.integers(radius[0], radius[1] + 1))
        else:
            r = radius
        v = int(rng.integers(1, 4))
        if any(_periodic_dist2(ctr, q[:3], n) < d_min * d_min for q in nuclei):
            continue
        nuclei.append((float(ctr[0]), float(ctr[1]), float(ctr[2]), float(r), v))
    for (x0, y0, z0, r, v) in nuclei:
        _paint(c, eta, n, (x0, y0, z0), r, v, c_in)
    return c, eta, nuclei


def _paint(c, eta, n, ctr, r, v, c_in):
    x0, y0, z0 = ctr
    lo = [int(np.floor(q - r)) for q in (x0, y0, z0)]
    hi = [int(np.ceil(q + r)) for q in (x0, y0, z0)]
    xs = np.arange(lo[0], hi[0] + 1)
    ys = np.arange(lo[1], hi[1] + 1)
    zs = np.arange(lo[2], hi[2] + 1)

    def md(idx, q):
        d = np.abs(idx - q)
        d = np.mod(d, n)
        return np.minimum(d, n - d)

    dz = md(zs, z0)[:, None, None]
    dy = md(ys, y0)[None, :, None]
    dxx = md(xs, x0)[None, None, :]
    inside = (dz * dz + dy * dy + dxx * dxx) <= r * r
    zi, yi, xi = np.nonzero(inside)
    gz, gy, gx = np.mod(zs[zi], n), np.mod(ys[yi], n), np.mod(xs[xi], n)
    eta[:, gz, gy, gx] = 0.0
    eta[v - 1, gz, gy, gx] = 1.0
    c[gz, gy, gx] = c_in


def two_particle(n=64, c0=0.16, variant=1, c_in=0.25):
    """Two seeds of one variant: radius 5 at (20, 31, 31), radius 6 at (41, 41, 41).

    The paper's 64^3, 0.5 nm two-particle geometry (2.5 nm seed at
    (10, 15.5, 15.5) nm and 3 nm seed at (20.5, 20.5, 20.5) nm) in grid units.
    No noise: the field is deterministic.
    """
    c = np.full((n, n, n), float(c0))
    eta = np.zeros((3, n, n, n))
    s = n / 64.0
    _paint(c, eta, n, (20 * s, 31 * s, 31 * s), 5 * s, variant, c_in)
    _paint(c, eta, n, (41 * s, 41 * s, 41 * s), 6 * s, variant, c_in)
    return c, eta


def single_mode(n, m=(1, 0, 0), amp=1e-3, c0=0.16, phase=0.0):
    """``c = c0 + amp cos(2 pi (m . r)/n + phase)`` with eta = 0 (one Fourier mode)."""
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    arg = 2.0 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / n + phase
    c = c0 + amp * np.cos(arg)
    return c, np.zeros((3, n, n, n))


# Named synthetic workloads -------------------------------------------------
_WORKLOADS = {
    # 32^3 IMEX Euler, dt 0.05, 200 steps; 4 nuclei radius 3
    "small32": dict(n=32, seed=1000, c0=0.16, n_nuclei=4, radius=3, d_min=8.0,
                    method="imex_euler", dt=0.05, steps=200),
    # 256^3 adaptive ARK4(3)6L to t=500; ~200 nuclei, radius 2..5, spacing 8
    "adaptive256": dict(n=256, seed=1001, c0=0.16, n_nuclei=200, radius=(2, 5),
                        d_min=8.0, method="ark436l", rtol=1e-6, atol=1e-9,
                        t_final=500.0),
    # 512^3 throughput workload; ~1600 nuclei
    "mixed512": dict(n=512, seed=1002, c0=0.16, n_nuclei=1600, radius=(2, 5),
                     d_min=8.0, method="ark436l", rtol=1e-5, atol=1e-9),
    # the 64^3 twin: same seed, nucleus count scaled by volume
    "twin64": dict(n=64, seed=1002, c0=0.16, n_nuclei=3, radius=(2, 5),
                   d_min=8.0, method="ark436l", rtol=1e-5, atol=1e-9),
}


def config(name, n=None):
    """Return ``(spec, c, eta)`` for a named workload; ``n`` overrides the size.

    Overriding ``n`` scales the nucleus count by volume (at least 1).
    """
    spec = dict(_WORKLOADS[name])
    if n is not None and n != spec["n"]:
        scale = (n / spec["n"]) ** 3
        spec["n_nuclei"] = max(1, int(round(spec["n_nuclei"] * scale)))
        spec["n"] = n
    c, eta, nuc = seeded_nuclei(spec["n"], spec["seed"], c0=spec["c0"],
                                n_nuclei=spec["n_nuclei"], radius=spec["radius"],
                                d_min=spec["d_min"])
    spec["nuclei"] = nuc
    return spec, c, eta


def ensemble_members(count=64, base_seed=2000, sizes=(48, 64, 96, 128),
                     make_fields=True):
    """Uneven-size ensemble: per member m, seed ``base_seed + m``.

    Draw order per member: size index, ``c0 ~ U(0.14, 0.18)``, nucleus count
    in [10, 80], then the fields as in :func:`seeded_nuclei` (radius 2..5,
    spacing 8) from the same generator.
    """
    out = []
    for m in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + m))
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        c0 = float(rng.uniform(0.14, 0.18))
        k = int(rng.integers(10, 81))
        item = dict(member=m, n=n, c0=c0, n_nuclei=k, seed=base_seed + m)
        if make_fields:
            c, eta, nuc = seeded_nuclei(n, None, c0=c0, n_nuclei=k, radius=(2, 5),
                                        d_min=8.0, rng=rng)
            item.update(c=c, eta=eta, nuclei=nuc)
        out.append(item)
    return out


def surrogate_run(r, n=128, base_seed=3000, nuclei=(10, 80)):
    """Initial condition of training run ``r`` for the learned surrogate: seed
    ``base_seed + r``, draw order ``c0 ~ U(0.14, 0.18)``, nucleus count in
    ``nuclei`` (inclusive), then the fields as in :func:`seeded_nuclei`
    (radius 2..5, spacing 8) -- the ensemble members' distribution at one
    fixed size."""
    rng = np.random.Generator(np.random.PCG64(base_seed + r))
    c0 = float(rng.uniform(0.14, 0.18))
    k = int(rng.integers(nuclei[0], nuclei[1] + 1))
    c, eta, nuc = seeded_nuclei(n, None, c0=c0, n_nuclei=k, radius=(2, 5), d_min=8.0, rng=rng)
    return dict(run=r, n=n, c0=c0, n_nuclei=k, seed=base_seed + r, c=c, eta=eta, nuclei=nuc)
