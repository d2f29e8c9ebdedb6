"""Writes c1_replay_256.json: the FP64 oracle's first 50 accepted steps of
adaptive ARK4(3)6L (rtol 1e-6, atol 1e-9, dt0 0.01) on the 256^3 seeded
workload (seed 1001, 200 nuclei, radius 2-5, spacing 8): every attempt
(t, dt, error norm, accepted), and of the state after the 50th step the
real-space values at 1024 seeded points per field, the per-field L2 norms,
the mass and the volume fraction.  A GPU test replays the accepted steps and
compares (the full 256^3 state is 0.5 GB; the sample stands in for it).

Calls only the oracle and the seeded input generator (SciPy's FFT on all
cores for speed):
    python tests/golden/make_c1_replay.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import pfinputs  # noqa: E402
from oracle import ark, diagnostics as dg, model as om, spectral as sp  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_replay_256.json")
STEPS = 50
SAMPLES = 1024
SAMPLE_SEED = 4242


def sample_points(n, count, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, n, size=(count, 3))


def main():
    sp.set_fft_backend("scipy", workers=os.cpu_count())
    spec, c, eta = pfinputs.config("adaptive256")
    n = c.shape[0]
    m = om.Model((n, n, n), pfinputs.default_params())
    y = om.to_kspace(c, eta)
    del c, eta
    integ = ark.Integrator(m, table="ark436l", adaptive=True, dt0=0.01, rtol=1e-6, atol=1e-9)
    t0 = time.time()
    y, t = integ.advance(y, 0.0, 500.0, max_steps=STEPS)
    print("%d steps, %d rejects, t = %.6f (%.0f s)" % (integ.stats["steps"], integ.stats["rejects"], t,
                                                        time.time() - t0), flush=True)
    u = sp.irfft3(y, m.shape)
    pts = sample_points(n, SAMPLES, SAMPLE_SEED)
    vf, vf_thr = dg.volume_fraction(m, y)
    out = dict(
        workload=dict(name="adaptive256", n=n, seed=spec["seed"], n_nuclei=spec["n_nuclei"]),
        method="ark436l", rtol=1e-6, atol=1e-9, dt0=0.01, steps=integ.stats["steps"],
        rejects=integ.stats["rejects"], t=t,
        attempts=[dict(t=a[0], dt=a[1], err=a[2], accepted=a[3]) for a in integ.stats["log"]],
        sample_seed=SAMPLE_SEED, points=pts.tolist(),
        values=[[float(u[f][tuple(p)]) for p in pts] for f in range(4)],
        l2=[float(np.sqrt(np.sum(u[f] ** 2))) for f in range(4)],
        mass=float(dg.mass(y, m.shape)), vf=float(vf), vf_threshold=float(vf_thr),
        note="written by tests/golden/make_c1_replay.py (oracle only)")
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
