"""Writes vf_curve_twin64.txt: the FP64 oracle's volume fraction, threshold
fraction, mass and free energy at t = 0, 1, ..., 20 on the 64^3 twin of the
512^3 seeded workload (same generator and seed, nucleus count scaled by
volume), advanced by adaptive ARK4(3)6L at rtol 1e-6, atol 1e-9.

Calls only the oracle and the seeded input generator:
    python tests/golden/make_vf_curve.py
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import pfinputs  # noqa: E402
from oracle import ark, diagnostics as dg, model as om  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "vf_curve_twin64.txt")


def main():
    spec, c, eta = pfinputs.config("twin64")
    n = c.shape[0]
    m = om.Model((n, n, n), pfinputs.default_params())
    y = om.to_kspace(c, eta)
    integ = ark.Integrator(m, table="ark436l", adaptive=True, dt0=0.01, rtol=1e-6, atol=1e-9)
    rows = []
    t = 0.0
    t0 = time.time()
    for k in range(0, 21):
        if k > 0:
            y, t = integ.advance(y, t, float(k))
        vf, thr = dg.volume_fraction(m, y)
        rows.append((float(k), vf, thr, dg.mass(y, m.shape), dg.free_energy(m, y), integ.stats["steps"],
                     integ.stats["rejects"]))
        print("t=%g vf=%.6e thr=%.6e steps=%d (%.0f s)" % (k, vf, thr, integ.stats["steps"], time.time() - t0),
              flush=True)
    with open(OUT, "w") as f:
        f.write("# oracle: 64^3 twin (seed %d, %d nuclei), adaptive ARK4(3)6L rtol 1e-6 atol 1e-9, dt0 0.01\n"
                % (spec["seed"], spec["n_nuclei"]))
        f.write("# written by tests/golden/make_vf_curve.py (oracle only)\n")
        f.write("# t vf vf_threshold mass F steps rejects\n")
        for r in rows:
            f.write("%g %.17e %.17e %.17e %.17e %d %d\n" % r)


if __name__ == "__main__":
    main()
