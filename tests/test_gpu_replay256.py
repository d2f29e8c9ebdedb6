"""The 256^3 adaptive workload against the FP64 oracle over its first 50
steps (Methods, "Time integration": the ARK step, its embedded error and the
WRMS norm; the step sequence is the oracle's).  Accept/reject decisions near
err = 1 can flip between two correct implementations, so the oracle's
accepted step sizes are replayed as fixed steps: the GPU's error norm of
every step, the time reached, the per-field L2 norms of the final state and
its values at 1024 seeded points per field are compared with the oracle's
(tests/golden/c1_replay_256.json, written by make_c1_replay.py from the
oracle alone)."""
import json
import os
import sys

import numpy as np
import pytest

import pfinputs

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_replay_256.json")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible GPU"
    return _t


def test_first_50_steps_at_256_match_oracle(torch, params):
    from paper_2609_36100_amd import Solver
    fx = json.load(open(FIXTURE))
    n = fx["workload"]["n"]
    _say("replay 256^3, %d steps" % fx["steps"])
    spec, c, eta = pfinputs.config(fx["workload"]["name"])
    assert spec["seed"] == fx["workload"]["seed"] and c.shape == (n, n, n)
    accepted = [a for a in fx["attempts"] if a["accepted"]]
    assert len(accepted) == fx["steps"] == 50
    with Solver(n, params, method=fx["method"], adaptive=False, rtol=fx["rtol"], atol=fx["atol"]) as s:
        s.set_state(c, eta)
        del c, eta
        for k, a in enumerate(accepted):
            acc, err, _ = s.step(a["dt"])
            assert acc
            assert abs(err - a["err"]) <= 1e-6 * a["err"], (k, err, a["err"])
        st = s.stats()
        assert abs(st["t"] - fx["t"]) <= 1e-12 * fx["t"]
        cg, etag = s.get_state()
    fields = [cg, etag[0], etag[1], etag[2]]
    idx = tuple(np.asarray(fx["points"]).T)
    for f in range(4):
        o = np.asarray(fx["values"][f])
        g = fields[f][idx]
        rel = np.linalg.norm(g - o) / max(np.linalg.norm(o), 1e-300)
        l2 = float(np.sqrt(np.sum(fields[f] ** 2)))
        print("field", f, "sampled rel-L2", rel, "norm", l2, fx["l2"][f], flush=True)
        assert rel <= 1e-10, (f, rel)
        assert abs(l2 - fx["l2"][f]) <= 1e-12 * max(fx["l2"][f], 1e-300), (f, l2, fx["l2"][f])
