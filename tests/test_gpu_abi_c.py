"""The C ABI from a plain C caller (tests/native/abi_c_client.c: host arrays,
no Python or HIP of its own) against the FP64 oracle: three IMEX Euler steps
at 16^3 from the seeded small workload, whole state within 1e-10."""
import os
import subprocess

import numpy as np
import pytest

import pfinputs
from oracle import ark as oark
from oracle import model as om
from oracle import spectral as osp

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_client_imex_euler_matches_oracle(tmp_path, params):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[case] C ABI client 16^3", flush=True)
    exe = str(tmp_path / "client")
    lib = os.path.join(ROOT, "paper_2609_36100_amd")
    r = subprocess.run(["gcc", "-std=c99", "-O1", "-I", os.path.join(ROOT, "include"), "-o", exe,
                        os.path.join(ROOT, "tests", "native", "abi_c_client.c"), "-L", lib, "-lpf",
                        "-Wl,-rpath," + lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    n = 16
    _, c, eta = pfinputs.config("small32", n=n)
    np.concatenate([c[None], eta]).astype(np.float64).tofile(tmp_path / "in.bin")
    out = subprocess.run([exe, str(n), str(tmp_path / "in.bin"), str(tmp_path / "out.bin")],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, (out.returncode, out.stderr)
    assert int(out.stdout.strip()) == 3
    got = np.fromfile(tmp_path / "out.bin", dtype=np.float64).reshape(4, n, n, n)
    m = om.Model((n, n, n), params)
    y = om.to_kspace(c, eta)
    for _ in range(3):
        y, _, _ = oark.ark_step(y, 0.05, oark.imex_euler(), m.f_explicit, m.implicit_symbol())
    want = osp.irfft3(y, (n, n, n))
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
