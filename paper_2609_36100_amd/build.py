"""Build libpf.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

The library carries the identifier of the sources it was built from
(``pf_build_id``): a SHA-256 over the kernel, runtime and header sources.
The binding recomputes it from the sources beside the library and refuses a
library built from other sources.
"""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("pf_runtime.hip", "pf_ensemble.hip", "pf_fno.hip")]
OUT = os.path.join(HERE, "libpf.so")
OBJDIR = os.path.join(HERE, "_build")


def source_files():
    """Every file that goes into libpf.so, in a fixed order."""
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) + glob.glob(os.path.join(HERE, "csrc", "*.hpp")))
    return files + [os.path.join(ROOT, "include", "pf.h")]


def source_id():
    """First 16 hex digits of SHA-256 over (relative path, contents) of the sources."""
    h = hashlib.sha256()
    for f in source_files():
        h.update(os.path.relpath(f, ROOT).encode())
        h.update(b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()[:16]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep hipcc from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose=True):
    """Compile every translation unit in parallel, then link libpf.so."""
    hipcc = os.environ.get("HIPCC", "hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    t0 = time.time()
    bid = source_id()
    procs = []
    objs = []
    for src in SRCS:
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append((src, subprocess.Popen([hipcc, *HIPCC_FLAGS, '-DPF_BUILD_ID="%s"' % bid, "-c", "-o", obj, src],
                                            stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    failed = False
    for src, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(err)
            failed = True
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = OUT + ".tmp"
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("link failed (%d)" % r.returncode)
    os.replace(tmp, OUT)
    if verbose:
        print("built %s (sources %s) in %.1fs" % (OUT, bid, time.time() - t0), flush=True)
    return OUT


if __name__ == "__main__":
    build()
