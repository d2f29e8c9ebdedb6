"""Host-only checks of libpf: it loads without a GPU and exports every symbol pf.h declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2609_36100_amd import _lib
    L = _lib.lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    # the Python binding binds exactly the declared entry points
    assert sorted(_lib.exported_symbols()) == names


def test_host_only_entry_points():
    from paper_2609_36100_amd import _lib
    L = _lib.lib()
    p = _lib.Params()
    assert L.pf_default_params(ctypes.byref(p)) == 0
    assert (p.C11, p.C12, p.C44) == (250.0, 150.0, 120.0)
    assert p.eps_star[1][1] == 0.0286 and p.eps_star[1][0] == 0.0067
    for n in (8, 16, 24, 32, 48, 56, 64, 96, 128, 168, 256, 336, 504, 512):
        assert L.pf_size_supported(n) == 1, n
    # not a multiple of 8, a prime factor above 7, beyond 512, or not in the compiled set
    for n in (6, 10, 12, 28, 88, 104, 112, 144, 1024, 7, 0, -8):
        assert L.pf_size_supported(n) == 0, n
    assert L.pf_status_string(-4) == b"PF_ERR_UNSUPPORTED_SIZE"
    assert L.pf_status_string(12345) == b"PF_UNKNOWN_STATUS"
    assert L.pf_init(None, None, None) == -1


def test_argument_checks_precede_any_device_work():
    """Invalid parameters are rejected on the host, before the library touches
    a device (so these run without a GPU)."""
    from paper_2609_36100_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()

    def init(**over):
        p = _lib.make_params(32, None)
        for k, v in over.items():
            setattr(p, k, v)
        return L.pf_init(ctypes.byref(p), None, ctypes.byref(h))

    assert init(dx=0.0) == -1
    assert init(M=-1.0) == -1
    assert init(precision=7) == -1
    assert init(method=5) == -1 and init(method=0) == -1
    assert init(method=_lib.PF_IMEX_EULER, adaptive=1) == -1      # no embedding to control with
    assert init(method=_lib.PF_ARK2, adaptive=1, atol=0.0) == -1
    assert init(mean_strain_mode=2) == -1
    assert init(norm_space=2) == -1 and init(norm_space=-1) == -1
    # inhomogeneous elasticity: FP64, prescribed mean strain, stable cubic constants
    inh = dict(elastic_inhom=1, C11p=375.0, C12p=225.0, C44p=180.0)
    assert init(precision=_lib.PF_MIXED, **inh) == -1
    assert init(mean_strain_mode=1, **inh) == -1
    assert init(**dict(inh, C12p=400.0)) == -1 and init(**dict(inh, C44p=0.0)) == -1
    assert init(el_max_iter=-1, **inh) == -1 and init(el_tol=-1.0, **inh) == -1
    assert init(elastic_inhom=2) == -1
    assert init(nx=7) == -4 and init(nz=88) == -4
    # ensembles: cubic supported sizes, one embedded method, one precision
    arr = (_lib.Params * 2)()
    arr[0] = _lib.make_params(32, None)
    arr[1] = _lib.make_params(48, None)
    assert L.pf_ensemble_init(0, arr, None, ctypes.byref(h)) == -1
    arr[1] = _lib.make_params(256, None)
    assert L.pf_ensemble_init(2, arr, None, ctypes.byref(h)) == -4
    arr[1] = _lib.make_params(48, None, method="imex_euler")
    assert L.pf_ensemble_init(2, arr, None, ctypes.byref(h)) == -1
    arr[1] = _lib.make_params(48, None, method="ark324l")
    assert L.pf_ensemble_init(2, arr, None, ctypes.byref(h)) == -1          # mixed methods
    arr[1] = _lib.make_params(48, None, norm_space=1)
    assert L.pf_ensemble_init(2, arr, None, ctypes.byref(h)) == -1          # k-space norm only
    arr[1] = _lib.make_params(48, dict(C11p=375.0, C12p=225.0, C44p=180.0))
    assert arr[1].elastic_inhom == 1
    assert L.pf_ensemble_init(2, arr, None, ctypes.byref(h)) == -1          # homogeneous elasticity only
    arr[1] = _lib.make_params(48, None, precision="mixed")
    assert L.pf_ensemble_init(2, arr, None, ctypes.byref(h)) == -1
    # the surrogate's shape limits
    for bad in [(12, 32, 12, 4, 128, 4, 4), (128, 30, 12, 4, 128, 4, 4), (128, 32, 11, 4, 128, 4, 4),
                (128, 32, 12, 4, 130, 4, 4), (16, 32, 12, 4, 128, 4, 4), (128, 32, 12, 0, 128, 4, 4)]:
        cfg = _lib.FnoConfig(*bad)
        assert L.pf_fno_create(ctypes.byref(cfg), None, ctypes.byref(h)) == -1, bad
    d = ctypes.c_double()
    assert L.pf_bandwidth_probe(1000, 5, None, ctypes.byref(d), ctypes.byref(d), ctypes.byref(d)) == -1
    assert L.pf_rel_l2(None, None, 10, None, ctypes.byref(d)) == -1


def test_params_struct_matches_header_layout():
    """sizeof of the ABI structs seen by ctypes equal the C compiler's."""
    from paper_2609_36100_amd import _lib
    src = ('#include "pf.h"\n#include <stdio.h>\n'
           'int main(){printf("%zu %zu %zu %zu\\n", sizeof(pf_params), sizeof(pf_stats), sizeof(pf_fno_config),'
           ' sizeof(pf_fno_stats));return 0;}\n')
    exe = "/tmp/pf_sizeof_check"
    r = subprocess.run(["gcc", "-x", "c", "-I", os.path.join(ROOT, "include"), "-o", exe, "-"],
                       input=src, text=True, capture_output=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True).stdout.split()
    assert int(out[0]) == ctypes.sizeof(_lib.Params)
    assert int(out[1]) == ctypes.sizeof(_lib.Stats)
    assert int(out[2]) == ctypes.sizeof(_lib.FnoConfig)
    assert int(out[3]) == ctypes.sizeof(_lib.FnoStats)


def test_fft_building_blocks_on_host():
    """Plans, radix DFTs, Stockham indexing and r2c/c2r packing against a naive DFT."""
    exe = "/tmp/pf_fft_host_check"
    r = subprocess.run(["hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-o", exe,
                        os.path.join(ROOT, "tests", "native", "fft_host_check.cpp")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    lines = [l.split() for l in out.stdout.strip().splitlines()]
    assert len(lines) >= 60
    for name, n, err in lines:
        assert float(err) < 1e-14, (name, n, err)


def test_plain_c_client_builds_and_reports_missing_device():
    """include/pf.h is plain C: a C99 client compiles and links against libpf.so;
    on a machine without a GPU its pf_init fails with PF_ERR_HIP, not a crash."""
    exe = "/tmp/pf_abi_c_client"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-O1", "-I", os.path.join(ROOT, "include"), "-o", exe,
                        os.path.join(ROOT, "tests", "native", "abi_c_client.c"),
                        "-L", os.path.join(ROOT, "paper_2609_36100_amd"), "-lpf",
                        "-Wl,-rpath," + os.path.join(ROOT, "paper_2609_36100_amd")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present: the GPU test runs this client")
    import numpy as np
    np.zeros(4 * 8 ** 3).tofile("/tmp/pf_abi_in.bin")
    out = subprocess.run([exe, "8", "/tmp/pf_abi_in.bin", "/tmp/pf_abi_out.bin"], capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 10 and "PF_ERR_HIP" in out.stderr, (out.returncode, out.stderr)


def test_every_bench_mode_has_its_driver():
    """bench.py's modes dispatch to module-level drivers; each must exist (a
    missing one would only show when that mode runs on a GPU)."""
    import bench
    for name in ("run_solver", "fft_bench", "cpu_baseline", "ensemble_bench", "time_to_t_bench",
                 "orders_bench", "oracle_timing", "fno_bench", "fno_step_bench", "measured_traffic"):
        assert callable(getattr(bench, name, None)), name
    src = open(os.path.join(ROOT, "bench.py")).read()
    for mode in ("ensemble", "time_to_t", "fno", "fno_step", "orders", "oracle_timing"):
        assert 'args.mode == "%s"' % mode in src, mode


def test_build_id_matches_sources_and_stale_library_is_refused(monkeypatch):
    """The library carries the hash of the sources it was built from; the
    binding refuses a library whose hash differs from the sources beside it."""
    from paper_2609_36100_amd import _lib, build
    L = _lib.lib()
    assert L.pf_build_id().decode() == build.source_id()
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "source_id", lambda: "0" * 16)
    with pytest.raises(ImportError, match="stale"):
        _lib.lib()
