#!/usr/bin/env python
"""Throughput of the ImEx-ARK stage cycle of the pseudospectral phase-field method.

Workload: the 512^3 precision-form configuration (about 1600 seeded spherical
nuclei of radius 2-5, spacing 8, c0 = 0.16 +- 0.005) advanced by fixed-step
ARK4(3)6L (6 explicit RHS stages per step), first in FP64 (`value`), then
with FP32 FFT/pointwise/elastic work and FP64 stage sums (`mixed`).  A step
is one full pass of the hot path: six stage-combine + implicit-solve +
explicit-RHS cycles and the update / embedded-error / WRMS finalize.  Inputs
are resident on the GPU before timing starts.

Prints ONE JSON line.  Extra objects:
  roofline      dominant kernel's algorithmic bytes per launch / average
                launch time (HIP events around each launch on the library's
                stream, inside the timed region) against 8 TB/s HBM, and
                against the streaming probe's copy rate below;
  hbm_probe     what plain streaming kernels draw from HBM on this device
                (copy, read-only, eleven reads + one write), GB/s;
  kernels       the same for every kernel class;
  mixed         the mixed-precision run of the same workload;
  fft           standalone forward + inverse 3D real FFT of 4 fields (FP64);
  time_to_t     time to simulated time t = 2 of the same 512^3 workload with
                adaptive ARK4(3)6L at rtol 1e-5 (atol 1e-8), FP64 and mixed,
                each against a plain FP64 rtol 1e-8 reference: wall time,
                steps, volume-fraction error and per-field state error, and the
                mixed form's gain over FP64;
  cpu_baseline  the FP64 CPU oracle on a bounded sample (one ARK4 step at
                128^3 of the same seeded generator), one thread.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mpts·stages/s at 512^3 (FP64 vs FP32-mixed); FFT HBM GB/s; time-to-t at tol"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


COUNTERS_MD = os.path.join(ROOT, "profiles", "ark4_stage_cycle_512_hbm_counters.md")


def measured_traffic():
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary,
    or None once the kernel sources differ from those the counters were taken on."""
    import hashlib
    try:
        text = open(COUNTERS_MD).read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        h = hashlib.sha256()
        for f in blob["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != blob["sources_sha256"]:
            return None
        return blob["traffic"]
    except (OSError, IndexError, ValueError, KeyError):
        return None


def kernel_table(rep):
    out = {}
    for name, (ms, n, b) in rep.items():
        avg_ms = ms / n
        gbs = (b / n) / (avg_ms * 1e-3) / 1e9
        out[name] = dict(launches=n, avg_ms=round(avg_ms, 4), total_ms=round(ms, 3),
                         bytes_per_launch=b / n, gbs=round(gbs, 1),
                         frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


def run_solver(torch, n, c, eta, precision, steps, warmup, dt, variants=None):
    from paper_2609_36100_amd import Solver
    s = Solver(n, None, method="ark436l", precision=precision, dt0=dt)
    # the state handed over in host memory (pageable NumPy arrays): the PCIe
    # copy and the forward transform, timed for the PCIe-inclusive figure
    ch, eh = (c.cpu().numpy(), eta.cpu().numpy()) if isinstance(c, torch.Tensor) else (c, eta)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    s.set_state(ch, eh)
    torch.cuda.synchronize()
    t_set = time.perf_counter() - ts
    del ch, eh
    tuning = s.autotune(3)          # tile plans, chosen before the timed region
    if variants:                    # fixed plans (e.g. to repeat a profiled run's choice)
        for k, v in enumerate(variants):
            s.set_tuning(k, v)
        tuning = s.tuning()
    log("%s tile plans: %s" % (precision, {k: (v["variant"], [round(x, 3) for x in v["ms"]]) for k, v in tuning.items()}))
    for _ in range(warmup):
        acc, _, _ = s.step(dt)
        assert acc
    torch.cuda.synchronize()
    s.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        acc, err, _ = s.step(dt)
        assert acc
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep = s.profile_report()
    s.profile(False)
    st = s.stats()
    tg = time.perf_counter()
    s.get_state()                   # back to host arrays: inverse transform and the PCIe copy
    t_get = time.perf_counter() - tg
    s.close()
    wall = t1 - t0
    stages = 6 * steps
    pcie = dict(set_state_s=round(t_set, 3), get_state_s=round(t_get, 3),
                value=round(n ** 3 * stages / (wall + t_set + t_get) / 1e6, 1))
    return dict(value=n ** 3 * stages / wall / 1e6, ms_per_step=1e3 * wall / steps, pcie=pcie,
                kernels=kernel_table(rep), n_rhs=st["n_rhs"], err_last=err,
                tuning={k: v["tile_cols"] for k, v in tuning.items()},
                variants={k: v["variant"] for k, v in tuning.items()})


def fft_bench(torch, n, reps=3):
    from paper_2609_36100_amd import Solver
    s = Solver(n, None)
    u = torch.randn((4, n, n, n), dtype=torch.float64, device="cuda")
    k = s.kspace_empty(4)
    back = torch.empty_like(u)
    s.fft3d(-1, 4, u, k)
    s.fft3d(+1, 4, k, back)
    torch.cuda.synchronize()
    s.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        s.fft3d(-1, 4, u, k)
        s.fft3d(+1, 4, k, back)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    rep = s.profile_report()
    s.close()
    tab = kernel_table(rep)
    tot_ms = sum(v[0] for v in rep.values()) / reps
    tot_b = sum(v[2] for v in rep.values()) / reps
    real_b = 4 * n ** 3 * 8.0
    return dict(fields=4, n=n, precision="f64", ms_fwd_inv=round(1e3 * wall, 3),
                pass_gbs=round(tot_b / (tot_ms * 1e-3) / 1e9, 1),
                pass_frac=round(tot_b / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                effective_gbs_1r1w=round(2 * 2 * real_b / wall / 1e9, 1),
                kernels=tab)


def host_cpu():
    """CPU model and the logical CPUs this process may run on (lscpu, else /proc/cpuinfo)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            model = platform.processor() or platform.machine()
    return dict(model=model, logical_cpus_visible=len(os.sched_getaffinity(0)), logical_cpus_host=os.cpu_count())


def cpu_baseline(n=128):
    """The FP64 oracle, as it stands, on one ARK4(3)6L step at n^3: NumPy's FFT on
    one thread (the value), and SciPy's FFT on every visible core beside it."""
    import numpy as np  # noqa: F401
    import pfinputs
    from oracle import ark as oark
    from oracle import model as om
    from oracle import spectral as osp
    host = host_cpu()
    spec, c, eta = pfinputs.config("mixed512", n=n)
    m = om.Model((n, n, n), pfinputs.default_params())
    m.B()  # one-time per-grid setup, not part of a step
    y = om.to_kspace(c, eta)
    L = m.implicit_symbol()
    osp.set_fft_backend("numpy")
    t0 = time.perf_counter()
    _, _, nexp = oark.ark_step(y, 0.1, oark.ark436l2sa(), m.f_explicit, L)
    wall = time.perf_counter() - t0
    workers = host["logical_cpus_visible"]
    try:
        osp.set_fft_backend("scipy", workers=workers)
        t1 = time.perf_counter()
        oark.ark_step(y, 0.1, oark.ark436l2sa(), m.f_explicit, L)
        wall_all = time.perf_counter() - t1
    finally:
        osp.set_fft_backend("numpy")
    return dict(value=round(n ** 3 * nexp / wall / 1e6, 4), unit="Mpts·stages/s", cores=1,
                kind="oracle",
                sample="one ARK4(3)6L step (6 stages) of the NumPy FP64 oracle at %d^3, same seeded "
                       "generator with the nucleus count scaled by volume; pocketfft, one thread; "
                       "%.1f s" % (n, wall),
                host=host,
                all_cores=dict(value=round(n ** 3 * nexp / wall_all / 1e6, 4), cores=workers,
                               sample="the same step with scipy.fft on %d workers (the pointwise and "
                                      "elastic NumPy work stays on one thread); %.1f s" % (workers, wall_all)))


def ensemble_bench(torch, count, t_final, rtol, atol, ref_members, precisions=("fp64", "mixed"),
                   batched_only=False):
    """64 uneven members: batched (one launch per pass, graph replay) vs one after another
    (batched_only: the batched runs alone, e.g. under a counter profiler)."""
    import pfinputs
    from paper_2609_36100_amd import Ensemble, Solver
    mem = pfinputs.ensemble_members(count)
    kw = dict(adaptive=True, dt0=0.1, rtol=rtol, atol=atol)
    pts = [m["n"] ** 3 for m in mem]
    out = dict(members=count, sizes=sorted(set(m["n"] for m in mem)), t_final=t_final, rtol=rtol, atol=atol)
    vf = {}
    for prec in precisions:
        log("ensemble batched %s" % prec)
        with Ensemble([dict(n=m["n"], precision=prec, **kw) for m in mem]) as E:
            for i, m in enumerate(mem):
                E.set_state(i, m["c"], m["eta"])
            tun = E.autotune(2)
            for i, m in enumerate(mem):     # the autotuner overwrote scratch only; restart cleanly
                E.set_state(i, m["c"], m["eta"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = E.advance(t_final)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            vf[prec] = [E.diagnostics(i)["vf"] for i in range(count)]
        stages = sum(p * s["n_rhs"] for p, s in zip(pts, st))
        out["batched_" + prec] = dict(wall_s=round(wall, 3), value=round(stages / wall / 1e6, 1),
                                      steps=sum(s["steps"] for s in st), rejects=sum(s["rejects"] for s in st),
                                      block_threads={k: v["block_threads"] for k, v in tun.items()})
        out["batched_" + prec]["member_point_stages"] = stages
    if batched_only:
        return out
    log("ensemble sequential plain fp64")
    wall = 0.0
    stages = 0
    vf_seq = []
    for i, m in enumerate(mem):
        with Solver(m["n"], None, method="ark436l", **kw) as s:
            s.set_state(m["c"], m["eta"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.advance(t_final)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            stages += pts[i] * st["n_rhs"]
            vf_seq.append(s.diagnostics()["vf"])
    out["sequential_fp64"] = dict(wall_s=round(wall, 3), value=round(stages / wall / 1e6, 1))
    out["speedup_batched_fp64_vs_sequential"] = round(wall / out["batched_fp64"]["wall_s"], 3)
    # volume-fraction error against a tighter-tolerance plain FP64 reference
    log("ensemble reference runs (rtol 1e-8) for %d members" % ref_members)
    errs = {k: [] for k in list(vf) + ["sequential_fp64"]}
    for i in range(min(ref_members, count)):
        m = mem[i]
        with Solver(m["n"], None, method="ark436l", adaptive=True, dt0=0.05, rtol=1e-8, atol=1e-11) as s:
            s.set_state(m["c"], m["eta"])
            s.advance(t_final)
            ref = s.diagnostics()["vf"]
        for k in vf:
            errs[k].append(abs(vf[k][i] - ref))
        errs["sequential_fp64"].append(abs(vf_seq[i] - ref))
    out["vf_error_max"] = {k: float("%.3e" % max(v)) for k, v in errs.items() if v}
    return out


def time_to_t_bench(torch, n, t_final, rtol, atol, precisions=("fp64", "mixed"), workload="adaptive256"):
    """Adaptive ARK4 run of a seeded n^3 workload to t_final; volume-fraction and
    per-field state errors against an rtol 1e-8 plain FP64 reference."""
    import pfinputs
    from paper_2609_36100_amd import Solver, rel_l2
    spec, c, eta = pfinputs.config(workload, n=n)
    out = dict(n=n, workload=workload, t_final=t_final, rtol=rtol, atol=atol, nuclei=spec["n_nuclei"])
    vf, states = {}, {}
    for prec in precisions:
        log("time-to-t %s" % prec)
        with Solver(n, None, method="ark436l", precision=prec, adaptive=True, dt0=0.01, rtol=rtol, atol=atol) as s:
            s.set_state(c, eta)
            s.autotune(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.advance(t_final)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            vf[prec] = s.diagnostics()["vf"]
            states[prec] = s.get_state_device().clone()
        out[prec] = dict(wall_s=round(wall, 3), steps=st["steps"], rejects=st["rejects"],
                         value=round(n ** 3 * st["n_rhs"] / wall / 1e6, 1), vf=vf[prec])
        log("time-to-t %s: %.2f s, %d steps" % (prec, wall, st["steps"]))
    log("time-to-t reference (rtol 1e-8)")
    with Solver(n, None, method="ark436l", adaptive=True, dt0=0.01, rtol=1e-8, atol=1e-11) as s:
        s.set_state(c, eta)
        for k in range(1, 21):   # in twentieths, with a progress line each
            st = s.advance(t_final * k / 20)
            log("reference: t = %g, %d steps" % (st["t"], st["steps"]))
        ref = s.diagnostics()["vf"]
        uref = s.get_state_device()
        for prec in precisions:
            out[prec]["vf_error"] = float("%.3e" % abs(vf[prec] - ref))
            out[prec]["state_rel_l2"] = [float("%.3e" % rel_l2(states[prec][f], uref[f])) for f in range(4)]
            # the target (vf error <= 1e-3) says little once vf has decayed below it; the
            # state's relative error is reported as the guard beside it
            out[prec]["meets_vf_tol"] = bool(out[prec]["vf_error"] <= 1e-3)
    out["vf_ref"] = ref
    if "fp64" in out and "mixed" in out:
        out["gain_mixed_vs_fp64"] = round(out["fp64"]["wall_s"] / out["mixed"]["wall_s"], 3)
    return out


def inhom_bench(torch, n, steps, dt, scale=1.5):
    """Inhomogeneous elasticity (Reuss stiffness, Hu-Chen iteration) on the n^3
    seeded workload: fixed-step ARK4(3)6L throughput at the loose (1e-6) and
    tight (1e-16, at most 50 updates) elasticity tolerances, updates per RHS,
    per-kernel-class table, against the homogeneous path on the same input."""
    import pfinputs
    from paper_2609_36100_amd import Solver
    spec, c, eta = pfinputs.config("mixed512", n=n)
    prm = pfinputs.default_params()
    out = dict(n=n, steps=steps, dt=dt, precipitate_stiffness_scale=scale, nuclei=spec["n_nuclei"])
    runs = [("homogeneous", dict(prm)),
            ("loose", dict(prm, C11p=scale * prm["C11"], C12p=scale * prm["C12"], C44p=scale * prm["C44"],
                           el_tol=1e-6, el_max_iter=50)),
            ("tight", dict(prm, C11p=scale * prm["C11"], C12p=scale * prm["C12"], C44p=scale * prm["C44"],
                           el_tol=1e-16, el_max_iter=50))]
    for name, model in runs:
        log("inhom bench %s" % name)
        with Solver(n, model, method="ark436l", dt0=dt) as s:
            s.set_state(c, eta)
            s.autotune(2)
            acc, _, _ = s.step(dt)                 # warm-up
            it0 = s.stats()["el_iterations"]
            torch.cuda.synchronize()
            s.profile(True)
            t0 = time.perf_counter()
            for _ in range(steps):
                acc, _, _ = s.step(dt)
                assert acc
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            rep = s.profile_report()
            s.profile(False)
            st = s.stats()
        upd = (st["el_iterations"] - it0) / (6.0 * steps)
        out[name] = dict(value=round(n ** 3 * 6 * steps / wall / 1e6, 1), ms_per_step=round(1e3 * wall / steps, 2),
                         updates_per_rhs=round(upd, 2), kernels=kernel_table(rep))
        log("%s: %.1f Mpts*stages/s, %.1f updates per RHS" % (name, out[name]["value"], upd))
    return out


def orders_bench(torch, n, t_final):
    """Work-precision of the four ImEx pairs on one seeded n^3 workload: state error
    at t_final against a tight ARK4 reference, explicit RHS evaluations and wall
    time (IMEX Euler with fixed steps, the embedded pairs adaptive over rtol)."""
    import numpy as np
    import pfinputs
    from paper_2609_36100_amd import Solver, rel_l2
    spec, c, eta = pfinputs.config("adaptive256", n=n)
    out = dict(n=n, t_final=t_final, nuclei=spec["n_nuclei"], runs={})
    log("orders: reference ARK4 rtol 1e-11")
    with Solver(n, None, method="ark436l", adaptive=True, dt0=1e-3, rtol=1e-11, atol=1e-14) as s:
        s.set_state(c, eta)
        s.advance(t_final)
        ref = s.get_state_device().clone()

    def run(method, **kw):
        with Solver(n, None, method=method, **kw) as s:
            s.set_state(c, eta)
            s.autotune(1) if n >= 128 else None
            s.set_state(c, eta)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = s.advance(t_final)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            u = s.get_state_device()
        err = max(rel_l2(u[f], ref[f]) for f in range(4) if float(ref[f].abs().max()) > 0)
        return dict(err=float("%.3e" % err), n_rhs=st["n_rhs"], steps=st["steps"], rejects=st["rejects"],
                    wall_s=round(wall, 4))

    for dt in (0.02, 0.01, 0.005, 0.0025):
        out["runs"].setdefault("imex_euler", []).append(dict(dt=dt, **run("imex_euler", dt0=dt)))
    for method in ("ark2", "ark324l", "ark436l"):
        for rtol in (1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
            r = run(method, adaptive=True, dt0=1e-3, rtol=rtol, atol=rtol * 1e-3)
            out["runs"].setdefault(method, []).append(dict(rtol=rtol, **r))
            log("orders: %s rtol %g: err %.2e, %d RHS, %.3f s" % (method, rtol, r["err"], r["n_rhs"], r["wall_s"]))

    # wall time each method needs for a given error, by log-log interpolation
    def cost_at(method, target):
        pts = sorted((r["err"], r["wall_s"]) for r in out["runs"][method] if r["err"] > 0)
        for (e0, w0), (e1, w1) in zip(pts, pts[1:]):
            if e0 <= target <= e1:
                f = (np.log(target) - np.log(e0)) / (np.log(e1) - np.log(e0))
                return float(np.exp(np.log(w0) + f * (np.log(w1) - np.log(w0))))
        return None
    gains = {}
    for target in (1e-7, 1e-8, 1e-9):
        w4 = cost_at("ark436l", target)
        row = {}
        for mth in ("imex_euler", "ark2", "ark324l"):
            w = cost_at(mth, target)
            row[mth] = round(w / w4, 3) if (w and w4) else None
        gains["%g" % target] = row
    out["ark4_speedup_at_error"] = gains
    return out


def oracle_timing(sizes_rhs=(64, 128, 256), sizes_step=(64, 128), threads=None):
    """The FP64 CPU oracle as it stands, timed on this host: one explicit RHS
    and one ARK4(3)6L step at several sizes, with NumPy's single-threaded FFT
    and with SciPy's FFT on all cores (same seeded generator as the 512^3
    workload, nucleus count scaled by volume)."""
    import subprocess
    import pfinputs
    from oracle import ark as oark
    from oracle import model as om
    from oracle import spectral as osp
    # the host share this process may use (the thread cap set for the job, at most the visible cores)
    cores = threads or min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16")))
    try:
        cpu = [l.split(":", 1)[1].strip() for l in subprocess.run(["lscpu"], capture_output=True, text=True)
               .stdout.splitlines() if l.startswith("Model name")][0]
    except Exception:
        cpu = platform.processor() or platform.machine()
    out = dict(cpu=cpu, cores=cores, rhs={}, ark4_step={})
    for backend, workers in (("numpy", 1), ("scipy", cores)):
        osp.set_fft_backend(backend, workers)
        for n in sizes_rhs:
            spec, c, eta = pfinputs.config("mixed512", n=n)
            m = om.Model((n, n, n), pfinputs.default_params())
            t0 = time.perf_counter()
            m.B()
            out["rhs"]["setup_%s_%d" % (backend, n)] = round(time.perf_counter() - t0, 3)
            y = om.to_kspace(c, eta)
            del c, eta
            t0 = time.perf_counter()
            m.rhs(y)
            wall = time.perf_counter() - t0
            out["rhs"]["%s_%d" % (backend, n)] = dict(s=round(wall, 3), mpts_stages=round(n ** 3 / wall / 1e6, 3))
            log("oracle rhs %s %d^3: %.2f s" % (backend, n, wall))
            if n in sizes_step:
                t0 = time.perf_counter()
                _, _, ne = oark.ark_step(y, 0.1, oark.ark436l2sa(), m.f_explicit, m.implicit_symbol())
                wall = time.perf_counter() - t0
                out["ark4_step"]["%s_%d" % (backend, n)] = dict(s=round(wall, 3),
                                                                mpts_stages=round(n ** 3 * ne / wall / 1e6, 3))
                log("oracle ark4 step %s %d^3: %.2f s" % (backend, n, wall))
    osp.set_fft_backend("numpy", 1)
    return out


def fno_bench(torch, t_final, runs, val_runs, snapshots, epochs, train_s, members, dt_ref_t, lr, ensemble=True):
    """Learned surrogate: plain-solver training data at 128^3, GPU training, held-out
    validation, then the 128^3 members of the uneven ensemble advanced to t_final
    with the checked surrogate against plain adaptive ARK4 (the gain test)."""
    import numpy as np
    import pfinputs
    from paper_2609_36100_amd import Solver, rel_l2
    from paper_2609_36100_amd import surrogate as sg
    n = 128
    out = dict(n=n, width=32, modes=12, layers=4, hidden=128)
    t0 = time.perf_counter()
    dt_ref, _ = sg.reference_dt(n, 0, dt_ref_t)
    delta = 10.0 * dt_ref
    out.update(dt_ref=dt_ref, delta=delta, dt_ref_window=dt_ref_t)
    log("dt_ref %.5f (mean accepted ARK4 step over [0, %g] of run 0), delta %.5f" % (dt_ref, dt_ref_t, delta))
    snaps, steps = sg.generate_snapshots(n, runs + val_runs, snapshots, delta, log=log)
    out["data"] = dict(runs=runs, val_runs=val_runs, snapshots=snapshots, pairs=runs * snapshots,
                       plain_steps=steps, wall_s=round(time.perf_counter() - t0, 1))
    scale = sg.increment_scale(snaps, runs)
    norm = sg.state_norm(snaps, runs)
    out["scale"] = [float("%.4e" % v) for v in scale]
    out["input_norm"] = dict(mean=[float("%.4e" % v) for v in norm[0]], std=[float("%.4e" % v) for v in norm[1]])
    f = sg.make_fno(n, 32, 12, 4, 128, seed=0, scale=scale, norm=norm)
    val = list(range(runs, runs + val_runs))
    e0, keep, inc0 = sg.validate(f, snaps, val)
    t1 = time.perf_counter()
    hist = sg.train(f, snaps, runs, epochs=epochs, lr=lr, batch=4, seed=0, log=log, time_limit=train_s)
    out["train"] = dict(epochs=len(hist), loss=[float("%.4e" % v) for v in hist],
                        wall_s=round(time.perf_counter() - t1, 1))
    e1, _, inc1 = sg.validate(f, snaps, val)
    out["validation_rel_l2_c"] = dict(untrained_mean=float("%.3e" % e0.mean()), trained_mean=float("%.3e" % e1.mean()),
                                      trained_max=float("%.3e" % e1.max()), no_change_mean=float("%.3e" % keep.mean()),
                                      frac_below_tol=float("%.3f" % (e1 <= 1e-3).mean()),
                                      increment_rel_err=[float("%.3f" % v) for v in inc1],
                                      increment_rel_err_untrained=[float("%.3f" % v) for v in inc0])
    log("validation rel-L2(c): trained %.3e (max %.3e), untrained %.3e, no change %.3e"
        % (e1.mean(), e1.max(), e0.mean(), keep.mean()))
    del snaps
    torch.cuda.empty_cache()
    # gain test on the ensemble's 128^3 members
    mem = [m for m in pfinputs.ensemble_members(64) if m["n"] == n][:members]
    # default horizon: the training window (snapshots x delta)
    n_adv = int(round(t_final / delta)) if t_final > 0 else snapshots
    t_end = n_adv * delta
    kw = dict(method="ark436l", adaptive=True, dt0=0.01, rtol=1e-6, atol=1e-9)
    res = []
    tot_plain = tot_sur = 0.0
    for i, m in enumerate(mem):
        with Solver(n, None, **kw) as s:
            s.set_state(m["c"], m["eta"])
            torch.cuda.synchronize()
            ta = time.perf_counter()
            st = s.advance(t_end)
            torch.cuda.synchronize()
            w_plain = time.perf_counter() - ta
            u_plain = s.get_state_device().clone()
            vf_plain = s.diagnostics()["vf"]
            s.set_state(m["c"], m["eta"])
            u = s.get_state_device().clone()
            s.set_dt(0.01)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            fs = sg.checked_advance(f, s, u, t_end, delta, check_every=5, tol=1e-3)
            torch.cuda.synchronize()
            w_sur = time.perf_counter() - ta
            s.set_state_device(u)
            vf_sur = s.diagnostics()["vf"]
        with Solver(n, None, method="ark436l", adaptive=True, dt0=0.01, rtol=1e-8, atol=1e-11) as r:
            r.set_state(m["c"], m["eta"])
            r.advance(t_end)
            u_ref = r.get_state_device()
            vf_ref = r.diagnostics()["vf"]
        tot_plain += w_plain
        tot_sur += w_sur
        d = fs.as_dict()
        res.append(dict(member=m["member"], plain_s=round(w_plain, 3), plain_steps=st["steps"],
                        surrogate_s=round(w_sur, 3), surrogate=d["surrogate"], checks=d["checks"],
                        fallbacks=d["fallbacks"], plain_advances=d["plain"],
                        check_err_max=float("%.3e" % d["err_max"]),
                        vf_err_plain=float("%.3e" % abs(vf_plain - vf_ref)),
                        vf_err_surrogate=float("%.3e" % abs(vf_sur - vf_ref)),
                        c_rel_l2_plain=float("%.3e" % rel_l2(u_plain[0], u_ref[0])),
                        c_rel_l2_surrogate=float("%.3e" % rel_l2(u[0], u_ref[0]))))
        log("member %d: plain %.2f s (%d steps), surrogate %.2f s (%d net, %d checks, %d fallbacks), "
            "vf err %.1e / %.1e" % (m["member"], w_plain, st["steps"], w_sur, d["surrogate"], d["checks"],
                                    d["fallbacks"], res[-1]["vf_err_plain"], res[-1]["vf_err_surrogate"]))
    out["gain"] = dict(t_final=t_end, members=len(mem), plain_s=round(tot_plain, 3), surrogate_s=round(tot_sur, 3),
                       speedup=round(tot_plain / tot_sur, 3) if tot_sur > 0 else None,
                       vf_err_max_plain=max(r["vf_err_plain"] for r in res),
                       vf_err_max_surrogate=max(r["vf_err_surrogate"] for r in res),
                       fallbacks=sum(r["fallbacks"] for r in res), per_member=res)
    if ensemble:
        # the whole uneven ensemble: every member on the batched plain solver, against the
        # same ensemble with its 128^3 members advanced by the surrogate inside it (one
        # batched network pass for all of them per interval; their checks and fallback
        # intervals through the ensemble's plain solver) and the other sizes by the plain
        # solver afterwards
        from paper_2609_36100_amd import Ensemble
        allm = pfinputs.ensemble_members(64)
        idx128 = [i for i, m in enumerate(allm) if m["n"] == n]
        walls = {}
        vf_end = {}
        for name in ("all_plain", "with_surrogate"):
            log("ensemble %s (%d members, %d of %d^3) to t=%g" % (name, len(allm), len(idx128), n, t_end))
            with Ensemble([dict(n=m["n"], **kw) for m in allm]) as E:
                for i, m in enumerate(allm):
                    E.set_state(i, m["c"], m["eta"])
                torch.cuda.synchronize()
                ta = time.perf_counter()
                if name == "with_surrogate":
                    est = f.ensemble_advance(E, idx128, n_adv, delta, check_every=5, tol=1e-3)
                E.advance(t_end)
                torch.cuda.synchronize()
                walls[name] = time.perf_counter() - ta
                vf_end[name] = [E.diagnostics(i)["vf"] for i in idx128]
        d = [x.as_dict() for x in est]
        out["gain"]["ensemble"] = dict(
            members=len(allm), members_128=len(idx128), all_plain_s=round(walls["all_plain"], 3),
            with_surrogate_s=round(walls["with_surrogate"], 3),
            speedup=round(walls["all_plain"] / walls["with_surrogate"], 3),
            surrogate_advances=sum(x["surrogate"] for x in d), checks=sum(x["checks"] for x in d),
            fallbacks=sum(x["fallbacks"] for x in d), plain_advances=sum(x["plain"] for x in d),
            vf_diff_max=float("%.3e" % max(abs(a - b) for a, b in zip(vf_end["all_plain"],
                                                                        vf_end["with_surrogate"]))))
    return out


def fno_step_bench(torch, n=128, reps=10):
    """The surrogate's kernels on their own: one training step (forward, loss,
    backward) and one surrogate advance at n^3 (width 32, 12 modes, 4 layers),
    with the dense-contraction flops they carry."""
    import numpy as np
    from paper_2609_36100_amd import surrogate as sg
    f = sg.make_fno(n, 32, 12, 4, 128, seed=0, scale=np.full(4, 1e-3, np.float32))
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.rand((4, n, n, n), dtype=torch.float32, device="cuda", generator=g)
    y = x + 1e-3 * torch.rand((4, n, n, n), dtype=torch.float32, device="cuda", generator=g)
    u = x.double().contiguous()
    w = torch.empty_like(u)
    for _ in range(2):
        f.grad(x, y)
        f.apply(u, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        f.grad(x, y)
    torch.cuda.synchronize()
    t_grad = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        f.adam_step(1e-4)
    torch.cuda.synchronize()
    t_adam = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        f.apply(u, w)
    torch.cuda.synchronize()
    t_apply = (time.perf_counter() - t0) / reps
    # flops of one forward pass (channel counts padded to 8 as the kernels run
    # them): lift; per layer the pointwise W, the six truncated-DFT GEMM
    # stages (x: 4 m w n^3 each way, y: 16 m^2 w n^2, z: 32 m^3 w n) and the
    # per-mode complex w x w mixing (32 m^3 w^2); projection
    P = n ** 3
    wd, m, L, h = 32, 12, 4, 128
    layer = 2 * P * wd * wd + 2 * (4 * m * wd * n ** 3 + 16 * m * m * wd * n * n + 32 * m ** 3 * wd * n) \
        + 32 * m ** 3 * wd * wd
    fwd = 2 * P * 8 * wd + L * layer + 2 * P * wd * h + 2 * P * h * 8
    # algorithmic bytes and flops per kind (the library's own accounting) of
    # one training step, one Adam step and one advance
    work = {}
    for name, call in (("grad", lambda: f.grad(x, y)), ("adam", lambda: f.adam_step(1e-4)),
                       ("apply", lambda: f.apply(u, w))):
        f.work(1)
        call()
        work[name] = {k: dict(gb=round(v["bytes"] / 1e9, 4), gflop=round(v["flops"] / 1e9, 3),
                              launches=v["launches"]) for k, v in f.work(0).items() if v["launches"]}
    torch.cuda.synchronize()
    # batched advances: B samples through one network pass
    batched = {}
    for B in (1, 4, 8):
        ub = u.unsqueeze(0).expand(B, -1, -1, -1, -1).contiguous()
        wb = torch.empty_like(ub)
        f.apply_batch(ub, wb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            f.apply_batch(ub, wb)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        batched[str(B)] = dict(ms=round(1e3 * tb, 3), ms_per_sample=round(1e3 * tb / B, 3),
                               tflops=round(B * fwd / tb / 1e12, 2))
        del ub, wb
    return dict(n=n, grad_ms=round(1e3 * t_grad, 3), adam_ms=round(1e3 * t_adam, 3), apply_ms=round(1e3 * t_apply, 3),
                forward_gflop=round(fwd / 1e9, 2),
                apply_tflops=round(fwd / t_apply / 1e12, 2), apply_batch=batched, work=work)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--variants", default=None,
                    help="throughput: fixed tile variants after autotuning, 'a,b,c,d' (FP64) or "
                         "'a,b,c,d/e,f,g,h' (FP64/mixed) for colfft, stage_invz, zpass_elastic, zpass_fwd_ac")
    ap.add_argument("--dt", type=float, default=0.1)
    ap.add_argument("--skip-mixed", action="store_true")
    ap.add_argument("--skip-fft", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-ttt", action="store_true", help="throughput: skip the time-to-t leg")
    ap.add_argument("--mode", choices=["throughput", "ensemble", "time_to_t", "fno", "fno_step", "orders",
                                       "oracle_timing", "inhom"], default="throughput")
    ap.add_argument("--runs", type=int, default=40, help="fno: training runs")
    ap.add_argument("--val-runs", type=int, default=4, help="fno: held-out runs")
    ap.add_argument("--snapshots", type=int, default=50, help="fno: snapshots per run")
    ap.add_argument("--epochs", type=int, default=6, help="fno: training epochs")
    ap.add_argument("--train-seconds", type=float, default=None, help="fno: stop training after this long")
    ap.add_argument("--fno-members", type=int, default=64, help="fno: at most this many 128^3 members")
    ap.add_argument("--dt-ref-window", type=float, default=10.0, help="fno: window for the mean ARK4 step")
    ap.add_argument("--lr", type=float, default=1e-3, help="fno: peak learning rate")
    ap.add_argument("--skip-ensemble", action="store_true", help="fno: skip the whole-ensemble comparison")
    ap.add_argument("--workload", default="adaptive256", choices=["adaptive256", "mixed512"],
                    help="time_to_t: seeded initial condition")
    ap.add_argument("--rtol", type=float, default=1e-6, help="time_to_t: relative tolerance (atol = rtol / 1000)")
    ap.add_argument("--t-final", type=float, default=None)
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--batched-only", action="store_true",
                    help="ensemble: the batched runs alone (no sequential or reference runs)")
    ap.add_argument("--rhs-sizes", default="64,128,256",
                    help="oracle_timing: grid sizes for the one-RHS timing (512 needs about 40 GB of host memory)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 4 GiB (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the stage cycle runs on a single MI355X; "
              "--gpus %d is not supported" % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    import pfinputs
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size: 4 GiB read + 4 GiB written per launch
        src = torch.ones(1 << 29, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": src.numel() * 8,
                          "copy_bytes_written_per_launch": src.numel() * 8, "launches": 3}))
        return
    if args.mode == "ensemble":
        r = ensemble_bench(torch, args.members, args.t_final or 100.0, 1e-6, 1e-9, ref_members=8,
                           batched_only=args.batched_only)
        print(json.dumps({"metric": METRIC, "mode": "ensemble", "unit": "Mpts·stages/s",
                          "value": r["batched_fp64"]["value"], "n_gpus": 1, "dtype": "f64",
                          "data": "synthetic", "higher_is_better": True,
                          "config": {"workload": "%d seeded members of sizes %s, adaptive ARK4(3)6L to t=%g"
                                                 % (args.members, r["sizes"], r["t_final"])},
                          "ensemble": r}), flush=True)
        return
    if args.mode == "fno":
        r = fno_bench(torch, args.t_final or 0.0, args.runs, args.val_runs, args.snapshots, args.epochs,
                      args.train_seconds, args.fno_members, args.dt_ref_window, args.lr,
                      ensemble=not args.skip_ensemble)
        g = r["gain"]
        print(json.dumps({"metric": METRIC, "mode": "fno", "unit": "s", "value": g["surrogate_s"],
                          "higher_is_better": False, "n_gpus": 1, "dtype": "bf16 network, f64 state",
                          "data": "synthetic",
                          "config": {"workload": "FNO surrogate (4 layers, width 32, 12 modes) at 128^3 inside the "
                                                 "uneven ensemble's 128^3 members, to t=%g, checks every 5th "
                                                 "advance at rel-L2(c) 1e-3" % g["t_final"]},
                          "fno": r}), flush=True)
        return
    if args.mode == "oracle_timing":
        r = oracle_timing(sizes_rhs=tuple(int(v) for v in args.rhs_sizes.split(",")))
        print(json.dumps({"metric": METRIC, "mode": "oracle_timing", "unit": "Mpts·stages/s", "value": None,
                          "higher_is_better": True, "n_gpus": 0, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "FP64 CPU oracle: one RHS and one ARK4 step at several sizes"},
                          "oracle_timing": r}), flush=True)
        return
    if args.mode == "fno_step":
        r = fno_step_bench(torch, args.n if args.n != 512 else 128)
        print(json.dumps({"metric": METRIC, "mode": "fno_step", "unit": "ms", "value": r["grad_ms"],
                          "higher_is_better": False, "n_gpus": 1, "dtype": "bf16 (fp32 accumulate)",
                          "data": "synthetic",
                          "config": {"workload": "FNO (4 layers, width 32, 12 modes, hidden 128) at %d^3: one "
                                                 "training step and one surrogate advance" % r["n"]},
                          "fno_step": r}), flush=True)
        return
    if args.mode == "orders":
        n = args.n if args.n != 512 else 128
        r = orders_bench(torch, n, args.t_final or 2.0)
        print(json.dumps({"metric": METRIC, "mode": "orders", "unit": "s", "value": None,
                          "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "%d^3, %d seeded nuclei, to t=%g: IMEX Euler, ARK2, ARK3(2)4L, "
                                                 "ARK4(3)6L work-precision" % (n, r["nuclei"], r["t_final"])},
                          "orders": r}), flush=True)
        return
    if args.mode == "inhom":
        r = inhom_bench(torch, args.n, args.steps, args.dt)
        print(json.dumps({"metric": METRIC, "mode": "inhom", "unit": "Mpts·stages/s", "value": r["loose"]["value"],
                          "higher_is_better": True, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "%d^3, %d seeded nuclei, ARK4(3)6L fixed dt=%g, Reuss stiffness with "
                                                 "precipitate constants x%g, Hu-Chen tolerance 1e-6 (loose) / 1e-16 "
                                                 "(tight)" % (args.n, r["nuclei"], args.dt,
                                                              r["precipitate_stiffness_scale"])},
                          "inhom": r}), flush=True)
        return
    if args.mode == "time_to_t":
        n = args.n if (args.n != 512 or args.workload != "adaptive256") else 256
        r = time_to_t_bench(torch, n, args.t_final or 500.0, args.rtol, args.rtol * 1e-3, workload=args.workload)
        print(json.dumps({"metric": METRIC, "mode": "time_to_t", "unit": "s", "value": r["fp64"]["wall_s"],
                          "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "%d^3 (%s), %d seeded nuclei, adaptive ARK4(3)6L rtol %g to t=%g"
                                                 % (n, args.workload, r["nuclei"], args.rtol, r["t_final"])},
                          "time_to_t": r}), flush=True)
        return
    n = args.n
    from paper_2609_36100_amd import bandwidth_probe
    probe = bandwidth_probe(1 << 30, 5)
    log("streaming probe (GB/s): copy %.0f, read %.0f, 11 reads + 1 write %.0f"
        % (probe["copy"], probe["read"], probe["multi"]))
    log("generating %d^3 seeded initial condition" % n)
    spec, c, eta = pfinputs.config("mixed512", n=n)
    ct = torch.from_numpy(c).cuda()
    et = torch.from_numpy(eta).cuda()
    del c, eta

    log("FP64 run: %d warmup + %d timed ARK4 steps" % (args.warmup, args.steps))
    var64 = var32 = None
    if args.variants:
        parts = [[int(x) for x in q.split(",")] for q in args.variants.split("/")]
        var64 = parts[0]
        var32 = parts[1] if len(parts) > 1 else None
    r64 = run_solver(torch, n, ct, et, "fp64", args.steps, args.warmup, args.dt, var64)
    log("FP64 %.1f Mpts*stages/s, %.1f ms/step" % (r64["value"], r64["ms_per_step"]))
    mixed = None
    if not args.skip_mixed:
        log("mixed run")
        rm = run_solver(torch, n, ct, et, "mixed", args.steps, args.warmup, args.dt, var32)
        log("mixed %.1f Mpts*stages/s, %.1f ms/step" % (rm["value"], rm["ms_per_step"]))
        mixed = dict(value=round(rm["value"], 2), ms_per_step=round(rm["ms_per_step"], 3),
                     dtype="f32 FFT/pointwise/elastic, f64 stage sums and error", kernels=rm["kernels"],
                     tuning=rm["tuning"], variants=rm["variants"],
                     speedup_vs_fp64=round(rm["value"] / r64["value"], 3))
    del ct, et
    torch.cuda.empty_cache()
    fft = None
    if not args.skip_fft:
        log("FFT run")
        fft = fft_bench(torch, n)
    kt = r64["kernels"]
    dom = max(kt, key=lambda k: kt[k]["total_ms"])
    d = kt[dom]
    tr = measured_traffic()
    traffic = None
    if tr is not None and args.n == 512 and ("%s/f64" % dom) in tr:
        traffic = tr["%s/f64" % dom]
    roofline = dict(bound="hbm", kernel=dom, achieved=d["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=d["frac"], traffic=traffic,
                    traffic_note="HBM bytes per launch from rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1 "
                                 "(copy-kernel calibration); algorithmic bytes per launch %.0f"
                                 % d["bytes_per_launch"],
                    probe_gbs=round(probe["copy"], 1),
                    frac_of_probe=round(d["gbs"] / probe["copy"], 4))
    ttt = None
    if not args.skip_ttt and n == 512:
        log("time-to-t leg: 512^3, adaptive ARK4 rtol 1e-5 to t = 2, FP64 / mixed / rtol 1e-8 reference")
        ttt = time_to_t_bench(torch, n, 2.0, 1e-5, 1e-8, workload="mixed512")
    cpu = None
    if not args.skip_cpu:
        log("CPU oracle sample")
        cpu = cpu_baseline()
    line = {
        "metric": METRIC,
        "value": round(r64["value"], 2),
        "unit": "Mpts·stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%d^3 ARK4(3)6L fixed dt=%g, %d seeded nuclei (radius 2-5, spacing 8), "
                               "6 stages per step" % (n, args.dt, spec["n_nuclei"]),
                   "grid": n, "stages_per_step": 6, "dt": args.dt, "tile_cols": r64["tuning"],
                   "tile_variants": r64["variants"]},
        "roofline": roofline,
        "kernels": kt,
        "mixed": mixed,
        "fft": fft,
        "time_to_t": ttt,
        "cpu_baseline": cpu,
        "hbm_probe": {k: round(v, 1) for k, v in probe.items()},
        # the same timed steps with the state handed over in host memory (pf_set_state
        # before, pf_get_state after, both through PCIe); context, never `value`
        "pcie_inclusive": dict(r64["pcie"], unit="Mpts·stages/s", steps=args.steps),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
