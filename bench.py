"""Benchmark of the DFS spectral Poisson solver on one MI355X.

Workload (one step = one complete solve, every stage of the hot path):
n = m = 10000 grid (1e8 degrees of freedom), f a seeded band-limited random
spherical-harmonic field with degree l <= 2000 and c_lM ~ N(0,1)/(1+l)^2,
float64 samples in and out, inputs resident in HBM before timing.

Prints ONE JSON line: DOF/s (whole job), the HIP-event roofline of the
dominant kernel, the CPU oracle baseline on the same workload, and the
accuracy of the timed result against the closed-form solution and the FP64
oracle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "sphere Poisson DOF/s at 1e-10 rel err (FP32+refine vs FP64); HBM GB/s"

WORKLOADS = {
    # name: (n, m, L, cfg seed)
    "sphere_poisson_n10000_m10000_l2000": (10000, 10000, 2000, 2),
    "sphere_poisson_n1024_m1024_l256": (1024, 1024, 256, 1),
}


def kernel_bytes(kind: str, n: int, m: int, precision: str, rank: int = 0) -> int:
    """Algorithmic HBM bytes of one launch (what the kernel must read and write);
    `rank`: the low-rank right-hand side's K (its two kernels)."""
    N = n // 2
    spec64 = m * (N + 1) * 16
    spec32 = m * (N + 1) * 8
    grid = m * n * 8
    table = {
        "lambda_fwd": grid + spec64,
        # mixed first solve: reads the spectrum of sin^2 f, writes its theta coefficients F and
        # the float32 solution spectrum
        "theta": 2 * spec64 if precision == "fp64" else 2 * spec64 + spec32,
        "lambda_inv": spec64 + grid,
        # mix: reads the float32 first solution, writes its float64 spectrum and
        # keeps the float32 rows (4 B per sample) in u for the update
        "lambda_mix": spec32 + spec64 + grid // 2,
        "theta_resid": 2 * spec64 + spec32,
        # update: reads the kept float32 rows and the correction spectrum, writes u
        "lambda_upd": grid // 2 + spec32 + grid,
        # tangential gradient: both float64 spectra read, three components written
        "lambda_grad": 2 * spec64 + 3 * grid,
        # low-rank right-hand side: the factors' half spectra (K rows of r in, K spectra out),
        # then the rank-K product (c, those spectra and sin^2 in, the float64 spectrum out)
        "lowrank_rows": rank * n * 8 + rank * (N + 1) * 16,
        "lowrank": rank * m * 8 + rank * (N + 1) * 16 + m * 8 + spec64,
    }
    return table[kind]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest() -> str:
    """sha256 of the solver's HIP sources: a measured traffic record applies only
    to the kernels it was taken on.  The Gaussian-elimination constructor
    (sp_ge*) is a translation unit of its own and takes no part in them."""
    import hashlib
    d = os.path.join(ROOT, "paper_1510_08094_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp", ".h")) and not name.startswith("sp_ge"):
            with open(os.path.join(d, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, precision: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summaries (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a plain
    copy), or None when no record matches these kernel sources."""
    import re
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    digest = source_digest()
    pat = re.compile(r"traffic-record kernel=(\S+) precision=(\S+) workload=(\S+) fetch_bytes=(\d+) "
                     r"write_bytes=(\d+) source_sha256=([0-9a-f]+)")
    for name in sorted(os.listdir(pdir)):
        with open(os.path.join(pdir, name), errors="replace") as fh:
            for line in fh:
                m = pat.search(line)
                if m and m.group(1) == kernel and m.group(2) == precision and m.group(3) == workload \
                        and m.group(6) == digest:
                    return int(m.group(4)) + int(m.group(5))
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="sphere_poisson_n10000_m10000_l2000")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-fp64-ref", action="store_true", help="skip timing the plain float64 solver")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-problem heterogeneous batch")
    ap.add_argument("--no-autotune", action="store_true", help="batch: radix orders by the fixed rule")
    ap.add_argument("--no-c4", action="store_true", help="skip the 16 x 2048^2 forward + adjoint measurement")
    ap.add_argument("--no-literal", action="store_true",
                    help="skip the mixed solve with float32 eliminations for every k > 0 and two corrections")
    ap.add_argument("--no-sweep", action="store_true", help="skip the O(mn) size sweep")
    ap.add_argument("--no-stream", action="store_true", help="skip the achievable-bandwidth kernels")
    ap.add_argument("--stream-only", action="store_true",
                    help="only run the achievable-bandwidth kernels (copy, read, write of 10^8 doubles)")
    ap.add_argument("--no-gradient", action="store_true", help="skip the tangential-gradient measurement")
    ap.add_argument("--no-lowrank", action="store_true", help="skip the low-rank right-hand side measurement")
    ap.add_argument("--no-eval", action="store_true", help="skip the pointwise-evaluation measurement")
    ap.add_argument("--no-ge", action="store_true", help="skip the Gaussian-elimination constructor measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time a plain 800 MB device-to-device copy (the reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        copy_calibration(args, torch)
        return
    if args.stream_only:
        import paper_1510_08094_amd as P
        print(json.dumps(bench_stream(args, P, torch)), flush=True)
        return

    import paper_1510_08094_amd as P
    import sh_inputs as S

    n, m, L, cfg = WORKLOADS[args.workload]
    dof = n * m
    log("bench: synthesising f (n=%d m=%d l<=%d)" % (n, m, L))
    t0 = time.time()
    if args.no_check:
        f, u_exact = S.sphere_field(cfg, 0, n, m, L), None
    else:
        f, u_exact = S.sphere_field(cfg, 0, n, m, L, with_solution=True)
    log("bench: inputs ready in %.1fs" % (time.time() - t0))

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    fg = torch.from_numpy(f).to(dev)
    ug = torch.empty_like(fg)
    plan = P.SpherePoisson(n, m, args.precision)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        plan.solve(fg, out=ug)
    torch.cuda.synchronize()
    log("bench: warmup done")
    plan.profile_enable(16 * args.steps)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        plan.solve(fg, out=ug)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    prof = plan.profile_read()
    plan.profile_enable(0)
    ms_per_step = total_ms / args.steps
    value = dof / (ms_per_step * 1e-3)
    log("bench: %.3f ms/step, %.3e DOF/s, kernels %s" % (ms_per_step, value, prof))

    fp64_ref = None
    if args.precision == "mixed" and not args.no_fp64_ref:
        # the plain float64 solver on the same input, same protocol (context for the mixed speed-up)
        p64 = P.SpherePoisson(n, m, "fp64")
        u64 = torch.empty_like(fg)
        for _ in range(args.warmup):
            p64.solve(fg, out=u64)
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(args.steps):
            p64.solve(fg, out=u64)
        s1.record(stream)
        torch.cuda.synchronize()
        ms64 = s0.elapsed_time(s1) / args.steps
        fp64_ref = {"ms_per_step": ms64, "dof_per_s": dof / (ms64 * 1e-3)}
        p64.close()
        del u64
        log("bench: float64 solver %.3f ms/step" % ms64)

    kernels = {}
    for kind, (tot, cnt) in prof.items():
        avg_ms = tot / cnt
        b = kernel_bytes(kind, n, m, args.precision)
        kernels[kind] = {"avg_ms": round(avg_ms, 5), "launches": cnt, "alg_bytes": b,
                         "alg_GBps": round(b / (avg_ms * 1e-3) / 1e9, 1)}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    achieved = kernels[dom]["alg_GBps"]

    out = {
        "metric": METRIC, "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic (seeded band-limited spherical-harmonic field)",
        "config": {"workload": args.workload, "n_lambda": n, "m_theta": m, "dof": dof, "l_max": L,
                   "precision": args.precision, "rhs": 1},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, args.precision, args.workload)},
        "kernels": kernels,
        "paper_context_dof_per_s": 1e8 / 60.0,
    }
    if fp64_ref is not None:
        out["fp64_solver"] = fp64_ref
        out["speedup_vs_fp64_solver"] = value / fp64_ref["dof_per_s"]

    if not args.no_check:
        torch.cuda.synchronize()
        u = ug.cpu().numpy()
        out["rel_err_vs_closed_form"] = float(np.linalg.norm(u - u_exact) / np.linalg.norm(u_exact))
        del u_exact
    else:
        u = None

    if not args.no_cpu_baseline:
        out["cpu_baseline"], u_or = cpu_baseline(f, dof, n, m)
        if u is not None:
            out["rel_err_vs_oracle"] = float(np.linalg.norm(u - u_or) / np.linalg.norm(u_or))
        del u_or
    plan.close()
    del fg, ug
    if not args.no_gradient:
        out["gradient"] = bench_gradient(args, P, torch, n, m)
    if not args.no_lowrank:
        out["lowrank"] = bench_lowrank(args, P, S, torch, np, n, m)
    if not args.no_eval:
        out["evaluation"] = bench_evaluate(args, P, S, torch, np)
    if not args.no_ge:
        out["ge"] = bench_ge(args, P, S, torch, np, n, m)
    if not args.no_literal and args.precision == "mixed":
        out["mixed_literal"] = bench_literal(args, P, torch, np, f, n, m, L, cfg)
    del f
    if not args.no_c4:
        out["c4"] = bench_c4(args, P, S, torch, np)
    if not args.no_sweep:
        out["sweep"] = bench_sweep(args, P, S, torch, np)
    if not args.no_stream:
        out["achievable"] = bench_stream(args, P, torch)
        out["roofline"]["frac_of_achievable"] = round(achieved / out["achievable"]["best_copy_GBps"], 4)
    if not args.no_batch:
        out["batch"] = bench_batch(args, P, S, torch, np)
    print(json.dumps(out), flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(f, dof, n, m):
    """The float64 oracle (reduced mode: numpy real FFT in lambda, scipy DCT /
    DST in theta, banded solves vectorised over k) timed on this host: one
    warm-up, then the median of three full solves, once with scipy.fft on every
    core (workers = os.cpu_count(); numpy's FFT stays single-threaded) and once
    on one core.  The thread count used is measured as process CPU time over
    wall time."""
    import resource
    import statistics

    import scipy.fft
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        blas = sorted({"%s:%d" % (i.get("internal_api", "?"), i.get("num_threads", 0)) for i in threadpool_info()})
    except Exception:  # noqa: BLE001 - optional introspection
        blas = []
    cores = os.cpu_count() or 1
    res = {}
    u_or = None
    for workers in (cores, 1):
        times, cpu = [], []
        with scipy.fft.set_workers(workers):
            for rep in range(4):
                r0 = resource.getrusage(resource.RUSAGE_SELF)
                t0 = time.perf_counter()
                u_or = O.solve_reduced(f)
                dt = time.perf_counter() - t0
                r1 = resource.getrusage(resource.RUSAGE_SELF)
                if rep:
                    times.append(dt)
                    cpu.append((r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime))
        med = statistics.median(times)
        res[workers] = {"value": dof / med, "seconds": med, "cpu_seconds": statistics.median(cpu),
                        "threads_used": round(statistics.median(cpu) / med, 2), "workers": workers}
        log("bench: oracle with %d workers: %.2f s per solve (%.2f threads busy)" % (workers, med,
                                                                                  res[workers]["threads_used"]))
    allc = res[cores]
    return ({"value": allc["value"], "unit": "DOF/s", "cores": cores, "kind": "oracle",
             "sample": "full %dx%d float64 solves by the reduced-mode oracle, median of 3 after a warm-up, "
                       "scipy.fft workers = %d (%.2f s each; process CPU time / wall time = %.2f)"
                       % (n, m, cores, allc["seconds"], allc["threads_used"]),
             "single_core": {"value": res[1]["value"], "unit": "DOF/s", "cores": 1, "seconds": res[1]["seconds"]},
             "threads_used": allc["threads_used"], "cpu_model": cpu_model(), "blas_threads": blas,
             "host_cpus": cores}, u_or)


def bench_literal(args, P, torch, np, fg_host, n, m, L, cfg):
    """The mixed solve with the literal precision split: float32 eliminations
    for every k > 0 (only k = 0 in float64) and two corrections, on the same
    workload: time per solve and error against the closed form (every 97th
    row)."""
    import sh_inputs as S
    fg = torch.from_numpy(fg_host).cuda()
    u = torch.empty_like(fg)
    plan = P.SpherePoisson(n, m, "mixed", max_refine=2, low_k_fp64=1)
    for _ in range(max(1, args.warmup)):
        plan.solve(fg, out=u)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    steps = max(1, args.steps // 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.solve(fg, out=u)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan.close()
    _, ue = S.sphere_field(cfg, 0, n, m, L, with_solution=True)
    err = float(np.linalg.norm(u.cpu().numpy() - ue) / np.linalg.norm(ue))
    log("bench: mixed literal (k >= 1 in float32, two corrections) %.3f ms/solve, rel err %.2e" % (ms, err))
    return {"workload": "sphere_poisson_n%d_m%d_l%d_mixed_fp32_all_k_two_corrections" % (n, m, L),
            "low_k_fp64": 1, "max_refine": 2, "ms_per_solve": ms, "dof_per_s": n * m / (ms * 1e-3),
            "rel_err_vs_closed_form": err}


def bench_c4(args, P, S, torch, np, count=16, n=2048, L=512):
    """16 right-hand sides at n = m = 2048, loss sum ||u(f) - u_obs||^2 with
    u_obs a seeded field l <= 512 plus N(0, 1e-3^2) noise: one step is the 16
    forward solves and the 16 adjoint solves of the loss gradient (inputs and
    the adjoint's right-hand sides resident).  Both precisions; the gradient
    of the first problem is checked against the oracle's."""
    import oracle as O
    m = n
    log("bench: synthesising the C4 problems")
    fs = [S.sphere_field(4, r, n, m, L) for r in range(count)]
    uobs = [S.sphere_field(4, r, n, m, L, tag=S.TAG_OBS) + S.noise(4, r, (m, n), 1e-3) for r in range(count)]
    fg = [torch.from_numpy(a).cuda() for a in fs]
    og = [torch.from_numpy(a).cuda() for a in uobs]
    res = {"workload": "c4_16_rhs_n2048_m2048_forward_adjoint", "rhs": count, "dof_per_step": 2 * count * n * m}
    for prec in ("fp64", "mixed"):
        plan = P.SpherePoisson(n, m, prec)
        us = [torch.empty_like(fg[0]) for _ in range(count)]
        gs = []
        for r in range(count):
            plan.solve(fg[r], out=us[r])
            gs.append(2.0 * (us[r] - og[r]))
        fb = [torch.empty_like(fg[0]) for _ in range(count)]
        torch.cuda.synchronize()

        def step():
            for r in range(count):
                plan.solve(fg[r], out=us[r])
            for r in range(count):
                plan.adjoint(gs[r], out=fb[r])

        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        steps = max(1, args.steps // 4)
        plan.profile_enable(16 * count * steps)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        prof = plan.profile_read()
        plan.profile_enable(0)
        plan.close()
        g0 = gs[0].cpu().numpy()
        ref = O.adjoint_reduced(g0)
        err = float(np.linalg.norm(fb[0].cpu().numpy() - ref) / np.linalg.norm(ref))
        kern = {}
        for k, (tot, cnt) in prof.items():
            alg = kernel_bytes(k, n, m, prec)
            avg = tot / cnt
            kern[k] = {"avg_ms": round(avg, 5), "launches": cnt, "alg_bytes": alg,
                       "alg_GBps": round(alg / (avg * 1e-3) / 1e9, 1)}
        log("bench: c4 %s %.3f ms/step (16 forward + 16 adjoint), gradient rel err %.2e" % (prec, ms, err))
        res[prec] = {"ms_per_step": ms, "dof_per_s": res["dof_per_step"] / (ms * 1e-3), "kernels": kern,
                     "gradient_rel_err_vs_oracle": err}
        del us, gs, fb
    return res


def bench_sweep(args, P, S, torch, np, sizes=(1024, 2048, 4096, 6144, 8192, 10000)):
    """Time per solve against the number of unknowns, n = m (the paper's
    complexity experiment, Section 5, Figure FastSphericalPoissonSolver right):
    both precisions, and the least-squares slope of log time against log(nm),
    over all sizes and over those from 4096 on (below that a solve does not
    fill the chip and fixed costs flatten the curve)."""
    res = {"workload": "sweep_n_eq_m", "sizes": list(sizes)}
    for prec in ("fp64", "mixed"):
        ms_list = []
        for n in sizes:
            f = torch.from_numpy(S.sphere_field(5, n, n, n, n // 5)).cuda()
            u = torch.empty_like(f)
            plan = P.SpherePoisson(n, n, prec)
            for _ in range(3):
                plan.solve(f, out=u)
            torch.cuda.synchronize()
            reps = 20 if n < 10000 else 5
            stream = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                plan.solve(f, out=u)
            e1.record(stream)
            torch.cuda.synchronize()
            ms_list.append(e0.elapsed_time(e1) / reps)
            plan.close()
            del f, u
        x = np.log([float(n) * n for n in sizes])
        y = np.log(ms_list)
        slope = float(np.polyfit(x, y, 1)[0])
        big = [i for i, n in enumerate(sizes) if n >= 4096]
        slope_big = float(np.polyfit(x[big], y[big], 1)[0])
        log("bench: sweep %s ms %s, slope %.3f (n >= 4096: %.3f)" % (prec, ["%.3f" % t for t in ms_list], slope,
                                                                      slope_big))
        res[prec] = {"ms_per_solve": ms_list, "dof_per_s": [n * n / (t * 1e-3) for n, t in zip(sizes, ms_list)],
                     "loglog_slope": slope, "loglog_slope_n_ge_4096": slope_big}
    return res


def bench_stream(args, P, torch, count=10 ** 8):
    """The library's streaming kernels (copy, read, write of 10^8 doubles,
    plain and non-temporal) and torch's device copy: the achievable HBM
    bandwidth the kernels' fractions are read against."""
    dev = torch.device("cuda", 0)
    x = torch.ones(count, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    part = torch.empty(int(P.library().sphere_poisson_stream_partials(count)), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    res = {"workload": "stream_1e8_doubles", "doubles": count}

    def timed(fn, nbytes):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        return {"ms": round(ms, 5), "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1)}

    nb = count * 8
    for nt in (False, True):
        tag = "_nt" if nt else ""
        res["copy" + tag] = timed(lambda: P.stream("copy", x, y, nt), 2 * nb)
        res["read" + tag] = timed(lambda: P.stream("read", x, part, nt), nb)
        res["write" + tag] = timed(lambda: P.stream("write", None, y, nt), nb)
    res["torch_copy"] = timed(lambda: y.copy_(x), 2 * nb)
    res["best_copy_GBps"] = max(res["copy"]["GBps"], res["copy_nt"]["GBps"])
    log("bench: achievable bandwidth %s" % {k: v for k, v in res.items() if isinstance(v, dict)})
    del x, y, part
    return res


def copy_calibration(args, torch):
    """A plain copy of 10^8 float64 values (800 MB read, 800 MB written): the
    kernel against which FETCH_SIZE / WRITE_SIZE counts are scaled."""
    dev = torch.device("cuda", 0)
    x = torch.ones(10 ** 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(args.warmup):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    nbytes = 2 * x.numel() * 8
    print(json.dumps({"copy_bytes_per_launch": nbytes, "read_bytes": nbytes // 2, "write_bytes": nbytes // 2,
                      "ms": ms, "GBps": nbytes / (ms * 1e-3) / 1e9}), flush=True)


def bench_gradient(args, P, torch, n, m):
    """Tangential gradient (d^t/dx, d^t/dy, d^t/dz of Section 4) of
    F = x y z + z^2 - 3 x^2 y on the workload grid, float64: time per call
    (inputs resident), library HIP-event kernel times, error against the
    closed form grad F - (p . grad F) p on every 97th row."""
    dev = torch.device("cuda", 0)
    # grid nodes theta_j = (j + 1/2) pi / m, lambda_i = -pi + 2 pi i / n
    th = ((torch.arange(m, dtype=torch.float64, device=dev) + 0.5) * (math.pi / m))[:, None]
    lam = (-math.pi + torch.arange(n, dtype=torch.float64, device=dev) * (2.0 * math.pi / n))[None, :]
    x, y, z = torch.cos(lam) * torch.sin(th), torch.sin(lam) * torch.sin(th), torch.cos(th).expand(m, n)
    f = (x * y * z + z * z - 3 * x * x * y).contiguous()
    plan = P.SpherePoisson(n, m, "fp64")
    outs = [torch.empty_like(f) for _ in range(3)]
    for _ in range(max(1, args.warmup)):
        plan.tangential_gradient(f, outs=outs)
    torch.cuda.synchronize()
    steps = max(1, args.steps // 2)
    plan.profile_enable(4 * steps)   # four launches per call: lambda forward, two theta passes, gradient
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.tangential_gradient(f, outs=outs)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    prof = plan.profile_read()
    plan.profile_enable(0)
    rows = torch.arange(0, m, 97, device=dev)
    xs, ys, zs = x[rows], y[rows], z[rows]
    Fx, Fy, Fz = ys * zs - 6 * xs * ys, xs * zs - 3 * xs * xs, xs * ys + 2 * zs
    rad = xs * Fx + ys * Fy + zs * Fz
    ref = (Fx - rad * xs, Fy - rad * ys, Fz - rad * zs)
    err = torch.sqrt(sum(((o[rows] - r) ** 2).sum() for o, r in zip(outs, ref)) / sum((r ** 2).sum() for r in ref))
    kinds = {"lambda_fwd": "lambda_fwd", "theta": "theta_deriv", "lambda_grad": "lambda_grad"}
    kern = {}
    for k, (tot, cnt) in prof.items():
        alg = kernel_bytes(k, n, m, "fp64")
        avg = tot / cnt
        kern[kinds.get(k, k)] = {"avg_ms": round(avg, 5), "launches": cnt, "alg_bytes": alg,
                                 "alg_GBps": round(alg / (avg * 1e-3) / 1e9, 1)}
    plan.close()
    log("bench: gradient %.3f ms/call, %.3e DOF/s, rel err %.2e" % (ms, n * m / (ms * 1e-3), float(err)))
    return {"workload": "tangential_gradient_n%d_m%d_fp64" % (n, m), "ms_per_call": ms,
            "dof_per_s": n * m / (ms * 1e-3), "alg_bytes_per_dof": 72, "kernels": kern,
            "rel_err_vs_closed_form": float(err)}


def bench_lowrank(args, P, S, torch, np, n, m, L=12):
    """Solve with the right-hand side given in low-rank form (rank K = 2L + 1:
    a band-limited field as its theta-profile / lambda-mode factors), both
    precisions: time per solve with the factors resident, library HIP-event
    kernel times, error against the closed-form solution on every 97th row."""
    K = 2 * L + 1
    d, C, R, u_exact = S.sphere_field_factors(21, 0, n, m, L, with_solution=True)
    dg, Cg, Rg = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (d, C, R))
    rows = np.arange(0, m, 97)
    res = {"workload": "lowrank_rhs_rank%d_n%d_m%d" % (K, n, m), "rank": K}
    for prec in ("mixed", "fp64"):
        plan = P.SpherePoisson(n, m, prec)
        u = torch.empty((m, n), dtype=torch.float64, device="cuda")
        for _ in range(max(1, args.warmup)):
            plan.solve_lowrank(dg, Cg, Rg, out=u)
        torch.cuda.synchronize()
        steps = max(1, args.steps // 2)
        plan.profile_enable(8 * steps)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            plan.solve_lowrank(dg, Cg, Rg, out=u)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        prof = plan.profile_read()
        plan.profile_enable(0)
        uh = u[torch.from_numpy(rows).cuda()].cpu().numpy()
        err = float(np.linalg.norm(uh - u_exact[rows]) / np.linalg.norm(u_exact[rows]))
        kern = {}
        for k, (tot, cnt) in prof.items():
            name = "lowrank_rows" if k == "lambda_fwd" else k
            alg = kernel_bytes(name, n, m, prec, rank=K)
            avg = tot / cnt
            kern[name] = {"avg_ms": round(avg, 5), "launches": cnt, "alg_bytes": alg,
                          "alg_GBps": round(alg / (avg * 1e-3) / 1e9, 1)}
        plan.close()
        del u
        log("bench: lowrank %s %.3f ms/solve, %.3e DOF/s, rel err %.2e" % (prec, ms, n * m / (ms * 1e-3), err))
        res[prec] = {"ms_per_solve": ms, "dof_per_s": n * m / (ms * 1e-3), "kernels": kern,
                     "rel_err_vs_closed_form": err}
    return res


def bench_evaluate(args, P, S, torch, np, n=150, m=150, L=12, npts=10 ** 6):
    """Pointwise evaluation of a rank-25 field given by its factors on the
    150 x 150 grid (the size of the paper's Poisson example) at 10^6 random
    points of the sphere: time per call (coefficients + evaluation), library
    HIP-event kernel times, and the evaluation kernel against the float64
    vector FMA peak (it is bound by arithmetic, not memory)."""
    K = 2 * L + 1
    d, C, R = S.sphere_field_factors(22, 0, n, m, L)
    rng = np.random.default_rng(23)
    v = rng.standard_normal((npts, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    dg, Cg, Rg, pg = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (d, C, R, v))
    out = torch.empty(npts, dtype=torch.float64, device="cuda")
    plan = P.SpherePoisson(n, m, "fp64")
    for _ in range(max(1, args.warmup)):
        plan.eval_lowrank(dg, Cg, Rg, pg, out=out)
    torch.cuda.synchronize()
    steps = max(1, args.steps // 2)
    plan.profile_enable(4 * steps)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.eval_lowrank(dg, Cg, Rg, pg, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    prof = plan.profile_read()
    plan.profile_enable(0)
    plan.close()
    # per point and factor: m Horner steps on two theta series (2 complex products + 2 adds,
    # 14 flops) and n/4 + 1 steps on two lambda series (16 flops), plus the combination
    N = n // 2
    flops = npts * K * (14 * m + 16 * (N // 2 + 1) + 8)
    ev = prof.get("eval", (float("nan"), 1))
    ev_ms = ev[0] / ev[1]
    peak = 78.6e12
    kern = {k: {"avg_ms": round(t / c, 5), "launches": c} for k, (t, c) in prof.items()}
    log("bench: evaluation %.3f ms/call (%d points, rank %d, %dx%d), eval kernel %.3f ms = %.1f TFLOP/s"
        % (ms, npts, K, n, m, ev_ms, flops / (ev_ms * 1e-3) / 1e12))
    return {"workload": "eval_lowrank_rank%d_n%d_m%d_points%d" % (K, n, m, npts), "ms_per_call": ms,
            "points_per_s": npts / (ms * 1e-3), "kernels": kern,
            "eval_roofline": {"bound": "alu", "achieved": flops / (ev_ms * 1e-3) / 1e12, "peak": peak / 1e12,
                              "unit": "TFLOP/s", "frac": flops / (ev_ms * 1e-3) / peak,
                              "flops_per_launch": flops}}


def bench_ge(args, P, S, torch, np, n, m, L=12):
    """Low-rank approximation by structure-preserving Gaussian elimination of a
    band-limited field of degree 12 (rank 25) sampled on the workload grid:
    time per call with the samples resident, steps until the tolerance stops
    the loop, reconstruction error on every 97th row, and the HBM rate of the
    whole call against its algorithmic bytes (one read of the grid for the
    first pivot search, then per step one read and one write: the update pass
    also scores the next step's candidates)."""
    f = torch.from_numpy(S.sphere_field(24, 0, n, m, L)).cuda()
    steps = 2 * L + 2
    for _ in range(max(1, args.warmup)):
        d, c, r, piv = P.ge_lowrank(f, steps, 0.01, 1e-12)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 4)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        d, c, r, piv = P.ge_lowrank(f, steps, 0.01, 1e-12)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    active = int((piv[:, 0] >= 0).sum())
    rows = torch.arange(0, m, 97, device=f.device)
    rec = (c[:, rows].T * d[None, :]) @ r
    err = float((rec - f[rows]).abs().max() / f.abs().max())
    # one search before the first step (8 B per sample), then per active step one update pass that also
    # scores the next step's candidates (16 B: read and write)
    alg = n * m * (8 + 16 * active)
    log("bench: ge %.3f ms/call (%d steps, %d active), rel err %.2e, %.0f GB/s" % (ms, steps, active, err,
                                                                                    alg / (ms * 1e-3) / 1e9))
    return {"workload": "ge_lowrank_rank%d_n%d_m%d" % (2 * L + 1, n, m), "ms_per_call": ms, "steps": steps,
            "active_steps": active, "rel_err_rows": err, "alg_bytes": alg, "alg_GBps": alg / (ms * 1e-3) / 1e9}


def bench_batch(args, P, S, torch, np):
    """512 right-hand sides, n, m i.i.d. uniform on {128, 192, ..., 2048}, band
    limit floor(min(n, m)/4), mixed precision, one graph launch per step."""
    sizes = S.batch_sizes(3, 512, [64 * j for j in range(2, 33)])
    log("bench: synthesising the 512-problem batch")
    t0 = time.time()
    fs = [torch.from_numpy(S.sphere_field(3, r, int(n), int(m), int(min(n, m)) // 4)).cuda()
          for r, (n, m) in enumerate(sizes)]
    us = [torch.empty_like(f) for f in fs]
    log("bench: batch inputs ready in %.1fs" % (time.time() - t0))
    dof = int(sum(int(n) * int(m) for n, m in sizes))
    # the batch plan: radix orders of every distinct size from the autotuner (measured now when the
    # cache has no entry), workspace, work lists and the captured graph; built once, outside the timing
    t0 = time.time()
    batch = P.SpherePoissonBatch(fs, us, "mixed", max_refine=1, autotune=not args.no_autotune)
    plan_s = time.time() - t0
    log("bench: batch plan built in %.1fs (autotune %s)" % (plan_s, not args.no_autotune))
    for _ in range(max(1, args.warmup)):
        batch.solve()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(1, args.steps // 4)
    e0.record(stream)
    for _ in range(steps):
        batch.solve()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    _, infos = batch.solve(with_info=True)
    batch.close()
    log("bench: batch %.3f ms/step, %.3e DOF/s" % (ms, dof / (ms * 1e-3)))
    return {"workload": "batch_512_rhs_n_m_uniform_128_2048_mixed", "rhs": 512, "dof": dof,
            "ms_per_step": ms, "dof_per_s": dof / (ms * 1e-3), "launches_per_step": 1,
            "autotuned": not args.no_autotune, "plan_seconds": plan_s,
            "max_est_rel_err": max(i["est_rel_err"] for i in infos)}


if __name__ == "__main__":
    main()
