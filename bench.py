#!/usr/bin/env python3
"""Benchmark: solved samples/s of the ensemble diffusion solve on one MI355X.

Workload (default): 128^3 hexahedra (2,146,689 nodes, 57,066,625 stored
entries), M = 10 KL terms, sigma = 0.3, ensemble size s = 32, FP32 CG inside
FP64 iterative refinement to a true relative residual of 1e-8 per sample,
the inner CG preconditioned by the ensemble multigrid V-cycle in FP32
(--precond jacobi: Jacobi instead).  One step = ensemble assembly (FP64
values, FP32 copy, load vector) + the multigrid set-up + the refined solve
of all 32 samples from a zero guess; inputs (graph, KL table, KL inputs y)
are resident in HBM before the timed region.

Printed: one JSON line with the contract fields plus
  roofline      the dominant kernel (the fine-level row passes of the cycle;
                with Jacobi, the FP32 ensemble SpMV of the inner CG):
                algorithmic bytes per launch / mean launch time from HIP
                events recorded on the launch stream during the timed steps;
  jacobi        the same timed step with the Jacobi preconditioner;
  cpu_baseline  the FP64 CPU oracle of the timed method on the host cores;
  context       FP64 ensemble CG (per-sample and coupled) and s one-sample
                GPU solves of the same samples, per-sample error against an
                FP64 solve, SpMV GB/s.
Other workloads: --workload mid|small|batch|learned|mg.
"""
from __future__ import annotations

import argparse
import hashlib
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SNAPSHOT_RTOL = 1e-10   # training solves of the learned guess
METRIC = "solved samples/s at 128^3, s=32, 1e-8 resid; ensemble SpMV HBM GB/s vs scalar"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_bytes(n, nnz, s, w):
    """Algorithmic bytes of one ensemble CRS product: values and column
    indices once, row offsets once, x read once, y written once."""
    return nnz * (s * w + 4.0) + 4.0 * (n + 1) + 2.0 * n * s * w


def kernel_source_hash():
    """Hash of the sources of the CG and cycle kernels with comments and all
    white space left out (an edit of comments or layout does not change what
    the counters were taken on)."""
    import re

    h = hashlib.sha256()
    for f in ("rowops.hpp", "cgcore.hpp", "cg.hip", "common.hpp", "mg.hip", "mg.hpp"):
        with open(os.path.join(ROOT, "paper_1511_03703_amd", "csrc", f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        text = "\n".join(re.sub(r"//.*", "", l) for l in text.splitlines())
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel_name):
    """HBM traffic per launch measured with rocprofv3 counters (see profiles/),
    valid only while the kernel sources are unchanged."""
    p = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    ent = d.get(kernel_name)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def host_env():
    """Where the numbers come from: the host's CPUs (model, count, the share
    this process may use, the OpenMP threads the oracle gets), the ROCm
    toolchain the library was compiled with, and the HIP runtime actually
    mapped into this process (torch loads its own libamdhip64, whose soname
    the library's dependency then resolves to)."""
    import ctypes

    import torch

    env = {"device": torch.cuda.get_device_name(0), "torch": torch.__version__, "torch_hip": torch.version.hip,
           "nproc": os.cpu_count(), "cpus_usable": len(os.sched_getaffinity(0)),
           "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        with open("/proc/cpuinfo") as fh:
            env["cpu_model"] = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        env["cpu_model"] = None
    try:
        with open("/opt/rocm/.info/version") as fh:
            env["rocm_toolchain"] = fh.read().strip()
    except OSError:
        env["rocm_toolchain"] = None
    with open("/proc/self/maps") as fh:
        libs = sorted({l.split()[-1] for l in fh if "libamdhip64" in l})
    env["hip_runtime_lib"] = libs
    try:
        hip = ctypes.CDLL("libamdhip64.so.7")
        v = ctypes.c_int()
        hip.hipRuntimeGetVersion(ctypes.byref(v))
        env["hip_runtime_version"] = v.value
        # peak engine and memory clocks and the compute units the runtime
        # reports (hipDeviceAttribute ClockRate = 5, MemoryClockRate = 60,
        # MultiprocessorCount = 63 in hip_runtime_api.h of ROCm 7)
        for key, attr, scale in (("gpu_clock_mhz", 5, 1e-3), ("mem_clock_mhz", 60, 1e-3), ("compute_units", 63, 1)):
            if hip.hipDeviceGetAttribute(ctypes.byref(v), attr, torch.cuda.current_device()) == 0:
                env[key] = v.value * scale if scale != 1 else v.value
    except OSError:
        env["hip_runtime_version"] = None
    return env


def oracle_threads(requested):
    """OpenMP threads of the CPU baseline: the requested count, or (0) the
    threads the oracle's OpenMP runtime offers this process, at most 32."""
    if requested > 0:
        return requested
    from oracle import oracle as orc
    return max(1, min(orc.max_threads(), 32))


def cpu_baseline(N, M, sigma, rtol, xi, iters_fp64, cap_iters, L=1.0, kappa0=1.0, f=1.0):
    """The FP64 oracle (graph, KL, assembly, Jacobi-CG) on the rows of `xi` in
    parallel, one sample per OpenMP thread, on the host cores.  Bounded: each
    solve runs `cap_iters` iterations; the oracle reports per-sample set-up
    and solve wall times, and the full solve is scaled with the per-sample
    FP64 iteration counts of the same samples.  Returns (samples/s, threads,
    per-sample full seconds, set-up s, capped-solve s)."""
    from oracle import oracle as orc

    threads = xi.shape[0]
    _, it, _, _, used, tm = orc.solve_samples(N, M, L, kappa0, sigma, f, xi, rtol, max_iter=cap_iters,
                                              want_x=False, timing=True)
    full = []
    for e in range(threads):
        t_iter = tm[e, 1] / max(int(it[e]), 1)
        full.append(tm[e, 0] + iters_fp64[e] * t_iter)
    return threads / max(full), int(used), full, float(tm[:, 0].max()), float(tm[:, 1].max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="default 5 (solve workloads), 1 (batch, learned)")
    ap.add_argument("--warmup", type=int, default=None, help="default 1 (solve workloads), 0 (batch, learned)")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "mid", "small", "batch", "learned", "mg", "newton", "assembly",
                             "coupled"])
    ap.add_argument("--pool-gib", type=float, default=192.0, help="batch: resident pool size")
    ap.add_argument("--batch-s", type=int, default=0, help="batch: fix s (skip the autotuner)")
    ap.add_argument("--batch-tile", type=int, default=4, help="batch: tile when --batch-s is given")
    ap.add_argument("--group", default="contrast", choices=["contrast", "draw"],
                    help="batch: form each mesh size's ensembles by coefficient contrast, or in draw order")
    ap.add_argument("--train-steps", type=int, default=32000, help="learned: Adam steps")
    ap.add_argument("--train-lr", type=float, default=3e-3, help="learned: initial Adam learning rate")
    ap.add_argument("--precond", default="mg", choices=["mg", "jacobi"],
                    help="headline/mid/small: preconditioner of the timed solve (default: multigrid)")
    ap.add_argument("--coarse", default="redisc", choices=["redisc", "galerkin"],
                    help="multigrid coarse operators: assembled on each mesh, or Galerkin products P^T A P")
    ap.add_argument("--mg-fp64", action="store_true",
                    help="mg: FP64 CG with an FP64 cycle instead of the FP32-in-FP64 refinement")
    ap.add_argument("--lr-halvings", type=int, default=5,
                    help="learned: the step count is split into this many + 1 equal stages, lr halved per stage")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-context", action="store_true", help="skip the FP64 / scalar comparison runs")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="CPU oracle threads and samples (0: what OpenMP offers the process, at most 32)")
    ap.add_argument("--cpu-cap-iters", type=int, default=25)
    ap.add_argument("--inner-rtol", type=float, default=None,
                    help="refinement inner tolerance (default: 1e-4 with multigrid, 1e-5 with Jacobi, the measured "
                         "optima at 128^3, s=32)")
    ap.add_argument("--check-every", type=int, default=16)
    ap.add_argument("--compact", action="store_true",
                    help="FP64 solve workloads: finish the last s/2 iterating samples in a compacted ensemble")
    ap.add_argument("--lin-rtol", type=float, default=None, help="newton: GMRES tolerance per Newton step")
    ap.add_argument("--jac-fp64", action="store_true", help="newton: keep the Jacobian in FP64 for GMRES")
    ap.add_argument("--newton-mg", default="adv", choices=["adv", "diffusion"],
                    help="newton: the multigrid cycle of D + alpha C (adv) or of the diffusion operator D")
    ap.add_argument("--forcing", default="ew", choices=["ew", "fixed"],
                    help="newton: GMRES tolerance per step, Eisenstat-Walker or fixed")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (hardware-counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the path is measured on one GPU's "
              f"share at its real shape; sharding over several GPUs is designed, not built.", file=sys.stderr)
        sys.exit(2)
    heavy = args.workload in ("batch", "learned")
    if args.steps is None:
        args.steps = 1 if heavy else 5
    if args.warmup is None:
        args.warmup = 0 if heavy else 1
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "learned":
        return run_learned(args)
    if args.workload == "mg":
        return run_mg(args)
    if args.workload == "newton":
        return run_newton(args)
    if args.workload == "assembly":
        return run_assembly(args)
    if args.workload == "coupled":
        return run_coupled(args)
    return run_solve(args)


def calibration_copy(args):
    """One plain device copy of --calib-copy-mb MiB (k_copy16: that many bytes
    read and written), whose FETCH_SIZE / WRITE_SIZE counters scale the
    counters of the kernels profiled in the same run."""
    if args.calib_copy_mb <= 0:
        return
    import torch

    from paper_1511_03703_amd import ens
    nb = args.calib_copy_mb << 20
    src = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    ens.stream_copy(src, dst)
    torch.cuda.synchronize()
    log(f"calibration copy of {nb} bytes done")
    del src, dst


def run_solve(args):
    import numpy as np
    import torch

    from paper_1511_03703_amd import ens
    import workloads

    w = {"headline": workloads.HEADLINE, "mid": workloads.MID, "small": workloads.SMALL}[args.workload]
    dev = "cuda"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    log(f"workload {w.name}: N={w.N} n={w.n} nnz={w.nnz} s={w.s} M={w.M} sigma={w.sigma} mixed={w.mixed}")
    g = ens.graph_build(w.N)
    kl = ens.kl_build(w.N, w.M, w.L)
    xi = torch.as_tensor(w.xi(), device=dev)
    vals = torch.empty((w.nnz, w.s), dtype=torch.float64, device=dev)
    v32 = torch.empty((w.nnz, w.s), dtype=torch.float32, device=dev) if w.mixed else None
    rhs = torch.empty((w.n, w.s), dtype=torch.float64, device=dev)
    x = torch.zeros((w.n, w.s), dtype=torch.float64, device=dev)
    jac_inner = args.inner_rtol if args.inner_rtol is not None else 1e-5
    opts = ens.cg_opts(rtol=w.rtol, mixed=w.mixed, inner_rtol=jac_inner, check_every=args.check_every,
                       compact=args.compact and not w.mixed)
    ws = torch.empty(ens.cg_workspace_bytes(g, w.s, opts), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    calibration_copy(args)

    use_mg = args.precond == "mg"
    mg = ens.Multigrid(w.N, w.M, w.s, fp32=w.mixed, L=w.L, device=dev) if use_mg else None
    # the multigrid solve takes a handful of iterations: poll every 4
    mg_inner = args.inner_rtol if args.inner_rtol is not None else 1e-4
    mg_opts = ens.cg_opts(rtol=w.rtol, mixed=w.mixed, inner_rtol=mg_inner, check_every=min(args.check_every, 4))

    def step_jacobi():
        ens.assemble(g, kl, xi, w.M, w.sigma, L=w.L, kappa0=w.kappa0, f=w.f, values=vals, values32=v32, rhs=rhs)
        x.zero_()
        return ens.cg(g, vals, rhs, x=x, values32=v32, opts=opts, workspace=ws)

    def step_mg():
        # fine assembly with the hierarchy's fine-level D^-1 and bound fused in,
        # then the coarse levels
        mg.assemble_setup(g, kl, xi, w.sigma, vals, rhs, values32=v32, kappa0=w.kappa0, f=w.f,
                          galerkin=args.coarse == "galerkin")
        x.zero_()
        return ens.cg_mg(g, vals, rhs, mg, x=x, values32=v32, opts=mg_opts, workspace=ws)

    step_ms = []

    def timed(step, steps, warmup):
        # profiling is on during the warmup too, so the timed steps repeat
        # exactly the warmup's host work; the interpreter's cyclic garbage
        # collector (a full pass over torch's objects takes tens of ms) is
        # run once here and paused until the timing ends
        ens.prof_enable(True)
        gc.collect()
        gc.disable()
        for i in range(warmup):
            tw = time.perf_counter()
            _, stats, st = step()
            log(f"warmup {i}: {(time.perf_counter() - tw) * 1e3:.1f} ms, status {st}, "
                f"iters {[t['iters'] for t in stats][:8]}...")
        torch.cuda.synchronize()
        ens.prof_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        marks = []
        for i in range(steps):
            _, stats, st = step()  # ends with the solver's own synchronisation
            marks.append(time.perf_counter())
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        gc.enable()
        ens.prof_enable(False)
        per = [round((b - a) * 1e3, 2) for a, b in zip([t0] + marks[:-1], marks)]
        log(f"ms per step: {per}")
        step_ms.clear()
        step_ms.extend(per)
        return el, stats

    def spmv_roofline():
        kid = ens.K_SPMV_F32 if w.mixed else ens.K_SPMV_F64
        pq = ens.prof_query(kid)
        wb = 4.0 if w.mixed else 8.0
        per = spmv_bytes(w.n, w.nnz, w.s, wb)
        avg = pq["total_ms"] / max(pq["launches"], 1)
        ach = per / (avg * 1e-3) / 1e9
        kname = f"k_cg_spmv_dot<{'float' if w.mixed else 'double'},{w.s}>"
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": load_traffic(kname), "kernel": kname,
                "bytes_per_launch": per, "avg_launch_ms": round(avg, 5), "launches": pq["launches"]}

    def mg_roofline():
        pr = ens.prof_query(ens.K_MG_ROW)
        ach = pr["bytes"] / (pr["total_ms"] * 1e-3) / 1e9 if pr["launches"] else 0.0
        kname = f"k_mg_row<{'float' if w.mixed else 'double'},{w.s},*>"
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": load_traffic(kname),
                "kernel": kname + " (fine-level Chebyshev and residual passes of the V-cycle)",
                "bytes_per_launch": round(pr["bytes"] / max(pr["launches"], 1)),
                "avg_launch_ms": round(pr["total_ms"] / max(pr["launches"], 1), 5), "launches": pr["launches"]}

    elapsed, stats = timed(step_mg if use_mg else step_jacobi, args.steps, args.warmup)
    head_steps = list(step_ms)
    roofline = mg_roofline() if use_mg else spmv_roofline()
    pa = ens.prof_query(ens.K_ASSEMBLE)
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    ok = all(t["status"] == 0 and t["rel_res"] <= w.rtol * (1 + 1e-6) for t in stats)
    value = args.steps * w.s / elapsed
    wb = 4.0 if w.mixed else 8.0

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-in-f64" if w.mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "mesh": f"{w.N}^3 Q1 hexahedra", "n": w.n, "nnz": w.nnz, "s": w.s,
                   "M": w.M, "sigma": w.sigma, "L": w.L, "rtol": w.rtol, "seed": w.seed,
                   "inner_rtol": (mg_inner if use_mg else jac_inner) if w.mixed else None,
                   "preconditioner": ("multigrid V-cycle (levels N, N/2, .. 4; order-2 Chebyshev; exact coarsest)"
                                      + (" in FP32 inside the FP64 refinement" if w.mixed else "")) if use_mg
                   else "Jacobi",
                   "coarse_operators": ({"redisc": "assembled on each mesh", "galerkin": "Galerkin P^T A P"}
                                        [args.coarse] if use_mg else None)},
        "roofline": roofline,
        "all_converged": ok,
        "iters": {"inner_total": [t["iters"] for t in stats], "outer": [t["outer_iters"] for t in stats]},
        # every level's assembly in one step (launches under 5 % of the
        # longest one are not recorded)
        "assembly_ms_per_step": round(pa["total_ms"] / max(args.steps, 1), 3),
        "step_ms": {"median": float(np.median(head_steps)), "min": min(head_steps), "max": max(head_steps)},
        "env": host_env(),
    }
    x_head = x.clone() if not args.no_context else None
    if use_mg and not args.no_context:
        # the same step with the Jacobi preconditioner (the oracle's method)
        el_j, st_j = timed(step_jacobi, args.steps, 1)
        out["jacobi"] = {"value": round(args.steps * w.s / el_j, 3), "ms_per_step": round(el_j / args.steps * 1e3, 3),
                         "inner_rtol": jac_inner if w.mixed else None,
                         "iters_inner_max": max(t["iters"] for t in st_j),
                         "all_converged": all(t["status"] == 0 and t["rel_res"] <= w.rtol * (1 + 1e-6) for t in st_j),
                         "roofline": spmv_roofline(),
                         "note": "identical workload, Jacobi instead of multigrid as the preconditioner"}

    iters_fp64 = None
    if not args.no_context:
        # FP64 ensemble CG of the same samples: reference solution at 1e-12 for
        # the per-sample error, and the FP64 timing at the target tolerance
        xr = torch.zeros_like(x)
        _, st12, _ = ens.cg(g, vals, rhs, x=xr, opts=ens.cg_opts(rtol=1e-12), workspace=None)
        xs = x_head.cpu().numpy()
        del x_head
        xrn = xr.cpu().numpy()
        err = [float(np.linalg.norm(xs[:, e] - xrn[:, e]) / np.linalg.norm(xrn[:, e])) for e in range(w.s)]
        x64 = torch.zeros_like(x)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, st64, _ = ens.cg(g, vals, rhs, x=x64, opts=ens.cg_opts(rtol=w.rtol, check_every=args.check_every))
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        iters_fp64 = [s["iters"] for s in st64]
        xcp = torch.zeros_like(x)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, stcp, _ = ens.cg(g, vals, rhs, x=xcp, opts=ens.cg_opts(rtol=w.rtol, check_every=args.check_every,
                                                                 coupled=True))
        torch.cuda.synchronize()
        tcp = time.perf_counter() - t1
        del xcp
        # s one-sample solves on the same GPU (sample-major layout)
        vsm = ens.relayout(vals, True)
        bsm = ens.relayout(rhs, True)
        del xr
        best = None
        for lanes in (0, 8, 16):  # 0: row tiles read by the whole workgroup
            xsm = torch.zeros_like(bsm)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            _, sst, _ = ens.scalar_cg(g, vsm, bsm, xsm, opts=ens.cg_opts(rtol=w.rtol, check_every=args.check_every),
                                      lanes_per_row=lanes)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t2
            if best is None or ts < best[0]:
                best = (ts, lanes, [s["iters"] for s in sst])
        conc = None
        for streams in (4, 8):
            xsm = torch.zeros_like(bsm)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            _, sst, _ = ens.scalar_cg_concurrent(g, vsm, bsm, xsm,
                                                 opts=ens.cg_opts(rtol=w.rtol, check_every=args.check_every),
                                                 lanes_per_row=best[1], streams=streams)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t2
            if conc is None or ts < conc[0]:
                conc = (ts, streams)
        del vsm, bsm, xsm
        # standalone SpMV bandwidth, ensemble vs one-sample kernel
        V = v32 if w.mixed else vals
        xv = torch.rand((w.n, w.s), dtype=V.dtype, device=dev)
        yv = torch.empty_like(xv)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            ens.spmv(g, V, xv, yv)
        e0.record()
        for _ in range(10):
            ens.spmv(g, V, xv, yv)
        e1.record()
        torch.cuda.synchronize()
        t_ens = e0.elapsed_time(e1) / 10
        vs1 = vals[:, 0].contiguous() if not w.mixed else v32[:, 0].contiguous()
        x1 = torch.rand(w.n, dtype=vs1.dtype, device=dev)
        y1 = torch.empty_like(x1)
        sc_times = {}
        for lanes in (0, 16):  # the faster one-sample product is the baseline
            for _ in range(3):
                ens.scalar_spmv(g, vs1, x1, y1, lanes_per_row=lanes)
            e0.record()
            for _ in range(10):
                ens.scalar_spmv(g, vs1, x1, y1, lanes_per_row=lanes)
            e1.record()
            torch.cuda.synchronize()
            sc_times[lanes] = e0.elapsed_time(e1) / 10
        sc_lanes = min(sc_times, key=sc_times.get)
        t_sc = sc_times[sc_lanes]
        # the STREAM-style triad a = b + q c on 3 x 4 GiB of FP64 (the
        # bandwidth the paper bounds its products with)
        na = (4 << 30) // 8
        ta = torch.empty(na, dtype=torch.float64, device=dev)
        tb = torch.rand(na, dtype=torch.float64, device=dev)
        tc = torch.rand(na, dtype=torch.float64, device=dev)
        for _ in range(2):
            ens.stream_triad(ta, tb, tc, 0.5)
        e0.record()
        for _ in range(5):
            ens.stream_triad(ta, tb, tc, 0.5)
        e1.record()
        torch.cuda.synchronize()
        triad_gbs = 3.0 * na * 8 / (e0.elapsed_time(e1) / 5) / 1e6
        # the read-only and copy ceilings on the same 4 GiB buffers
        for _ in range(2):
            ens.stream_read(tb)
        e0.record()
        for _ in range(5):
            ens.stream_read(tb)
        e1.record()
        torch.cuda.synchronize()
        read_gbs = na * 8 / (e0.elapsed_time(e1) / 5) / 1e6
        for _ in range(2):
            ens.stream_copy(tb, ta)
        e0.record()
        for _ in range(5):
            ens.stream_copy(tb, ta)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 2.0 * na * 8 / (e0.elapsed_time(e1) / 5) / 1e6
        write_gbs = write_ceiling(ta)
        del ta, tb, tc
        b_ens = spmv_bytes(w.n, w.nnz, w.s, wb)
        b_sc = spmv_bytes(w.n, w.nnz, 1, wb)
        jac_rate = out["jacobi"]["value"] if use_mg else value
        out["context"] = {
            "per_sample_error_vs_fp64": {"max": max(err), "median": float(np.median(err)),
                                          "reference": "GPU FP64 ensemble Jacobi-CG to 1e-12"},
            "fp64_ensemble_cg": {"seconds": round(t64, 4), "samples_per_s": round(w.s / t64, 3),
                                 "iters": iters_fp64},
            "fp64_coupled_ensemble_cg": {"seconds": round(tcp, 4), "samples_per_s": round(w.s / tcp, 3),
                                         "iters": stcp[0]["iters"],
                                         "max_sample_rel_res": max(t["rel_res"] for t in stcp),
                                         "note": "one alpha/beta for the ensemble; stop on the residual over all "
                                                 "samples"},
            "scalar_gpu_fp64": {"seconds": round(best[0], 4), "samples_per_s": round(w.s / best[0], 3),
                                "lanes_per_row": best[1], "iters": best[2],
                                "speedup_jacobi_refinement_ensemble": round(jac_rate / (w.s / best[0]), 3),
                                "speedup_fp64_ensemble": round(best[0] / t64, 3),
                                "speedup_headline_solve": round(value / (w.s / best[0]), 3)},
            "scalar_gpu_fp64_concurrent": {"seconds": round(conc[0], 4), "samples_per_s": round(w.s / conc[0], 3),
                                           "streams": conc[1], "lanes_per_row": best[1],
                                           "speedup_jacobi_refinement_ensemble": round(jac_rate / (w.s / conc[0]),
                                                                                       3),
                                           "speedup_fp64_ensemble": round(conc[0] / t64, 3),
                                           "speedup_headline_solve": round(value / (w.s / conc[0]), 3)},
            "speedup_note": ("the one-sample baselines run Jacobi-CG; speedup_jacobi_refinement_ensemble and "
                             "speedup_fp64_ensemble compare the same method (the ensemble gain), "
                             "speedup_headline_solve compares the timed headline solve with them"),
            "spmv": {"ensemble_ms": round(t_ens, 5), "ensemble_GBs": round(b_ens / t_ens / 1e6, 1),
                     "ensemble_GFLOPs": round(2.0 * w.nnz * w.s / t_ens / 1e6, 1),
                     "scalar_ms": round(t_sc, 5), "scalar_GBs": round(b_sc / t_sc / 1e6, 1),
                     "scalar_lanes_per_row": sc_lanes,
                     "scalar_ms_by_lanes_per_row": {str(k): round(v, 5) for k, v in sc_times.items()},
                     "speedup_s_times_scalar_over_ensemble": round(w.s * t_sc / t_ens, 3),
                     "dtype": "f32" if w.mixed else "f64"},
            "triad_GBs": round(triad_gbs, 1),
            "read_GBs": round(read_gbs, 1),
            "copy_GBs": round(copy_gbs, 1),
            "write_GBs": round(write_gbs, 1),
        }
        del xv, yv, x1, y1

    if not args.no_cpu_baseline and use_mg:
        from oracle import oracle as orc
        threads = min(oracle_threads(args.cpu_threads), w.s)
        log("CPU oracle baseline (multigrid PCG) ...")
        t0 = time.perf_counter()
        _, it, _, _, _ = orc.ens_mg_pcg(w.N, w.M, w.L, w.kappa0, w.sigma, w.f, w.xi()[:threads], rtol=w.rtol)
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": threads / tc, "unit": "samples/s", "cores": min(threads, orc.max_threads()), "kind": "oracle",
            "sample": (f"{threads} samples of the same workload, one per OpenMP thread: the oracle's FP64 "
                       f"multigrid PCG (it has no FP32 path) from graph and assembly of every level to {w.rtol:g}, "
                       f"iterations {[int(v) for v in it]}"),
            "seconds_measured": round(tc, 2)}
    elif not args.no_cpu_baseline:
        its = iters_fp64 if iters_fp64 is not None else [300] * w.s
        threads = min(oracle_threads(args.cpu_threads), w.s)
        log("CPU oracle baseline ...")
        t0 = time.perf_counter()
        v, used, _, t_set, t_cg = cpu_baseline(w.N, w.M, w.sigma, w.rtol, w.xi()[:threads], its,
                                               args.cpu_cap_iters, w.L, w.kappa0, w.f)
        out["cpu_baseline"] = {
            "value": v, "unit": "samples/s", "cores": used, "kind": "oracle",
            "sample": (f"{threads} samples of the same workload, one per OpenMP thread; set-up (graph+KL+assembly) "
                       f"{t_set:.1f} s, Jacobi-CG capped at {args.cpu_cap_iters} iterations ({t_cg:.1f} s); full "
                       f"FP64 solve to {w.rtol:g} scaled with the per-sample FP64 iteration counts "
                       f"{[int(i) for i in its[:threads]]}"),
            "seconds_measured": round(time.perf_counter() - t0, 2)}

    out.setdefault("env", host_env())
    print(json.dumps(out), flush=True)


def cg_iteration_bytes(n, nnz, s, w):
    """Algorithmic bytes of one Jacobi-CG iteration of an ensemble: the
    product q = A p (with p.q), the update pass (reads x, p, q, r, D^-1,
    writes x, r) and the direction pass (reads r, D^-1, p, writes p)."""
    return spmv_bytes(n, nnz, s, w) + 11.0 * n * s * w


def run_batch(args):
    """256 sample groups on meshes drawn from {32,48,64,96}^3, FP64 Jacobi-CG
    to 1e-8, streamed through a resident pool in waves of batched solves."""
    import numpy as np
    import torch

    from paper_1511_03703_amd import batchpool, ens
    import workloads as W

    dev = "cuda"
    torch.cuda.set_device(0)
    meshes = W.batch_meshes()
    G, M, sigma, rtol = len(meshes), W.BATCH_M, W.BATCH_SIGMA, W.BATCH_RTOL
    counts = {int(N): int((meshes == N).sum()) for N in W.BATCH_MESHES}
    log(f"batch: {G} groups, meshes {counts}, M={M} sigma={sigma} rtol={rtol}")
    tune = None
    if args.batch_s:
        s, tile = args.batch_s, args.batch_tile
    else:
        distinct = list(W.BATCH_MESHES)
        xi_tune = np.stack([W.draw_xi(W.BATCH_TUNE_SEED + i, 32, M) for i in range(len(distinct))])
        t0 = time.perf_counter()
        s, tile, scores = ens.batch_autotune(distinct, M, sigma, xi_tune,
                                             opts=ens.batch_opts(rtol=rtol, check_every=args.check_every))
        tune = {"seconds": round(time.perf_counter() - t0, 2),
                "scores_samples_per_s": {f"s{a}_tile{b}": round(v, 2) for (a, b), v in scores.items()},
                "trial": "32 samples per mesh size, each candidate solves them to the target tolerance"}
        log(f"autotuner: s={s} tile={tile} ({tune['seconds']} s)")
    opts = ens.batch_opts(rtol=rtol, check_every=args.check_every, tile=tile)
    xi = torch.as_tensor(W.draw_xi(W.BATCH_XI_SEED, G * s, M).reshape(G, s, M), device=dev)
    pool_bytes = int(args.pool_gib * (1 << 30))
    pool = batchpool.BatchPool(ens, meshes, s, M, pool_bytes)
    log(f"pool {args.pool_gib} GiB: {len(pool.waves)} waves of {[w.count for w in pool.waves]} groups")

    wave_times = []

    def on_wave(wv, groups, stats):
        wave_times.append(time.perf_counter())

    grouped = args.group == "contrast"

    def step(**kw):
        # the grouping (coefficient extremes on the device, host ordering,
        # regrouped inputs) is part of the timed step
        xg = pool.group_by_contrast(xi, sigma)[0] if grouped else xi
        return pool.run(xg, sigma, opts, **kw)

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_g = time.perf_counter()
    if grouped:
        pool.group_by_contrast(xi, sigma)
    torch.cuda.synchronize()
    t_group = time.perf_counter() - t_g
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    for i in range(args.steps):
        wave_times.clear()
        stats, rc = step(on_wave=on_wave)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gc.enable()
    per_step = elapsed / args.steps
    ok = rc == ens.ENS_OK and all(t["status"] == 0 and t["rel_res"] <= rtol * (1 + 1e-6) for st in stats
                                  for t in st)
    # algorithmic bytes of the iterations each group ran (a group's kernels
    # stream its whole ensemble while any of its samples is active)
    tot_bytes = 0.0
    iters_by_mesh = {int(N): [] for N in W.BATCH_MESHES}
    for N, st in zip(meshes, stats):
        n, nnz = batchpool.mesh_sizes(int(N))
        k = max(t["iters"] for t in st)
        tot_bytes += k * cg_iteration_bytes(n, nnz, s, 8.0)
        iters_by_mesh[int(N)].extend(t["iters"] for t in st)
    achieved = tot_bytes / per_step / 1e9
    value = G * s / per_step
    out = {
        "metric": "solved samples/s, 256 groups on {32,48,64,96}^3 meshes, FP64 to 1e-8",
        "value": round(value, 3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(per_step * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "q1_batch_256groups_fp64", "groups": G, "meshes": counts, "s": s, "tile": tile,
                   "M": M, "sigma": sigma, "rtol": rtol, "mesh_seed": W.BATCH_MESH_SEED,
                   "xi_seed": W.BATCH_XI_SEED, "pool_gib": args.pool_gib, "waves": len(pool.waves),
                   "check_every": args.check_every},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole batched step (assembly + every CG phase of every wave)",
                     "bytes": tot_bytes,
                     "note": "algorithmic bytes of the CG iterations run, over the step's wall time"},
        "all_converged": bool(ok),
        "iters": {str(N): {"median": float(np.median(v)), "max": int(max(v))} for N, v in iters_by_mesh.items()
                  if v},
        "grouping": {
            "by": ("coefficient contrast kmax/kmin over the mesh's Gauss points, per mesh size" if grouped
                   else "draw order"),
            "seconds": round(t_group, 4) if grouped else 0.0,
            # an ensemble iterates as long as its slowest sample: the sum of
            # the groups' maxima is what the batch pays; sorting each mesh
            # size's samples by their actual counts would give the least
            "summed_group_max_iters": int(sum(max(t["iters"] for t in st) for st in stats)),
            "summed_group_max_iters_ideal": int(sum(
                np.sort(np.asarray(v))[k * s:(k + 1) * s].max() for v in iters_by_mesh.values() if v
                for k in range(len(v) // s))),
            "summed_sample_iters": int(sum(t["iters"] for st in stats for t in st))},
        "autotune": tune,
    }
    if not args.no_context:
        # the same groups one at a time through the single-ensemble solver
        log("sequential single-ensemble solves of the same groups ...")
        cg = ens.cg_opts(rtol=rtol, check_every=args.check_every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        seq_ok = True
        for gi, N in enumerate(meshes):
            g, kl = pool.graphs[int(N)]
            n, nnz = batchpool.mesh_sizes(int(N))
            vals, off = pool._carve(0, 8 * nnz * s, (nnz, s))
            b, off = pool._carve(off, 8 * n * s, (n, s))
            x, off = pool._carve(off, 8 * n * s, (n, s))
            ens.assemble(g, kl, xi[gi], M, sigma, values=vals, rhs=b)
            x.zero_()
            _, st1, rc1 = ens.cg(g, vals, b, x=x, opts=cg, workspace=pool.pool[off:])
            seq_ok &= rc1 == ens.ENS_OK
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t1
        out["context"] = {"sequential_ens_cg": {"seconds": round(t_seq, 3),
                                                "samples_per_s": round(G * s / t_seq, 3),
                                                "all_converged": bool(seq_ok),
                                                "batched_speedup": round(t_seq / per_step, 3)}}
    if not args.no_cpu_baseline:
        log("CPU oracle baseline ...")
        t0 = time.perf_counter()
        per_mesh = {}
        used_max = 0
        nth = oracle_threads(args.cpu_threads)
        for N in W.BATCH_MESHES:
            its = iters_by_mesh[int(N)] or [200]
            xi_c = W.draw_xi(W.BATCH_XI_SEED, nth, M)
            med = [int(np.median(its))] * nth
            _, used, full, _, _ = cpu_baseline(int(N), M, sigma, rtol, xi_c, med, args.cpu_cap_iters)
            per_mesh[int(N)] = float(np.mean(full))
            used_max = max(used_max, used)
        # the whole batch on `used` cores, one sample per core at a time
        t_cpu = sum(s * per_mesh[int(N)] for N in meshes) / used_max
        out["cpu_baseline"] = {
            "value": G * s / t_cpu, "unit": "samples/s", "cores": used_max, "kind": "oracle",
            "sample": (f"{nth} samples per mesh size, one per OpenMP thread, Jacobi-CG capped at "
                       f"{args.cpu_cap_iters} iterations and scaled to each mesh's median GPU FP64 iteration "
                       f"count; per-sample seconds {{N: s}} = "
                       f"{ {k: round(v, 2) for k, v in per_mesh.items()} }, summed over the 256 x s samples"),
            "seconds_measured": round(time.perf_counter() - t0, 2)}
    out.setdefault("env", host_env())
    print(json.dumps(out), flush=True)


def run_learned(args):
    """64^3 mesh, M=10, s=32: POD (r=32) of 2048 FP64 solves, a BF16-MFMA
    network trained on the device, and its prediction as the CG initial guess
    on 1024 held-out samples, against zero-guess CG on the same samples."""
    import numpy as np
    import torch

    from paper_1511_03703_amd import ens
    from paper_1511_03703_amd.learned import LearnedGuess
    import workloads as W

    w = W.LEARNED
    dev = "cuda"
    torch.cuda.set_device(0)
    s, M, rtol = w.s, w.M, w.rtol
    g = ens.graph_build(w.N)
    kl = ens.kl_build(w.N, M, w.L)
    n = g.n
    vals = torch.empty((g.nnz, s), dtype=torch.float64, device=dev)
    rhs = torch.empty((n, s), dtype=torch.float64, device=dev)
    x = torch.zeros((n, s), dtype=torch.float64, device=dev)
    train_xi = W.draw_xi(W.LEARNED_TRAIN_SEED, W.LEARNED_TRAIN, M)
    test_xi = W.draw_xi(W.LEARNED_TEST_SEED, W.LEARNED_TEST, M)
    phase = {}

    # training solves (the snapshots)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Sm = torch.empty((n, W.LEARNED_TRAIN), dtype=torch.float64, device=dev)
    snap_opts = ens.cg_opts(rtol=SNAPSHOT_RTOL, check_every=args.check_every)
    for j in range(W.LEARNED_TRAIN // s):
        xj = torch.as_tensor(train_xi[j * s:(j + 1) * s], device=dev)
        ens.assemble(g, kl, xj, M, w.sigma, values=vals, rhs=rhs)
        x.zero_()
        _, st, rc = ens.cg(g, vals, rhs, x=x, opts=snap_opts)
        assert rc == ens.ENS_OK, st
        ens.pod_collect(x, Sm, j * s)
    torch.cuda.synchronize()
    phase["training_solves_s"] = round(time.perf_counter() - t0, 3)
    log(f"{W.LEARNED_TRAIN} training solves in {phase['training_solves_s']} s")

    lg = LearnedGuess(r=32, device=dev)
    t0 = time.perf_counter()
    T = lg.fit_basis(Sm, eig_seed=W.LEARNED_INIT_SEED)
    torch.cuda.synchronize()
    phase["pod_s"] = round(time.perf_counter() - t0, 3)
    lam = lg.lam.cpu().numpy()
    del Sm
    X32 = torch.as_tensor(train_xi.astype(np.float32), device=dev)
    t0 = time.perf_counter()
    loss = lg.fit_network(X32, T, steps=args.train_steps, init_seed=W.LEARNED_INIT_SEED,
                          order_seed=W.LEARNED_INIT_SEED + 1, lr=args.train_lr, halvings=args.lr_halvings)
    torch.cuda.synchronize()
    phase["train_s"] = round(time.perf_counter() - t0, 3)
    ln = loss.cpu().numpy()
    log(f"POD {phase['pod_s']} s, training {args.train_steps} steps {phase['train_s']} s, loss "
        f"{ln[:10].mean():.3e} -> {ln[-50:].mean():.3e}")

    # held-out evaluation: zero guess vs learned guess, assembly included in both
    opts = ens.cg_opts(rtol=rtol, check_every=args.check_every)
    ws = torch.empty(ens.cg_workspace_bytes(g, s, opts), dtype=torch.uint8, device=dev)
    xz = torch.zeros_like(x)
    xl = torch.zeros_like(x)
    chunks = W.LEARNED_TEST // s
    test_dev = torch.as_tensor(test_xi, device=dev)
    test32 = torch.as_tensor(test_xi.astype(np.float32), device=dev)
    it_zero, it_learn, err_guess, diff_final, res_learn, pod_floor = [], [], [], [], [], []
    Phi_h = lg.Phi.cpu().numpy()

    def eval_pass(collect):
        t_z = t_l = 0.0
        for j in range(chunks):
            xj = test_dev[j * s:(j + 1) * s]
            torch.cuda.synchronize()
            ta = time.perf_counter()
            ens.assemble(g, kl, xj, M, w.sigma, values=vals, rhs=rhs)
            xz.zero_()
            _, stz, rcz = ens.cg(g, vals, rhs, x=xz, opts=opts, workspace=ws)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            ens.assemble(g, kl, xj, M, w.sigma, values=vals, rhs=rhs)
            lg.guess(test32[j * s:(j + 1) * s], x0=xl)
            if collect:
                g0 = xl.cpu().numpy()
            _, stl, rcl = ens.cg(g, vals, rhs, x=xl, opts=opts, workspace=ws)
            torch.cuda.synchronize()
            tc = time.perf_counter()
            t_z += tb - ta
            t_l += tc - tb
            if collect:
                assert rcz == ens.ENS_OK and rcl == ens.ENS_OK
                a, b = xz.cpu().numpy(), xl.cpu().numpy()
                for e in range(s):
                    nz = np.linalg.norm(a[:, e])
                    it_zero.append(stz[e]["iters"])
                    it_learn.append(stl[e]["iters"])
                    err_guess.append(float(np.linalg.norm(g0[:, e] - a[:, e]) / nz))
                    diff_final.append(float(np.linalg.norm(b[:, e] - a[:, e]) / nz))
                    res_learn.append(stl[e]["rel_res"])
                    pod_floor.append(float(np.linalg.norm(a[:, e] - Phi_h @ (Phi_h.T @ a[:, e])) / nz))
        return t_z, t_l

    eval_pass(collect=True)  # untimed: per-sample iterations and errors
    # the best guess the basis holds, Phi Phi^T x* of the zero-guess solution:
    # the bound on what any predictor of the POD coefficients can save
    it_pod = []
    zero_mu = torch.zeros(lg.r, dtype=torch.float64, device=dev)
    one_sd = torch.ones(lg.r, dtype=torch.float64, device=dev)
    for j in range(chunks):
        xj = test_dev[j * s:(j + 1) * s]
        ens.assemble(g, kl, xj, M, w.sigma, values=vals, rhs=rhs)
        xz.zero_()
        ens.cg(g, vals, rhs, x=xz, opts=opts, workspace=ws)
        C = ens.pod_project(lg.Phi, xz)
        ens.pod_reconstruct(lg.Phi, C.float().contiguous(), zero_mu, one_sd, x0=xl)
        _, stp, _ = ens.cg(g, vals, rhs, x=xl, opts=opts, workspace=ws)
        it_pod += [t_["iters"] for t_ in stp]
    for _ in range(args.warmup):
        eval_pass(collect=False)
    ens.prof_reset()
    ens.prof_enable(True)
    gc.collect()
    gc.disable()
    t_zero = t_learn = 0.0
    for _ in range(args.steps):
        tz, tl = eval_pass(collect=False)
        t_zero += tz
        t_learn += tl
    gc.enable()
    ens.prof_enable(False)
    pq = ens.prof_query(ens.K_SPMV_F64)
    nt = W.LEARNED_TEST * args.steps
    value = nt / t_learn
    per_launch = spmv_bytes(n, g.nnz, s, 8.0)
    avg_ms = pq["total_ms"] / max(pq["launches"], 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    saved = np.array(it_zero) - np.array(it_learn)
    out = {
        "metric": "solved samples/s at 64^3, s=32, 1e-8 resid, learned initial guess",
        "value": round(value, 3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_learn / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (network bf16/f32)", "data": "synthetic",
        "config": {"workload": w.name, "mesh": f"{w.N}^3 Q1 hexahedra", "n": n, "nnz": g.nnz, "s": s, "M": M,
                   "sigma": w.sigma, "rtol": rtol, "train_solves": W.LEARNED_TRAIN, "held_out": W.LEARNED_TEST,
                   "pod_r": 32, "snapshot_rtol": SNAPSHOT_RTOL, "mlp": "10-256-256-32 GELU", "adam_steps": args.train_steps, "batch": 256,
                   "lr": args.train_lr, "lr_halvings": args.lr_halvings,
                   "targets": "POD coefficients centred, one common scale"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(f"k_cg_spmv_dot<double,{s}>"),
                     "kernel": f"k_cg_spmv_dot<double,{s}>", "bytes_per_launch": per_launch,
                     "avg_launch_ms": round(avg_ms, 5), "launches": pq["launches"]},
        "learned": {
            "zero_guess_samples_per_s": round(nt / t_zero, 3),
            "speedup": round(t_zero / t_learn, 3),
            "iters_zero": {"mean": float(np.mean(it_zero)), "median": float(np.median(it_zero))},
            "iters_learned": {"mean": float(np.mean(it_learn)), "median": float(np.median(it_learn))},
            "iters_pod_projected": {"mean": float(np.mean(it_pod)), "median": float(np.median(it_pod)),
                                    "note": "CG from Phi Phi^T x* (FP32 coefficients): the bound for the basis"},
            "iters_saved": {"mean": float(saved.mean()), "median": float(np.median(saved)),
                            "min": int(saved.min()), "max": int(saved.max())},
            "initial_guess_rel_error": {"median": float(np.median(err_guess)), "max": float(max(err_guess))},
            "pod_floor_rel_error": {"median": float(np.median(pod_floor)), "max": float(max(pod_floor))},
            "final_rel_diff_vs_zero_guess": {"median": float(np.median(diff_final)),
                                             "max": float(max(diff_final))},
            "max_rel_res": float(max(res_learn)),
            "pod_eigenvalues": [float(v) for v in lam[:4]] + [float(lam[-1])],
            "train_loss_first_last": [float(ln[:10].mean()), float(ln[-50:].mean())],
            "phases_s": phase,
        },
    }
    if not args.no_cpu_baseline:
        log("CPU oracle baseline ...")
        t0 = time.perf_counter()
        threads = min(oracle_threads(args.cpu_threads), s)
        v, used, _, t_set, t_cg = cpu_baseline(w.N, M, w.sigma, rtol, test_xi[:threads], it_zero[:threads],
                                               args.cpu_cap_iters, w.L, w.kappa0, w.f)
        out["cpu_baseline"] = {
            "value": v, "unit": "samples/s", "cores": used, "kind": "oracle",
            "sample": (f"{threads} held-out samples, zero-guess FP64 Jacobi-CG (the oracle has no learned guess), "
                       f"one per OpenMP thread; set-up {t_set:.1f} s, CG capped at {args.cpu_cap_iters} "
                       f"iterations ({t_cg:.1f} s), scaled to the GPU zero-guess iteration counts"),
            "seconds_measured": round(time.perf_counter() - t0, 2)}
    out.setdefault("env", host_env())
    print(json.dumps(out), flush=True)


def run_mg(args):
    """The headline samples (128^3, s = 32, M = 10, sigma = 0.3) solved in
    FP64 to 1e-8 by CG preconditioned with the ensemble multigrid V-cycle.
    One step = FP64 assembly + hierarchy set-up + the solve."""
    import numpy as np
    import torch

    from paper_1511_03703_amd import ens
    import workloads as W

    w = W.HEADLINE
    dev = "cuda"
    torch.cuda.set_device(0)
    g = ens.graph_build(w.N)
    kl = ens.kl_build(w.N, w.M, w.L)
    xi = torch.as_tensor(w.xi(), device=dev)
    mixed = not args.mg_fp64
    vals = torch.empty((w.nnz, w.s), dtype=torch.float64, device=dev)
    v32 = torch.empty((w.nnz, w.s), dtype=torch.float32, device=dev) if mixed else None
    rhs = torch.empty((w.n, w.s), dtype=torch.float64, device=dev)
    x = torch.zeros((w.n, w.s), dtype=torch.float64, device=dev)
    mg = ens.Multigrid(w.N, w.M, w.s, fp32=mixed, L=w.L, device=dev)
    # a handful of iterations: poll every 4 so few launches run after convergence
    check = min(args.check_every, 4)
    inner = args.inner_rtol if args.inner_rtol is not None else 1e-4
    opts = ens.cg_opts(rtol=w.rtol, check_every=check, mixed=mixed, inner_rtol=inner)
    ws = torch.empty(ens.cg_workspace_bytes(g, w.s, opts), dtype=torch.uint8, device=dev)
    log(f"mg workload: N={w.N} s={w.s} hierarchy {mg.buffer.numel() / 2**30:.2f} GiB")

    def step():
        mg.assemble_setup(g, kl, xi, w.sigma, vals, rhs, values32=v32, kappa0=w.kappa0, f=w.f,
                          galerkin=args.coarse == "galerkin")
        x.zero_()
        return ens.cg_mg(g, vals, rhs, mg, x=x, values32=v32, opts=opts, workspace=ws)

    ens.prof_enable(True)
    gc.collect()
    gc.disable()
    for i in range(args.warmup):
        _, stats, st = step()
        log(f"warmup {i}: status {st}, iters {[t['iters'] for t in stats][:8]}...")
    torch.cuda.synchronize()
    ens.prof_reset()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, stats, st = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gc.enable()
    ens.prof_enable(False)
    pr = ens.prof_query(ens.K_MG_ROW)
    ps = ens.prof_query(ens.K_SPMV_F32 if mixed else ens.K_SPMV_F64)
    ok = all(t["status"] == 0 and t["rel_res"] <= w.rtol * (1 + 1e-6) for t in stats)
    achieved = pr["bytes"] / (pr["total_ms"] * 1e-3) / 1e9 if pr["launches"] else 0.0
    out = {
        "metric": ("solved samples/s at 128^3, s=32, 1e-8 resid, multigrid-preconditioned "
                   + ("FP32 CG inside FP64 refinement" if mixed else "FP64 CG")),
        "value": round(args.steps * w.s / elapsed, 3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32-in-f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": "q1_128cube_s32_mg_mixed" if mixed else "q1_128cube_s32_mg_fp64", "mesh": f"{w.N}^3 Q1 hexahedra", "n": w.n, "nnz": w.nnz,
                   "s": w.s, "M": w.M, "sigma": w.sigma, "rtol": w.rtol, "seed": w.seed,
                   "levels": "128,64,32,16,8,4", "smoother": "Chebyshev order 2 on [lmax/4, lmax]",
                   "coarse": "dense inverse of the 4^3 interior block", "check_every": check,
                   "coarse_operators": {"redisc": "assembled on each mesh", "galerkin": "Galerkin P^T A P"}[
                       args.coarse],
                   "inner_rtol": inner if mixed else None},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_mg_row<32,*> (fine-level Chebyshev and residual passes)",
                     "launches": pr["launches"],
                     "avg_launch_ms": round(pr["total_ms"] / max(pr["launches"], 1), 5),
                     "bytes_per_launch": round(pr["bytes"] / max(pr["launches"], 1))},
        "all_converged": bool(ok),
        "iters": [t["iters"] for t in stats],
        "outer_iters": [t["outer_iters"] for t in stats],
        "cg_spmv_GBs": round(ps["bytes"] / (ps["total_ms"] * 1e-3) / 1e9, 1) if ps["launches"] else None,
    }
    if not args.no_context:
        xs = x.clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x.zero_()
        _, stj, _ = ens.cg(g, vals, rhs, x=x, opts=ens.cg_opts(rtol=w.rtol, check_every=args.check_every))
        torch.cuda.synchronize()
        tj = time.perf_counter() - t1
        # per-sample error against an FP64 multigrid solve to 1e-12
        mg64 = ens.Multigrid(w.N, w.M, w.s, L=w.L, device=dev).setup(g, vals, xi, w.sigma, kappa0=w.kappa0, f=w.f)
        xr = torch.zeros_like(x)
        ens.cg_mg(g, vals, rhs, mg64, x=xr, opts=ens.cg_opts(rtol=1e-12, check_every=4), workspace=None)
        a, r_ = xs.cpu().numpy(), xr.cpu().numpy()
        err = [float(np.linalg.norm(a[:, e] - r_[:, e]) / np.linalg.norm(r_[:, e])) for e in range(w.s)]
        del mg64, xr
        out["context"] = {"jacobi_fp64_ensemble_cg": {"seconds_solve_only": round(tj, 4),
                                                      "iters_max": max(t["iters"] for t in stj)},
                          "per_sample_error_vs_fp64": {"max": max(err), "median": float(np.median(err)),
                                                       "reference": "GPU FP64 multigrid CG to 1e-12"}}
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        threads = min(oracle_threads(args.cpu_threads), w.s)
        log("CPU oracle baseline (multigrid PCG) ...")
        t0 = time.perf_counter()
        _, it, rr, st_o, _ = orc.ens_mg_pcg(w.N, w.M, w.L, w.kappa0, w.sigma, w.f, w.xi()[:threads], rtol=w.rtol)
        tc = time.perf_counter() - t0
        cores = min(threads, orc.max_threads())
        out["cpu_baseline"] = {
            "value": threads / tc, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": (f"{threads} samples of the same workload, one per OpenMP thread (of {orc.max_threads()} "
                       f"available): hierarchy set-up and multigrid PCG to {w.rtol:g} in full, "
                       f"iterations {[int(v) for v in it]}"),
            "seconds_measured": round(tc, 2)}
    out.setdefault("env", host_env())
    print(json.dumps(out), flush=True)


def assembly_bytes(n, nnz, s, fp64=True, fp32=True, rhs=True, dinv32=False):
    """Algorithmic bytes written by one ensemble assembly: the [nnz][s]
    values (FP64 and / or FP32), the [n][s] load vector, an FP32 D^-1 of a
    fused multigrid set-up; the inputs (KL table, y, row offsets) are
    negligible."""
    return nnz * s * (8.0 * fp64 + 4.0 * fp32) + n * s * (8.0 * rhs + 4.0 * dinv32)


def write_ceiling(buf):
    """Write-only stream rate (GB/s) over the buffer: 2 untimed passes, 5
    timed ones."""
    import torch

    from paper_1511_03703_amd import ens
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        ens.stream_write(buf, 1)
    e0.record()
    for _ in range(5):
        ens.stream_write(buf, 2)
    e1.record()
    torch.cuda.synchronize()
    return buf.numel() * buf.element_size() / (e0.elapsed_time(e1) / 5) / 1e6


def run_assembly(args):
    """The two assembly kernels at the headline size (128^3, s = 32, the
    headline samples), each timed alone: the linear ensemble assembly of A
    (FP64 and FP32 copy) and f (ens_assemble, Alg. assembly), and the
    nonlinear residual with the FP32 Jacobian (ens_nl_assemble, as each
    Newton step of the newton workload forms them) at a seeded state u."""
    import numpy as np
    import torch

    from paper_1511_03703_amd import ens
    import workloads as W

    w = W.HEADLINE
    dev = "cuda"
    torch.cuda.set_device(0)
    g = ens.graph_build(w.N)
    kl = ens.kl_build(w.N, w.M, w.L)
    xi = torch.as_tensor(w.xi(), device=dev)
    vals = torch.empty((w.nnz, w.s), dtype=torch.float64, device=dev)
    v32 = torch.empty((w.nnz, w.s), dtype=torch.float32, device=dev)
    rhs = torch.empty((w.n, w.s), dtype=torch.float64, device=dev)
    prob = ens.nl_problem(w.M, w.sigma, W.NEWTON_ALPHA, W.NEWTON_BETA, W.NEWTON_VEL, L=w.L, kappa0=w.kappa0, f=w.f)
    u = torch.as_tensor(W.draw_vector(1090, (w.n, w.s), 0.0, 0.05), device=dev)
    F = torch.empty((w.n, w.s), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    calibration_copy(args)

    def lin():
        ens.assemble(g, kl, xi, w.M, w.sigma, L=w.L, kappa0=w.kappa0, f=w.f, values=vals, values32=v32, rhs=rhs)

    def nonlin():
        ens.nl_assemble(g, kl, xi, prob, u, want_jac=False, want_jac32=True, values32=v32, F=F)

    out_k = {}
    for name, fn, kid in (("assemble", lin, ens.K_ASSEMBLE), ("nl_assemble", nonlin, ens.K_NL_ASSEMBLE)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ens.prof_enable(True)
        ens.prof_reset()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ens.prof_enable(False)
        pq = ens.prof_query(kid)
        avg_ms = pq["total_ms"] / max(pq["launches"], 1)
        by = pq["bytes"] / max(pq["launches"], 1)
        out_k[name] = {"ms_per_launch": round(avg_ms, 4), "launches": pq["launches"],
                       "bytes_per_launch": round(by), "GBs": round(by / (avg_ms * 1e-3) / 1e9, 1),
                       "wall_ms_per_step": round(el / args.steps * 1e3, 3)}
        log(f"{name}: {avg_ms:.3f} ms per launch, {by / (avg_ms * 1e-3) / 1e9:.1f} GB/s")
    a = out_k["assemble"]
    out = {
        "metric": "ensemble Q1 assembly of A (FP64 + FP32 copy) and f at 128^3, s=32: assembled samples/s",
        "value": round(w.s / (a["ms_per_launch"] * 1e-3), 3), "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": a["ms_per_launch"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "q1_128cube_s32_assembly", "mesh": f"{w.N}^3 Q1 hexahedra", "n": w.n, "nnz": w.nnz,
                   "s": w.s, "M": w.M, "sigma": w.sigma, "seed": w.seed,
                   "nl": {"alpha": W.NEWTON_ALPHA, "beta": W.NEWTON_BETA, "u": "U[0, 0.05] seed 1090",
                          "jacobian": "FP32"}},
        "roofline": {"bound": "hbm", "achieved": a["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(a["GBs"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_assemble_tile<32,0,false>", "bytes_per_launch": a["bytes_per_launch"],
                     "avg_launch_ms": a["ms_per_launch"], "launches": a["launches"]},
        "kernels": out_k,
    }
    del vals, v32, rhs, u, F
    wb = torch.empty((4 << 30) // 8, dtype=torch.float64, device=dev)
    wgbs = write_ceiling(wb)
    del wb
    out["context"] = {"write_GBs": round(wgbs, 1),
                      "assemble_floor_ms_at_write_ceiling": round(a["bytes_per_launch"] / (wgbs * 1e6), 4),
                      "assemble_frac_of_write_ceiling": round(a["GBs"] / wgbs, 4)}
    log(f"write ceiling {wgbs:.1f} GB/s: assembly at {a['GBs'] / wgbs:.3f} of it")
    out.setdefault("env", host_env())
    print(json.dumps(out), flush=True)


def run_coupled(args):
    """The coupled ensemble CG (one alpha, beta and stopping test for the
    whole commuted system, as the paper's solver runs it) against the
    per-sample ensemble CG on the headline samples (128^3, s = 32, FP64
    Jacobi-CG to 1e-8) as sigma rises: the coupled iteration count follows
    the union of the samples' spectra (Sec. 3.7), the per-sample one the
    slowest sample.  One step = both solves at every sigma."""
    import numpy as np
    import torch

    from paper_1511_03703_amd import ens
    import workloads as W

    w = W.HEADLINE
    dev = "cuda"
    torch.cuda.set_device(0)
    g = ens.graph_build(w.N)
    kl = ens.kl_build(w.N, w.M, w.L)
    xi = torch.as_tensor(w.xi(), device=dev)
    vals = torch.empty((w.nnz, w.s), dtype=torch.float64, device=dev)
    rhs = torch.empty((w.n, w.s), dtype=torch.float64, device=dev)
    x = torch.zeros((w.n, w.s), dtype=torch.float64, device=dev)
    ws = torch.empty(ens.cg_workspace_bytes(g, w.s, ens.cg_opts()), dtype=torch.uint8, device=dev)
    sigmas = (0.0, 0.1, 0.2, 0.3)  # sigma = 0: identical samples, where the two solves coincide
    rows = []
    total_s, total_t = 0, 0.0
    for sigma in sigmas:
        ens.assemble(g, kl, xi, w.M, sigma, L=w.L, kappa0=w.kappa0, f=w.f, values=vals, rhs=rhs)
        res = {"sigma": sigma}
        for name, coupled in (("per_sample", False), ("coupled", True)):
            opts = ens.cg_opts(rtol=w.rtol, check_every=args.check_every, coupled=coupled)
            best = None
            for rep in range(args.warmup + args.steps):
                x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st, rc = ens.cg(g, vals, rhs, x=x, opts=opts, workspace=ws)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                if rep >= args.warmup:
                    best = t if best is None else min(best, t)
            its = [t_["iters"] for t_ in st]
            # the coupled solve stops on the ensemble's residual, so single
            # samples may end a little above rtol: their largest is reported
            res[name] = {"iters_max": max(its), "iters_min": min(its), "seconds": round(best, 4),
                         "samples_per_s": round(w.s / best, 3),
                         "all_converged": all(t_["status"] == 0 for t_ in st),
                         "max_sample_rel_res": max(t_["rel_res"] for t_ in st)}
            if coupled:
                total_s += w.s
                total_t += best
        res["coupled_over_slowest_sample"] = round(res["coupled"]["iters_max"] / res["per_sample"]["iters_max"], 3)
        rows.append(res)
        log(f"sigma {sigma}: per-sample {res['per_sample']['iters_min']}-{res['per_sample']['iters_max']} iterations "
            f"({res['per_sample']['seconds']} s), coupled {res['coupled']['iters_max']} ({res['coupled']['seconds']} s)")
    out = {
        "metric": "solved samples/s at 128^3, s=32, 1e-8: coupled ensemble CG (the paper's solve), sigma 0-0.3",
        "value": round(total_s / total_t, 3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total_t / len(sigmas) * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "q1_128cube_s32_coupled_sweep", "mesh": f"{w.N}^3 Q1 hexahedra", "n": w.n,
                   "nnz": w.nnz, "s": w.s, "M": w.M, "sigmas": list(sigmas), "rtol": w.rtol, "seed": w.seed,
                   "preconditioner": "Jacobi", "check_every": args.check_every},
        "sweep": rows,
    }
    out.setdefault("env", host_env())
    print(json.dumps(out), flush=True)


def run_newton(args):
    """The nonlinear problem (advection alpha v.grad u and reaction beta u^2
    on) for the headline samples: one step = the diffusion matrix for the
    preconditioner, the multigrid set-up, and Newton's method with
    multigrid-preconditioned GMRES from u = 0 to |F(u)| <= 1e-8 |load|."""
    import numpy as np
    import torch

    from paper_1511_03703_amd import ens
    import workloads as W

    w = W.NEWTON
    dev = "cuda"
    torch.cuda.set_device(0)
    g = ens.graph_build(w.N)
    kl = ens.kl_build(w.N, w.M, w.L)
    xi = torch.as_tensor(w.xi(), device=dev)
    prob = ens.nl_problem(w.M, w.sigma, W.NEWTON_ALPHA, W.NEWTON_BETA, W.NEWTON_VEL, L=w.L, kappa0=w.kappa0, f=w.f)
    mg32 = not args.mg_fp64
    # an FP32 hierarchy needs no FP64 fine matrix: it is not formed
    K = None if mg32 else torch.empty((w.nnz, w.s), dtype=torch.float64, device=dev)
    K32 = torch.empty((w.nnz, w.s), dtype=torch.float32, device=dev) if mg32 else None
    rhs = torch.empty((w.n, w.s), dtype=torch.float64, device=dev)
    u = torch.zeros((w.n, w.s), dtype=torch.float64, device=dev)
    mg = ens.Multigrid(w.N, w.M, w.s, fp32=mg32, L=w.L, device=dev)
    ew = args.forcing == "ew"
    lin_rtol = args.lin_rtol if args.lin_rtol is not None else (W.NEWTON_ETA_MAX if ew else W.NEWTON_LIN_RTOL)
    jac32 = not args.jac_fp64
    opts = ens.newton_opts(rtol=w.rtol, lin_rtol=lin_rtol, restart=W.NEWTON_RESTART, jac32=jac32,
                           forcing=ens.FORCING_EW if ew else ens.FORCING_FIXED)
    ws = torch.empty(ens.newton_workspace_bytes(g, w.s, opts), dtype=torch.uint8, device=dev)
    log(f"newton workload: N={w.N} s={w.s} workspace {ws.numel() / 2**30:.1f} GiB, "
        f"hierarchy {mg.buffer.numel() / 2**30:.2f} GiB")

    adv = args.newton_mg == "adv"

    def step():
        if adv:
            mg.assemble_setup_adv(g, kl, xi, prob, K, rhs, values32=K32)
        else:
            mg.assemble_setup(g, kl, xi, w.sigma, K, rhs, values32=K32, kappa0=w.kappa0, f=w.f)
        u.zero_()
        return ens.newton(g, kl, xi, prob, u=u, opts=opts, mg=mg, mg_values=K32 if mg32 else K, workspace=ws)

    ens.prof_enable(True)
    gc.collect()
    gc.disable()
    for i in range(args.warmup):
        _, stats, st = step()
        log(f"warmup {i}: status {st}, newton {[t['newton_iters'] for t in stats][:8]}..., "
            f"gmres {[t['lin_iters'] for t in stats][:8]}...")
    torch.cuda.synchronize()
    ens.prof_reset()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, stats, st = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gc.enable()
    ens.prof_enable(False)
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    kernels = {f"k_mg_row<{'float' if mg32 else 'double'},32,*> (fine-level V-cycle passes)": ens.K_MG_ROW,
               "k_nl_assemble<32,8,*> (residual and Jacobian)": ens.K_NL_ASSEMBLE,
               "k_gm_spmv<32> (GMRES product w = A z)": ens.K_GM_SPMV,
               "k_gm_dots/k_gm_axpy<32> (Gram-Schmidt passes)": ens.K_GM_ORTH,
               "k_assemble_tile<32,*,true> (the preconditioner's matrices, every level)": ens.K_ASSEMBLE}
    prof = {k: ens.prof_query(v) for k, v in kernels.items()}
    per_kernel = {k: {"ms_per_step": round(p["total_ms"] / args.steps, 3), "launches": p["launches"],
                      "GBs": round(p["bytes"] / (p["total_ms"] * 1e-3) / 1e9, 1) if p["launches"] else None}
                  for k, p in prof.items()}
    dom = max((k for k in prof if k.startswith(("k_mg_row", "k_gm_spmv", "k_gm_dots"))),
              key=lambda k: prof[k]["total_ms"])
    pd = prof[dom]
    achieved = pd["bytes"] / (pd["total_ms"] * 1e-3) / 1e9 if pd["launches"] else 0.0
    ok = all(t["status"] == 0 and t["rel_res"] <= w.rtol * (1 + 1e-6) for t in stats)
    out = {
        "metric": "solved samples/s at 128^3, s=32: nonlinear (alpha=10, beta=100) Newton to 1e-8 residual",
        "value": round(args.steps * w.s / elapsed, 3), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "mesh": f"{w.N}^3 Q1 hexahedra", "n": w.n, "nnz": w.nnz, "s": w.s, "M": w.M,
                   "sigma": w.sigma, "alpha": W.NEWTON_ALPHA, "beta": W.NEWTON_BETA,
                   "velocity": [round(v, 6) for v in W.NEWTON_VEL], "f": w.f, "rtol": w.rtol, "seed": w.seed,
                   "linear_solver": f"GMRES({W.NEWTON_RESTART}) to "
                                    + (f"Eisenstat-Walker forcing terms (eta_max {lin_rtol:g})" if ew
                                       else f"{lin_rtol:g}") + ", right-preconditioned by "
                                    + ("the multigrid V-cycle of the advection-diffusion operator D + alpha C "
                                       "(every level rediscretized)" if adv
                                       else "the multigrid V-cycle of the diffusion operator")
                                    + (" in FP32" if mg32 else " in FP64")
                                    + ("; Jacobian stored in FP32" if jac32 else "; Jacobian in FP64")},
        # the fine-level FP32 cycle passes are the same launches (kernel,
        # mesh, ensemble size) as in the headline step, whose HBM counters
        # are on record
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic("k_mg_row<float,32,*>") if dom.startswith("k_mg_row<float,32") else None,
                     "kernel": dom,
                     "launches": pd["launches"], "avg_launch_ms": round(pd["total_ms"] / max(pd["launches"], 1), 5),
                     "bytes_per_launch": round(pd["bytes"] / max(pd["launches"], 1))},
        "all_converged": bool(ok),
        "newton_iters": [t["newton_iters"] for t in stats],
        "gmres_iters": [t["lin_iters"] for t in stats],
        "kernels": per_kernel,
    }
    if not args.no_cpu_baseline:
        # A full oracle solve takes about 90 s per sample at 128^3, so the
        # bounded sample is the first Newton step (hierarchy, residual and
        # Jacobian, GMRES, update, and the next residual) of `threads`
        # samples, scaled by the Newton steps the samples take.
        from oracle import oracle as orc
        threads = min(oracle_threads(args.cpu_threads), w.s)
        log("CPU oracle baseline (first Newton step) ...")
        t0 = time.perf_counter()
        _, ni, li, rr, st_o, _ = orc.ens_newton(w.N, w.M, w.L, w.kappa0, w.sigma, w.f, W.NEWTON_ALPHA,
                                                np.array(W.NEWTON_VEL), W.NEWTON_BETA, w.xi()[:threads],
                                                prec=orc.PREC_MG_ADV if adv else orc.PREC_MG, rtol=w.rtol,
                                                max_newton=1, lin_rtol=lin_rtol,
                                                restart=W.NEWTON_RESTART,
                                                forcing=orc.FORCING_EW if ew else orc.FORCING_FIXED)
        tc = time.perf_counter() - t0
        steps_full = float(np.mean([t["newton_iters"] for t in stats[:threads]]))
        cores = min(threads, orc.max_threads())
        out["cpu_baseline"] = {
            "value": threads / (tc * steps_full), "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": (f"the first Newton step of {threads} samples of the same workload (one per OpenMP thread: "
                       f"the oracle's hierarchy, residual and Jacobian, multigrid-preconditioned GMRES(30) to "
                       f"{lin_rtol:g} with {[int(v) for v in li]} iterations, update, next residual) in "
                       f"{tc:.1f} s, scaled by the {steps_full:g} Newton steps these samples take"
                       + (" (an overestimate of the oracle's speed: later steps solve to tighter tolerances)"
                          if ew else "")),
            "seconds_measured": round(tc, 2)}
    out.setdefault("env", host_env())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
