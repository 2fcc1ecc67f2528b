"""Throughput benchmark of the semi-Lagrangian Monte-Carlo step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c3|c2|c1]
                [--precision fp64|fp32_refine|bf16split_refine] [--no-cpu-baseline]
                [--schedule perorder|fused|perorder_graph|fused_graph|auto]
python bench.py --serve [--serve-requests R] [--serve-rate HZ] [--serve-kmax K] [--serve-mmax M]

One "step" is one pass of the whole hot path (Wiener increments, node moves,
advected fits, trace exchange, constrained remap) over every sample of the
workload.  The timed region holds exactly K steps with the samples resident
in HBM; the value is Monte-Carlo node-updates per second (elements x nodes x
samples x steps / seconds).  Prints one JSON line.

The default workload is the largest one that fits one GPU: the 2-D 128 x 128
mixed-order (N in {6, 8, 10}) solid-body rotation with 512 samples, float64.
Before the warm-up the same handle takes a few untimed check steps; samples
0..P-1 after them are compared with the float64 CPU oracle run over the same
steps (``l2_vs_oracle``), and the oracle's run time gives ``cpu_baseline``
(one host thread on one sample, and P worker processes side by side).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X = {"fp64_vector_tflops": 78.6, "fp64_mfma_tflops": 78.6, "fp32_mfma_tflops": 157.3,
          "bf16_mfma_tflops": 2500.0, "hbm_gbs": 8000.0}


def fit_flops_1d(N):
    """Float64 operations of one 1-D element fit and step in the nodal form the kernel
    runs (multiply-add = 2, division = 1): moves 3N, carried values N, node products
    for the barycentric weights 1.5N(N-1) (each difference once), their reciprocals
    2.5N (one reciprocal per four), the two edge Lagrange rows 12N - 4, traces and S 10N,
    multipliers 14, corrected and weighted values 5N, evaluation at the N Gauss nodes
    5N^2 - 5N (differences, then a Horner scheme over the prefix products)."""
    return (13 * N * N + 54 * N + 20) // 2

def fit_flops_2d_phase2(N):
    """Algorithmic float64 operations of one 2-D fit in the second (constrained) phase:
    Gram n^2 (n+1) (symmetric), right side 2n^2, Cholesky n^3/3, two solves 4n^2,
    C_r^T = C^T U_r 2 n T R, Y = L^-1 C_r^T n^2 R, S = Y^T Y n R (R+1), Cholesky of S R^3/3,
    multiplier solves 2R^2, Y lambda 2nR, L^-T solve 2n^2, evaluation at the nodes 2nN
    (sum-factorised)  --  n = N^2, T = 4N, R = 4N - 4."""
    n, T, R = N * N, 4 * N, 4 * N - 4
    return n * n * (n + 1) + 2 * n * n + n ** 3 / 3.0 + 4 * n * n + 2 * n * T * R + n * n * R \
        + n * R * (R + 1) + R ** 3 / 3.0 + 2 * R * R + 2 * n * R + 2 * n * n + 2 * n * N


def fit_flops_2d_ref(N, phase, iters, ncomp=1):
    """Float64 operations of one 2-D fit with the reference-preconditioned solver, as
    the kernels perform them (multiply-add = 2), for `iters` conjugate-gradient
    iterations:  n = N^2, T = 4N, m = N - 2 (bubble functions per direction).
    Phase 1 (Richardson iteration on V c = f, each iteration counted): moves and
      carried values 8n, 1-D tables 12 n N;  V0^-1 v (Kronecker): 4N^3 + 2n;
      residual f - V c: 2n(N^2 + N) + n;  traces 2T(N^2 + N); p0 at the Gauss
      nodes 2n(N^2 + N).
    Phase 2: moves 8n; bubble tables (Legendre recurrence of m terms, times
      x(1 - x)) 2(n + N)(5m + 4); the two 1-D Gram matrices 4 m^2 N + 12 N and
      their Gauss-Jordan inverses 4 m^3; jump data T, the jump projected through
      the four corner conditions 16N + 32 + 4T + 40 (eight end values, a 4 x 4
      solve, the correction, the corner values);
      transfinite lift at the moved nodes n(20N + 20) and at the Gauss nodes 14n;
      Vz p: 2n(m^2 + m);  Vz^T r: 2n m^2 + n m;  Kronecker preconditioner 4 m^3;
      evaluation 2n(m^2 + m) + 3n.
    With ncomp components the moves, tables and Gram inverses are done once per
    fit and the rest once per component."""
    n, T = N * N, 4 * N
    if phase == 1:
        geom = 8 * n + 12 * n * N
        v0 = 4 * N ** 3 + 2 * n
        per_it = 2 * n * (N * N + N) + n + v0
        out = 2 * T * (N * N + N) + 2 * n * (N * N + N)
        return geom + ncomp * (v0 + iters * per_it + out)
    m = N - 2
    geom = 8 * n + 2 * (n + N) * (5 * m + 4) + 4 * m * m * N + 12 * N + 4 * m ** 3 + 4 * N * m
    lift = T + (16 * N + 32 + 4 * T + 40) + n * (20 * N + 20) + 14 * n + 3 * n
    if m == 0:
        return geom + ncomp * (lift + 3 * n)
    zv = 2 * n * (m * m + m)
    zvt = 2 * n * m * m + n * m
    pinv = 4 * m ** 3
    start = zvt + pinv + zv + zvt + m * m + pinv + 4 * m * m
    per_it = zv + zvt + 2 * m * m + 4 * m * m + pinv + 4 * m * m + 2 * m * m
    return geom + ncomp * (lift + start + iters * per_it + zv + 3 * n)


SCHEDULES = {"perorder": (0, 0), "fused": (1, 0), "perorder_graph": (0, 1), "fused_graph": (1, 1)}


def kernel_name(wl, fused=0, solver=1):
    if wl.dim == 1:
        return "resident_1d"
    if fused:
        return "fit2d_fused_phase2"
    return "fit2r_phase2" if solver == 2 else "fit2d_phase2"


def kernel_sources_digest(wl):
    """Digest of the sources the dominant kernel is built from, comments and
    blank lines left out (a stored HBM traffic measurement is only valid for
    the kernel it was taken on; a comment does not change the kernel)."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2009_07340_amd", "csrc")
    names = ["sl_internal.hpp", "philox.hpp", "fit1d.hpp"]
    names += ["k1d.hip"] if wl.dim == 1 else ["k2d.hip", "k2r.hip", "blocks.hpp", "kshared.hip"]
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(csrc, n)) as f:
            for line in f:
                code = re.sub(r"//.*", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def stored_traffic(wl, kname, precision, ncomp=1):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), or
    None when none matches this kernel source, workload, precision and number
    of components."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    key = f"{kname}|{wl.name}|{precision}" + (f"|nc{ncomp}" if ncomp > 1 else "")
    e = table.get(key)
    if not e or e.get("source_digest") != kernel_sources_digest(wl):
        return None
    return e["hbm_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's step count, at most 20 in 2-D)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--check-steps", type=int, default=None,
                    help="untimed steps compared with the oracle before the warm-up (default 2 in 2-D, 20 in 1-D)")
    ap.add_argument("--check-samples", type=int, default=None,
                    help="samples compared with the oracle (default: one per worker process)")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--samples", type=int, default=None)
    ap.add_argument("--ncomp", type=int, default=1,
                    help="components of a vector-valued field sharing the moved points (node-updates count each)")
    ap.add_argument("--solver", default="auto", choices=["auto", "factor", "reference"],
                    help="2-D least-squares solver (auto: reference for fp64, factor for the mixed modes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--schedule", default="perorder", choices=list(SCHEDULES) + ["auto"],
                    help="2-D launch schedule (auto: the library's autotuner picks)")
    ap.add_argument("--path", default="general", choices=["general", "shared"],
                    help="2-D: the general path, or the shared-geometry path (constant u and D, one order; "
                         "reported on its own, never as the general path's figure)")
    ap.add_argument("--serve", action="store_true", help="run the serving stream instead")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-kmax", type=int, default=64)
    ap.add_argument("--serve-mmax", type=int, default=128)
    ap.add_argument("--serve-steps-scale", type=float, default=1.0)
    ap.add_argument("--serve-max-active", type=int, default=32)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by samples, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    from paper_2009_07340_amd import workloads as W

    if args.serve:
        return serve_bench(args)
    wl = W.WORKLOADS[args.workload]()
    if args.samples:
        wl.samples = args.samples
    steps = args.steps if args.steps is not None else (min(wl.steps, 20) if wl.dim == 2 else wl.steps)
    check_steps = args.check_steps if args.check_steps is not None else (2 if wl.dim == 2 else min(200, wl.steps))
    workers = cpu_share()
    per_worker = 1 if wl.dim == 2 else 8
    check_samples = min(wl.samples, args.check_samples or workers * per_worker)
    # The oracle leg runs first, in worker processes started before this
    # process touches the GPU: the check samples over the check steps, and
    # the timings of the CPU baseline.
    oracle = None
    if not args.no_cpu_baseline and check_steps > 0:
        oracle = oracle_leg(args.workload, wl.samples, check_samples, check_steps, workers, per_worker)
    # the GPU library (and torch's HIP runtime) only from here on
    import torch
    from paper_2009_07340_amd import binding as B
    from paper_2009_07340_amd.problem import Problem
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    nbytes = Problem.required_bytes(wl, args.precision, solver=args.solver, ncomp=args.ncomp)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)       # device memory from torch
    prob = Problem(wl, precision=args.precision, dev_ws=ws.data_ptr(), ws_bytes=nbytes,
                   hip_stream=stream.cuda_stream, solver=args.solver, ncomp=args.ncomp)
    prob.set_fields()
    fused = 0
    if wl.dim == 2 and args.path == "shared":
        B.sl_set_schedule(prob.h, 0, 0, 0, 1)
    elif wl.dim == 2:
        if args.schedule == "auto":
            sched = B.sl_autotune(prob.h, wl.dt, 1)
            print(f"[bench] autotuner: {sched}", file=sys.stderr, flush=True)
        else:
            B.sl_set_schedule(prob.h, *SCHEDULES[args.schedule], 0)
        fused = B.sl_get_schedule(prob.h)["fused"]
    solver = B.sl_diag(prob.h)["solver"]
    print(f"[bench] {wl.name}: K={wl.K} samples={wl.samples} dt={wl.dt} check={check_steps} warmup={args.warmup} "
          f"steps={steps}", file=sys.stderr, flush=True)
    l2 = None
    if check_steps > 0:
        prob.step(wl.dt, check_steps)             # untimed: compared with the oracle
        got = prob.samples(0, check_samples)[:, :prob.nodes]     # component 0 (the workload's own field)
        if oracle is not None:
            ref = oracle["ref"]
            dif = np.abs(got - ref)
            l2 = {"rel_l2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                  "max_abs_over_max_ref": float(dif.max() / np.abs(ref).max()),
                  "samples": check_samples, "steps": check_steps, "tol": 1e-11}
            l2["pass"] = bool(l2["rel_l2"] <= 1e-11 and l2["max_abs_over_max_ref"] <= 1e-11)
            print(f"[bench] vs oracle after {check_steps} steps on {check_samples} samples: rel L2 "
                  f"{l2['rel_l2']:.3e}, max|d|/max|ref| {l2['max_abs_over_max_ref']:.3e}", file=sys.stderr, flush=True)
    if args.warmup:
        prob.step(wl.dt, args.warmup)
    torch.cuda.synchronize()
    d0 = B.sl_diag(prob.h)
    B.sl_profile(prob.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.step(wl.dt, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kname = "shared_update" if args.path == "shared" else kernel_name(wl, fused, solver)
    launches, kms = B.sl_kernel_time(prob.h, kname)
    d1 = B.sl_diag(prob.h)
    others = {}
    for other in ("fit2d_phase1", "fit2d_phase2", "fit2r_phase1", "fit2r_phase2", "fit2d_fused_phase1",
                  "fit2d_fused_phase2", "resident_1d", "shared_build", "shared_traces", "shared_update"):
        if other != kname:
            n_o, ms_o = B.sl_kernel_time(prob.h, other)
            if n_o:
                others[other] = {"launches": n_o, "ms": round(ms_o, 4)}
    B.sl_profile(prob.h, False)
    sched_used = B.sl_get_schedule(prob.h) if wl.dim == 2 else None
    elapsed = t1 - t0
    nodes_per_sample = prob.nodes
    node_updates = float(nodes_per_sample) * wl.samples * args.ncomp * steps
    value = node_updates / elapsed
    mean = prob.mean()
    finite = bool(np.all(np.isfinite(mean)))
    print(f"[bench] timed {steps} steps in {elapsed * 1e3:.2f} ms; {kname}: {launches} launches {kms:.2f} ms; {others} "
          f"mean finite={finite} max|mean|={float(np.max(np.abs(mean))):.4g}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel
    if wl.dim == 1:
        N = int(wl.order)
        flops = fit_flops_1d(N) * wl.K * wl.samples * args.ncomp * steps
        achieved = flops / (kms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": MI355X["fp64_vector_tflops"],
                "unit": "TFLOP/s", "frac": round(achieved / MI355X["fp64_vector_tflops"], 4),
                "traffic": stored_traffic(wl, kname, args.precision, args.ncomp),
                "kernel": kname, "kernel_ms": round(kms, 4), "launches": launches,
                "flops_per_fit_step": round(fit_flops_1d(N), 1)}
    elif args.path == "shared":
        # dense float64 products on the matrix cores: per element-sample 2 n (n + T) for the update
        # (T = 4N edge points), and 2 T n for the traces (reported beside it)
        N = int(wl.order)
        n, T = N * N, 4 * N
        per_launch = 2.0 * n * (n + T) * wl.K * wl.samples * args.ncomp
        achieved = per_launch * launches / (kms * 1e-3) / 1e12
        n_t, ms_t = B.sl_kernel_time(prob.h, "shared_traces")
        n_b, ms_b = B.sl_kernel_time(prob.h, "shared_build")
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": MI355X["fp64_mfma_tflops"],
                "unit": "TFLOP/s", "frac": round(achieved / MI355X["fp64_mfma_tflops"], 4),
                "traffic": stored_traffic(wl, kname, "shared", args.ncomp),
                "kernel": kname, "kernel_ms": round(kms, 4), "launches": launches,
                "flops_per_launch": per_launch, "flops_per_element_sample": 2 * n * (n + T),
                "traces_kernel": {"ms": round(ms_t, 4), "launches": n_t,
                                  "tflops": round(2.0 * T * n * wl.K * wl.samples * args.ncomp * n_t / (ms_t * 1e-3) / 1e12, 3)
                                  if ms_t else None},
                "build_kernel_ms": round(ms_b, 4)}
    elif solver == 2:
        # float64 VALU work of the reference solver with the iteration counts of the
        # timed steps; the roofline is the one of the phase that takes longer
        fits = wl.K * wl.samples * args.ncomp * steps
        it2 = (d1["solver_iterations"][1] - d0["solver_iterations"][1]) / fits
        it1 = (d1["solver_iterations"][0] - d0["solver_iterations"][0]) / fits
        orders = wl.order_array()
        phases = {}
        for ph, it in ((1, it1), (2, it2)):
            name = f"fit2d_fused_phase{ph}" if fused else f"fit2r_phase{ph}"   # the persistent kernel's label
            n_l, ms_l = (launches, kms) if name == kname else B.sl_kernel_time(prob.h, name)
            pl = sum(fit_flops_2d_ref(int(N), ph, it, args.ncomp) for N in orders) * wl.samples
            phases[name] = {"launches": n_l, "ms": round(ms_l, 4), "flops_per_launch": pl,
                            "tflops": round(pl * n_l / (ms_l * 1e-3) / 1e12, 3) if ms_l else None}
        kname = max(phases, key=lambda k: phases[k]["ms"])
        launches, kms, per_launch = phases[kname]["launches"], phases[kname]["ms"], phases[kname]["flops_per_launch"]
        others = {k: v for k, v in others.items() if k != kname}
        for k, v in phases.items():
            if k != kname:
                others[k] = v
        achieved = per_launch * launches / (kms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": MI355X["fp64_vector_tflops"],
                "unit": "TFLOP/s", "frac": round(achieved / MI355X["fp64_vector_tflops"], 4),
                "traffic": stored_traffic(wl, kname, args.precision, args.ncomp),
                "kernel": kname, "kernel_ms": round(kms, 4), "launches": launches,
                "flops_per_launch": per_launch, "mean_iterations": [round(it1, 3), round(it2, 3)],
                "unconverged": [d1["solver_unconverged"][0] - d0["solver_unconverged"][0],
                                d1["solver_unconverged"][1] - d0["solver_unconverged"][1]],
                "other_kernels": others}
    else:
        orders = wl.order_array()
        per_launch = sum(fit_flops_2d_phase2(int(N)) for N in orders) * wl.samples * args.ncomp
        flops = per_launch * launches
        achieved = flops / (kms * 1e-3) / 1e12
        peak = MI355X["fp64_mfma_tflops"] if args.precision == "fp64" else MI355X["fp32_mfma_tflops"]
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": stored_traffic(wl, kname, args.precision, args.ncomp),
                "kernel": kname, "kernel_ms": round(kms, 4), "launches": launches,
                "flops_per_launch": per_launch, "other_kernels": others}

    if args.pmc_calibrate:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 1073741824 bytes read, 1073741824 written", file=sys.stderr, flush=True)

    cpu = oracle["cpu_baseline"] if oracle is not None else None
    prob.close()
    out = {
        "metric": "MC node-updates/s at fixed L2 error vs FP64 oracle",
        "value": value, "unit": "node-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else args.precision, "data": "synthetic",
        "config": {"workload": wl.name, "dim": wl.dim, "elements": wl.K, "order": int(wl.order) if np.isscalar(wl.order) else "mixed",
                   "samples": wl.samples, "dt": wl.dt, "dt_specified": wl.dt_specified, "precision": args.precision,
                   "fits_per_step": wl.K * wl.samples * args.ncomp, "nodes_per_sample": nodes_per_sample,
                   "ncomp": args.ncomp,
                   "element_sample_fits_per_s": wl.K * wl.samples * steps / elapsed},
        "roofline": roof,
        "cpu_baseline": cpu,
        "l2_vs_oracle": l2,
    }
    if wl.dim == 2:
        out["config"]["schedule"] = sched_used
        out["config"]["solver"] = "shared-geometry path" if args.path == "shared" else {1: "factor", 2: "reference"}[solver]
        out["config"]["path"] = args.path
    print(json.dumps(out), flush=True)


def serve_bench(args):
    """The serving stream (Poisson arrivals, mixed 1-D / 2-D requests) through the
    continuous-batching loop; one JSON line with p50/p99 latency and throughput."""
    import torch
    from paper_2009_07340_amd import binding as B
    from paper_2009_07340_amd import serve
    from paper_2009_07340_amd import workloads as W
    torch.cuda.set_device(0)
    stream = W.serving_requests(n=args.serve_requests, rate=args.serve_rate, kmax=args.serve_kmax,
                                mmax=args.serve_mmax)
    reqs = serve.requests_from_stream(stream, precision=args.precision, steps_scale=args.serve_steps_scale)
    s_batch, s_admit = torch.cuda.Stream(), torch.cuda.Stream()
    srv = serve.Server(B, max_active=args.serve_max_active, chunk_steps=16,
                       batch_stream=s_batch.cuda_stream, admit_stream=s_admit.cuda_stream)
    print(f"[serve] {len(reqs)} requests at {args.serve_rate}/s, K <= {args.serve_kmax}, M <= {args.serve_mmax}, "
          f"budget {srv.budget / 2**30:.1f} GiB", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    srv.run(reqs)
    wall = time.perf_counter() - t0
    st = serve.summarize(reqs)
    unsupported = sum(1 for r in reqs if r.error and "admission" in r.error)
    out = {
        "metric": "serving p50/p99 latency", "value": st["p99_latency_s"], "unit": "s",
        "higher_is_better": False, "n_gpus": 1,
        "dtype": "f64" if args.precision == "fp64" else f"{args.precision} (2-D), f64 (1-D)", "data": "synthetic",
        "p50_latency_s": st["p50_latency_s"], "p99_latency_s": st["p99_latency_s"],
        "p50_queue_wait_s": st["p50_queue_wait_s"], "arrival_rate_per_s": args.serve_rate,
        "completed": st["completed"], "failed": st["failed"], "unsupported_shapes": unsupported,
        "makespan_s": st["makespan_s"], "wall_s": wall, "node_updates_per_s": st["node_updates_per_s"],
        "sustained_completions_per_s": st["completed_per_s"], "peak_active": srv.peak_active,
        "iterations": srv.iterations, "peak_used_bytes": srv.peak_used,
        "config": {"workload": "serving stream", "requests": args.serve_requests, "rate": args.serve_rate,
                   "kmax": args.serve_kmax, "mmax": args.serve_mmax, "steps_scale": args.serve_steps_scale,
                   "max_active": args.serve_max_active, "chunk_steps": 16},
    }
    print(json.dumps(out), flush=True)


def cpu_share():
    """Worker processes for the oracle leg: the host cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_job(job):
    """One worker of the oracle leg: the float64 oracle, one host thread, on the
    given global samples of a workload for `steps` steps from its initial field.
    Returns (samples x nodes array, seconds)."""
    key, samples, steps = job
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import sl
    from paper_2009_07340_amd import workloads as W
    wl = W.WORKLOADS[key]()
    x0, x1, y0, y1 = wl.box
    mesh = sl.Mesh(dim=wl.dim, kx=wl.kx, ky=wl.ky, x0=x0, x1=x1, y0=y0, y1=y1, order=wl.order_array(), bc=wl.bc)
    ax = []
    for e in range(mesh.K):
        N = int(mesh.order[e])
        ax += [0, 0] if mesh.dim == 1 else [0] * (2 * N) + [1] * (2 * N)
    a = wl.sample_fields(mesh.node_coords(), mesh.edge_coords(), np.array(ax))
    f = sl.Fields(u=a["u"], D=a["D"], divu=a["divu"], un=a["un"], Dn=a["Dn"], ghost=a["ghost"])
    samples = np.asarray(samples, dtype=np.int64)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        phi = sl.run(mesh, f, a["phi0"], wl.dt, steps, wl.seed, samples)
        el = time.perf_counter() - t0
    return phi, el


def oracle_leg(key, total_samples, check_samples, check_steps, workers, per_worker):
    """The oracle on the host: reference values of samples 0..check_samples-1
    after check_steps steps, and the CPU baseline.

    One host thread: the first per_worker samples over one step (2-D) or the
    check steps (1-D), alone.  `workers` threads: one process per host core,
    each running per_worker of the check samples over the check steps at the
    same time; the rate is all their node-updates over the wall time."""
    import multiprocessing as mp
    import numpy as np
    from paper_2009_07340_amd import workloads as W
    wl = W.WORKLOADS[key]()
    jobs = [(key, list(range(s0, min(s0 + per_worker, check_samples))), check_steps)
            for s0 in range(0, check_samples, per_worker)]
    single_steps = 1 if wl.dim == 2 else check_steps
    ctx = mp.get_context("spawn")           # fresh interpreters: nothing of this process's runtime is inherited
    with ctx.Pool(processes=min(workers, len(jobs))) as pool:
        _, t_single = pool.apply(_oracle_job, ((key, list(range(per_worker)), single_steps),))
        t0 = time.perf_counter()
        out = pool.map(_oracle_job, jobs, chunksize=1)
        wall = time.perf_counter() - t0
    ref = np.concatenate([o[0] for o in out], axis=0)
    nodes = ref.shape[1]
    single = float(nodes) * per_worker * single_steps / t_single
    multi = float(nodes) * check_samples * check_steps / wall
    print(f"[bench] cpu oracle: 1 thread {per_worker} samples x {single_steps} steps in {t_single:.2f} s; "
          f"{len(jobs)} processes {check_samples} samples x {check_steps} steps in {wall:.2f} s",
          file=sys.stderr, flush=True)
    cpu = {"value": multi, "unit": "node-updates/s", "cores": min(workers, len(jobs)), "kind": "oracle",
           "sample": f"samples 0..{check_samples - 1} of {total_samples} x the first {check_steps} of "
                     f"{wl.steps} steps, all {wl.K} elements, one sample group per process (samples are "
                     f"independent, so the rate scales to the full run)",
           "single_thread": {"value": single, "cores": 1,
                             "sample": f"{per_worker} sample(s) x {single_steps} step(s), one process alone"}}
    return {"ref": ref, "cpu_baseline": cpu}


if __name__ == "__main__":
    main()
