#!/usr/bin/env python
"""Benchmark of the IBSN hot path on one MI355X.

Workload: m = n = 10^4 points uniform in [0,1]^2 on both sides (seed 1000), squared
Euclidean cost divided by its maximum (800 MB FP64), uniform weights, eta = 1e-2.

A step is one outer iteration of Algorithm 2 (every row of the hot path: outer update
of the implicit centre, Sinkhorn warm-up when the gradient is large, sparsified
Newton-CG with Armijo steps, the inexact stop test and the certificate).  Warm-up
steps run from X^0 = a b^T untimed; the timed steps resume from that state.

`time_to_gap` compares the two precision forms on the same instance from X^0: plain FP64
runs `--gap-outer` outer iterations and reaches a certified relative gap G; the
mixed-precision form (FP32 exponentials and sparse values, FP64 sums, FP64 near
convergence) then runs until its certified gap is <= G.  Both wall times are reported.

JSON line: `value` is the whole-job streaming throughput of the timed steps, i.e.
the algorithmic bytes of every dense m x n pass the steps made divided by their wall
time (inputs resident in HBM).  `roofline` reports the row-LSE (eval) kernel: its
algorithmic bytes per launch over its average launch time, measured with HIP events
recorded on the library's stream around each launch.  `cpu_baseline` times the CPU
oracle's eval pass on the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# HBM counters of the LSE pass (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a copy of known
# size); used only while they describe the dense-pass source that is built
TRAFFIC_MD = os.path.join(ROOT, "profiles", "eval_uniform10000_hbm_counters.md")
METRIC = ("time to 1e-8 OT gap at n=10k (plain vs warm-start+FP32); LSE-pass HBM GB/s")
HBM_PEAK_GBS = 8000.0


def pass_bytes(m: int, n: int) -> float:
    """Algorithmic bytes of one dense pass: the FP64 cost once plus the m- and n-vectors
    it reads or writes (w, a, M, S, partial-sum inputs: 4 m-vectors and 5 n-vectors)."""
    return 8.0 * m * n + 8.0 * (4 * m + 5 * n)


def cg_roofline(m: int, n: int, rep: dict, kt: dict):
    """The CG iterations' sparse gathers: per iteration the row gather reads each stored
    entry of the sparsified factor (int32 column + FP64 value) and the column gather its
    transpose (int32 row + FP64 value), i.e. 24 bytes per stored entry outside the dense
    row, 8 bytes per dense-row entry read twice, plus the n- and m-vectors they read and
    write (8 (6n + 2m) bytes).  Time per iteration from the CG solves' HIP events (host
    polling between chunks of iterations included)."""
    iters = rep["cg"]
    if not iters or not kt.get("cg", (0, 0))[1]:
        return None
    nnz = rep["nnz_mean"]
    per_iter = 24.0 * max(nnz - n, 0.0) + 16.0 * n + 8.0 * (6 * n + 2 * m)
    ms_per_iter = kt["cg"][0] / iters
    achieved = per_iter / (ms_per_iter * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "CG iteration (row gather + column gather + update)",
            "bytes_per_iteration": per_iter, "ms_per_iteration": ms_per_iter}


def cpu_baseline(inst, seconds: float):
    """The oracle's eval pass (eqs. 5-8) on the same 10^4 workload, repeated for about
    `seconds` of CPU time; GB/s in the same algorithmic bytes as `value`."""
    import numpy as np

    import oracle

    m, n = inst.C.shape
    gamma = np.zeros(n)
    s = np.log(inst.b)
    q = oracle.center_quantum(inst.C, s, gamma, inst.eta, 0)
    t0 = time.perf_counter()
    passes = 0
    while True:
        oracle.eval_pass(inst.C, inst.a, inst.b, inst.eta, gamma, s=s, q=q)
        passes += 1
        if time.perf_counter() - t0 >= seconds or passes >= 50:
            break
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": passes * pass_bytes(m, n) / dt / 1e9, "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{passes} oracle eval passes (row LSE, P^T a, objective) at m=n={n}, "
                      f"{dt:.1f} s"}


def time_to_gap(ibsn, ctx, prob, outer: int):
    """Plain FP64 for `outer` outer iterations from X^0 sets the gap target G; the mixed
    form runs from X^0 until its certified relative gap is <= G."""
    import torch

    def run(precision, **kw):
        pr = ibsn.Problem(prob.C, prob.a, prob.b, prob.eta, precision=precision)
        opt = ibsn.default_options(marg_tol=0.0, **kw)
        ctx.kernel_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ibsn.solve(ctx, pr, opt)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = ctx.kernel_times()
        ctx.kernel_timing(False)
        rep = res["report"]
        return {"seconds": dt, "rel_gap": rep["rel_gap"],
                "kernel_ms": {k: {"total": v[0], "launches": v[1],
                                  "avg": (v[0] / v[1]) if v[1] else None}
                              for k, v in kt.items() if v[1]},
                "outer": rep["outer"], "newton": rep["newton"], "cg": rep["cg"],
                "dense_passes": rep["passes"], "mixed_passes": rep["mixed_passes"],
                "status": res["status"]}

    plain = run(ibsn.PREC_F64, max_outer=outer, gap_tol=0.0)
    target = plain["rel_gap"]
    mixed = run(ibsn.PREC_MIXED, max_outer=2 * outer, gap_tol=target)
    return {"target_rel_gap": target, "start": "X^0 = a b^T, gamma = 0",
            "plain_f64": plain, "mixed": mixed,
            "mixed_over_plain_time": mixed["seconds"] / plain["seconds"]}


def time_to_1e8(ibsn, ctx, n: int, eta: float):
    """Wall time to a certified relative gap of 1e-8 from X^0, plain FP64 and the mixed
    form, on uniform points at size n (seed 0) with the given eta: a size and eta at which
    the target is reachable in seconds (at n = 10^4 and eta = 1e-2 it needs ~10^7 outer
    iterations)."""
    import torch

    from paper_2603_07156_amd import workloads
    inst = workloads.uniform_points(n, 0, eta=eta)
    dev = torch.device("cuda", 0)
    C = torch.from_numpy(inst.C).to(dev)
    a = torch.from_numpy(inst.a).to(dev)
    b = torch.from_numpy(inst.b).to(dev)
    out = {"workload": f"uniform points in [0,1]^2, m=n={n}, eta={eta:g}, seed 0, from X^0",
           "target_rel_gap": 1e-8}
    for name, prec in (("plain_f64", ibsn.PREC_F64), ("mixed", ibsn.PREC_MIXED)):
        pr = ibsn.Problem(C, a, b, eta, precision=prec)
        opt = ibsn.default_options(max_outer=5000, gap_tol=1e-8, marg_tol=0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ibsn.solve(ctx, pr, opt)
        torch.cuda.synchronize()
        rep = res["report"]
        out[name] = {"seconds": time.perf_counter() - t0, "status": res["status"],
                     "rel_gap": rep["rel_gap"], "outer": rep["outer"], "newton": rep["newton"],
                     "cg": rep["cg"], "t_cg": rep["t_cg"]}
    return out


def batch_solves(ibsn, count: int, outer: int = 20):
    """The batched workload (grid histograms, sizes m, n in [64, 2048], seed 300, eta 1e-2):
    `outer` outer iterations per problem, with one context and with four contexts on their
    own streams (ibsn_solve_batch)."""
    import torch

    from paper_2603_07156_amd import workloads
    batch = workloads.grid_histogram_batch(count, 300)
    dev = torch.device("cuda", 0)
    probs = [ibsn.Problem(torch.from_numpy(b.C).to(dev), torch.from_numpy(b.a).to(dev),
                          torch.from_numpy(b.b).to(dev), b.eta) for b in batch]
    opt = ibsn.default_options(max_outer=outer, gap_tol=0.0, marg_tol=0.0)
    res = {"workload": f"{count} grid-histogram problems, m,n in [64, 2048], sum m n = "
                       f"{sum(b.C.size for b in batch):.3g}, eta 1e-2, {outer} outer iterations each"}
    for workers in (1, 4):
        ctxs = [ibsn.Context(0, stream=torch.cuda.Stream()) for _ in range(workers)]
        ibsn.solve_batch(ctxs, probs[:workers], opt)   # warm the workspaces
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = ibsn.solve_batch(ctxs, probs, opt)
        dt = time.perf_counter() - t0
        res[f"contexts_{workers}"] = {"seconds": dt, "problems_per_s": count / dt,
                                      "failed": sum(1 for o in outs if o["status"] < 0)}
        for c in ctxs:
            c.close()
    res["speedup_4_over_1"] = res["contexts_1"]["seconds"] / res["contexts_4"]["seconds"]
    return res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=60)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--gap-outer", type=int, default=100,
                    help="outer iterations of the plain run that sets the common gap target")
    ap.add_argument("--ttg-n", type=int, default=1024,
                    help="size of the time-to-1e-8-gap runs (0 = skip); eta set by --ttg-eta")
    ap.add_argument("--ttg-eta", type=float, default=1e-5)
    ap.add_argument("--batch", type=int, default=64,
                    help="problems of the batched grid-histogram workload (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the hot path is not sharded across GPUs in this "
              "build (see the design notes for how it would shard); run with --gpus 1",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2603_07156_amd import ibsn, probe, workloads

    dev = torch.device("cuda", 0)
    inst = workloads.uniform_points(args.n, args.seed)
    m, n = inst.C.shape
    ctx = ibsn.Context(0)
    prob = ibsn.Problem(torch.from_numpy(inst.C).to(dev), torch.from_numpy(inst.a).to(dev),
                        torch.from_numpy(inst.b).to(dev), inst.eta)
    torch.cuda.synchronize()

    # warm-up steps from X^0 (untimed)
    opt = ibsn.default_options(max_outer=max(args.warmup, 1), gap_tol=0.0, marg_tol=0.0)
    w = ibsn.solve(ctx, prob, opt)
    state = (w["r"], w["s"], w["k"])
    gamma = w["gamma"]
    torch.cuda.synchronize()

    # timed steps
    opt = ibsn.default_options(max_outer=args.steps, gap_tol=0.0, marg_tol=0.0)
    ctx.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ibsn.solve(ctx, prob, opt, gamma0=gamma, state=state)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = ctx.kernel_times()
    ctx.kernel_timing(False)
    rep = res["report"]
    steps = int(rep["outer"])

    pb = pass_bytes(m, n)
    value = rep["passes"] * pb / dt / 1e9
    eval_ms, eval_n = kt["eval"]
    eval_avg_ms = eval_ms / max(eval_n, 1)
    achieved = pb / (eval_avg_ms * 1e-3) / 1e9 if eval_n else None

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / max(steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"uniform points in [0,1]^2, m=n={n}, squared-Euclidean cost / max, "
                               f"uniform weights, eta={inst.eta}, seed {args.seed}; a step is one "
                               f"IBSN outer iteration (k = {args.warmup}..{args.warmup + steps - 1})",
                   "m": m, "n": n, "eta": inst.eta},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": probe.read_traffic(TRAFFIC_MD) if args.n == 10000 else None,
                     "kernel": "row-LSE eval pass (k_eval)", "bytes_per_launch": pb,
                     "avg_launch_ms": eval_avg_ms, "launches": eval_n},
        "solve": {"outer_per_s": steps / dt, "dense_passes": rep["passes"],
                  "newton": rep["newton"], "cg": rep["cg"], "sinkhorn": rep["sinkhorn"],
                  "backtracks": rep["backtracks"], "rel_gap_end": rep["rel_gap"],
                  "grad_norm_end": rep["grad_norm"], "k_end": res["k"],
                  "nnz_mean": rep["nnz_mean"], "nnz_last": rep["nnz_last"],
                  "density_mean": rep["nnz_mean"] / (m * n)},
        "roofline_cg": cg_roofline(m, n, rep, kt),
        "kernel_ms": {k: {"total": v[0], "launches": v[1],
                          "avg": (v[0] / v[1]) if v[1] else None} for k, v in kt.items()},
    }
    if args.gap_outer > 0:
        ttg = time_to_gap(ibsn, ctx, prob, args.gap_outer)
        out["time_to_gap"] = ttg
        # the LSE pass of the mixed form (FP32 exponentials, FP64 sums): same bytes
        mk = ttg["mixed"]["kernel_ms"].get("eval_mixed")
        if mk:
            ach = pb / (mk["avg"] * 1e-3) / 1e9
            out["roofline_mixed_eval"] = {
                "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "kernel": "row-LSE eval pass, mixed-precision form (k_eval<..., MX>)",
                "bytes_per_launch": pb, "avg_launch_ms": mk["avg"], "launches": mk["launches"]}
    if args.ttg_n > 0:
        out["time_to_1e-8_gap"] = time_to_1e8(ibsn, ctx, args.ttg_n, args.ttg_eta)
    if args.batch > 0:
        out["batch"] = batch_solves(ibsn, args.batch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
