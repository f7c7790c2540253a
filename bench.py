#!/usr/bin/env python
"""Benchmark of the IBSN hot path on one MI355X.

Workload (the metric's instance): m = n = 10^4 points uniform in [0,1]^2 on both sides
(seed 1000), squared Euclidean cost divided by its maximum (800 MB FP64), uniform weights,
eta = 1e-6.  At this eta plain FP64 IBSN reaches a certified relative gap of 1e-8 in a few
hundred outer iterations, seconds on one GPU (at eta = 1e-2 the same gap needs ~10^7 outer
iterations; on this instance eta = 1e-6 was the fastest of 1e-5 ... 1e-7).

A step is one outer iteration of Algorithm 2 (every row of the hot path: the implicit
centre and its outer update, the Sinkhorn warm-up when the gradient is large, the eval
(row LSE) pass, sparsification, Newton-CG, the Armijo trial passes, the inexact stop test
with Algorithm 3's rounding, and the certificate).  W warm-up steps run from X^0 = a b^T
untimed; the K timed steps resume from that state.

JSON line:
  value          LSE-pass throughput of the timed steps: algorithmic bytes of the eval
                 kernel per launch over its mean launch time (HIP events recorded on the
                 library's stream around each launch), in GB/s.  `roofline` is the same
                 kernel against the 8 TB/s peak.
  time_to_1e-8_gap  the metric's time half at m = n = 10^4: wall time from X^0 to a
                 certified relative gap <= 1e-8, plain FP64 and the precision form (FP32
                 exponentials and sparse values with FP64 sums), each from zero
                 initialisation, and both forms again from the learned warm start (its
                 features and network forward pass inside the timed region) when trained
                 weights are present; counts and the gap reached.
  gap_within_budget  both forms from zero at eta = 1e-2 on the same cost: the certified
                 relative gap each reaches within 0.25, 0.5, 1 and 2 s (at most 400 outer
                 iterations).
  paper_workloads  the paper's Table 1 runs at m = n = 10^4 (IBSN to Delta_kkt < 1e-11 or
                 300 outer iterations) and Table 2 (E)IBSN runs on Square, with the paper's
                 own figures (other hardware) beside them as context.
  cpu_baseline   the oracle's eval pass on the same instance, on the host's cores, for a
                 bounded time, in the unit of `value`; and the oracle's time to a certified
                 1e-8 gap at m = n = 512 (same generator and eta), the GPU's beside it.
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
CG_TRAFFIC_MD = os.path.join(ROOT, "profiles", "cg_uniform10000_hbm_counters.md")
METRIC = ("time to 1e-8 OT gap at n=10k (plain vs warm-start+FP32); LSE-pass HBM GB/s")
HBM_PEAK_GBS = 8000.0
ETA = 1e-6
# trained parameters of the learned warm start (paper_2603_07156_amd/train_warmstart.py)
WS_WEIGHTS = os.path.join(ROOT, "paper_2603_07156_amd", "warmstart_uniform_eta1e-6.npz")


def pass_bytes(m: int, n: int) -> float:
    """Algorithmic bytes of one dense pass (probe.algorithmic_bytes: the FP64 cost once,
    4 m-vectors and 6 n-vectors)."""
    import probe
    return probe.algorithmic_bytes(m, n)


def cg_roofline(m: int, n: int, rep: dict, kt: dict):
    """The CG iterations' sparse gathers: per iteration the row gather reads each stored
    entry of the sparsified factor (int32 column + FP64 value) and the column gather its
    transpose (int32 row + FP64 value), i.e. 24 bytes per stored entry outside the dense
    row, 8 bytes per dense-row entry read twice, plus the n- and m-vectors they read and
    write (8 (6n + 2m) bytes).  Time per iteration from the CG solves' HIP events (host
    polling between chunks of iterations included), in the form the automatic choice took
    for each solve (late in a solve one barrier per iteration on P'^T diag(a) P', whose
    entries stay in LDS; the bytes above are those of the two-hop product)."""
    iters = rep["cg"]
    if not iters or not kt.get("cg", (0, 0))[1]:
        return None
    nnz = rep["nnz_mean"]
    per_iter = 24.0 * max(nnz - n, 0.0) + 16.0 * n + 8.0 * (6 * n + 2 * m)
    ms_per_iter = kt["cg"][0] / iters
    achieved = per_iter / (ms_per_iter * 1e-3) / 1e9
    import probe_cg
    counters = probe_cg.read_traffic(CG_TRAFFIC_MD)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "CG iteration (automatic form: one barrier on P'^T diag(a) P' late in "
                      "a solve, two on the row and column gathers before)",
            "bytes_per_iteration": per_iter, "ms_per_iteration": ms_per_iter,
            "nnz_mean": nnz,
            # HBM counters of the three-launch form at a late state of this instance (the
            # one-launch form is a cooperative launch, which the profiler did not survive)
            "counters_three_launch_form": None if counters is None else {
                "traffic_bytes_per_iteration": counters[0],
                "algorithmic_bytes_per_iteration": counters[1],
                "summary": os.path.relpath(CG_TRAFFIC_MD, ROOT)}}


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
                      f"eta={inst.eta:g}, {dt:.1f} s"}


def cpu_time_to_gap(ibsn, ctx, n: int = 512, eta: float = ETA, gap: float = 1e-8):
    """The oracle's plain FP64 solve from X^0 to a certified relative gap on the host's
    cores, at a size it finishes in seconds (the metric's generator, seed 1000), with the
    GPU's plain FP64 solve of the same instance beside it."""
    import torch

    import oracle
    from paper_2603_07156_amd import workloads

    inst = workloads.uniform_points(n, 1000, eta=eta)
    t0 = time.perf_counter()
    o = oracle.solve(inst.C, inst.a, inst.b, eta, options=oracle.default_options(
        max_outer=20000, gap_tol=gap, marg_tol=0.0))
    t_cpu = time.perf_counter() - t0
    dev = torch.device("cuda", 0)
    pr = ibsn.Problem(torch.from_numpy(inst.C).to(dev), torch.from_numpy(inst.a).to(dev),
                      torch.from_numpy(inst.b).to(dev), eta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = ibsn.solve(ctx, pr, ibsn.default_options(max_outer=20000, gap_tol=gap, marg_tol=0.0))
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    ro, rg = o["report"], g["report"]
    return {"workload": f"uniform points m=n={n}, eta={eta:g}, seed 1000, to a certified "
                        f"relative gap <= {gap:g} from X^0, plain FP64",
            "oracle_seconds": t_cpu, "oracle_outer": ro["outer"], "oracle_newton": ro["newton"],
            "oracle_rel_gap": ro["rel_gap"], "oracle_status": o["status"],
            "gpu_seconds": t_gpu, "gpu_outer": rg["outer"], "gpu_newton": rg["newton"],
            "gpu_rel_gap": rg["rel_gap"]}


def kt_dict(kt):
    return {k: {"total": v[0], "launches": v[1], "avg": (v[0] / v[1]) if v[1] else None}
            for k, v in kt.items() if v[1]}


def solve_to_gap(ibsn, ctx, prob, precision, gap=1e-8, max_outer=20000, gamma0_fn=None,
                 problem=None):
    """Wall time from X^0 to a certified relative gap <= `gap`, starting the first
    subproblem from gamma = 0 or from gamma0_fn() (called inside the timed region).
    `problem`: a prepared problem to solve instead of prob's stored cost in `precision`."""
    import torch

    pr = problem if problem is not None else ibsn.Problem(prob.C, prob.a, prob.b, prob.eta,
                                                          precision=precision)
    opt = ibsn.default_options(max_outer=max_outer, gap_tol=gap, marg_tol=0.0)
    ctx.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gamma0 = gamma0_fn() if gamma0_fn else None
    t_ws = time.perf_counter() - t0
    res = ibsn.solve(ctx, pr, opt, gamma0=gamma0, trace_cap=max_outer)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = ctx.kernel_times()
    ctx.kernel_timing(False)
    rep = res["report"]
    # where the time goes: cumulative seconds and gap after the first outer iterations
    tr = res["trace"] or []
    cum, acc = {}, 0.0
    marks = {1, 2, 5, 10, 20, 50, 100, 200, 500, 1000, 2000, 5000}
    for t in tr:
        acc += t["t_total"]
        if t["k"] + 1 in marks or t is tr[-1]:
            cum[str(t["k"] + 1)] = {"seconds": acc, "rel_gap": t["rel_gap"],
                                    "newton": t["newton"], "backtracks": t["backtracks"],
                                    "sinkhorn": t["sinkhorn"]}
    return {"seconds": dt, "warm_start_seconds": t_ws if gamma0_fn else None,
            "status": res["status"], "rel_gap": rep["rel_gap"],
            "by_outer": cum,
            "primal": rep["primal"], "dual": rep["dual"], "outer": rep["outer"],
            "newton": rep["newton"], "cg": rep["cg"], "sinkhorn": rep["sinkhorn"],
            "backtracks": rep["backtracks"], "dense_passes": rep["passes"],
            "mixed_passes": rep["mixed_passes"],
            "t_eval": rep["t_eval"], "t_sparsify": rep["t_sparsify"], "t_cg": rep["t_cg"],
            "t_linesearch": rep["t_linesearch"], "t_stop": rep["t_stop"],
            "kernel_ms": kt_dict(kt)}


def gap_within_budget(ibsn, ctx, prob, eta, budgets=(0.25, 0.5, 1.0, 2.0), max_outer=400):
    """Both arms from gamma = 0 (plain FP64 and the FP32 form; the trained warm start is for
    eta = 1e-6 and is not used) on the same stored cost at another eta: the certified
    relative gap each has reached within each wall-time budget, read from the solve's
    per-outer-iteration records (cumulative outer-iteration time), over at most max_outer
    outer iterations."""
    import torch

    out = {"eta": eta, "budgets_s": list(budgets), "max_outer": max_outer,
           "start": "gamma = 0, no warm start"}
    for name, prec in (("plain_f64", ibsn.PREC_F64), ("mixed_fp32", ibsn.PREC_MIXED)):
        pr = ibsn.Problem(prob.C, prob.a, prob.b, eta, precision=prec)
        opt = ibsn.default_options(max_outer=max_outer, gap_tol=0.0, marg_tol=0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ibsn.solve(ctx, pr, opt, trace_cap=max_outer)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        acc, at = 0.0, {}
        for t in res["trace"] or []:
            acc += t["t_total"]
            for b in budgets:
                if acc <= b:
                    at[b] = {"rel_gap": t["rel_gap"], "outer": t["k"] + 1}
        rep = res["report"]
        out[name] = {"at_budget": {f"{b:g}": at.get(b) for b in budgets},
                     "seconds": dt, "outer": rep["outer"], "newton": rep["newton"],
                     "final_rel_gap": rep["rel_gap"]}
        print(f"gap within budget, eta {eta:g}, {name}: {dt:.2f} s, {rep['outer']} outer, "
              f"final gap {rep['rel_gap']:.3g}", file=sys.stderr, flush=True)
    return out


def points_problem(ibsn, inst, prob, precision, scale=None):
    """The same instance with its cost formed from the points in every pass (no m x n
    array): C_ij = scale |x_i - y_j|^2 with scale = 1 / max, the stored cost to rounding."""
    import numpy as np
    import torch

    from paper_2603_07156_amd import workloads
    dev = prob.C.device
    x = torch.from_numpy(np.ascontiguousarray(inst.x)).to(dev)
    y = torch.from_numpy(np.ascontiguousarray(inst.y)).to(dev)
    if scale is None:
        scale = workloads.points_scale(inst.x, inst.y)
    return ibsn.Problem.from_points(x, y, prob.a, prob.b, prob.eta, scale, precision)


def warm_start_fn(ibsn, ctx, prob, inst):
    """gamma0 of the first subproblem from the trained network (features, forward, centring
    and scaling all in the library's kernels), or None when no trained weights exist."""
    import numpy as np
    import torch

    if not os.path.exists(WS_WEIGHTS) or inst.x is None:
        return None, None
    d = np.load(WS_WEIGHTS)
    ws = ibsn.WarmStart(ctx)
    ws.set_params(d["params"])
    x = torch.from_numpy(np.ascontiguousarray(inst.x)).to(prob.C.device)
    y = torch.from_numpy(np.ascontiguousarray(inst.y)).to(prob.C.device)
    m, n = inst.C.shape

    def fn():
        fs, fte, fth, scale = ws.features(prob, x, y)
        return ws.predict(m, n, fs, fte, fth, scale)
    info = {"weights": os.path.relpath(WS_WEIGHTS, ROOT), "trained_n": int(d["n"]),
            "trained_eta": float(d["eta"]), "train_instances": int(d["train"]),
            "val_r2": float(d["val_r2"])}
    return fn, (ws, info)


# The paper's own figures (Apple M2 Pro, one process, NumPy; Tables 1 and 2), as context for
# the same workloads run here; different hardware and software, not a target.
PAPER_TABLE1 = {   # IBSN, eta = 1e-4, Delta_kkt < 1e-11 or 300 outer iterations, m = n = 10^4
    "uniform": {"newton": 170, "cg_seconds": 16.82, "seconds": 921.60, "abs_gap": 3.63e-9},
    "square": {"newton": 300, "cg_seconds": 267.15, "seconds": 2205.74, "abs_gap": 1.59e-7},
}
PAPER_TABLE2 = {   # (E)IBSN on Square, eta = 1e-4, ||g|| < 1e-9
    1000: {"mean_cg": 163.6, "newton": 11, "seconds": 0.54},
    5000: {"mean_cg": 290.4, "newton": 13, "seconds": 23.64},
    10000: {"mean_cg": 241.2, "newton": 13, "seconds": 88.63},
}


def paper_tables(ibsn, ctx):
    """The paper's Table 1 runs at m = n = 10^4 (Uniform: C_ij ~ U(0,1); Square:
    C_ij = (i - j)^2; a, b ~ U(0,1) normalised; seed 0) and its Table 2 (E)IBSN runs on
    Square, with the paper's figures beside them."""
    import torch

    from paper_2603_07156_amd import workloads
    dev = torch.device("cuda", 0)

    def run(inst, opt):
        pr = ibsn.Problem(torch.from_numpy(inst.C).to(dev), torch.from_numpy(inst.a).to(dev),
                          torch.from_numpy(inst.b).to(dev), 1e-4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ibsn.solve(ctx, pr, opt)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    out = {"note": "paper figures: Apple M2 Pro, NumPy, one process (context only)",
           "table1": {}, "table2": {}}
    for gen in ("uniform", "square"):
        inst = getattr(workloads, "paper_" + gen)(10000, 0)
        r, dt = run(inst, ibsn.default_options(max_outer=300, gap_tol=0.0, marg_tol=0.0,
                                               kkt_tol=1e-11))
        rep = r["report"]
        out["table1"][gen] = {"seconds": dt, "outer": rep["outer"], "newton": rep["newton"],
                              "cg_seconds": rep["t_cg"], "kkt": rep["kkt"],
                              "rel_gap": rep["rel_gap"],
                              "abs_gap_bound": rep["primal"] - rep["dual"],
                              "paper": PAPER_TABLE1[gen]}
    for n in (1000, 5000, 10000):
        inst = workloads.paper_square(n, 0)
        r, dt = run(inst, ibsn.default_options(eot=1, eot_tol=1e-9, max_newton=500))
        rep = r["report"]
        out["table2"][str(n)] = {"seconds": dt, "newton": rep["newton"],
                                 "mean_cg": rep["cg"] / max(rep["newton"], 1),
                                 "sinkhorn": rep["sinkhorn"], "grad_norm": rep["grad_norm"],
                                 "status": r["status"], "paper": PAPER_TABLE2[n]}
    return out


def batch_solves(ibsn, count: int, outer: int = 20, gap: float = 0.0, workers_list=(1, 4)):
    """The batched workload (grid histograms, sizes m, n in [64, 2048], seed 300, eta 1e-2):
    `outer` outer iterations per problem, or (gap > 0) each problem solved to a certified
    relative gap <= gap with at most `outer` outer iterations, with one context and with four
    contexts on their own streams (ibsn_solve_batch)."""
    import torch

    from paper_2603_07156_amd import workloads
    batch = workloads.grid_histogram_batch(count, 300)
    dev = torch.device("cuda", 0)
    probs = [ibsn.Problem(torch.from_numpy(b.C).to(dev), torch.from_numpy(b.a).to(dev),
                          torch.from_numpy(b.b).to(dev), b.eta) for b in batch]
    opt = ibsn.default_options(max_outer=outer, gap_tol=gap, marg_tol=0.0)
    stop = (f"to a certified relative gap <= {gap:g} (at most {outer} outer iterations)" if gap > 0
            else f"{outer} outer iterations each")
    res = {"workload": f"{count} grid-histogram problems, m,n in [64, 2048], sum m n = "
                       f"{sum(b.C.size for b in batch):.3g}, eta 1e-2, {stop}"}
    for workers in workers_list:
        ctxs = [ibsn.Context(0, stream=torch.cuda.Stream()) for _ in range(workers)]
        ibsn.solve_batch(ctxs, probs[:workers], opt)   # warm the workspaces
        torch.cuda.synchronize()
        # batches of more than 128 problems run in chunks of 128 calls of ibsn_solve_batch,
        # each chunk's end reported as it comes (the workers idle at each chunk's tail)
        outs, t0 = [], time.perf_counter()
        for c0 in range(0, count, 128):
            outs += ibsn.solve_batch(ctxs, probs[c0:c0 + 128], opt)
            if count > 128:
                print(f"batch: {len(outs)}/{count} problems, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
        dt = time.perf_counter() - t0
        res[f"contexts_{workers}"] = {"seconds": dt, "problems_per_s": count / dt,
                                      "failed": sum(1 for o in outs if o["status"] < 0),
                                      "reached_gap": sum(1 for o in outs if o["status"] == 0),
                                      "outer_total": sum(int(o["report"]["outer"])
                                                         for o in outs)}
        for c in ctxs:
            c.close()
    if "contexts_1" in res and "contexts_4" in res:
        res["speedup_4_over_1"] = res["contexts_1"]["seconds"] / res["contexts_4"]["seconds"]
    return res


def cfg3_legs(ibsn, ctx, outer: int = 5):
    """The 20000 x 20000 configuration (3-D unit-cube points vs an 8-component mixture,
    uniform weights, eta = 1e-2): `outer` outer iterations from X^0 with the cost formed from
    the points in every pass (rows split into two column blocks) in the FP64 and the FP32
    form, and with the cost stored in FP32 (1.6 GB) on whole rows and on split rows; the time
    per outer iteration and each pass's mean time."""
    import numpy as np
    import torch

    from paper_2603_07156_amd import workloads
    dev = torch.device("cuda", 0)
    N = 20000
    rng = np.random.default_rng(200)
    x = rng.random((N, 3))
    y = workloads._gmm(rng, N, 8, 3, 0.08)
    scale = workloads.points_scale(x, y)
    xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    ab = torch.full((N,), 1.0 / N, dtype=torch.float64, device=dev)
    # the stored FP32 cost: the same squared distances, formed on the device
    C32 = torch.empty((N, N), dtype=torch.float32, device=dev)
    for i0 in range(0, N, 2000):
        d = xd[i0:i0 + 2000, None, :] - yd[None, :, :]
        C32[i0:i0 + 2000] = ((d * d).sum(-1) * scale).to(torch.float32)
    torch.cuda.synchronize()
    legs = {}
    cases = [("points_f64", ibsn.Problem.from_points(xd, yd, ab, ab, 1e-2, scale), 0),
             ("points_mixed", ibsn.Problem.from_points(xd, yd, ab, ab, 1e-2, scale,
                                                       ibsn.PREC_MIXED), 0),
             ("stored_f32_mixed_whole_rows", ibsn.Problem(C32, ab, ab, 1e-2,
                                                          precision=ibsn.PREC_MIXED), 0),
             ("stored_f32_mixed_split_10240", ibsn.Problem(C32, ab, ab, 1e-2,
                                                           precision=ibsn.PREC_MIXED), 10240)]
    opt = ibsn.default_options(max_outer=outer, gap_tol=0.0, marg_tol=0.0)
    for name, pr, cols in cases:
        ctx.set_row_split(cols)
        ibsn.solve(ctx, pr, ibsn.default_options(max_outer=1, gap_tol=0.0, marg_tol=0.0))
        ctx.kernel_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ibsn.solve(ctx, pr, opt)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = kt_dict(ctx.kernel_times())
        ctx.kernel_timing(False)
        rep = res["report"]
        legs[name] = {"seconds": dt, "outer": rep["outer"], "s_per_outer": dt / rep["outer"],
                      "newton": rep["newton"], "sinkhorn": rep["sinkhorn"],
                      "rel_gap": rep["rel_gap"], "pass_ms": {k: v["avg"] for k, v in kt.items()}}
        print(f"cfg3 {name}: {dt:.2f} s for {rep['outer']} outer iterations", file=sys.stderr,
              flush=True)
    ctx.set_row_split(0)
    ev = legs["stored_f32_mixed_whole_rows"]["pass_ms"].get("eval_mixed")
    evs = legs["stored_f32_mixed_split_10240"]["pass_ms"].get("eval_mixed")
    alg = 4.0 * N * N + 8.0 * 10 * N   # the FP32 cost once and the row and column vectors
    return {"workload": f"3-D unit-cube points (seed 200) vs an 8-component mixture, m=n={N}, "
                        f"uniform weights, eta=1e-2, {outer} outer iterations from X^0",
            "legs": legs,
            "eval_mixed_stored_f32_GBs": {"whole_rows": alg / (ev * 1e-3) / 1e9 if ev else None,
                                          "split_rows": alg / (evs * 1e-3) / 1e9 if evs else None,
                                          "bytes": alg,
                                          "note": "algorithmic bytes (the cost read once) over "
                                                  "the pass time; split rows read the cost twice"}}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=10000)
    ap.add_argument("--eta", type=float, default=ETA)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttg", action="store_true", help="skip the time-to-1e-8-gap runs")
    ap.add_argument("--cg", choices=("auto", "launches", "persistent"), default="auto",
                    help="CG form of the context (ibsn_set_cg_kernel; auto: one cooperative "
                         "launch per CG solve where supported)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose the dense-pass tiles with ibsn_autotune on the metric instance "
                         "before the timed runs (the choice is reported)")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the runs of the paper's Table 1 and Table 2 workloads")
    ap.add_argument("--batch-gap", type=float, default=0.0,
                    help="solve the batched problems to this certified gap instead of 20 outer "
                         "iterations (at most 5000), four contexts only")
    ap.add_argument("--cfg3", action="store_true",
                    help="also run the 20000 x 20000 points / FP32-cost configuration")
    ap.add_argument("--batch", type=int, default=32,
                    help="problems of the batched grid-histogram workload (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the hot path on one GPU and "
              "does not shard it across GPUs (the design notes say how it would); run with "
              "--gpus 1", file=sys.stderr)
        return 2

    import torch

    import probe
    from paper_2603_07156_amd import ibsn, workloads

    dev = torch.device("cuda", 0)
    inst = workloads.uniform_points(args.n, args.seed, eta=args.eta)
    m, n = inst.C.shape
    ctx = ibsn.Context(0)
    ctx.set_cg_kernel({"auto": ibsn.CG_AUTO, "launches": ibsn.CG_LAUNCHES,
                       "persistent": ibsn.CG_PERSISTENT}[args.cg])
    prob = ibsn.Problem(torch.from_numpy(inst.C).to(dev), torch.from_numpy(inst.a).to(dev),
                        torch.from_numpy(inst.b).to(dev), inst.eta)
    tuned = None
    if args.autotune:
        tuned = ctx.autotune(prob)
        ctx.autotune(ibsn.Problem(prob.C, prob.a, prob.b, prob.eta, precision=ibsn.PREC_MIXED))
    torch.cuda.synchronize()
    workload = (f"uniform points in [0,1]^2, m=n={n}, squared-Euclidean cost / max (FP64), "
                f"uniform weights, eta={inst.eta:g}, seed {args.seed}")

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
    eval_ms, eval_n = kt["eval"]
    eval_avg_ms = eval_ms / max(eval_n, 1)
    achieved = pb / (eval_avg_ms * 1e-3) / 1e9 if eval_n else None
    k0 = max(args.warmup, 1)

    out = {
        "metric": METRIC,
        "value": achieved,
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
        "config": {"workload": workload + f"; a step is one IBSN outer iteration "
                               f"(k = {k0}..{k0 + steps - 1}); value is the LSE (eval) pass's "
                               f"HBM throughput over the timed steps",
                   "m": m, "n": n, "eta": inst.eta, "cg": args.cg, "tiles": tuned},
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
        "kernel_ms": kt_dict(kt),
    }
    if not args.no_ttg:
        ttg = {"workload": workload + ", from X^0 (gamma = 0)", "target_rel_gap": 1e-8}
        ttg["plain_f64"] = solve_to_gap(ibsn, ctx, prob, ibsn.PREC_F64)
        ttg["mixed_fp32"] = solve_to_gap(ibsn, ctx, prob, ibsn.PREC_MIXED)
        ttg["mixed_over_plain_time"] = ttg["mixed_fp32"]["seconds"] / ttg["plain_f64"]["seconds"]
        fn, held = warm_start_fn(ibsn, ctx, prob, inst)
        if fn:
            ttg["warm_start"] = held[1]
            ttg["warm_f64"] = solve_to_gap(ibsn, ctx, prob, ibsn.PREC_F64, gamma0_fn=fn)
            ttg["warm_mixed_fp32"] = solve_to_gap(ibsn, ctx, prob, ibsn.PREC_MIXED, gamma0_fn=fn)
            ttg["warm_mixed_over_plain_time"] = (ttg["warm_mixed_fp32"]["seconds"]
                                                 / ttg["plain_f64"]["seconds"])
            # the FP32 form with the cost formed from the points: no 800 MB FP64 stream
            pts = points_problem(ibsn, inst, prob, ibsn.PREC_MIXED)
            fn_pts, held_pts = warm_start_fn(ibsn, ctx, pts, inst)
            ttg["warm_mixed_fp32_points"] = solve_to_gap(ibsn, ctx, prob, ibsn.PREC_MIXED,
                                                         gamma0_fn=fn_pts, problem=pts)
            ttg["warm_mixed_fp32_points"]["cost"] = ("formed from the points in every pass "
                                                     "(scale = 1 / max |x_i - y_j|^2)")
            ttg["warm_f64_points"] = solve_to_gap(
                ibsn, ctx, prob, ibsn.PREC_F64, gamma0_fn=fn_pts,
                problem=points_problem(ibsn, inst, prob, ibsn.PREC_F64, pts.cost_scale))
            ttg["warm_f64_points"]["cost"] = ttg["warm_mixed_fp32_points"]["cost"]
            held_pts[0].free()
            held[0].free()
        out["time_to_1e-8_gap"] = ttg
        try:
            out["gap_within_budget"] = gap_within_budget(ibsn, ctx, prob, 1e-2)
        except Exception as e:   # reported in the line; the rest of the bench still runs
            out["gap_within_budget"] = {"eta": 1e-2, "error": repr(e)}
        mk = ttg["mixed_fp32"]["kernel_ms"].get("eval_mixed")
        if mk:
            ach = pb / (mk["avg"] * 1e-3) / 1e9
            out["roofline_mixed_eval"] = {
                "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "kernel": "row-LSE eval pass, mixed-precision form (k_eval<..., MX>)",
                "bytes_per_launch": pb, "avg_launch_ms": mk["avg"], "launches": mk["launches"]}
    if not args.no_paper:
        out["paper_workloads"] = paper_tables(ibsn, ctx)
    if args.cfg3:
        out["cfg3_20000"] = cfg3_legs(ibsn, ctx)
    if args.batch > 0:
        if args.batch_gap > 0:
            out["batch"] = batch_solves(ibsn, args.batch, outer=5000, gap=args.batch_gap,
                                        workers_list=(4,))
        else:
            out["batch"] = batch_solves(ibsn, args.batch)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
        out["cpu_baseline"]["time_to_1e-8_gap"] = cpu_time_to_gap(ibsn, ctx)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
