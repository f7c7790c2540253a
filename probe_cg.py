"""HBM byte counters of the CG kernels in their three-launch form (row gather, column
gather, update), at a late state of the metric instance.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o fetch -- python3 probe_cg.py
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o write -- python3 probe_cg.py
    python3 probe_cg.py --summarize <dir>/fetch_counter_collection.csv \\
        <dir>/write_counter_collection.csv > profiles/<name>.md

The probe solves m = n = 10^4 uniform points (seed 1000, eta = 1e-6) for five outer
iterations (CG capped at 10 iterations; past the first subproblem the sparsified factor
keeps a few entries per row), sparsifies at that state with the solver's rho, and runs 100 CG iterations on
(H_rho + ||g|| I) x = -g as three kernel launches each (the one-launch form is a
cooperative launch, under which the profiler did not write its results); then five device
copies of 800 MB whose bytes are known calibrate the counters.  The summary takes the last
100 dispatches of each CG kernel (the probe's own); the factor's size goes to a sidecar
file that it reads.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)
COPY_BYTES = 800_000_000
N = 10000
SEED = 1000
ETA = 1e-6
INFO = os.path.join(HERE, "gpurun_out", "probe_cg_info.json")
PROBE_ITERS = 100
KERNELS = (("row gather", "k_row_gather"), ("column gather", "k_col_gather"),
           ("update", "k_cg_update"))


# the three-launch CG kernels are built from this file
CG_SRC = os.path.join(HERE, "paper_2603_07156_amd", "csrc", "sparse_ops.hip")


def source_hash() -> str:
    import hashlib
    with open(CG_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def read_traffic(md_path: str):
    """(traffic, algorithmic) bytes per iteration from a summary written by --summarize, or
    None if it is missing or was made for a different source of the CG kernels."""
    if not os.path.exists(md_path):
        return None
    vals, h = {}, None
    with open(md_path) as f:
        for line in f:
            for key in ("traffic_bytes_per_iteration", "algorithmic_bytes_per_iteration"):
                if line.startswith(key + ":"):
                    vals[key] = float(line.split(":", 1)[1])
            if line.startswith("CG source sha256:"):
                h = line.split(":", 1)[1].strip()
    if h != source_hash() or len(vals) != 2:
        return None
    return vals["traffic_bytes_per_iteration"], vals["algorithmic_bytes_per_iteration"]


def iteration_bytes(m: int, n: int, nnz: float) -> float:
    """Algorithmic bytes of one CG iteration (as bench.py's roofline_cg): 24 bytes per stored
    entry outside the dense row (index and value, in the rows and in the transpose), 16 per
    dense-row entry, and 8 (6 n + 2 m) for the vectors."""
    return 24.0 * max(nnz - n, 0.0) + 16.0 * n + 8.0 * (6 * n + 2 * m)


def run_probe() -> None:
    import torch

    from paper_2603_07156_amd import ibsn, workloads

    dev = torch.device("cuda", 0)
    inst = workloads.uniform_points(N, SEED, eta=ETA)
    ctx = ibsn.Context(0)
    ctx.set_cg_kernel(ibsn.CG_LAUNCHES)
    pr = ibsn.Problem(torch.from_numpy(inst.C).to(dev), torch.from_numpy(inst.a).to(dev),
                      torch.from_numpy(inst.b).to(dev), ETA)
    # CG capped at 10 iterations on the way (fewer counted dispatches before the probe's own)
    res = ibsn.solve(ctx, pr, ibsn.default_options(max_outer=5, gap_tol=0.0, marg_tol=0.0,
                                                   cg_maxit=10))
    gamma = res["gamma"]
    ctr = ibsn.Center(int(res["k"]), res["r"], res["s"], 1.0)
    ctr.quantum = ibsn.center_quantum(ctx, pr, ctr, gamma)
    ev = ibsn.subproblem_eval(ctx, pr, ctr, gamma)
    gn = float(ev["g"].norm())
    rho = ETA * gn / (N * N)
    csr = ibsn.sparsify(ctx, pr, ctr, gamma, ev["M"], ev["S"], rho)
    x, it = ibsn.cg(ctx, csr, pr.a, ETA, gn, -ev["g"], 0.0, PROBE_ITERS)
    nnz = int(csr.nnz)
    os.makedirs(os.path.dirname(INFO), exist_ok=True)
    with open(INFO, "w") as f:
        json.dump({"m": N, "n": N, "nnz": nnz, "iterations": int(it), "k": int(res["k"]),
                   "rho": rho, "grad_norm": gn}, f)
    x1 = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    y1 = torch.empty_like(x1)
    for _ in range(5):
        y1.copy_(x1)
    torch.cuda.synchronize()
    print(f"probe done: {it} CG iterations at nnz {nnz}, 5 copies of {COPY_BYTES} bytes",
          flush=True)


def _per_kernel(path: str) -> dict:
    out: dict = {}
    with open(path) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Dispatch_Id"]))
        for r in rows:
            name = r["Kernel_Name"]
            key = "copy" if "copyBuffer" in name else None
            for label, tag in KERNELS:
                if tag in name:
                    key = label
            if key:
                out.setdefault(key, []).append(float(r["Counter_Value"]))
    # the probe's own CG is the last PROBE_ITERS dispatches of each CG kernel
    for label, _ in KERNELS:
        if label in out:
            out[label] = out[label][-PROBE_ITERS:]
    return out


def summarize(fetch_csv: str, write_csv: str) -> str:
    fe, wr = _per_kernel(fetch_csv), _per_kernel(write_csv)
    with open(INFO) as f:
        info = json.load(f)
    cf = sorted(fe["copy"][-5:])[2]
    cw = sorted(wr["copy"][-5:])[2]
    f_fetch = COPY_BYTES / (cf * 1024.0)
    f_write = COPY_BYTES / (cw * 1024.0)
    lines = [
        f"# CG kernels (three-launch form), uniform points m = n = {N}, eta = {ETA:g}: HBM "
        "counters",
        "",
        "Commands (from the repository root, one MI355X; each counter in its own run):",
        "",
        "```",
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_cg_fetch -o fetch -- "
        "python3 probe_cg.py",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_cg_write -o write -- "
        "python3 probe_cg.py",
        "python3 probe_cg.py --summarize "
        "gpurun_out/pmc_cg_fetch/fetch_counter_collection.csv "
        "gpurun_out/pmc_cg_write/write_counter_collection.csv",
        "```",
        "",
        f"State: outer iteration k = {info['k']}, rho = {info['rho']:.3g}, stored entries "
        f"{info['nnz']}, {info['iterations']} CG iterations.",
        "",
        "| quantity | value |",
        "|---|---:|",
        f"| copy of {COPY_BYTES} B: FETCH_SIZE (KiB) | {cf:.1f} |",
        f"| copy of {COPY_BYTES} B: WRITE_SIZE (KiB) | {cw:.1f} |",
        f"| scale factor FETCH_SIZE -> bytes | {f_fetch:.4f} x 1024 |",
        f"| scale factor WRITE_SIZE -> bytes | {f_write:.4f} x 1024 |",
    ]
    total = 0.0
    for label, _ in KERNELS:
        if label not in fe or label not in wr:
            continue
        ef = sum(fe[label]) / len(fe[label]) * 1024.0 * f_fetch
        ew = sum(wr[label]) / len(wr[label]) * 1024.0 * f_write
        total += ef + ew
        lines.append(f"| {label}: HBM bytes fetched / written per launch (mean of "
                     f"{len(fe[label])}) | {ef:.4g} / {ew:.4g} |")
    alg = iteration_bytes(info["m"], info["n"], info["nnz"])
    lines += [f"| one iteration (three launches): HBM bytes | {total:.4g} |",
              f"| one iteration: algorithmic bytes | {alg:.4g} |", "",
              f"traffic_bytes_per_iteration: {total:.6e}",
              f"algorithmic_bytes_per_iteration: {alg:.6e}",
              f"CG source sha256: {source_hash()}", ""]
    return "\n".join(lines)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    args = ap.parse_args()
    if args.summarize:
        print(summarize(*args.summarize))
        return 0
    run_probe()
    return 0


if __name__ == "__main__":
    sys.exit(main())
