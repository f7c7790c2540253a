"""HBM byte counters of the transpose's two fills (per entry and by 32-row block) on a dense
sparsified factor.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o fetch -- python3 probe_csc.py
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o write -- python3 probe_csc.py
    python3 probe_csc.py --summarize <dir>/fetch_counter_collection.csv \\
        <dir>/write_counter_collection.csv > profiles/<name>.md

The probe takes m = n = 10^4 uniform points (seed 1000) at eta = 1e-2, the first
subproblem at gamma = 0 from the centre X^0 = a b^T, and sparsifies with the paper's rho
(eta ||g|| / (m n)): the factor keeps a large share of the entries, as early in a solve at
this eta.  It builds the factor REPS times with each fill forced (per entry, then by
block), then five device copies of 800 MB whose bytes are known calibrate the counters.
Each fill's figure is the median over its REPS dispatches; its algorithmic bytes are 24
per stored entry outside the dense row (int32 column and FP64 value read from the row
slots, int32 row and FP64 value written to the transpose).
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)
COPY_BYTES = 800_000_000
N = 10000
SEED = 1000
ETA = 1e-2
REPS = 5
INFO = os.path.join(HERE, "gpurun_out", "probe_csc_info.json")
KERNELS = (("per-entry fill", "k_csc_fill<"), ("block fill", "k_csc_fill_block"))


def run_probe() -> None:
    import torch

    from paper_2603_07156_amd import ibsn, workloads

    dev = torch.device("cuda", 0)
    inst = workloads.uniform_points(N, SEED, eta=ETA)
    ctx = ibsn.Context(0)
    pr = ibsn.Problem(torch.from_numpy(inst.C).to(dev), torch.from_numpy(inst.a).to(dev),
                      torch.from_numpy(inst.b).to(dev), ETA)
    r = torch.empty(N, dtype=torch.float64, device=dev)
    s = torch.empty(N, dtype=torch.float64, device=dev)
    ibsn.center_init(ctx, pr, r, s)
    gamma = torch.zeros(N, dtype=torch.float64, device=dev)
    ctr = ibsn.Center(0, r, s, 1.0)
    ctr.quantum = ibsn.center_quantum(ctx, pr, ctr, gamma)
    ev = ibsn.subproblem_eval(ctx, pr, ctr, gamma)
    rho = ETA * float(ev["g"].norm()) / (N * N)
    times = {}
    nnz = 0
    for mode, label in ((ibsn.CSC_ENTRY, "per-entry fill"), (ibsn.CSC_BLOCK, "block fill")):
        ctx.set_csc_fill(mode)
        ts = []
        for _ in range(REPS):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            csr = ibsn.sparsify(ctx, pr, ctr, gamma, ev["M"], ev["S"], rho)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            nnz = int(csr.nnz)
            csr.free()
        times[label] = sorted(ts)[REPS // 2]
    ctx.set_csc_fill(ibsn.CSC_AUTO)
    os.makedirs(os.path.dirname(INFO), exist_ok=True)
    with open(INFO, "w") as f:
        json.dump({"m": N, "n": N, "nnz": nnz, "rho": rho, "sparsify_s": times}, f)
    x1 = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    y1 = torch.empty_like(x1)
    for _ in range(5):
        y1.copy_(x1)
    torch.cuda.synchronize()
    print(f"probe done: nnz {nnz} ({nnz / (N * N):.3f} of the entries), {REPS} builds per fill, "
          f"5 copies of {COPY_BYTES} bytes", flush=True)


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
    return out


def summarize(fetch_csv: str, write_csv: str) -> str:
    fe, wr = _per_kernel(fetch_csv), _per_kernel(write_csv)
    with open(INFO) as f:
        info = json.load(f)
    cf = sorted(fe["copy"][-5:])[2]
    cw = sorted(wr["copy"][-5:])[2]
    f_fetch = COPY_BYTES / (cf * 1024.0)
    f_write = COPY_BYTES / (cw * 1024.0)
    alg = 24.0 * max(info["nnz"] - info["n"], 0)
    lines = [
        f"# Transpose fills, uniform points m = n = {N}, eta = {ETA:g}, first subproblem: HBM "
        "counters",
        "",
        "Commands (from the repository root, one MI355X; each counter in its own run):",
        "",
        "```",
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_csc_fetch -o fetch -- "
        "python3 probe_csc.py",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_csc_write -o write -- "
        "python3 probe_csc.py",
        "python3 probe_csc.py --summarize "
        "gpurun_out/pmc_csc_fetch/fetch_counter_collection.csv "
        "gpurun_out/pmc_csc_write/write_counter_collection.csv",
        "```",
        "",
        f"Factor: rho = {info['rho']:.3g}, {info['nnz']} stored entries "
        f"({info['nnz'] / (info['m'] * info['n']):.3f} of m n); algorithmic bytes of a fill "
        f"24 (nnz - n) = {alg:.4g}.",
        "",
        "| quantity | value |",
        "|---|---:|",
        f"| copy of {COPY_BYTES} B: FETCH_SIZE (KiB) | {cf:.1f} |",
        f"| copy of {COPY_BYTES} B: WRITE_SIZE (KiB) | {cw:.1f} |",
        f"| scale factor FETCH_SIZE -> bytes | {f_fetch:.4f} x 1024 |",
        f"| scale factor WRITE_SIZE -> bytes | {f_write:.4f} x 1024 |",
    ]
    for label, _ in KERNELS:
        if label not in fe or label not in wr:
            continue
        ef = sorted(fe[label])[len(fe[label]) // 2] * 1024.0 * f_fetch
        ew = sorted(wr[label])[len(wr[label]) // 2] * 1024.0 * f_write
        lines.append(f"| {label}: HBM bytes fetched / written per launch (median of "
                     f"{len(fe[label])}) | {ef:.4g} / {ew:.4g} |")
        lines.append(f"| {label}: HBM bytes over algorithmic bytes | {(ef + ew) / alg:.3f} |")
    for label, t in info["sparsify_s"].items():
        lines.append(f"| whole sparsify call with the {label}, wall time under the profiler "
                     f"(median) | {t * 1e3:.2f} ms |")
    lines.append("")
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
