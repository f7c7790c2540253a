"""HBM byte counters of the LSE pass (the row log-sum-exp eval kernel).

Two counter runs, each on its own (rocprofv3 collects one counter group per run):

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o fetch -- python3 probe.py
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o write -- python3 probe.py

then

    python3 probe.py --summarize <dir>/fetch_counter_collection.csv \
        <dir>/write_counter_collection.csv > profiles/<name>.md

The probe runs the eval kernel five times on the m = n = 10^4 uniform-points workload
(the benchmark's) and five plain device-to-device copies of 800 MB, whose bytes are known:
the counters of the copies give the factor that turns FETCH_SIZE / WRITE_SIZE (KiB per
dispatch) into bytes, and that factor is applied to the eval kernel's counters.  The
summary records a hash of the LSE-pass source, so that a reader (bench.py) can tell
whether the counters still describe the kernel that is built.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)
# the LSE-pass kernel is built from these two files
DENSE_SRC = [os.path.join(HERE, "paper_2603_07156_amd", "csrc", f)
             for f in ("dense_common.h", "dense_eval.hip")]
COPY_BYTES = 800_000_000
N = 10000
SEED = 1000


def source_hash() -> str:
    h = hashlib.sha256()
    for p in DENSE_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def algorithmic_bytes(m: int, n: int) -> float:
    """Bytes one dense pass must move: the FP64 cost once, 4 m-vectors (a, M, S, the log of
    the row sums) and 6 n-vectors (w, its low parts, the column partials and sums)."""
    return 8.0 * m * n + 8.0 * (4 * m + 6 * n)


def run_probe() -> None:
    import torch

    from paper_2603_07156_amd import ibsn, workloads

    dev = torch.device("cuda", 0)
    inst = workloads.uniform_points(N, SEED)
    ctx = ibsn.Context(0)
    pr = ibsn.Problem(torch.from_numpy(inst.C).to(dev), torch.from_numpy(inst.a).to(dev),
                      torch.from_numpy(inst.b).to(dev), inst.eta)
    ctr = ibsn.Center.initial(ctx, pr)
    gamma = torch.zeros(N, dtype=torch.float64, device=dev)
    for _ in range(5):
        ibsn.subproblem_eval(ctx, pr, ctr, gamma, want_obj=False, want_lse=False)
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print("probe done: 5 eval launches, 5 copies of", COPY_BYTES, "bytes", flush=True)


def _per_kernel(path: str) -> dict:
    out: dict = {}
    with open(path) as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Dispatch_Id"]))
        for r in rows:
            name = r["Kernel_Name"]
            key = "eval" if "k_eval" in name else ("copy" if "copyBuffer" in name else None)
            if key:
                out.setdefault(key, []).append(float(r["Counter_Value"]))
    return out


def summarize(fetch_csv: str, write_csv: str) -> str:
    fe, wr = _per_kernel(fetch_csv), _per_kernel(write_csv)
    # the probe's five device copies are the last five copy dispatches (earlier ones move
    # the inputs from the host); their median
    cf = sorted(fe["copy"][-5:])[2]
    cw = sorted(wr["copy"][-5:])[2]
    f_fetch = COPY_BYTES / (cf * 1024.0)
    f_write = COPY_BYTES / (cw * 1024.0)
    ef = sum(fe["eval"]) / len(fe["eval"])
    ew = sum(wr["eval"]) / len(wr["eval"])
    fetch_b = ef * 1024.0 * f_fetch
    write_b = ew * 1024.0 * f_write
    alg = algorithmic_bytes(N, N)
    lines = [
        f"# LSE pass (k_eval), uniform points m = n = {N}, FP64 cost: HBM counters",
        "",
        "Commands (from the repository root, one MI355X; each counter in its own run):",
        "",
        "```",
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d gpurun_out/pmc_fetch -o fetch -- "
        "python3 probe.py",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d gpurun_out/pmc_write -o write -- "
        "python3 probe.py",
        "python3 probe.py --summarize "
        "gpurun_out/pmc_fetch/fetch_counter_collection.csv "
        "gpurun_out/pmc_write/write_counter_collection.csv",
        "```",
        "",
        "| quantity | value |",
        "|---|---:|",
        f"| copy of {COPY_BYTES} B: FETCH_SIZE (KiB) | {cf:.1f} |",
        f"| copy of {COPY_BYTES} B: WRITE_SIZE (KiB) | {cw:.1f} |",
        f"| scale factor FETCH_SIZE -> bytes | {f_fetch:.4f} x 1024 |",
        f"| scale factor WRITE_SIZE -> bytes | {f_write:.4f} x 1024 |",
        f"| eval: FETCH_SIZE per launch (KiB, mean of {len(fe['eval'])}) | {ef:.1f} |",
        f"| eval: WRITE_SIZE per launch (KiB, mean of {len(wr['eval'])}) | {ew:.1f} |",
        f"| eval: HBM bytes fetched per launch | {fetch_b:.4g} |",
        f"| eval: HBM bytes written per launch | {write_b:.4g} |",
        f"| eval: algorithmic bytes per launch | {alg:.4g} |",
        "",
        f"traffic_bytes_per_launch: {fetch_b + write_b:.6e}",
        f"LSE-pass source sha256: {source_hash()}",
        "",
    ]
    return "\n".join(lines)


def read_traffic(md_path: str):
    """Traffic per launch from a summary written by --summarize, or None if the file is
    missing or was made for a different LSE-pass source."""
    if not os.path.exists(md_path):
        return None
    traffic, h = None, None
    with open(md_path) as f:
        for line in f:
            if line.startswith("traffic_bytes_per_launch:"):
                traffic = float(line.split(":", 1)[1])
            elif line.startswith("LSE-pass source sha256:"):
                h = line.split(":", 1)[1].strip()
    if traffic is None or h != source_hash():
        return None
    return traffic


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
