"""Train the learned warm start (ibsn_ws_*) on pairs the solver generates.

    python -m paper_2603_07156_amd.train_warmstart --train 192 --out warmstart.npz

Instances: uniform points in [0,1]^2 on both sides with uniform weights (the generator of the
small configuration), m = n = --n (1024), eta = --eta; training seeds 10000.., validation
seeds 900000...  Target of each instance: the dual gamma of its first proximal subproblem
(ibsn_solve with one outer iteration from gamma = 0, centred), divided by the instance's
scale (ibsn_ws_features: u s, the cost of the typical nearest-source distance), the unit
the network predicts in.  Training: Adam on the per-instance centred squared error, batches
of --batch instances, cosine learning-rate decay.
Everything runs in the library's kernels (the solver for the targets, the BF16 MFMA network
for the features, the forward and backward passes); this script only drives them.
The parameters are written as a NumPy .npz (keys: params, eta, n, train, val_loss, val_r2).
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def make_pairs(ib, ctx, n, eta, seeds, contexts):
    """Features and targets of the instances with these seeds: (fs, fte, fth, target, scale)
    device tensors stacked by instance."""
    import numpy as np
    import torch

    from paper_2603_07156_amd import workloads

    dev = torch.device("cuda", 0)
    probs, pts = [], []
    for s in seeds:
        inst = workloads.uniform_points(n, s, eta=eta)
        probs.append(ib.Problem(torch.from_numpy(inst.C).to(dev), torch.from_numpy(inst.a).to(dev),
                                torch.from_numpy(inst.b).to(dev), eta))
        pts.append((torch.from_numpy(np.ascontiguousarray(inst.x)).to(dev),
                    torch.from_numpy(np.ascontiguousarray(inst.y)).to(dev)))
    opt = ib.default_options(max_outer=1, gap_tol=0.0, marg_tol=0.0)
    outs = ib.solve_batch(contexts, probs, opt)
    ws = ib.WarmStart(ctx, seed=0)   # only its feature kernel is used here
    F, T, S = [], [], []
    for pr, (x, y), o in zip(probs, pts, outs):
        if o["status"] < 0:
            raise RuntimeError(f"solve failed: {o['status']}")
        fs, fte, fth, scale = ws.features(pr, x, y)
        g = o["gamma"]
        T.append(((g - g.mean()) / scale).to(torch.float32))
        F.append((fs, fte, fth))
        S.append(scale)
    ws.free()
    fs = torch.cat([f[0] for f in F])
    fte = torch.cat([f[1] for f in F])
    fth = torch.cat([f[2] for f in F])
    return fs, fte, fth, torch.cat(T), S


def evaluate(ws, data, n, B):
    """Mean loss and the fraction of the target variance explained (R^2) over the set."""
    import torch
    fs, fte, fth, tg, _ = data
    cnt = tg.numel() // n
    sse, sst = 0.0, 0.0
    for b0 in range(0, cnt, B):
        bb = min(B, cnt - b0)
        o = ws.forward(bb, n, n, fs[b0 * n:(b0 + bb) * n], fte[b0 * n:(b0 + bb) * n],
                       fth[b0 * n:(b0 + bb) * n]).double().view(bb, n)
        t = tg[b0 * n:(b0 + bb) * n].double().view(bb, n)
        oc = o - o.mean(1, keepdim=True)
        sse += float(((oc - t) ** 2).sum())
        sst += float((t ** 2).sum())
    return sse / (cnt * n), 1.0 - sse / sst


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--eta", type=float, default=1e-6)
    ap.add_argument("--train", type=int, default=192)
    ap.add_argument("--val", type=int, default=16)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--contexts", type=int, default=4)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=os.path.join(HERE, "warmstart_uniform_eta1e-6.npz"))
    args = ap.parse_args()

    import numpy as np
    import torch

    from paper_2603_07156_amd import ibsn as ib

    ctx = ib.Context(0)
    ctxs = [ib.Context(0, stream=torch.cuda.Stream()) for _ in range(args.contexts)]
    t0 = time.time()
    train, chunk = [], 32
    for c0 in range(0, args.train, chunk):
        seeds = range(10000 + c0, 10000 + min(args.train, c0 + chunk))
        train.append(make_pairs(ib, ctx, args.n, args.eta, seeds, ctxs))
        print(f"pairs {min(args.train, c0 + chunk)}/{args.train} {time.time() - t0:.1f}s",
              flush=True)
    train = tuple(torch.cat([d[i] for d in train]) for i in range(4)) + (
        sum((d[4] for d in train), []),)
    val = make_pairs(ib, ctx, args.n, args.eta, range(900000, 900000 + args.val), ctxs)
    print(f"data ready {time.time() - t0:.1f}s", flush=True)

    ws = ib.WarmStart(ctx, seed=args.seed)
    n, B = args.n, args.batch
    rng = np.random.default_rng(args.seed)
    fs, fte, fth, tg, _ = train
    cnt = tg.numel() // n
    for step in range(args.steps):
        idx = torch.from_numpy(rng.choice(cnt, B, replace=False)).to(fs.device)
        rows = (idx[:, None] * n + torch.arange(n, device=fs.device)[None]).reshape(-1)
        lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / args.steps))
        loss, _ = ws.train_step(B, n, n, fs[rows].contiguous(), fte[rows].contiguous(),
                                fth[rows].contiguous(), tg[rows].contiguous(), lr)
        if step % 250 == 0 or step == args.steps - 1:
            vl, r2 = evaluate(ws, val, n, B)
            print(f"step {step} lr {lr:.2e} loss {loss:.4g} val_loss {vl:.4g} val_r2 {r2:.4f} "
                  f"{time.time() - t0:.1f}s", flush=True)
    vl, r2 = evaluate(ws, val, n, B)
    np.savez(args.out, params=ws.params(), eta=args.eta, n=args.n, train=args.train,
             val_loss=vl, val_r2=r2)
    print(f"saved {args.out}: val_loss {vl:.4g} val_r2 {r2:.4f}", flush=True)
    ws.free()
    for c in ctxs:
        c.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
