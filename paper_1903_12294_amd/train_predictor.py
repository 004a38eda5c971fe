"""Train the brick-activity predictor on masks the plain grower produces.

    python -m paper_1903_12294_amd.train_predictor --out paper_1903_12294_amd/predictor.npy

Variants are the 128^3 x 32 workload (16 moving blobs, 262,144 particles,
8 seeds) regenerated with data seeds 1000..1199; the first 180 train, the last
20 validate.  Each variant is grown by the plain GPU grower; its brick-step
labels ("holds a member") and the network inputs come from the library.
Training is Adam in the library's kernels, one variant per step, fixed order.

Writes the fp32 parameters (.npy, no pickle) and a JSON record beside them
with the losses, the validation precision / recall at the chosen logit
threshold, and the seeds.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def evaluate(net, data, thr: float) -> dict:
    """Precision / recall of 'logit >= thr' against the brick labels."""
    tp = fp = fn = 0
    for x, y in data:
        z = net.forward(x)
        p = z >= thr
        yb = y.bool()
        tp += int((p & yb).sum())
        fp += int((p & ~yb).sum())
        fn += int((~p & yb).sum())
    return dict(precision=tp / max(tp + fp, 1), recall=tp / max(tp + fn, 1), tp=tp, fp=fp, fn=fn)


def choose_threshold(net, data, min_recall: float) -> float:
    """Largest logit threshold whose validation recall stays >= min_recall."""
    import torch
    zs, ys = [], []
    for x, y in data:
        zs.append(net.forward(x).flatten())
        ys.append(y.flatten().bool())
    z = torch.cat(zs)
    y = torch.cat(ys)
    pos = z[y].sort().values
    if pos.numel() == 0:
        return 0.0
    k = int(np.floor((1.0 - min_recall) * pos.numel()))
    return float(pos[min(k, pos.numel() - 1)].item())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--variants", type=int, default=200)
    ap.add_argument("--val", type=int, default=20)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--min-recall", type=float, default=0.995)
    ap.add_argument("--init-seed", type=int, default=0)
    args = ap.parse_args()

    import torch

    from .learned import Net, init_params, make_dataset, train

    seeds = list(range(args.seed0, args.seed0 + args.variants))
    t0 = time.time()
    data = make_dataset(seeds, config=2, log=lambda m: log(f"[data] {m}"))
    log(f"[data] {len(data)} variants in {time.time() - t0:.1f}s")
    tr, va = data[:-args.val], data[-args.val:]
    net = Net(0)
    try:
        net.set_params(init_params(args.init_seed))
        hist = train(net, tr, epochs=args.epochs, lr=args.lr,
                     log=lambda m: log(f"[train] {m}"))
        torch.cuda.synchronize()
        thr = choose_threshold(net, va, args.min_recall)
        ev_val = evaluate(net, va, thr)
        ev_train = evaluate(net, tr, thr)
        params = net.get_params()
    finally:
        net.close()
    np.save(args.out, params.astype(np.float32), allow_pickle=False)
    pos = sum(int(y.sum()) for _, y in data)
    tot = sum(y.numel() for _, y in data)
    rec = dict(workload="128^3 x 32, 16 blobs, 262144 particles, 8 seeds, thresholds 0.3/0.3",
               seeds=[seeds[0], seeds[-1]], n_train=len(tr), n_val=len(va), epochs=args.epochs,
               lr=args.lr, init_seed=args.init_seed, positive_fraction=pos / tot,
               loss_first=hist[0], loss_last=hist[-1], logit_threshold=thr,
               min_recall=args.min_recall, val=ev_val, train_metrics=ev_train,
               seconds=round(time.time() - t0, 1))
    with open(os.path.splitext(args.out)[0] + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    log(f"[done] threshold {thr:.4f} val {ev_val} loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
