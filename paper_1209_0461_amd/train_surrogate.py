"""Build the surrogate's training set with the exact integral and train the network on the
GPU, then write the weight blob.

    python -m paper_1209_0461_amd.train_surrogate --out paper_1209_0461_amd/data/surrogate_pm256.npy

Prints one JSON line: training loss, held-out (10%) error of y = ln(R (1 + k/k_fs)^2),
which is also the relative error of R (maximum, RMS, 99.9th percentile, and the 99.9th
percentile per range of ln k), and the time of each phase.
"""
import argparse
import json
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rows", type=int, default=8_000_000)
    ap.add_argument("--epochs", type=int, default=1000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--chunk", type=int, default=50, help="epochs per training call")
    ap.add_argument("--loop-seeds", default="7001,7002,7003",
                    help="seeds of particle runs whose stored histories add rows (empty: none)")
    ap.add_argument("--loop-masses", default="0.04,0.1,0.2,0.3,0.45,0.6,0.7")
    ap.add_argument("--loop-steps", default="32,40,56,72")
    ap.add_argument("--loop-repeat", type=int, default=8,
                    help="copies of the loop rows in the training set (their weight)")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    import torch
    from . import binding
    from .binding import PMNu
    from .surrogate import build_loop_rows, build_training_set

    t0 = time.perf_counter()
    x, y = build_training_set(args.rows, seed=args.seed)
    n_loop = 0
    if args.loop_seeds:
        xl, yl = build_loop_rows([int(v) for v in args.loop_seeds.split(",")],
                                 [float(v) for v in args.loop_masses.split(",")],
                                 [int(v) for v in args.loop_steps.split(",")])
        n_loop = int(xl.shape[0])
        x = torch.cat([x] + [xl] * args.loop_repeat)
        y = torch.cat([y] + [yl] * args.loop_repeat)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n = x.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(args.seed)
    order = torch.randperm(n, generator=gen).cuda()
    n_hold = n // 10
    xh, yh = x[order[:n_hold]].contiguous(), y[order[:n_hold]].contiguous()
    xt, yt = x[order[n_hold:]].contiguous(), y[order[n_hold:]].contiguous()
    ctx = PMNu(16, 8, 64.0, 8, 16, [0.3])
    binding.pm_nu_surrogate_init(ctx.h, xt, yt, args.seed)
    import sys
    done, loss = 0, float("nan")
    while done < args.epochs:               # in parts, with a progress line after each
        part = min(args.chunk, args.epochs - done)
        loss = binding.pm_nu_surrogate_train_part(ctx.h, xt, yt, done, part, args.epochs,
                                                  args.batch, args.lr, args.seed)
        done += part
        print(f"epoch {done}/{args.epochs}: loss {loss:.3e} ({time.perf_counter() - t1:.0f} s)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pred = torch.empty_like(yh)
    binding.pm_nu_surrogate_predict(ctx.h, xh, pred)
    err = (pred - yh).abs().cpu().numpy().astype(np.float64)
    lnk = xh[:, 0].cpu().numpy()
    edges = np.linspace(np.floor(lnk.min()), np.ceil(lnk.max()), 9)
    per_k = {}
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (lnk >= lo) & (lnk < hi)
        if sel.sum() > 100:
            per_k[f"[{lo:.2f},{hi:.2f})"] = float(np.quantile(err[sel], 0.999))
    blob = binding.pm_nu_surrogate_save(ctx.h)
    np.save(args.out, blob)
    ctx.close()
    print(json.dumps({"rows": int(n), "loop_rows": n_loop, "loop_repeat": args.loop_repeat,
                      "train_rows": int(n - n_hold), "epochs": args.epochs,
                      "train_loss_std": loss, "holdout_max_abs_err_lnR": float(err.max()),
                      "holdout_rms_err_lnR": float(np.sqrt(np.mean(err ** 2))),
                      "holdout_p999_err_lnR": float(np.quantile(err, 0.999)),
                      "holdout_p999_by_lnk": per_k,
                      "dataset_s": t1 - t0, "train_s": t2 - t1, "out": args.out}))


if __name__ == "__main__":
    main()
