"""Build the surrogate's training set with the exact integral and train the network on the
GPU, then write the weight blob.

    python -m paper_1209_0461_amd.train_surrogate --out paper_1209_0461_amd/data/surrogate_pm256.npy

Prints one JSON line: training loss, held-out (10%) error of y = ln(R (1 + k/k_fs)^2),
which is also the relative error of R, and the time of each phase.
"""
import argparse
import json
import time

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rows", type=int, default=4_000_000)
    ap.add_argument("--epochs", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    import torch
    from . import binding
    from .binding import PMNu
    from .surrogate import build_training_set

    t0 = time.perf_counter()
    x, y = build_training_set(args.rows, seed=args.seed)
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
    loss = binding.pm_nu_surrogate_train(ctx.h, xt, yt, args.epochs, args.batch, args.lr,
                                         args.seed)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pred = torch.empty_like(yh)
    binding.pm_nu_surrogate_predict(ctx.h, xh, pred)
    err = (pred - yh).abs().cpu().numpy().astype(np.float64)
    blob = binding.pm_nu_surrogate_save(ctx.h)
    np.save(args.out, blob)
    ctx.close()
    print(json.dumps({"rows": int(n), "train_rows": int(n - n_hold), "epochs": args.epochs,
                      "train_loss_std": loss, "holdout_max_abs_err_lnR": float(err.max()),
                      "holdout_rms_err_lnR": float(np.sqrt(np.mean(err ** 2))),
                      "holdout_p999_err_lnR": float(np.quantile(err, 0.999)),
                      "dataset_s": t1 - t0, "train_s": t2 - t1, "out": args.out}))


if __name__ == "__main__":
    main()
