"""Training-set construction and training of the surrogate network through the C ABI.

The training rows come from the library's exact history integral (pm_nu_surrogate_dataset
runs it), on the bin geometry and node grid of the 256^3 workload; the network is
trained by the library's own kernels (pm_nu_surrogate_train). This module only moves
arrays between those calls.
"""
import numpy as np

from . import binding
from .binding import PMNu

# the 256^3 workload's geometry and history grid
PM256 = dict(n_mesh=256, box=512.0, n_kbins=64, n_hist=200, a_lo=0.01, a_hi=1.0, substeps=8)


def build_training_set(n_rows, seed=4000, geometry=PM256, boxes_per_batch=16, j_min=120,
                       p_last=0.25, omega_m=0.3, hubble=0.7):
    """Rows (x [n][11], y [n]) as device tensors, at most n_rows, from random histories."""
    import torch
    from synth import log_spaced_nodes
    from synth.history import growth
    from synth.surrogate_cases import surrogate_batch
    g = geometry
    nodes = log_spaced_nodes(g["a_lo"], g["a_hi"], g["n_hist"])
    growth_nodes = growth(nodes, omega_m)
    rng = np.random.default_rng(seed)
    ctx = PMNu(g["n_mesh"], 1, g["box"], g["n_kbins"], g["n_hist"] + 2,
               np.full(boxes_per_batch, 0.3), omega_m=omega_m, hubble=hubble,
               substeps=g["substeps"])
    _, counts, kmean = ctx.bins()
    nb = boxes_per_batch * g["n_kbins"]
    xb = torch.empty((nb, binding.SUR_IN), device="cuda")
    yb = torch.empty(nb, device="cuda")
    xs, ys, have, batches = [], [], 0, 0
    import sys
    import time
    t0 = time.perf_counter()
    while have < n_rows:
        j = g["n_hist"] - 1 if rng.random() < p_last else int(rng.integers(j_min, g["n_hist"]))
        masses, hists, powers = surrogate_batch(kmean, nodes, j, boxes_per_batch, rng,
                                                omega_m, hubble, growth_nodes=growth_nodes)
        for b in range(boxes_per_batch):
            binding.pm_nu_set_mass(ctx.h, b, masses[b])
            ctx.set_history(b, hists[b])
            binding.pm_nu_set_power(ctx.h, b, powers[b])
        binding.pm_nu_surrogate_dataset(ctx.h, nodes[j], xb, yb)
        keep = torch.isfinite(yb)
        xs.append(xb[keep].clone())
        ys.append(yb[keep].clone())
        have += int(keep.sum())
        batches += 1
        if batches % 200 == 0:
            print(f"training set: {have} rows after {batches} batches, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx.close()
    return torch.cat(xs)[:n_rows].contiguous(), torch.cat(ys)[:n_rows].contiguous()


def train(ctx, x, y, epochs=40, batch=4096, lr=2e-3, seed=7, init=True):
    """Initialise (optionally) and train the network of ctx on (x, y); returns the loss."""
    if init:
        binding.pm_nu_surrogate_init(ctx.h, x, y, seed)
    return binding.pm_nu_surrogate_train(ctx.h, x, y, epochs, batch, lr, seed)
