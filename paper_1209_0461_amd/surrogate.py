"""Training-set construction and training of the surrogate network through the C ABI.

The training rows come from the library's exact history integral (pm_nu_surrogate_dataset
runs it), on the bin geometry and node grid of the 256^3 workload; the network is
trained by the library's own kernels (pm_nu_surrogate_train). This module only moves
arrays between those calls.
"""
import numpy as np

from . import binding
from .binding import PMNu

# the 256^3 workload's geometry; the stored histories of the training cases span node
# counts n_hist_range (log-uniform) from a first node in a_lo_range (16 log-spaced values)
# to a_hi, so that the network sees a range of spacings of the stored nodes
PM256 = dict(n_mesh=256, box=512.0, n_kbins=64, n_hist_range=(40, 400),
             a_lo_range=(0.005, 0.03), a_hi=1.0, substeps=8)
LAG_MAX = 2.1   # the inputs' longest lag in ln a below the last stored node


def build_training_set(n_rows, seed=4000, geometry=PM256, boxes_per_batch=16, p_last=0.25,
                       omega_m=0.3, hubble=0.7):
    """Rows (x [n][16], y [n]) as device tensors, at most n_rows, from random histories: per
    batch a node count and a first node drawn log-uniformly, and the current node anywhere
    from where the inputs exist to the last node (the last one with probability p_last)."""
    import torch
    from synth import log_spaced_nodes
    from synth.history import growth
    from synth.surrogate_cases import surrogate_batch
    g = geometry
    rng = np.random.default_rng(seed)
    j_lo, j_hi = g["n_hist_range"]
    ctx = PMNu(g["n_mesh"], 1, g["box"], g["n_kbins"], j_hi + 2,
               np.full(boxes_per_batch, 0.3), omega_m=omega_m, hubble=hubble,
               substeps=g["substeps"])
    grids = {}
    _, counts, kmean = ctx.bins()
    nb = boxes_per_batch * g["n_kbins"]
    xb = torch.empty((nb, binding.SUR_IN), device="cuda")
    yb = torch.empty(nb, device="cuda")
    xs, ys, have, batches = [], [], 0, 0
    import sys
    import time
    t0 = time.perf_counter()
    while have < n_rows:
        n_hist = int(round(np.exp(rng.uniform(np.log(j_lo), np.log(j_hi)))))
        a_lo = float(np.geomspace(*g["a_lo_range"], 16)[rng.integers(16)])
        key = (n_hist, a_lo)
        if key not in grids:
            nd = log_spaced_nodes(a_lo, g["a_hi"], n_hist)
            grids[key] = (nd, growth(nd, omega_m))
        nodes, growth_nodes = grids[key]
        step = np.log(nodes[1] / nodes[0])
        j_min = int(np.ceil(LAG_MAX / step)) + 2     # the last stored node j - 1 reaches back
        if j_min >= n_hist:
            continue
        j = n_hist - 1 if rng.random() < p_last else int(rng.integers(j_min, n_hist))
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


def build_loop_rows(seeds, masses, step_counts, a_i=0.02, sigma=0.1, geometry=PM256,
                    omega_m=0.3):
    """Rows (x, y) from the history that the time-stepping loop of Sec. 4.3 itself stores:
    for every seed one set of 2LPT initial conditions of the workload's particle count at
    a_i, then for every mass and step count a run from a_i to 1 (log-spaced steps, exact
    response), with the rows of every step whose stored history reaches the inputs' last
    lag. Synthetic histories miss how a particle run's measured amplitudes grow (mode
    coupling at low k, the mesh's own growth beyond its Nyquist frequency); these rows
    carry it."""
    import sys
    import torch
    from synth import zeldovich_ics
    from synth.history import free_streaming_k, growth, hubble_rate
    g = geometry
    n_side = g["n_mesh"]
    f_i = float(growth(np.array([a_i]), omega_m)[1][0])
    n_max = max(step_counts) + 4
    ctx = None
    xs, ys = [], []
    for seed in seeds:
        pos0, vel0 = zeldovich_ics(n_side, g["box"], sigma, seed, a_i, second_order=True)
        if ctx is None:
            ctx = PMNu(g["n_mesh"], pos0.shape[0], g["box"], g["n_kbins"], n_max, [masses[0]],
                       omega_m=omega_m, substeps=g["substeps"])
            _, counts, kmean = ctx.bins()
            ok = counts > 0
            B = g["n_kbins"]
            xb = torch.empty((B, binding.SUR_IN), device="cuda")
            yb = torch.empty(B, device="cuda")
        p0 = torch.from_numpy(pos0).cuda()
        v0 = torch.from_numpy(vel0).cuda()
        for mass in masses:
            binding.pm_nu_set_mass(ctx.h, 0, float(mass))
            fn = mass / (93.14 * omega_m * 0.49)
            for n_steps in step_counts:
                steps = np.geomspace(a_i, 1.0, n_steps + 1)
                p, v = p0.clone(), v0.clone()
                acc = torch.zeros_like(p)
                ctx.deposit(p)
                pc = np.sqrt(ctx.spectrum(0)["p_cdm"])
                rnu = np.where(ok, 1.0 / (1.0 + np.where(ok, kmean, 1.0)
                                          / free_streaming_k(a_i, mass / 3, omega_m)) ** 2, 0.0)
                pnu = pc * rnu
                theta = np.full(B, -f_i * a_i * hubble_rate(a_i, omega_m))
                ctx.set_history(0, dict(a=np.array([a_i]), pm_half=((1 - fn) * pc + fn * pnu)[None],
                                        pnu_half=pnu[None], pnu_half_init=pnu,
                                        theta_over_delta_init=theta))
                ctx.step(p, acc, a_i)
                for j in range(1, n_steps + 1):
                    ctx.advance(p, v, acc, steps[j - 1:j + 1])
                    if np.log(steps[j - 1] / a_i) < LAG_MAX:
                        continue
                    ctx.deposit(p)
                    binding.pm_nu_surrogate_dataset(ctx.h, steps[j], xb, yb)
                    keep = torch.isfinite(yb)
                    xs.append(xb[keep].clone())
                    ys.append(yb[keep].clone())
            print(f"loop rows: seed {seed}, M_nu {mass:.3f}: {sum(len(t) for t in ys)} rows",
                  file=sys.stderr, flush=True)
    if ctx is not None:
        ctx.close()
    return torch.cat(xs).contiguous(), torch.cat(ys).contiguous()


def train(ctx, x, y, epochs=40, batch=4096, lr=2e-3, seed=7, init=True):
    """Initialise (optionally) and train the network of ctx on (x, y); returns the loss."""
    if init:
        binding.pm_nu_surrogate_init(ctx.h, x, y, seed)
    return binding.pm_nu_surrogate_train(ctx.h, x, y, epochs, batch, lr, seed)
