"""Shared driver of the GPU parity tests: run one configuration through the C ABI and
through the FP64 oracle on the same seeded inputs."""
import numpy as np

from synth import log_spaced_nodes, synthetic_history, zeldovich_lattice

TOL_FORCE_RMS = 1e-4      # force RMS relative error
TOL_NU = 1e-6             # P_nu^{1/2} max relative error over non-empty bins


def rms_rel(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.sum((np.asarray(got, np.float64) - ref) ** 2) / np.sum(ref ** 2)))


def edge_positions(box, n_mesh):
    """Coordinates on nodes, at 0, just below L, and outside [0, L) (wrapped)."""
    cell = box / n_mesh
    L = np.float32(box)
    below = np.nextafter(L, np.float32(0))
    pts = [[0.0, 0.0, 0.0], [below, below, below], [cell, 2 * cell, 3 * cell],
           [-0.3 * cell, 0.5 * box, 0.25 * box], [box + 0.7 * cell, 1.5 * cell, -2.2 * cell],
           [0.5 * cell, below, 0.0]]
    return np.asarray(pts, dtype=np.float32)


def make_inputs(n_side, box, sigma, seed, extra_random=0, edges=False, n_mesh=None):
    pos = zeldovich_lattice(n_side, box, sigma, seed)
    parts = [pos]
    if extra_random:
        rng = np.random.default_rng(seed + 12345)
        parts.append(rng.uniform(0, box, size=(extra_random, 3)).astype(np.float32))
    if edges:
        parts.append(edge_positions(box, n_mesh or n_side))
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def oracle_case(pos, n_mesh, box, nb, J, a_lo, a_now, m_nu, Q=8, iters=1, deconv=True):
    import oracle.step as ostep
    nodes = log_spaced_nodes(a_lo, a_now, J)
    sp = ostep.spectrum(pos, n_mesh, box, nb)
    hist = synthetic_history(sp["k_mean"], np.sqrt(sp["p_cdm"]), nodes, m_nu)
    ref = ostep.full_step(pos, n_mesh, box, nb, hist, a_now, m_nu, substeps=Q,
                          iterations=iters, deconvolve=deconv, return_grids=True)
    return hist, ref


def gpu_case(pos_boxes, n_mesh, box, nb, J, a_now, masses, hists, Q=8, iters=1, deconv=True,
             want_modes=True):
    """Run deposit/response/force through the C ABI; pos_boxes (n_boxes, Np, 3)."""
    import torch
    from paper_1209_0461_amd import PMNu, binding
    nbox, npart = pos_boxes.shape[0], pos_boxes.shape[1]
    ctx = PMNu(n_mesh, npart, box, nb, J + 4, masses, substeps=Q, iterations=iters,
               deconvolve=deconv)
    for b in range(nbox):
        ctx.set_history(b, hists[b])
    p = torch.from_numpy(np.ascontiguousarray(pos_boxes)).cuda()
    acc = torch.zeros_like(p)
    out = {"boxes": []}
    ctx.deposit(p)
    m = n_mesh ** 3
    rho = [torch.empty(m, device="cuda") for _ in range(nbox)]
    modes = [torch.empty(n_mesh * n_mesh * (n_mesh // 2 + 1) * 2, device="cuda")
             for _ in range(nbox)] if want_modes else None
    for b in range(nbox):
        binding.pm_nu_copy_density(ctx.h, b, rho[b])
        if want_modes:
            binding.pm_nu_copy_modes(ctx.h, b, modes[b])
    ctx.response(a_now)
    ctx.force(p, acc, a_now)
    grids = [[torch.empty(m, device="cuda") for _ in range(3)] for _ in range(nbox)]
    for b in range(nbox):
        for ax in range(3):
            binding.pm_nu_copy_force_grid(ctx.h, b, ax, grids[b][ax])
    torch.cuda.synchronize()
    accn = acc.cpu().numpy()
    for b in range(nbox):
        sp = ctx.spectrum(b)
        a, pm, pn = ctx.history(b)
        d = dict(rho=rho[b].cpu().numpy().reshape((n_mesh,) * 3), acc=accn[b],
                 grids=np.stack([g.cpu().numpy().reshape((n_mesh,) * 3) for g in grids[b]]),
                 hist_a=a, hist_pm=pm, hist_pnu=pn, **sp)
        if want_modes:
            mm = modes[b].cpu().numpy().reshape(n_mesh, n_mesh, n_mesh // 2 + 1, 2)
            d["modes"] = mm[..., 0] + 1j * mm[..., 1]
        out["boxes"].append(d)
    out["bins"] = ctx.bins()
    ctx.close()
    return out
