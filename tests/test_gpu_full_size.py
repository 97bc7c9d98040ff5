"""Parity at the workloads' full sizes, in the launch configuration the benchmark times.

* pm256: 256^3 particles on a 256^3 mesh (Morton order, autotuned launch shapes) at each of
  the workload's three neutrino masses, compared with the full FP64 oracle step (every
  bin, every particle).
* batch64x64: 64 boxes of 64^3 particles with different masses and seeds, stepped by a
  captured HIP graph; every box compared with the oracle.
* pm512: 512^3 particles on a 512^3 mesh (autotuned), against the oracle's results stored
  by tests/golden/make_pm512_oracle.py: every bin, 16384 sampled particles and 4096 sampled
  nodes of the acceleration grids; the deposit must take the patch path throughout.
* N = 512 mesh with 64^3 particles: chunks far larger than any LDS tile, so the patch
  deposit's side grid and the direct gather carry the whole step.
"""
import json
import os

import numpy as np
import pytest

from gpu_cases import TOL_FORCE_RMS, TOL_NU, rms_rel

pytestmark = pytest.mark.gpu


def _hist_from_oracle(pos, n_mesh, box, nb, nodes, m):
    import oracle.step as ostep
    from synth import synthetic_history
    sp = ostep.spectrum(pos, n_mesh, box, nb)
    return synthetic_history(sp["k_mean"], np.sqrt(sp["p_cdm"]), nodes, m)


def _compare(gpu_acc, sp, ref, label):
    ok = ref["counts"] > 0
    prel = np.abs(sp["p_cdm"][ok] / ref["p_cdm"][ok] - 1.0).max()
    nrel = np.abs(sp["pnu_half"][ok] / ref["pnu_half"][ok] - 1.0).max()
    ferr = rms_rel(gpu_acc, ref["acc"])
    print(f"{label}: P_cdm {prel:.2e}  P_nu^1/2 {nrel:.2e}  force rms {ferr:.2e}", flush=True)
    assert prel <= 2e-6, label
    assert nrel <= TOL_NU, label
    assert ferr <= TOL_FORCE_RMS, label


@pytest.mark.parametrize("m,seed", [(0.15, 256), (0.3, 257), (0.6, 258)])
def test_pm256_full_step_matches_oracle(m, seed):
    import torch
    import oracle.step as ostep
    from paper_1209_0461_amd import PMNu, binding
    from synth import CONFIGS, log_spaced_nodes, zeldovich_lattice
    cfg = CONFIGS["pm256"]
    print(f"pm256 M_nu={m} seed={seed}", flush=True)
    pos = zeldovich_lattice(256, cfg["box"], cfg["sigma_cells"], seed)
    nodes = log_spaced_nodes(cfg["a_lo"], cfg["a_now"], cfg["n_hist"])
    hist = _hist_from_oracle(pos, 256, cfg["box"], cfg["n_kbins"], nodes, m)
    ref = ostep.full_step(pos, 256, cfg["box"], cfg["n_kbins"], hist, cfg["a_now"], m,
                          substeps=cfg["substeps"])
    ctx = PMNu(256, pos.shape[0], cfg["box"], cfg["n_kbins"], cfg["n_hist"] + 2, [m])
    ctx.set_history(0, hist)
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    binding.pm_nu_autotune(ctx.h, p, acc, cfg["a_now"])   # leaves the node a_now computed
    binding.pm_nu_side_grid_uses(ctx.h)
    ctx.step(p, acc, cfg["a_now"])
    torch.cuda.synchronize()
    _compare(acc.cpu().numpy(), ctx.spectrum(0), ref, f"pm256 M_nu={m}")
    if json.loads(binding.pm_nu_tuning(ctx.h))["deposit_mode"] >= 6:
        assert binding.pm_nu_side_grid_uses(ctx.h) == 0    # every chunk through its patch
    ctx.close()


def test_batched_boxes_through_a_graph_match_oracle():
    import torch
    import oracle.step as ostep
    from paper_1209_0461_amd import PMNu, binding
    from synth import CONFIGS, batched_lattices, log_spaced_nodes
    cfg = CONFIGS["batch64x64"]
    pos, masses = batched_lattices(cfg)
    nb, n_mesh, box = cfg["n_kbins"], cfg["n_mesh"], cfg["box"]
    nodes = log_spaced_nodes(cfg["a_lo"], cfg["a_now"], cfg["n_hist"])
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = PMNu(n_mesh, pos.shape[1], box, nb, cfg["n_hist"] + 2, masses)
        p = torch.from_numpy(pos).cuda()
        acc = torch.zeros_like(p)
        hists = [_hist_from_oracle(pos[b], n_mesh, box, nb, nodes, masses[b])
                 for b in range(len(masses))]
        for b, h in enumerate(hists):
            ctx.set_history(b, h)
        binding.pm_nu_graph_capture(ctx.h, p, acc, cfg["a_now"])
        for _ in range(3):
            binding.pm_nu_graph_launch(ctx.h)
        stream.synchronize()
        got = acc.cpu().numpy()
        for b in range(len(masses)):
            ref = ostep.full_step(pos[b], n_mesh, box, nb, hists[b], cfg["a_now"],
                                  float(masses[b]), substeps=cfg["substeps"])
            _compare(got[b], ctx.spectrum(b), ref, f"box {b} (M_nu={masses[b]:.3f})")
    ctx.close()


def test_mesh_512_code_path_matches_oracle():
    import torch
    import oracle.step as ostep
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, zeldovich_lattice
    n_mesh, box, nb, m = 512, 1000.0, 128, 0.3
    pos = zeldovich_lattice(64, box, 0.3, 512)
    nodes = log_spaced_nodes(0.01, 1.0, 60)
    hist = _hist_from_oracle(pos, n_mesh, box, nb, nodes, m)
    ref = ostep.full_step(pos, n_mesh, box, nb, hist, 1.0, m)
    ctx = PMNu(n_mesh, pos.shape[0], box, nb, 64, [m])
    ctx.set_history(0, hist)
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    ctx.step(p, acc, 1.0)
    torch.cuda.synchronize()
    assert binding.pm_nu_side_grid_uses(ctx.h) > 0        # chunks far wider than a tile
    _compare(acc.cpu().numpy(), ctx.spectrum(0), ref, "N=512")
    ctx.close()


GOLD512 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pm512_oracle.npz")


def test_pm512_full_step_matches_stored_oracle():
    import hashlib
    import torch
    from paper_1209_0461_amd import PMNu, binding
    from synth import CONFIGS, log_spaced_nodes, synthetic_history, zeldovich_lattice
    g = np.load(GOLD512)
    c = CONFIGS["pm512"]
    n, box, nb, J, m = c["n_mesh"], c["box"], c["n_kbins"], c["n_hist"], c["m_nu"][0]
    print(f"pm512: {c['n_side']}^3 particles, seed {c['seeds'][0]}", flush=True)
    pos = zeldovich_lattice(c["n_side"], box, c["sigma_cells"], c["seeds"][0])
    assert hashlib.sha256(pos.tobytes()).hexdigest() == str(g["pos_sha256"]), \
        "the regenerated input differs from the one the stored oracle results were made from"
    nodes = log_spaced_nodes(c["a_lo"], c["a_now"], J)
    hist = synthetic_history(g["k_mean"], np.sqrt(g["p_cdm"]), nodes, m)
    ctx = PMNu(n, pos.shape[0], box, nb, J + 2, [m], substeps=c["substeps"])
    edges, counts, kmean = ctx.bins()
    assert np.array_equal(edges, g["edges"]) and np.array_equal(counts, g["counts"])
    ctx.set_history(0, hist)
    p = torch.from_numpy(pos).cuda()
    del pos
    acc = torch.zeros_like(p)
    binding.pm_nu_autotune(ctx.h, p, acc, c["a_now"])   # leaves the node a_now computed
    tuning = json.loads(binding.pm_nu_tuning(ctx.h))
    binding.pm_nu_side_grid_uses(ctx.h)
    ctx.step(p, acc, c["a_now"])
    grid = torch.empty(n ** 3, device="cuda")
    gsample = []
    idx = torch.from_numpy(g["node_index"]).cuda()
    for ax in range(3):
        binding.pm_nu_copy_force_grid(ctx.h, 0, ax, grid)
        gsample.append(grid[idx].double().cpu().numpy())
    torch.cuda.synchronize()
    sp = ctx.spectrum(0)
    a_np = acc[torch.from_numpy(g["particle_index"]).cuda()].double().cpu().numpy()
    _, hpm, _ = ctx.history(0)
    uses = binding.pm_nu_side_grid_uses(ctx.h)
    ctx.close()
    ok = g["counts"] > 0
    prel = np.abs(sp["p_cdm"][ok] / g["p_cdm"][ok] - 1.0).max()
    nrel = np.abs(sp["pnu_half"][ok] / g["pnu_half"][ok] - 1.0).max()
    rrel = np.abs(sp["ratio"][ok] / g["ratio"][ok] - 1.0).max()
    hrel = np.abs(hpm[-1][ok] / g["pm_half_now"][ok] - 1.0).max()
    ferr = rms_rel(a_np, g["acc"])
    gerr = rms_rel(np.stack(gsample, 1), g["grid"])
    print(f"pm512 {tuning}: P_cdm {prel:.2e} P_nu^1/2 {nrel:.2e} R {rrel:.2e} node {hrel:.2e} "
          f"force rms {ferr:.2e} (16384 particles) grids {gerr:.2e} (4096 nodes) "
          f"side-grid uses {uses}", flush=True)
    assert len(hpm) == J
    assert prel <= 2e-6 and rrel <= 2e-5 and hrel <= 2e-6
    assert nrel <= TOL_NU
    assert ferr <= TOL_FORCE_RMS and gerr <= TOL_FORCE_RMS
    if tuning["deposit_mode"] >= 6:
        assert uses == 0, "a 512^3 lattice chunk left the patch path"
