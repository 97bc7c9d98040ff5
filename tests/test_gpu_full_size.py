"""Parity at the workloads' full sizes, in the launch configuration the benchmark times.

* pm256: 256^3 particles on a 256^3 mesh (Morton order, autotuned launch shapes), compared
  element by element with the full FP64 oracle step.
* batch64x64: 64 boxes of 64^3 particles with different masses and seeds, stepped by a
  captured HIP graph; four sampled boxes compared with the oracle.
* N = 512 mesh: the 512-point radix plan and tile shapes, with 64^3 particles.
"""
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


def test_pm256_full_step_matches_oracle():
    import torch
    import oracle.step as ostep
    from paper_1209_0461_amd import PMNu, binding
    from synth import CONFIGS, log_spaced_nodes, zeldovich_lattice
    cfg = CONFIGS["pm256"]
    m, seed = 0.3, 257
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
    ctx.step(p, acc, cfg["a_now"])
    torch.cuda.synchronize()
    _compare(acc.cpu().numpy(), ctx.spectrum(0), ref, "pm256")
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
        for b in (0, 17, 40, 63):
            ref = ostep.full_step(pos[b], n_mesh, box, nb, hists[b], cfg["a_now"],
                                  float(masses[b]), substeps=cfg["substeps"])
            _compare(got[b], ctx.spectrum(b), ref, f"box {b} (M_nu={masses[b]:.3f})")
    ctx.close()


def test_mesh_512_code_path_matches_oracle():
    import torch
    import oracle.step as ostep
    from paper_1209_0461_amd import PMNu
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
    _compare(acc.cpu().numpy(), ctx.spectrum(0), ref, "N=512")
    ctx.close()
