"""Parity on self-consistent stored histories (the loop of Sec. 4.3 (iii)-(iv)).

The library grows the history node by node: the CDM amplitude of node j is handed over
with pm_nu_set_power and pm_nu_response at a_j computes P_nu^{1/2}(a_j) from the earlier
nodes by eq. (P-final) and stores P_M^{1/2} = (1 - f_nu) P_cdm^{1/2} + f_nu P_nu^{1/2}.
The oracle replays the same nodes (oracle.response.replay_history). Every stored row is
compared, then one full step on the grown history.

Inputs: the oracle's binned P_cdm of the particles scaled by the linear growth factor to
every node (synth.growth_history), the initial neutrino amplitude of Appendix A
(synth.free_streaming_ic) and the growing-mode [theta/delta]_i.

Also: a lattice with no displacement has P_cdm = 0 in every bin; with neutrinos the
history still gives P_nu != 0, and the force must come out exactly zero.
"""
import numpy as np
import pytest

from gpu_cases import TOL_FORCE_RMS, TOL_NU, rms_rel

pytestmark = pytest.mark.gpu


def _replayed_case(pos, n_mesh, box, nb, J, a_lo, a_now, m, Q=8, label=""):
    import torch
    import oracle.step as ostep
    from oracle.response import replay_history
    from paper_1209_0461_amd import PMNu, binding
    from synth import free_streaming_ic, growth_history, log_spaced_nodes

    print(f"{label}: N={n_mesh} np={pos.shape[0]} B={nb} J={J} M_nu={m}", flush=True)
    nodes = log_spaced_nodes(a_lo, a_now, J)
    sp = ostep.spectrum(pos, n_mesh, box, nb)
    k, counts = sp["k_mean"], sp["counts"]
    cdm, theta = growth_history(np.sqrt(sp["p_cdm"]), nodes)
    ic = free_streaming_ic(k, cdm[0], nodes[0], m)
    # oracle: replay of the stored nodes, then the step at a_now on that history
    pm, pnu = replay_history(k, counts, cdm[:-1], nodes[:-1], ic, theta, m, 0.3, 0.7, Q)
    hist = dict(a=nodes[:-1], pm_half=pm, pnu_half=pnu, pnu_half_init=ic,
                theta_over_delta_init=theta)
    ref = ostep.full_step(pos, n_mesh, box, nb, hist, a_now, m, substeps=Q)

    # library: start a run at a_i (one node, recomputed from the initial amplitude), then
    # one response per stored node from its CDM amplitude
    ctx = PMNu(n_mesh, pos.shape[0], box, nb, J + 2, [m], substeps=Q)
    ctx.set_history(0, dict(a=nodes[:1], pm_half=np.zeros((1, nb)), pnu_half=ic[None, :],
                            pnu_half_init=ic, theta_over_delta_init=theta))
    for j in range(J - 1):
        binding.pm_nu_set_power(ctx.h, 0, cdm[j] ** 2)
        ctx.response(nodes[j])
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    ctx.step(p, acc, a_now)
    torch.cuda.synchronize()
    ga, gpm, gpn = ctx.history(0)
    g = ctx.spectrum(0)
    ctx.close()

    ok = counts > 0
    assert len(ga) == J and np.allclose(ga, nodes, rtol=1e-15)
    rows_pm = np.abs(gpm[:-1, ok] / pm[:, ok] - 1.0).max()
    rows_nu = np.abs(gpn[1:-1, ok] / pnu[1:, ok] - 1.0).max()
    assert np.allclose(gpn[0], ic, rtol=1e-14, atol=0)  # node 0: the initial amplitude
    prel = np.abs(g["p_cdm"][ok] / ref["p_cdm"][ok] - 1.0).max()
    nrel = np.abs(g["pnu_half"][ok] / ref["pnu_half"][ok] - 1.0).max()
    hrel = np.abs(gpm[-1, ok] / ref["pm_half_now"][ok] - 1.0).max()
    ferr = rms_rel(acc.cpu().numpy(), ref["acc"])
    print(f"  stored rows: P_M {rows_pm:.2e}, P_nu {rows_nu:.2e}; step: P_cdm {prel:.2e}, "
          f"P_nu {nrel:.2e}, node {hrel:.2e}, force rms {ferr:.2e}", flush=True)
    assert rows_pm <= TOL_NU and rows_nu <= TOL_NU, label
    assert prel <= 2e-6, label
    assert nrel <= TOL_NU, label
    assert hrel <= 2e-6, label
    assert ferr <= TOL_FORCE_RMS, label


def test_replayed_history_tiny32():
    from synth import CONFIGS, zeldovich_lattice
    c = CONFIGS["tiny32"]
    pos = zeldovich_lattice(c["n_side"], c["box"], c["sigma_cells"], 3)
    _replayed_case(pos, c["n_mesh"], c["box"], c["n_kbins"], c["n_hist"], c["a_lo"],
                   c["a_now"], 0.3, c["substeps"], "tiny32 replayed")


def test_replayed_history_pm256():
    from synth import CONFIGS, zeldovich_lattice
    c = CONFIGS["pm256"]
    pos = zeldovich_lattice(c["n_side"], c["box"], c["sigma_cells"], 257)
    _replayed_case(pos, c["n_mesh"], c["box"], c["n_kbins"], c["n_hist"], c["a_lo"],
                   c["a_now"], 0.3, c["substeps"], "pm256 replayed")


@pytest.mark.parametrize("mode", [0, 2])
def test_undisplaced_lattice_gives_exactly_zero_force(mode):
    """delta = 0 exactly (each particle of a cell-centre lattice puts 1/8 on 8 nodes), so
    P_cdm = 0 in every bin while P_nu from the history is not: R must read 0, the force 0."""
    import os
    import torch
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, synthetic_history
    n, box, nb = 32, 128.0, 16
    g = (np.arange(n) + 0.5) * (box / n)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    ctx = PMNu(n, pos.shape[0], box, nb, 24, [0.3])
    _, counts, kmean = ctx.bins()
    nodes = log_spaced_nodes(0.01, 0.5, 16)
    ctx.set_history(0, synthetic_history(kmean, np.ones(nb), nodes, 0.3))
    if mode:
        blob = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "paper_1209_0461_amd", "data", "surrogate_pm256.npy")
        binding.pm_nu_surrogate_load(ctx.h, np.load(blob))
        binding.pm_nu_set_response_mode(ctx.h, mode)
    p = torch.from_numpy(pos).cuda()
    acc = torch.full_like(p, 7.0)
    ctx.step(p, acc, 0.5)
    torch.cuda.synchronize()
    sp = ctx.spectrum(0)
    ctx.close()
    ok = counts > 0
    print(f"mode {mode}: max P_cdm {sp['p_cdm'].max():.1e}, min P_nu {sp['pnu_half'][ok].min():.2e}",
          flush=True)
    assert np.all(sp["p_cdm"] == 0.0)
    assert np.all(sp["pnu_half"][ok] > 0.0)
    assert np.all(sp["ratio"] == 0.0)
    a = acc.cpu().numpy()
    assert np.all(np.isfinite(a)) and np.all(a == 0.0)
