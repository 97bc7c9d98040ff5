"""Parity of the HIP path (through the C ABI) with the FP64 oracle, stage by stage.

Tolerances: force RMS relative error <= 1e-4 and P_nu^{1/2} max relative error <= 1e-6
(the accuracy targets of the step); FP32 stages are checked at the level FP32 arithmetic
allows (density 2e-6 of the peak, modes 1e-5 of the peak, binned power 2e-6: the density
is accumulated exactly in fixed point and only delta is rounded to FP32).
Integer work (bin edges, mode counts) must be bit-exact.
"""
import numpy as np
import pytest

from gpu_cases import (TOL_FORCE_RMS, TOL_NU, gpu_case, make_inputs, oracle_case, rms_rel)

pytestmark = pytest.mark.gpu


def _check_box(g, ref, hist_len, label):
    ok = ref["counts"] > 0
    # density (fixed-point sums of FP64 weights; unit mass per particle)
    assert np.abs(g["rho"] - ref["rho"]).max() <= 1e-7 * ref["rho"].max(), label
    assert abs(g["rho"].astype(np.float64).sum() / ref["rho"].sum() - 1.0) < 1e-6, label
    # forward FFT modes, numpy rfftn layout
    if "modes" in g:
        scale = np.abs(ref["delta_k"]).max()
        assert np.abs(g["modes"] - ref["delta_k"]).max() <= 1e-5 * scale, label
    # binned power (FP64 sums of FP32 modes)
    prel = np.abs(g["p_cdm"][ok] / ref["p_cdm"][ok] - 1.0)
    assert prel.max() <= 2e-6, (label, prel.max())
    assert np.all(g["p_cdm"][~ok] == 0)
    # neutrino amplitude of eq. (P-final), FP64
    nrel = np.abs(g["pnu_half"][ok] / ref["pnu_half"][ok] - 1.0)
    print(f"  {label}: P_cdm max rel {prel.max():.2e}, P_nu max rel {nrel.max():.2e}",
          flush=True)
    assert nrel.max() <= TOL_NU, (label, nrel.max())
    rrel = np.abs(g["ratio"][ok] / ref["ratio"][ok] - 1.0)
    assert rrel.max() <= 2e-5, (label, rrel.max())
    # history row appended at a_now
    assert len(g["hist_a"]) == hist_len + 1, label
    hrel = np.abs(g["hist_pm"][-1][ok] / ref["pm_half_now"][ok] - 1.0)
    assert hrel.max() <= 1e-5, (label, hrel.max())
    # acceleration grids and particle accelerations
    assert rms_rel(g["grids"], ref["grids"]) <= TOL_FORCE_RMS, label
    ferr = rms_rel(g["acc"], ref["acc"])
    assert ferr <= TOL_FORCE_RMS, (label, ferr)
    return ferr, nrel.max()


CASES = [
    # n_side, n_mesh, box, bins, J, a_lo, a_now, m_nu, sigma, seed, Q, iters, deconv, extra, edges
    (32, 32, 128.0, 32, 16, 0.01, 0.5, 0.3, 0.2, 0, 8, 1, True, 0, False),
    (32, 32, 128.0, 32, 16, 0.01, 0.5, 0.3, 0.2, 1, 1, 1, True, 0, False),
    (32, 32, 128.0, 32, 16, 0.01, 0.5, 0.3, 0.2, 2, 8, 2, True, 0, False),
    (32, 32, 128.0, 32, 16, 0.01, 0.5, 0.3, 0.2, 3, 8, 1, False, 0, False),
    (32, 32, 128.0, 32, 16, 0.01, 0.5, 0.3, 0.2, 4, 8, 1, True, 37, True),
    (8, 8, 32.0, 5, 6, 0.02, 0.3, 0.6, 0.3, 5, 4, 1, True, 13, True),
    (16, 16, 64.0, 12, 10, 0.01, 1.0, 0.15, 0.3, 6, 8, 1, True, 0, True),
    (32, 64, 256.0, 48, 30, 0.01, 1.0, 0.45, 0.3, 7, 8, 1, True, 999, False),
    (64, 128, 256.0, 40, 24, 0.01, 0.8, 0.3, 0.3, 8, 8, 1, True, 0, False),
    (64, 64, 256.0, 48, 100, 0.01, 1.0, 0.05, 0.3, 9, 8, 1, True, 0, False),
]


@pytest.mark.parametrize("case", CASES, ids=[f"N{c[1]}-np{c[0]}-s{c[9]}" for c in CASES])
def test_step_matches_oracle(case):
    (ns, nm, box, nb, J, alo, anow, mnu, sig, seed, Q, it, dec, extra, edges) = case
    print(f"case N={nm} np={ns} seed={seed} Q={Q} iters={it} deconv={dec}", flush=True)
    pos = make_inputs(ns, box, sig, seed, extra_random=extra, edges=edges, n_mesh=nm)
    hist, ref = oracle_case(pos, nm, box, nb, J, alo, anow, mnu, Q, it, dec)
    out = gpu_case(pos[None], nm, box, nb, J, anow, [mnu], [hist], Q, it, dec)
    edges_, counts, kmean = out["bins"]
    assert np.array_equal(edges_, ref["edges"])
    assert np.array_equal(counts, ref["counts"])
    ok = counts > 0
    # FP64 means summed in different orders (numpy by mode, the library by |n|^2)
    assert np.allclose(kmean[ok], ref["k_mean"][ok], rtol=1e-12, atol=0)
    ferr, nerr = _check_box(out["boxes"][0], ref, J - 1, str(case))
    print(f"  force rms rel {ferr:.2e}  nu max rel {nerr:.2e}", flush=True)


def test_batched_boxes_with_different_masses():
    nm, box, nb, J, anow = 32, 128.0, 24, 20, 1.0
    masses = [0.05, 0.3, 0.6]
    pos_b, hists, refs = [], [], []
    for i, m in enumerate(masses):
        p = make_inputs(32, box, 0.3, 100 + i)
        h, r = oracle_case(p, nm, box, nb, J, 0.01, anow, m)
        pos_b.append(p)
        hists.append(h)
        refs.append(r)
    out = gpu_case(np.stack(pos_b), nm, box, nb, J, anow, masses, hists)
    for i in range(len(masses)):
        _check_box(out["boxes"][i], refs[i], J - 1, f"box {i}")


def test_single_particle_box_matches_oracle():
    """The degenerate box of one particle (the smallest input the call accepts): bins, the
    density, the spectrum and P_nu^{1/2} as in every case; the acceleration grids at the RMS
    bar; the particle's own (CIC self-) force against the grids' scale, since it is not
    bounded away from zero."""
    nm, box, nb, J, a_now, m_nu = 16, 64.0, 12, 8, 0.5, 0.3
    pos = np.array([[17.3, 40.11, 5.7]], dtype=np.float32)
    print(f"case single particle N={nm}", flush=True)
    hist, ref = oracle_case(pos, nm, box, nb, J, 0.02, a_now, m_nu)
    out = gpu_case(pos[None], nm, box, nb, J, a_now, [m_nu], [hist])
    edges_, counts, _ = out["bins"]
    assert np.array_equal(edges_, ref["edges"]) and np.array_equal(counts, ref["counts"])
    g = out["boxes"][0]
    ok = ref["counts"] > 0
    assert np.abs(g["rho"] - ref["rho"]).max() <= 1e-7 * ref["rho"].max()
    assert np.abs(g["p_cdm"][ok] / ref["p_cdm"][ok] - 1.0).max() <= 2e-6
    assert np.abs(g["pnu_half"][ok] / ref["pnu_half"][ok] - 1.0).max() <= TOL_NU
    assert rms_rel(g["grids"], ref["grids"]) <= TOL_FORCE_RMS
    scale = np.abs(np.asarray(ref["grids"])).max()
    assert np.abs(np.asarray(g["acc"], np.float64) - ref["acc"]).max() <= 1e-5 * scale


def test_zero_mass_is_plain_pm():
    nm, box = 32, 128.0
    pos = make_inputs(32, box, 0.2, 21)
    hist, ref = oracle_case(pos, nm, box, 16, 8, 0.05, 0.5, 0.0)
    out = gpu_case(pos[None], nm, box, 16, 8, 0.5, [0.0], [hist])
    assert rms_rel(out["boxes"][0]["acc"], ref["acc"]) <= TOL_FORCE_RMS


def test_non_finite_position_is_skipped_and_reported():
    import torch
    from paper_1209_0461_amd import PMNu, PMNuError, binding
    import oracle.pm as opm
    nm, box = 16, 64.0
    pos = make_inputs(16, box, 0.2, 31)
    bad = pos.copy()
    bad[7] = [np.nan, 1.0, 1.0]
    ctx = PMNu(nm, len(bad), box, 8, 8, [0.3])
    p = torch.from_numpy(bad).cuda()
    ctx.deposit(p)
    rho = torch.empty(nm ** 3, device="cuda")
    binding.pm_nu_copy_density(ctx.h, 0, rho)
    with pytest.raises(PMNuError) as e:
        ctx.spectrum(0)
    assert e.value.code == -8
    ctx.spectrum(0)   # the flag is cleared once reported
    ref = opm.cic_deposit(np.delete(pos, 7, axis=0), nm, box)
    assert np.abs(rho.cpu().numpy().reshape(ref.shape) - ref).max() < 1e-5
    ctx.close()


def test_call_order_is_enforced():
    import torch
    from paper_1209_0461_amd import PMNu, PMNuError
    ctx = PMNu(16, 4096, 64.0, 8, 8, [0.3])
    p = torch.from_numpy(make_inputs(16, 64.0, 0.2, 1)).cuda()
    acc = torch.zeros_like(p)
    with pytest.raises(PMNuError) as e:
        ctx.response(0.5)
    assert e.value.code == -4
    with pytest.raises(PMNuError) as e:
        ctx.force(p, acc, 0.5)
    assert e.value.code in (-1, -4)
    ctx.deposit(p)
    with pytest.raises(PMNuError) as e:   # no history stored yet
        ctx.response(0.5)
    assert e.value.code == -5
    ctx.close()


def test_recompute_at_same_time_is_idempotent():
    """A second step at the same a_now recomputes (does not append) the current node."""
    import torch
    from paper_1209_0461_amd import PMNu
    nm, box, nb, J = 32, 128.0, 16, 12
    pos = make_inputs(32, box, 0.2, 41)
    hist, ref = oracle_case(pos, nm, box, nb, J, 0.01, 0.5, 0.3)
    ctx = PMNu(nm, len(pos), box, nb, J + 2, [0.3])
    ctx.set_history(0, hist)
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    results = []
    for _ in range(3):
        ctx.step(p, acc, 0.5)
        torch.cuda.synchronize()
        results.append((acc.cpu().numpy().copy(), ctx.spectrum(0)["pnu_half"].copy()))
        assert len(ctx.history(0)[0]) == J
    for a, pn in results[1:]:
        assert rms_rel(a, results[0][0]) < 1e-6
        assert np.allclose(pn, results[0][1], rtol=1e-12, atol=0)
    assert rms_rel(results[-1][0], ref["acc"]) <= TOL_FORCE_RMS
    ctx.close()


def test_graph_replay_matches_eager():
    import torch
    from paper_1209_0461_amd import PMNu, binding
    nm, box, nb, J = 32, 128.0, 16, 12
    pos = make_inputs(32, box, 0.2, 51)
    hist, ref = oracle_case(pos, nm, box, nb, J, 0.01, 0.5, 0.3)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = PMNu(nm, len(pos), box, nb, J + 2, [0.3])
        ctx.set_history(0, hist)
        p = torch.from_numpy(pos).cuda()
        acc = torch.zeros_like(p)
        ctx.step(p, acc, 0.5)
        stream.synchronize()
        eager = acc.cpu().numpy().copy()
        binding.pm_nu_graph_capture(ctx.h, p, acc, 0.5)
        for rep in range(3):
            acc.zero_()
            binding.pm_nu_graph_launch(ctx.h)
            stream.synchronize()
            got = acc.cpu().numpy()
            assert rms_rel(got, eager) < 1e-6, rep
            assert rms_rel(got, ref["acc"]) <= TOL_FORCE_RMS
            # eager work between replays
            ctx.step(p, acc, 0.5)
            stream.synchronize()
        # a setting changed after capture discards the graph; a new capture follows it
        pnu_fit = ctx.spectrum(0)["pnu_half"]
        binding.pm_nu_set_kernel(ctx.h, 1)
        with pytest.raises(binding.PMNuError, match="setting changed"):
            binding.pm_nu_graph_launch(ctx.h)
        binding.pm_nu_graph_capture(ctx.h, p, acc, 0.5)
        binding.pm_nu_graph_launch(ctx.h)
        stream.synchronize()
        ok = ref["counts"] > 0
        pnu_ser = ctx.spectrum(0)["pnu_half"]
        assert np.abs(pnu_ser[ok] / pnu_fit[ok] - 1).max() > 1e-4
    ctx.close()


def test_timing_records_every_stage():
    import torch
    from paper_1209_0461_amd import PMNu, binding
    nm, box, nb, J = 32, 128.0, 16, 12
    pos = make_inputs(32, box, 0.2, 61)
    hist, _ = oracle_case(pos, nm, box, nb, J, 0.01, 0.5, 0.3)
    ctx = PMNu(nm, len(pos), box, nb, J + 2, [0.3])
    ctx.set_history(0, hist)
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    binding.pm_nu_set_timing(ctx.h, True)
    common = ("cic_deposit", "fft_fwd_x_bin", "nu_response", "cic_interp")
    # N = 32: the first two forward and the first two inverse passes run as one kernel each
    # by default, as two on request
    # (fused forward, fused inverse x+y, fused inverse y+z) -> the stages that run
    passes = {(1, 0, 1): ("fft_fwd_zy", "inv_x_green", "inv_yz"),
              (1, 1, 0): ("fft_fwd_zy", "inv_xy_green", "fft_inv_z"),
              (0, 0, 0): ("fft_fwd_z", "fft_fwd_y", "inv_x_green", "fft_inv_y", "fft_inv_z")}
    every = set(sum(passes.values(), ()))
    for (zy, xy, yz), stages in passes.items():
        binding.pm_nu_set_forward_zy(ctx.h, zy)
        binding.pm_nu_set_inverse_xy(ctx.h, xy)
        binding.pm_nu_set_inverse_yz(ctx.h, yz)
        for _ in range(2):
            ctx.step(p, acc, 0.5)
        t = binding.pm_nu_read_timing(ctx.h)
        for stage in common + stages:
            ms, n = t[stage]
            assert n == 2 and ms > 0, (zy, xy, yz, stage)
        assert all(t[s][1] == 0 for s in every - set(stages)), (zy, xy, yz)
        assert binding.pm_nu_read_timing(ctx.h)["cic_deposit"][1] == 0
    ctx.close()


@pytest.mark.parametrize("order", ["morton", "c", "shuffled"])
def test_every_launch_mode_matches_oracle(order):
    """All deposit and interpolation modes, on particle orders that take the LDS paths
    (Morton), partly the fallback (C order: slab chunks) and only the fallback (shuffled)."""
    import torch
    from paper_1209_0461_amd import PMNu, binding
    from synth import zeldovich_lattice
    nm, box, nb, J = 32, 128.0, 16, 10
    pos = zeldovich_lattice(32, box, 0.3, 71, order="morton" if order == "morton" else "c")
    if order == "shuffled":
        pos = pos[np.random.default_rng(3).permutation(len(pos))]
    pos = np.ascontiguousarray(np.concatenate([pos, make_inputs(8, box, 0.2, 5)[:77]]))
    hist, ref = oracle_case(pos, nm, box, nb, J, 0.02, 0.7, 0.3)
    ctx = PMNu(nm, len(pos), box, nb, J + 2, [0.3])
    ctx.set_history(0, hist)
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    for dm, im, ib in ((0, 0, 256), (1, 1, 256), (2, 2, 256), (3, 3, 256), (1, 0, 512),
                       (0, 2, 256), (4, 0, 1024), (5, 1, 256), (6, 1, 256), (6, 0, 256), (7, 1, 256),
                       (8, 1, 256), (9, 1, 256)):
        binding.pm_nu_set_launch(ctx.h, dm, 256, im, ib)
        ctx.step(p, acc, 0.7)
        torch.cuda.synchronize()
        ok = ref["counts"] > 0
        sp = ctx.spectrum(0)
        assert np.abs(sp["p_cdm"][ok] / ref["p_cdm"][ok] - 1).max() <= 2e-6, (order, dm, im, ib)
        assert rms_rel(acc.cpu().numpy(), ref["acc"]) <= TOL_FORCE_RMS, (order, dm, im, ib)
    ctx.close()


def test_spectrum_after_deposit_alone_matches_oracle():
    """The binned power is available right after pm_nu_deposit, before any response, in a
    fresh context (it used to be produced only by the response)."""
    import torch
    from paper_1209_0461_amd import PMNu
    import oracle.step as ostep
    nm, box, nb = 32, 128.0, 24
    pos = make_inputs(32, box, 0.3, 81)
    ref = ostep.spectrum(pos, nm, box, nb)
    ctx = PMNu(nm, len(pos), box, nb, 8, [0.3])
    assert np.all(ctx.spectrum(0)["p_cdm"] == 0)          # nothing deposited yet
    ctx.deposit(torch.from_numpy(pos).cuda())
    got = ctx.spectrum(0)["p_cdm"]
    ok = ref["counts"] > 0
    assert np.abs(got[ok] / ref["p_cdm"][ok] - 1).max() <= 2e-6
    ctx.close()


@pytest.mark.parametrize("deposit_mode", [6, 8])
def test_patch_deposit_side_grid_on_crowded_cells(deposit_mode):
    """Deposit mode 6 (and 8, its fused form) with 40 chunks of particles packed into a few cells: the coarse cell's
    patch list overflows, those chunks go through the side grid, and the result still
    matches the oracle; a following deposit of an ordinary lattice finds the side grid
    cleared. In the last input half of the chunks straddle two coarse cells of which only
    one overflows: such a chunk's patch serves the other cell, and only its part in the full
    cell goes through the side grid."""
    import torch
    from paper_1209_0461_amd import PMNu, binding
    from synth import zeldovich_lattice
    nm, box, nb, J = 32, 128.0, 16, 10
    rng = np.random.default_rng(12)
    crowd = (40.0 + 10.0 * rng.random((40 * 4096, 3))).astype(np.float32)   # 2.5 cells wide
    lattice = zeldovich_lattice(32, box, 0.3, 72)
    lattice = np.concatenate([lattice] * 5)[: len(crowd)]   # same count, ordinary spread
    straddle = crowd.copy()                                 # x nodes 15-17: cells 0 and 1
    straddle[: 20 * 4096, 0] += 20.0
    ctx = PMNu(nm, len(crowd), box, nb, J + 2, [0.3])
    binding.pm_nu_set_launch(ctx.h, deposit_mode, 256, 1, 256)
    binding.pm_nu_set_keep_density(ctx.h, 1)
    assert binding.pm_nu_side_grid_uses(ctx.h) == 0
    # (five overlapping copies of a lattice also fill the coarse cells' lists: no claim there)
    for pos, side in ((crowd, True), (lattice, None), (straddle, True)):
        hist, ref = oracle_case(pos, nm, box, nb, J, 0.02, 0.7, 0.3)
        ctx.set_history(0, hist)
        p = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
        acc = torch.zeros_like(p)
        ctx.step(p, acc, 0.7)
        torch.cuda.synchronize()
        ok = ref["counts"] > 0
        sp = ctx.spectrum(0)
        assert np.abs(sp["p_cdm"][ok] / ref["p_cdm"][ok] - 1).max() <= 2e-6
        assert rms_rel(acc.cpu().numpy(), ref["acc"]) <= TOL_FORCE_RMS
        rho = torch.empty(nm ** 3, device="cuda")
        binding.pm_nu_copy_density(ctx.h, 0, rho)
        assert abs(float(rho.double().sum()) / len(pos) - 1.0) < 1e-5
        uses = binding.pm_nu_side_grid_uses(ctx.h)
        assert side is None or (uses > 0) == side, uses
    ctx.close()


@pytest.mark.parametrize("which", ["hierarchy_normal_eV", "hierarchy_inverted_eV"])
def test_mass_hierarchy_matches_oracle(which):
    """Species with their own masses (Sec. 6.2: the paper's normal and inverted hierarchies
    of M_nu = 0.1 eV), each with its own initial amplitude; the surrogate must step aside."""
    import json
    import os
    import torch
    import oracle.step as ostep
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, synthetic_history
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    masses = np.array(gold[which]["value"])
    M = float(masses.sum())
    nm, box, nb, J = 32, 128.0, 16, 12
    pos = make_inputs(32, box, 0.2, 91)
    sp = ostep.spectrum(pos, nm, box, nb)
    nodes = log_spaced_nodes(0.02, 0.8, J)
    hist = synthetic_history(sp["k_mean"], np.sqrt(sp["p_cdm"]), nodes, M)
    ics = np.stack([hist["pnu_half_init"] * (1.0 + 0.2 * s) for s in range(len(masses))])
    import oracle.response as ores
    r = ores.nu_amplitude(sp["k_mean"], sp["counts"], np.sqrt(sp["p_cdm"]), hist["a"],
                          hist["pm_half"], hist["pnu_half"][-1], hist["pnu_half_init"],
                          hist["theta_over_delta_init"], 0.8, M, 0.3, 0.7, 8, species=masses,
                          pnu_half_init_species=ics)
    forces = ostep.forces(pos, sp["delta_k"], nm, box, sp["k_mean"], sp["counts"], r["ratio"],
                          r["f_nu"], 0.8, 0.3, True)
    ctx = PMNu(nm, len(pos), box, nb, J + 2, [M], response_mode=2)
    binding.pm_nu_surrogate_load(ctx.h, np.load(os.path.join(
        os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1209_0461_amd",
        "data", "surrogate_pm256.npy")))
    ctx.set_history(0, hist)
    binding.pm_nu_set_species(ctx.h, 0, masses, ics)
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    ctx.step(p, acc, 0.8)
    torch.cuda.synchronize()
    ok = sp["counts"] > 0
    got = ctx.spectrum(0)
    assert np.abs(got["pnu_half"][ok] / r["pnu_half"][ok] - 1).max() <= TOL_NU
    assert rms_rel(acc.cpu().numpy(), forces) <= TOL_FORCE_RMS
    exact, sur = binding.pm_nu_get_surrogate_check(ctx.h, 0, nb)
    assert np.array_equal(exact, sur)          # the network is not used for a hierarchy
    # and the hierarchy differs from the same total mass in three equal species
    eq = ores.nu_amplitude(sp["k_mean"], sp["counts"], np.sqrt(sp["p_cdm"]), hist["a"],
                           hist["pm_half"], hist["pnu_half"][-1], hist["pnu_half_init"],
                           hist["theta_over_delta_init"], 0.8, M, 0.3, 0.7, 8)
    assert np.abs(got["pnu_half"][ok] / eq["pnu_half"][ok] - 1).max() > 100 * TOL_NU
    ctx.close()


@pytest.mark.parametrize("masses", [None, "hierarchy_inverted_eV"])
def test_relativistic_background_matches_oracle(masses):
    """The background of Sec. 4.4 (radiation, massless species, and the energy density of
    eq. (relativistic)) in the time grid, early enough (a <= 0.1) that it matters."""
    import json
    import os
    import torch
    import oracle.response as ores
    import oracle.step as ostep
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, synthetic_history
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    sp_m = None if masses is None else np.array(gold[masses]["value"])
    M = 0.3 if sp_m is None else float(sp_m.sum())
    nm, box, nb, J, a_now = 32, 128.0, 16, 16, 0.1
    pos = make_inputs(32, box, 0.2, 57)
    sp = ostep.spectrum(pos, nm, box, nb)
    nodes = log_spaced_nodes(0.005, a_now, J)
    hist = synthetic_history(sp["k_mean"], np.sqrt(sp["p_cdm"]), nodes, M)
    args = (sp["k_mean"], sp["counts"], np.sqrt(sp["p_cdm"]), hist["a"], hist["pm_half"],
            hist["pnu_half"][-1], hist["pnu_half_init"], hist["theta_over_delta_init"], a_now,
            M, 0.3, 0.7, 8)
    r = ores.nu_amplitude(*args, species=sp_m, relativistic=True)
    flat = ores.nu_amplitude(*args, species=sp_m)
    forces = ostep.forces(pos, sp["delta_k"], nm, box, sp["k_mean"], sp["counts"], r["ratio"],
                          r["f_nu"], a_now, 0.3, True)
    ctx = PMNu(nm, len(pos), box, nb, J + 2, [M], response_mode=2)
    binding.pm_nu_surrogate_load(ctx.h, np.load(os.path.join(
        os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1209_0461_amd",
        "data", "surrogate_pm256.npy")))
    ctx.set_history(0, hist)
    if sp_m is not None:
        binding.pm_nu_set_species(ctx.h, 0, sp_m)
    binding.pm_nu_set_background(ctx.h, 1)
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    ctx.step(p, acc, a_now)
    torch.cuda.synchronize()
    ok = sp["counts"] > 0
    got = ctx.spectrum(0)
    assert np.abs(got["pnu_half"][ok] / r["pnu_half"][ok] - 1).max() <= TOL_NU
    assert np.abs(got["pnu_half"][ok] / flat["pnu_half"][ok] - 1).max() > 100 * TOL_NU
    assert rms_rel(acc.cpu().numpy(), forces) <= TOL_FORCE_RMS
    exact, sur = binding.pm_nu_get_surrogate_check(ctx.h, 0, nb)
    assert np.array_equal(exact, sur)          # the network is not used off its background
    # back to matter + Lambda: the oracle's flat result again (a fresh history row)
    binding.pm_nu_set_background(ctx.h, 0)
    ctx.set_history(0, hist)
    if sp_m is not None:
        binding.pm_nu_set_species(ctx.h, 0, sp_m)
    ctx.step(p, acc, a_now)
    torch.cuda.synchronize()
    got = ctx.spectrum(0)
    assert np.abs(got["pnu_half"][ok] / flat["pnu_half"][ok] - 1).max() <= TOL_NU
    ctx.close()


def test_background_rejects_bad_flag():
    from paper_1209_0461_amd import PMNu, binding
    ctx = PMNu(16, 8, 64.0, 8, 4, [0.1])
    assert binding.ERRORS[binding.load_library().pm_nu_set_background(ctx.h, 2)] == "EINVAL"
    assert b"relativistic" in binding.load_library().pm_nu_last_error()
    ctx.close()


def test_kernel_values_match_oracle():
    """I(x) on the device against the oracle: the fit (same formula, FP64) and the exact
    series of Appendix C (accelerated on the device, Euler-transformed in the oracle)."""
    import torch
    from oracle import kernel
    from paper_1209_0461_amd import binding
    x = np.concatenate([np.linspace(0.0, 5.0, 2001), np.geomspace(5.0, 1e4, 3000)])
    xd = torch.from_numpy(x).cuda()
    out = torch.empty_like(xd)
    binding.pm_nu_kernel_values(xd, out, series=False)
    torch.cuda.synchronize()
    fit = out.cpu().numpy()
    assert np.abs(fit / kernel.I_fit(x) - 1).max() <= 1e-13
    binding.pm_nu_kernel_values(xd, out, series=True)
    torch.cuda.synchronize()
    ser = out.cpu().numpy()
    ref = kernel.I_series(x)
    small = x <= 1e3
    assert np.abs(ser[small] / ref[small] - 1).max() <= 1e-11
    assert np.abs(ser[~small] / ref[~small] - 1).max() <= 1e-8   # the oracle's own rounding
    assert ser[0] == pytest.approx(1.0, rel=1e-15)
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    binding.pm_nu_kernel_values(empty, empty, series=True)      # n = 0 is a no-op


@pytest.mark.parametrize("iters,masses,relativistic",
                         [(1, None, False), (3, None, False),
                          (2, "hierarchy_normal_eV", True)])
def test_exact_kernel_matches_oracle(iters, masses, relativistic):
    """The exact I(x) of Appendix C in eq. (P-final), with 1-3 iterations of Appendix B, and
    combined with a hierarchy and the relativistic background."""
    import json
    import os
    import torch
    import oracle.response as ores
    import oracle.step as ostep
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, synthetic_history
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    sp_m = None if masses is None else np.array(gold[masses]["value"])
    M = 0.3 if sp_m is None else float(sp_m.sum())
    nm, box, nb, J, a_now = 32, 128.0, 16, 16, 0.5
    pos = make_inputs(32, box, 0.2, 61)
    sp = ostep.spectrum(pos, nm, box, nb)
    nodes = log_spaced_nodes(0.01, a_now, J)
    hist = synthetic_history(sp["k_mean"], np.sqrt(sp["p_cdm"]), nodes, M)
    args = (sp["k_mean"], sp["counts"], np.sqrt(sp["p_cdm"]), hist["a"], hist["pm_half"],
            hist["pnu_half"][-1], hist["pnu_half_init"], hist["theta_over_delta_init"], a_now,
            M, 0.3, 0.7, 8)
    kw = dict(iterations=iters, species=sp_m, relativistic=relativistic)
    r = ores.nu_amplitude(*args, kernel="series", **kw)
    fit = ores.nu_amplitude(*args, **kw)
    forces = ostep.forces(pos, sp["delta_k"], nm, box, sp["k_mean"], sp["counts"], r["ratio"],
                          r["f_nu"], a_now, 0.3, True)
    ctx = PMNu(nm, len(pos), box, nb, J + 2, [M], iterations=iters)
    ctx.set_history(0, hist)
    if sp_m is not None:
        binding.pm_nu_set_species(ctx.h, 0, sp_m)
    binding.pm_nu_set_background(ctx.h, relativistic)
    binding.pm_nu_set_kernel(ctx.h, 1)
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    ctx.step(p, acc, a_now)
    torch.cuda.synchronize()
    ok = sp["counts"] > 0
    got = ctx.spectrum(0)
    err = np.abs(got["pnu_half"][ok] / r["pnu_half"][ok] - 1).max()
    print(f"  exact kernel, iterations {iters}: P_nu max rel {err:.2e}", flush=True)
    assert err <= TOL_NU
    assert np.abs(got["pnu_half"][ok] / fit["pnu_half"][ok] - 1).max() > 100 * TOL_NU
    assert rms_rel(acc.cpu().numpy(), forces) <= TOL_FORCE_RMS
    ctx.close()


def test_kernel_flag_is_checked():
    from paper_1209_0461_amd import PMNu, binding
    ctx = PMNu(16, 8, 64.0, 8, 4, [0.1])
    assert binding.ERRORS[binding.load_library().pm_nu_set_kernel(ctx.h, 5)] == "EINVAL"
    ctx.close()


@pytest.mark.parametrize("masses,relativistic,deposit_mode",
                         [((0.3,), False, 4), ((0.3,), False, 6), ((0.1, 0.6), True, 6)])
def test_advance_matches_oracle(masses, relativistic, deposit_mode):
    """Several kick-drift-kick steps through the C ABI (positions, velocities, forces and the
    history rows each step stores) against the oracle's loop, per box."""
    import torch
    import oracle.step as ostep
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, synthetic_history, zeldovich_ics
    nm, box, nb, a0 = 32, 128.0, 16, 0.1
    steps = np.geomspace(a0, 0.2, 5)
    nbox = len(masses)
    ics = [zeldovich_ics(32, box, 0.3, 71 + b, a0) for b in range(nbox)]
    pos = np.stack([p for p, _ in ics])
    vel = np.stack([v for _, v in ics])
    ctx = PMNu(nm, pos.shape[1], box, nb, 20, list(masses))
    binding.pm_nu_set_launch(ctx.h, deposit_mode, 256, 1, 256)
    binding.pm_nu_set_background(ctx.h, relativistic)
    refs = []
    for b in range(nbox):
        sp = ostep.spectrum(pos[b], nm, box, nb)
        hist = synthetic_history(sp["k_mean"], np.sqrt(sp["p_cdm"]),
                                 log_spaced_nodes(0.01, a0, 10), masses[b])
        ctx.set_history(b, hist)
        r = ostep.full_step(pos[b], nm, box, nb, hist, a0, masses[b], relativistic=relativistic)
        h = dict(hist)
        h["a"] = np.append(hist["a"], a0)
        h["pm_half"] = np.vstack([hist["pm_half"], r["pm_half_now"]])
        h["pnu_half"] = np.vstack([hist["pnu_half"], r["pnu_half"]])
        refs.append(ostep.advance(pos[b], vel[b], r["acc"], h, steps, nm, box, nb, masses[b],
                                  relativistic=relativistic))
    p = torch.from_numpy(pos).cuda()
    v = torch.from_numpy(vel).cuda()
    acc = torch.zeros_like(p)
    ctx.step(p, acc, a0)
    binding.pm_nu_advance(ctx.h, p, v, acc, steps)
    torch.cuda.synchronize()
    pg, vg, ag = p.cpu().numpy(), v.cpu().numpy(), acc.cpu().numpy()
    cell = box / nm
    for b in range(nbox):
        x1, u1, g1, h1 = refs[b]
        dx = np.mod(pg[b] - x1 + box / 2, box) - box / 2
        assert np.abs(dx).max() <= 1e-4 * cell, (b, np.abs(dx).max())
        assert np.all((pg[b] >= 0) & (pg[b] < box))
        assert rms_rel(vg[b], u1) <= 1e-4, b
        assert rms_rel(ag[b], g1) <= TOL_FORCE_RMS, b
        a, pm, pn = ctx.history(b)
        assert np.allclose(a[-len(steps):], steps, rtol=1e-15)
        ok = pn[-1] > 0
        for j in range(1, len(steps) + 1):
            assert np.abs(pn[-j][ok] / h1["pnu_half"][-j][ok] - 1).max() <= 1e-5, (b, j)
            assert np.abs(pm[-j][ok] / h1["pm_half"][-j][ok] - 1).max() <= 1e-5, (b, j)
        print(f"  box {b}: |dx|max/cell {np.abs(dx).max() / cell:.1e}, "
              f"u rms {rms_rel(vg[b], u1):.1e}", flush=True)
    # the history is full after (capacity - stored) more steps
    with pytest.raises(binding.PMNuError, match="history"):
        binding.pm_nu_advance(ctx.h, p, v, acc, np.geomspace(0.2, 0.5, 10))
    ctx.close()


@pytest.mark.parametrize("n_mesh,n_side,box", [(32, 32, 128.0), (64, 64, 256.0), (128, 64, 400.0)])
def test_fused_patch_pass_equals_separate_passes(n_mesh, n_side, box):
    """Deposit modes 8 and 9 (the coarse-cell sums and the z pass in one kernel) give the
    modes and forces of modes 6 and 7 (reduce kernel, then the z pass) bit for bit: the
    sums are exact integers and every later operation is the same. Also with chunks that
    go through the side grid (random particles appended), with several boxes, and with
    delta kept for reading back (the same density as mode 6; without asking for it the
    read-back is refused)."""
    import torch
    from paper_1209_0461_amd import PMNu, PMNuError, binding
    from synth import log_spaced_nodes, synthetic_history
    nbox, nb, J = 2, 16, 10
    pos = np.stack([make_inputs(n_side, box, 0.3, 90 + b, extra_random=3000) for b in range(nbox)])
    ctx = PMNu(n_mesh, pos.shape[1], box, nb, J + 2, [0.3, 0.1])
    nodes = log_spaced_nodes(0.02, 0.7, J)
    _, counts, kmean = ctx.bins()
    for b in range(nbox):
        ctx.set_history(b, synthetic_history(kmean, np.where(counts > 0, 1.0, 0.0), nodes, 0.3))
    p = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    nmode = n_mesh * n_mesh * (n_mesh // 2 + 1) * 2

    def run(mode, keep):
        binding.pm_nu_set_launch(ctx.h, mode, 256, 1, 256)
        binding.pm_nu_set_keep_density(ctx.h, keep)
        acc = torch.zeros_like(p)
        ctx.step(p, acc, 0.7)
        ctx.deposit(p)                              # the modes are read after a deposit
        modes = [torch.empty(nmode, device="cuda") for _ in range(nbox)]
        for b in range(nbox):
            binding.pm_nu_copy_modes(ctx.h, b, modes[b])
        rho = torch.empty(n_mesh ** 3, device="cuda")
        if keep or mode < 8:
            binding.pm_nu_copy_density(ctx.h, 1, rho)
        else:
            with pytest.raises(PMNuError) as e:
                binding.pm_nu_copy_density(ctx.h, 1, rho)
            assert e.value.code == -4
            rho = None
        torch.cuda.synchronize()
        uses = binding.pm_nu_side_grid_uses(ctx.h)
        return acc.cpu().numpy(), [m.cpu().numpy() for m in modes], rho, uses

    for sep, fus in ((6, 8), (7, 9)):
        a0, m0, r0, u0 = run(sep, 0)
        a1, m1, r1, u1 = run(fus, 1)
        a2, m2, r2, u2 = run(fus, 0)
        assert u0 > 0 and u0 == u1 == u2            # the side grid took part, the same way
        for mm in (m1, m2):
            assert all(np.array_equal(x, y) for x, y in zip(m0, mm)), (sep, fus)
        assert np.array_equal(a0, a1) and np.array_equal(a0, a2), (sep, fus)
        assert torch.equal(r0, r1)
        assert r2 is None
    ctx.close()


@pytest.mark.parametrize("n_mesh,n_side,box", [(16, 16, 64.0), (32, 32, 128.0), (64, 64, 256.0)])
def test_fused_inverse_xy_equals_separate_passes(n_mesh, n_side, box):
    """For N <= 64 the Green's function and the x and y inverse passes run as one kernel per
    k_z slab, or the y and z passes as one kernel per x-plane; the forces equal those of the
    three separate passes bit for bit (two boxes with different masses)."""
    import torch
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, synthetic_history
    nbox, nb, J = 2, 16, 10
    pos = np.stack([make_inputs(n_side, box, 0.3, 40 + b) for b in range(nbox)])
    ctx = PMNu(n_mesh, pos.shape[1], box, nb, J + 2, [0.3, 0.6])
    nodes = log_spaced_nodes(0.02, 0.7, J)
    _, counts, kmean = ctx.bins()
    for b in range(nbox):
        ctx.set_history(b, synthetic_history(kmean, np.where(counts > 0, 1.0, 0.0), nodes,
                                             [0.3, 0.6][b]))
    p = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    out = []
    # (inverse x+y, inverse y+z): x+y fused, three passes, x+y fused again, y+z fused
    for xy, yz in ((1, 0), (0, 0), (1, 0), (0, 1), (1, 1)):
        binding.pm_nu_set_inverse_xy(ctx.h, xy)
        binding.pm_nu_set_inverse_yz(ctx.h, yz)
        acc = torch.zeros_like(p)
        ctx.step(p, acc, 0.7)
        torch.cuda.synchronize()
        out.append(acc.cpu().numpy())
    ctx.close()
    assert all(np.array_equal(out[0], o) for o in out[1:])
    assert np.all(np.isfinite(out[0])) and np.abs(out[0]).max() > 0


@pytest.mark.parametrize("n_mesh,n_side,box", [(8, 8, 32.0), (16, 16, 64.0), (32, 32, 128.0),
                                               (64, 64, 256.0), (128, 64, 400.0)])
def test_fused_forward_zy_equals_separate_passes(n_mesh, n_side, box):
    """For N <= 128 the z and y forward passes run as one kernel per x-plane; the modes and
    forces equal those of the two separate passes bit for bit, from the fixed-point density
    (deposit modes 0 and 4) and from the patch deposit's delta (mode 6, whose registry the
    fused kernel clears as the z pass does: the second step would otherwise differ)."""
    import torch
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, synthetic_history
    nbox, nb, J = 2, 16, 10
    pos = np.stack([make_inputs(n_side, box, 0.3, 70 + b, extra_random=500) for b in range(nbox)])
    ctx = PMNu(n_mesh, pos.shape[1], box, nb, J + 8, [0.3, 0.6])
    nodes = log_spaced_nodes(0.02, 0.7, J)
    _, counts, kmean = ctx.bins()
    for b in range(nbox):
        ctx.set_history(b, synthetic_history(kmean, np.where(counts > 0, 1.0, 0.0), nodes,
                                             [0.3, 0.6][b]))
    p = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    nmode = n_mesh * n_mesh * (n_mesh // 2 + 1) * 2

    def run(mode, fused):
        binding.pm_nu_set_launch(ctx.h, mode, 256, 1, 256)
        binding.pm_nu_set_forward_zy(ctx.h, fused)
        accs = []
        for _ in range(2):                          # a second step reuses the registry
            acc = torch.zeros_like(p)
            ctx.step(p, acc, 0.7)
            accs.append(acc)
        ctx.deposit(p)                              # the modes are read after a deposit
        modes = [torch.empty(nmode, device="cuda") for _ in range(nbox)]
        for b in range(nbox):
            binding.pm_nu_copy_modes(ctx.h, b, modes[b])
        torch.cuda.synchronize()
        return [a.cpu().numpy() for a in accs], [m.cpu().numpy() for m in modes]

    for mode in (0, 4, 6):
        a0, m0 = run(mode, 0)
        a1, m1 = run(mode, 1)
        assert all(np.array_equal(x, y) for x, y in zip(m0, m1)), mode
        assert all(np.array_equal(x, y) for x, y in zip(a0, a1)), mode
        assert np.all(np.isfinite(a1[0])) and np.abs(a1[0]).max() > 0
    ctx.close()
