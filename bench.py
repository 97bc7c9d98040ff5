"""Benchmark of the PM + linear-response-neutrino step on one MI355X.

Workload (default): 256^3 particles (Zel'dovich lattice, k^-2 spectrum, RMS displacement
0.3 cells) on a 256^3 mesh in a 512 Mpc/h box, 64 log k-bins, a 200-node history over
a in [0.01, 1] (199 stored + the current step at a = 1), Q = 8 quadrature steps per
interval, M_nu = 0.3 eV. A step is deposit -> response -> force for every particle; each
timed step recomputes the node a = 1 from the same stored history.

Prints one JSON line. `value` is steps/s of the whole step with inputs resident in HBM;
`roofline` is the dominant kernel's algorithmic bytes per launch over its mean launch
time from HIP events recorded on the library's stream inside the timed region;
`cpu_baseline` is the FP64 oracle timed on this host on one full step (single-threaded
NumPy). After the 256^3 workload, `other_workloads` carries the same measurement of the
512^3 box and of the 64 boxes of 64^3 (through a HIP graph), each timed on its own.

    python bench.py [--steps K] [--warmup W] [--workload pm256|pm512|tiny32|batch64x64]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PM+nu steps/sec and particle-updates/s at 256^3; %HBM peak; surrogate vs integral"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {
    "cic_deposit": "grid_kernels.hip", "cic_interp": "grid_kernels.hip",
    "zero_mesh": "grid_kernels.hip", "fft_fwd_z": "fft_kernels.hip",
    "fft_fwd_y": "fft_kernels.hip", "fft_fwd_x_bin": "fft_kernels.hip",
    "inv_x_green": "fft_kernels.hip", "fft_inv_y": "fft_kernels.hip",
    "inv_xy_green": "fft_kernels.hip",
    "fft_inv_z": "fft_kernels.hip", "nu_response": "response_kernels.hip",
    "patch_reduce": "grid_kernels.hip",
    "kick_drift": "advance_kernels.hip", "patch_fwd_z": "fft_kernels.hip",
    "fft_fwd_zy": "fft_kernels.hip", "inv_yz": "fft_kernels.hip",
}


def stage_bytes(n_mesh, n_part, nbox, nbins, n_hist, n_partial, deposit_mode=0):
    """Algorithmic bytes per launch of every kernel: each input read once, each output
    written once (FP32 grids, complex64 modes, FP32 positions/accelerations). The patch
    deposit (modes 6..9) splits the deposit into reading the positions (cic_deposit) and
    writing the density contrast (patch_reduce), which the fused modes (8, 9) never write:
    their patch_fwd_z goes from the deposit to the z-transformed modes. For N <= 128
    fft_fwd_zy is the z and y passes in one kernel (delta in, the y-transformed modes out);
    for N <= 64 inv_yz is the y and z inverse passes in one kernel (F1, F2 in, the
    acceleration grid out)."""
    m = n_mesh ** 3 * nbox
    mh = n_mesh * n_mesh * (n_mesh // 2 + 1) * nbox
    npt = n_part * nbox
    patch = deposit_mode >= 6
    return {
        "zero_mesh": 4 * m,
        "cic_deposit": 12 * npt + (0 if patch else 4 * m),
        "patch_reduce": 4 * m,
        "fft_fwd_z": 4 * m + 8 * mh,
        "fft_fwd_zy": 4 * m + 8 * mh,
        "patch_fwd_z": 8 * mh,
        "fft_fwd_y": 16 * mh,
        "fft_fwd_x_bin": 16 * mh + 8 * n_partial * nbins * nbox,
        "nu_response": 8 * nbox * nbins * (2 * n_hist + n_partial + 8),
        "inv_x_green": 8 * mh + 16 * mh,
        "fft_inv_y": 16 * mh + 24 * mh,
        "inv_xy_green": 8 * mh + 24 * mh,
        "fft_inv_z": 24 * mh + 12 * m,
        "inv_yz": 16 * mh + 12 * m,
        "cic_interp": 12 * npt + 12 * m + 12 * npt,
    }


def step_algorithmic_bytes(n_mesh, n_part, nbox, nbins, n_hist):
    """Whole step: read positions twice and write accelerations (36 N_p), the density
    grid written and read and the three force grids written and read (32 M), the modes
    written and read once (16 M_h), plus the history (8 J B)."""
    m = n_mesh ** 3 * nbox
    mh = n_mesh * n_mesh * (n_mesh // 2 + 1) * nbox
    return 36 * n_part * nbox + 32 * m + 16 * mh + 8 * n_hist * nbins * nbox


def source_sha(name):
    p = os.path.join(ROOT, "paper_1209_0461_amd", "csrc", name)
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_name(stage, tuning, n_mesh):
    """Name (with template arguments) of the kernel a stage launches, as rocprofv3 lists it."""
    dep = {1: "<1024, 3328, 256>", 2: "<2048, 5120, 256>", 3: "<4096, 9216, 256>",
           4: "<4096, 9216, 512>", 5: "<8192, 18432, 1024>"}
    itp = {1: "<1024, 2048, false>", 2: "<2048, 4608, false>", 3: "<4096, 8192, false>"}
    if stage == "cic_deposit":
        m = tuning["deposit_mode"]
        if m >= 6:
            return "deposit_patch_kernel<4096, %d, 512>" % (9216 if m in (7, 9) else 6144)
        return "deposit_tiled_kernel" + dep[m] if m else "deposit_kernel"
    if stage == "cic_interp":
        m = tuning["interp_mode"]
        if m:
            return "interp_tiled_kernel" + itp[m]
        return "interp_kernel<%d, false>" % max(1, min(4, tuning["interp_block"] // 256))
    fixed = {"zero_mesh": "fill_zero_kernel", "nu_response": "response_kernel",
             "patch_reduce": "patch_reduce_kernel<8>"}
    if stage in fixed:
        return fixed[stage]
    tiles = tuning.get("fft_tiles", {})
    fft = {"fft_fwd_y": ("fwd_y_kernel", "fwd_y"), "inv_x_green": ("inv_x_kernel", "inv_x"),
           "fft_inv_y": ("inv_y_kernel", "inv_y"), "fft_inv_z": ("inv_z_kernel", "inv_z")}
    if stage == "inv_xy_green":
        return "inv_xy_kernel<%d>" % n_mesh
    if stage == "inv_yz":
        return "inv_yz_kernel<%d>" % n_mesh
    if stage == "patch_fwd_z":
        return "patch_fwd_z_kernel<%d>" % n_mesh
    if stage == "fft_fwd_zy":
        return "fwd_zy_kernel<%d, %s>" % (n_mesh, "true" if tuning["deposit_mode"] >= 6
                                          else "false")
    if stage == "fft_fwd_z":
        return "fwd_z_kernel<%d, %s, %d>" % (n_mesh, "true" if tuning["deposit_mode"] >= 6
                                             else "false", tiles.get("fwd_z", 0))
    if stage == "fft_fwd_x_bin":
        return "fwd_x_bin_kernel<%d, false, true, %d>" % (n_mesh, tiles.get("fwd_x", 0))
    name, key = fft[stage]
    return "%s<%d, %d>" % (name, n_mesh, tiles.get(key, 0))


def load_traffic(workload, stage, kernel):
    """Measured HBM bytes per launch (profiles/traffic.json), or None when there is no
    record for this kernel or its source changed after the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)[workload]["kernels"][stage][kernel]
        if rec.get("source_sha") != source_sha(KERNEL_SOURCES[stage]):
            return None
        return rec["bytes_per_launch"]
    except Exception:
        return None


def make_workload(name, mass_index, order):
    from synth import CONFIGS, batched_lattices, zeldovich_lattice
    cfg = dict(CONFIGS[name])
    if cfg["n_boxes"] == 1:
        m = cfg["m_nu"][mass_index % len(cfg["m_nu"])]
        seed = cfg["seeds"][mass_index % len(cfg["seeds"])]
        pos = zeldovich_lattice(cfg["n_side"], cfg["box"], cfg["sigma_cells"], seed,
                                order=order)[None]
        masses = np.array([m])
    else:
        pos, masses = batched_lattices(cfg, order=order)
    return cfg, np.ascontiguousarray(pos), masses


SURROGATE_BLOB = os.path.join(ROOT, "paper_1209_0461_amd", "data", "surrogate_pm256.npy")


def measure_surrogate(ctx, binding, pos, acc, a_now, steps, stream, timing_exact, names):
    """Same step with the surrogate response: accuracy of R against the exact integral
    (check mode, every box and non-empty bin), the step's rate with the network beside its
    rate with the integral (the same eager loop, no event pairs) and the network's kernel
    time (event pairs around it alone)."""
    binding.pm_nu_surrogate_load(ctx.h, np.load(SURROGATE_BLOB))
    binding.pm_nu_set_response_mode(ctx.h, 2)
    ctx.step(pos, acc, a_now)
    _, counts, _ = ctx.bins()
    ok = counts > 0
    errs = []
    for b in range(ctx.n_boxes):
        ex, su = binding.pm_nu_get_surrogate_check(ctx.h, b, ctx.cfg.n_kbins)
        errs.append(np.abs(su[ok] / ex[ok] - 1.0))
    errs = np.concatenate(errs)
    def rate(mode):
        # the same eager step in both response modes, no event pairs, at least 100 steps
        binding.pm_nu_set_response_mode(ctx.h, mode)
        for _ in range(3):
            ctx.step(pos, acc, a_now)
        stream.synchronize()
        n = max(steps, 100)
        t0 = time.perf_counter()
        for _ in range(n):
            ctx.step(pos, acc, a_now)
        stream.synchronize()
        return n / (time.perf_counter() - t0)

    exact_rate = rate(0)
    sur_rate = rate(1)
    # the network's kernel time: event pairs around it alone, in a loop of their own
    binding.pm_nu_read_timing(ctx.h)
    binding.pm_nu_set_timing(ctx.h, True)
    binding.pm_nu_set_timing_mask(ctx.h, 1 << names.index("surrogate"))
    for _ in range(steps):
        ctx.step(pos, acc, a_now)
    stream.synchronize()
    t = binding.pm_nu_read_timing(ctx.h)
    binding.pm_nu_set_timing(ctx.h, False)
    binding.pm_nu_set_response_mode(ctx.h, 0)
    sur_ms = t["surrogate"][0] / max(1, t["surrogate"][1])
    ex_ms = timing_exact["nu_response"][0] / max(1, timing_exact["nu_response"][1])
    return {"steps_per_s": sur_rate, "ms_per_step": 1e3 / sur_rate,
            "steps_per_s_exact_same_loop": exact_rate,
            "response_ms_exact": ex_ms, "response_ms_surrogate": sur_ms,
            "R_max_rel_err": float(errs.max()), "R_rms_rel_err": float(np.sqrt(np.mean(errs ** 2))),
            "bar": 1e-3}


def measure_variants(ctx, binding, pos, acc, a_now, stream, names, steps=20):
    """Appendix C (the exact I(x) in place of the fit) and Appendix B (more iterations of
    the implicit current node): the response kernel's time and the change each makes to
    P_nu^{1/2} and to the force, against the default step (fit, one iteration)."""
    import torch

    def run(series, iterations):
        binding.pm_nu_set_kernel(ctx.h, series)
        binding.pm_nu_set_iterations(ctx.h, iterations)
        for _ in range(3):
            ctx.step(pos, acc, a_now)
        stream.synchronize()
        binding.pm_nu_read_timing(ctx.h)
        binding.pm_nu_set_timing_mask(ctx.h, 1 << names.index("nu_response"))
        for _ in range(steps):
            ctx.step(pos, acc, a_now)
        stream.synchronize()
        t = binding.pm_nu_read_timing(ctx.h)
        binding.pm_nu_set_timing(ctx.h, False)
        pn = np.concatenate([ctx.spectrum(b)["pnu_half"] for b in range(ctx.n_boxes)])
        return t["nu_response"][0] / max(1, t["nu_response"][1]), pn, acc.clone()

    base_ms, base_pn, base_acc = run(0, 1)
    ok = base_pn != 0
    out = {"fit_1_iteration": {"response_ms": base_ms}}
    for name, series, iterations in (("exact_kernel", 1, 1), ("fit_2_iterations", 0, 2),
                                     ("exact_kernel_2_iterations", 1, 2)):
        ms, pn, a = run(series, iterations)
        out[name] = {"response_ms": ms,
                     "pnu_half_max_rel_change": float(np.abs(pn[ok] / base_pn[ok] - 1).max()),
                     "force_rms_rel_change": float(torch.sqrt(((a - base_acc) ** 2).sum()
                                                              / (base_acc ** 2).sum()))}
    binding.pm_nu_set_kernel(ctx.h, 0)
    binding.pm_nu_set_iterations(ctx.h, 1)
    return out


def measure_loop(cfg, pos, masses, stream, tuning, n_steps=50, a_start=0.5):
    """The loop of Sec. 4.3 through pm_nu_advance: n_steps kick-drift-kick steps from a_start
    to cfg["a_now"] after a stored history from cfg["a_lo"] to a_start, on a context of its
    own. Reports steps/s of the whole loop (host time grid and uploads included) and the
    time of the interpolation, which carries the leapfrog (HIP events)."""
    import torch
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, synthetic_history
    nbox = pos.shape[0]
    J = cfg["n_hist"]
    ctx = PMNu(cfg["n_mesh"], pos.shape[1], cfg["box"], cfg["n_kbins"], J + n_steps + 2,
               list(masses), substeps=cfg["substeps"])
    binding.pm_nu_set_launch(ctx.h, tuning["deposit_mode"], tuning["deposit_block"],
                             tuning["interp_mode"], tuning["interp_block"])   # the step's shapes
    p = pos.clone()
    vel = torch.zeros_like(p)
    acc = torch.zeros_like(p)
    ctx.deposit(p)
    _, _, kmean = ctx.bins()
    nodes = log_spaced_nodes(cfg["a_lo"], a_start, J)
    for b in range(nbox):
        h = synthetic_history(kmean, np.sqrt(ctx.spectrum(b)["p_cdm"]), nodes, float(masses[b]))
        ctx.set_history(b, h)
    ctx.step(p, acc, a_start)
    a_steps = np.geomspace(a_start, cfg["a_now"], n_steps + 1)
    ctx.advance(p, vel, acc, a_steps[:3])        # warm-up (also moves the history on)
    stream.synchronize()
    names = list(binding.pm_nu_read_timing(ctx.h))
    binding.pm_nu_set_timing_mask(ctx.h, 1 << names.index("cic_interp"))
    t0 = time.perf_counter()
    ctx.advance(p, vel, acc, a_steps[2:])
    stream.synchronize()
    dt = time.perf_counter() - t0
    t = binding.pm_nu_read_timing(ctx.h)
    binding.pm_nu_set_timing(ctx.h, False)
    n = n_steps - 2
    it_ms = t["cic_interp"][0] / max(1, t["cic_interp"][1])
    # interpolation with the leapfrog applied: x, u in and x, u out per particle besides the
    # 8 corners of the acceleration grid (the grid counted once, as in the step)
    it_bytes = (48 * pos.shape[1] + 12 * cfg["n_mesh"] ** 3) * nbox
    finite = bool(torch.isfinite(p).all() and torch.isfinite(vel).all())
    ctx.close()
    return {"steps": n, "a": [float(a_steps[2]), float(a_steps[-1])],
            "steps_per_s": n / dt, "ms_per_step": 1e3 * dt / n,
            "interp_leapfrog_ms": it_ms, "interp_leapfrog_gbs": it_bytes / (it_ms * 1e-3) / 1e9,
            "particle_updates_per_s": n / dt * pos.shape[1] * nbox, "finite": finite,
            "note": "HIP events around the interpolation only, which applies each step's "
                    "kick and next drift; each step's time grid is built on the host and "
                    "copied in stream order"}


def cpu_baseline(cfg, pos, masses, hists):
    """Time the FP64 oracle on one full step of box 0 (single-threaded NumPy)."""
    import oracle.step as ostep
    t0 = time.perf_counter()
    ostep.full_step(pos[0], cfg["n_mesh"], cfg["box"], cfg["n_kbins"], hists[0], cfg["a_now"],
                    float(masses[0]), substeps=cfg["substeps"])
    dt = time.perf_counter() - t0
    nbox = pos.shape[0]
    return {"value": 1.0 / (dt * nbox), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one full FP64 oracle step of one {cfg['n_mesh']}^3 box "
                      f"({pos.shape[1]} particles), {dt:.1f} s, single-threaded NumPy"
                      + (f"; scaled to {nbox} boxes" if nbox > 1 else "")}


def measure_workload(name, args, dev, full):
    """Time the step of one workload on this GPU. `full` adds the surrogate, the kernel
    variants, the stepping loop and the oracle's CPU timing (the headline workload);
    otherwise only steps/s, the step's share of the roofline and its dominant kernel."""
    import torch
    from paper_1209_0461_amd import PMNu, binding
    from synth import log_spaced_nodes, synthetic_history
    cfg, pos_np, masses = make_workload(name, args.mass_index, args.order)
    nbox, npart = pos_np.shape[0], pos_np.shape[1]
    n_mesh, nbins, J = cfg["n_mesh"], cfg["n_kbins"], cfg["n_hist"]
    a_now = cfg["a_now"]
    nodes = log_spaced_nodes(cfg["a_lo"], a_now, J)
    graph = args.graph if full else nbox > 1
    steps = args.steps
    warmup = args.warmup

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = PMNu(n_mesh, npart, cfg["box"], nbins, J + 2, masses, substeps=cfg["substeps"])
        pos = torch.from_numpy(pos_np).to(dev)
        acc = torch.zeros_like(pos)
        # stored history: synthetic linear growth scaled to this run's measured spectrum
        ctx.deposit(pos)
        _, _, kmean = ctx.bins()
        hists = []
        for b in range(nbox):
            pc = ctx.spectrum(b)["p_cdm"]
            h = synthetic_history(kmean, np.sqrt(pc), nodes, float(masses[b]))
            ctx.set_history(b, h)
            hists.append(h)
        if not args.no_autotune:
            binding.pm_nu_autotune(ctx.h, pos, acc, a_now)
        tuning = json.loads(binding.pm_nu_tuning(ctx.h))
        for _ in range(warmup):
            ctx.step(pos, acc, a_now)
        if graph:
            binding.pm_nu_graph_capture(ctx.h, pos, acc, a_now)
            for _ in range(warmup):
                binding.pm_nu_graph_launch(ctx.h)
        stream.synchronize()
        # per-stage profile: an event pair around every kernel, on untimed eager steps
        binding.pm_nu_read_timing(ctx.h)
        binding.pm_nu_set_timing(ctx.h, True)
        for _ in range(min(steps, 10)):
            ctx.step(pos, acc, a_now)
        stream.synchronize()
        timing = binding.pm_nu_read_timing(ctx.h)
        names = list(timing)
        dom = max((k for k in names if timing[k][1] > 0), key=lambda k: timing[k][0])
        # timed region: events only around the dominant kernel (graph replays carry none)
        binding.pm_nu_set_timing_mask(ctx.h, 0 if graph else 1 << names.index(dom))
        stream.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            if graph:
                binding.pm_nu_graph_launch(ctx.h)
            else:
                ctx.step(pos, acc, a_now)
        stream.synchronize()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        timed = binding.pm_nu_read_timing(ctx.h)
        binding.pm_nu_set_timing(ctx.h, False)
        if timed[dom][1] > 0:
            dom_ms, dom_source = timed[dom][0] / timed[dom][1], "timed region"
        else:
            dom_ms, dom_source = timing[dom][0] / timing[dom][1], "eager profile steps"
        sp = ctx.spectrum(0)
        finite = bool(torch.isfinite(acc).all()) and bool(np.isfinite(sp["ratio"]).all())
        surrogate = variants = loop = None
        if full and os.path.exists(SURROGATE_BLOB) and not args.no_surrogate and not graph:
            surrogate = measure_surrogate(ctx, binding, pos, acc, a_now, steps, stream,
                                          timing, names)
        if full and not args.no_variants:
            variants = measure_variants(ctx, binding, pos, acc, a_now, stream, names)
        if full and not args.no_loop and not graph:
            loop = measure_loop(cfg, pos, masses, stream, tuning)
        ctx.close()
        del pos, acc
    torch.cuda.empty_cache()

    n_partial = (n_mesh // tuning["fft_tiles"]["fwd_x"]) * (n_mesh // 2 + 1)
    sb = stage_bytes(n_mesh, npart, nbox, nbins, J, n_partial, tuning["deposit_mode"])
    stages = {k: {"ms_per_launch": v[0] / v[1], "launches": v[1],
                  "gbs": sb.get(k, 0) / (v[0] / v[1] * 1e-3) / 1e9 if k in sb else None}
              for k, v in timing.items() if v[1] > 0}
    value = steps / dt
    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * dt / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "dtype_detail": "FP32 deposit/FFT/Green/interpolation; FP64 k-bin sums and the "
                        "neutrino history integral",
        "data": "synthetic",
        "config": {"workload": f"{name}: {nbox} x {npart} particles on {n_mesh}^3, "
                               f"L={cfg['box']} Mpc/h, {nbins} k-bins, {J} history nodes "
                               f"over a in [{cfg['a_lo']}, {a_now}], Q={cfg['substeps']}, "
                               f"M_nu={','.join(f'{m:.3g}' for m in masses[:4])}"
                               + ("..." if nbox > 4 else "") + " eV",
                   "n_mesh": n_mesh, "n_particles": npart * nbox, "n_boxes": nbox,
                   "graph": bool(graph), "particle_order": args.order,
                   "launch": tuning},
        "particle_updates_per_s": value * npart * nbox,
        "finite": finite,
    }
    step_bytes = step_algorithmic_bytes(n_mesh, npart, nbox, nbins, J)
    out["step_hbm"] = {"algorithmic_bytes": step_bytes,
                       "achieved_gbs": step_bytes * value / 1e9,
                       "frac": step_bytes * value / 1e9 / HBM_PEAK_GBS}
    if stages:
        ach = sb[dom] / (dom_ms * 1e-3) / 1e9
        kname = kernel_name(dom, tuning, n_mesh)
        traffic = load_traffic(name, dom, kname)
        out["roofline"] = {"bound": "hbm", "kernel": dom, "kernel_name": kname,
                           "ms_per_launch": dom_ms, "timing": f"HIP events, {dom_source}",
                           "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS,
                           "traffic": traffic,
                           "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, "
                                           "copy-calibrated)",
                           "algorithmic_bytes_per_launch": sb[dom]}
        out["stages"] = stages
        out["stages_note"] = ("per-stage HIP event pairs around every kernel on "
                              f"{min(steps, 10)} eager steps before the timed region")
    if surrogate is not None:
        out["surrogate"] = surrogate
    if variants is not None:
        out["variants"] = variants
    if loop is not None:
        out["loop"] = loop
    if full and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, pos_np, masses, hists)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="pm256")
    ap.add_argument("--mass-index", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true", help="replay the step as a HIP graph")
    ap.add_argument("--order", default="morton", choices=["morton", "c"],
                    help="particle order of the synthetic lattice (space-filling curve or C)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate-versus-integral measurement")
    ap.add_argument("--no-loop", action="store_true",
                    help="skip the time-stepping loop measurement")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the exact-kernel and second-iteration measurement")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the 512^3 and batched workloads after the main one")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the step is "
              "single-GPU in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1209_0461_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_1209_0461_amd import build
        build.build()
    dev = torch.device("cuda:0")

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe}))
        return

    out = measure_workload(args.workload, args, dev, full=True)
    if not args.no_others and args.workload == "pm256":
        # the other single-GPU workloads, each in its own timed region, reported beside
        # the headline (the 512^3 box eagerly, the 64 small boxes through a HIP graph)
        out["other_workloads"] = {}
        for other in ("pm512", "batch64x64"):
            print(f"bench: {other}", file=sys.stderr, flush=True)
            o = measure_workload(other, args, dev, full=False)
            out["other_workloads"][other] = {
                k: o[k] for k in ("value", "unit", "steps", "ms_per_step",
                                  "particle_updates_per_s", "step_hbm", "roofline", "config",
                                  "finite") if k in o}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
