"""The launch-shape autotuner: every FFT tile candidate computes the step the oracle does,
the tuner reports its choice, and a cached choice is read back instead of re-timed.

The three tile candidates of each of the six FFT passes are run together as
fft = (v, v, v, v, v, v) for v = 0, 1, 2 (the passes are independent, so this covers every
candidate of every pass) at the mesh sizes where the candidates differ (N >= 64)."""
import json

import numpy as np
import pytest

from gpu_cases import TOL_FORCE_RMS, TOL_NU, make_inputs, oracle_case, rms_rel

pytestmark = pytest.mark.gpu

CASES = [  # n_side, n_mesh, box, bins, J, a_now, M_nu, seed
    (32, 64, 256.0, 48, 30, 1.0, 0.45, 31),
    (64, 128, 256.0, 40, 24, 0.8, 0.3, 32),
    (64, 256, 512.0, 64, 20, 1.0, 0.3, 33),
    (64, 512, 1000.0, 128, 16, 1.0, 0.3, 34),
]


@pytest.mark.parametrize("case", CASES, ids=[f"N{c[1]}" for c in CASES])
def test_every_fft_tile_candidate_matches_oracle(case):
    import torch
    from paper_1209_0461_amd import PMNu, binding
    ns, nm, box, nb, J, a_now, m, seed = case
    pos = make_inputs(ns, box, 0.3, seed)
    hist, ref = oracle_case(pos, nm, box, nb, J, 0.01, a_now, m)
    ok = ref["counts"] > 0
    ctx = PMNu(nm, pos.shape[0], box, nb, J + 4, [m])
    p = torch.from_numpy(pos).cuda()
    accs = []
    for v in (0, 1, 2):
        ctx.set_history(0, hist)
        binding.pm_nu_set_fft_tiles(ctx.h, [v] * 6)
        tiles = json.loads(binding.pm_nu_tuning(ctx.h))["fft_tiles"]
        acc = torch.zeros_like(p)
        ctx.step(p, acc, a_now)
        torch.cuda.synchronize()
        sp = ctx.spectrum(0)
        prel = np.abs(sp["p_cdm"][ok] / ref["p_cdm"][ok] - 1).max()
        nrel = np.abs(sp["pnu_half"][ok] / ref["pnu_half"][ok] - 1).max()
        ferr = rms_rel(acc.cpu().numpy(), ref["acc"])
        print(f"N={nm} candidate {v} {tiles}: P_cdm {prel:.2e} P_nu {nrel:.2e} force {ferr:.2e}",
              flush=True)
        assert prel <= 2e-6 and nrel <= TOL_NU and ferr <= TOL_FORCE_RMS
        accs.append(acc.cpu().numpy())
    # each line's transform is the same sequence of operations whatever the tile, up to the
    # compiler's choice of fused multiply-adds in each instantiation: the candidates agree
    # with each other to FP32 rounding
    for a in accs[1:]:
        assert rms_rel(a, accs[0]) < 2e-6
    with pytest.raises(binding.PMNuError):
        binding.pm_nu_set_fft_tiles(ctx.h, [0, 0, 3, 0, 0, 0])
    ctx.close()


def test_autotune_reports_fft_choice_and_reloads_it_from_the_cache(tmp_path):
    import time
    import torch
    from paper_1209_0461_amd import PMNu, binding
    ns, nm, box, nb, J, a_now, m = 64, 128, 256.0, 40, 24, 0.8, 0.3
    pos = make_inputs(ns, box, 0.3, 35)
    hist, ref = oracle_case(pos, nm, box, nb, J, 0.01, a_now, m)
    cache = str(tmp_path / "tuning.jsonl")
    p = torch.from_numpy(pos).cuda()
    acc = torch.zeros_like(p)
    ctx = PMNu(nm, pos.shape[0], box, nb, J + 4, [m])
    ctx.set_history(0, hist)
    t0 = time.perf_counter()
    binding.pm_nu_autotune(ctx.h, p, acc, a_now, cache)
    t_tune = time.perf_counter() - t0
    first = json.loads(binding.pm_nu_tuning(ctx.h))
    assert len(first["fft"]) == 6 and set(first["fft_tiles"]) == {
        "fwd_z", "fwd_y", "fwd_x", "inv_x", "inv_y", "inv_z"}
    assert rms_rel(acc.cpu().numpy(), ref["acc"]) <= TOL_FORCE_RMS   # left a full step
    ctx.close()
    with open(cache) as f:
        lines = [json.loads(l) for l in f if l.strip()]
    assert len(lines) == 1 and lines[0]["fft"] == first["fft"]
    assert lines[0]["key"].endswith(f"/N{nm}/boxes1/np{pos.shape[0]}")
    # a second context with the same key takes the cached choice without timing anything
    ctx = PMNu(nm, pos.shape[0], box, nb, J + 4, [m])
    ctx.set_history(0, hist)
    binding.pm_nu_set_launch(ctx.h, 0, 256, 0, 256)
    binding.pm_nu_set_fft_tiles(ctx.h, [2, 1, 2, 1, 2, 1])
    t0 = time.perf_counter()
    binding.pm_nu_autotune(ctx.h, p, acc, a_now, cache)
    t_cached = time.perf_counter() - t0
    assert json.loads(binding.pm_nu_tuning(ctx.h)) == first
    print(f"autotune {t_tune * 1e3:.0f} ms, from the cache {t_cached * 1e3:.1f} ms {first}",
          flush=True)
    ctx.step(p, acc, a_now)
    torch.cuda.synchronize()
    assert rms_rel(acc.cpu().numpy(), ref["acc"]) <= TOL_FORCE_RMS
    ctx.close()
    # every launch shape the library accepts is taken from the cache, the fused patch
    # deposit (mode 9) and other tiles included
    lines[0].update(deposit_mode=9, fft=[2, 1, 2, 1, 2, 1])
    with open(cache, "w") as f:
        f.write(json.dumps(lines[0]) + "\n")
    ctx = PMNu(nm, pos.shape[0], box, nb, J + 4, [m])
    ctx.set_history(0, hist)
    binding.pm_nu_autotune(ctx.h, p, acc, a_now, cache)
    third = json.loads(binding.pm_nu_tuning(ctx.h))
    assert third["deposit_mode"] == 9 and third["fft"] == [2, 1, 2, 1, 2, 1], third
    ctx.step(p, acc, a_now)
    torch.cuda.synchronize()
    assert rms_rel(acc.cpu().numpy(), ref["acc"]) <= TOL_FORCE_RMS
    ctx.close()
