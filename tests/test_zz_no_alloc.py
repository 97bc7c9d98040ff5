"""The no-allocation entry point (pm_nu_binned_power_noalloc) against the context's stage
(ii) (pm_nu_deposit + pm_nu_get_spectrum) on the same inputs: two calls in a row, the
second with a smaller mesh, fewer bins and fewer particles, then the first again. Both
sides sum the density exactly in fixed point and bin in FP64, so P_cdm agrees to rounding
of the FP64 bin sums (1e-12 here; the parity bar against the oracle is 2e-6)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _context_power(pos, n_mesh, box, nb):
    import torch
    from paper_1209_0461_amd import PMNu
    ctx = PMNu(n_mesh, pos.shape[0], box, nb, 8, [0.3])
    ctx.deposit(torch.from_numpy(pos).cuda())
    p = ctx.spectrum(0)["p_cdm"]
    _, counts, _ = ctx.bins()
    ctx.close()
    return p, counts


def _noalloc_power(pos, n_mesh, box, nb):
    import torch
    from paper_1209_0461_amd import binding
    p = torch.full((nb,), -1.0, dtype=torch.float64, device="cuda")
    binding.pm_nu_binned_power_noalloc(torch.from_numpy(pos).cuda(), n_mesh, box, nb, p)
    torch.cuda.synchronize()
    return p.cpu().numpy()


def test_noalloc_binned_power_matches_context():
    from synth import zeldovich_lattice
    import oracle.step as ostep
    cases = [(64, 64, 256.0, 48, 0.3, 21),     # n_side, n_mesh, box, bins, sigma, seed
             (16, 32, 128.0, 20, 0.25, 22),     # smaller: mesh, bins and particles
             (64, 64, 256.0, 48, 0.3, 21)]
    for ns, nm, box, nb, sig, seed in cases:
        pos = zeldovich_lattice(ns, box, sig, seed)
        print(f"no-alloc spectrum: N={nm} B={nb} np={pos.shape[0]}", flush=True)
        ref, counts = _context_power(pos, nm, box, nb)
        got = _noalloc_power(pos, nm, box, nb)
        ok = counts > 0
        assert np.all(got[~ok] == 0.0)
        rel = np.abs(got[ok] / ref[ok] - 1.0).max()
        orc = ostep.spectrum(pos, nm, box, nb)["p_cdm"]
        rel_o = np.abs(got[ok] / orc[ok] - 1.0).max()
        print(f"  vs context {rel:.2e}, vs oracle {rel_o:.2e}", flush=True)
        assert rel <= 1e-12
        assert rel_o <= 2e-6


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    from paper_1209_0461_amd import binding
    pos = torch.zeros((8, 3), dtype=torch.float32, device="cuda")
    for nm, nb in ((128, 16), (48, 16), (32, 300)):
        p = torch.zeros(nb, dtype=torch.float64, device="cuda")
        with pytest.raises(binding.PMNuError) as e:
            binding.pm_nu_binned_power_noalloc(pos, nm, 100.0, nb, p)
        assert e.value.code == -1
