"""Write pm512_oracle.npz: the FP64 oracle's results for one step of the 512^3 workload, for
the GPU parity test at that size (the oracle needs minutes and tens of GB there, so its
results are stored once instead of recomputed in every GPU run).

Workload: 512^3 particles (Zel'dovich lattice, k^-2 spectrum, RMS displacement 0.3 cells,
seed 512, Morton order) on a 512^3 mesh, L = 1000 Mpc/h, 128 k-bins, a 400-node history on
a in [0.01, 1] (399 stored nodes, the step at a = 1), Q = 8, M_nu = 0.3 eV in three equal
species. The history is synth.synthetic_history scaled to the oracle's own P_cdm.

Stored: the bin geometry and edges, P_cdm, P_nu^{1/2}, R and the new history node of every
bin; the accelerations of 16384 particles and the three acceleration grids at 4096 nodes,
both drawn with numpy's default_rng(5120); the SHA-256 of the FP32 positions, so that the
test can tell that it regenerated the same input.

This script calls only oracle/ (and synth/ for the seeded input):

    python tests/golden/make_pm512_oracle.py        # about 3 minutes, ~30 GB of memory
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pm512_oracle.npz")
SAMPLE_SEED = 5120
N_PART_SAMPLE = 16384
N_NODE_SAMPLE = 4096


def main():
    import oracle.response as oresp
    import oracle.step as ostep
    from synth import CONFIGS, log_spaced_nodes, synthetic_history, zeldovich_lattice
    c = CONFIGS["pm512"]
    n, box, nb, J, m = c["n_mesh"], c["box"], c["n_kbins"], c["n_hist"], c["m_nu"][0]
    t0 = time.perf_counter()
    pos = zeldovich_lattice(c["n_side"], box, c["sigma_cells"], c["seeds"][0])
    sha = hashlib.sha256(pos.tobytes()).hexdigest()
    print(f"input {pos.shape} sha256 {sha[:16]} ({time.perf_counter() - t0:.0f} s)", flush=True)
    sp = ostep.spectrum(pos, n, box, nb)
    del sp["rho"]
    print(f"spectrum ({time.perf_counter() - t0:.0f} s)", flush=True)
    nodes = log_spaced_nodes(c["a_lo"], c["a_now"], J)
    hist = synthetic_history(sp["k_mean"], np.sqrt(sp["p_cdm"]), nodes, m)
    r = oresp.nu_amplitude(sp["k_mean"], sp["counts"], np.sqrt(sp["p_cdm"]), hist["a"],
                           hist["pm_half"], hist["pnu_half"][-1], hist["pnu_half_init"],
                           hist["theta_over_delta_init"], c["a_now"], m, 0.3, 0.7,
                           c["substeps"])
    rng = np.random.default_rng(SAMPLE_SEED)
    pidx = np.sort(rng.choice(pos.shape[0], N_PART_SAMPLE, replace=False))
    nidx = np.sort(rng.choice(n ** 3, N_NODE_SAMPLE, replace=False))
    acc, grids = ostep.forces(pos[pidx], sp["delta_k"], n, box, sp["k_mean"], sp["counts"],
                              r["ratio"], r["f_nu"], c["a_now"], 0.3, return_grids=True)
    gs = grids.reshape(3, -1)[:, nidx].T.copy()
    print(f"forces ({time.perf_counter() - t0:.0f} s)", flush=True)
    np.savez_compressed(OUT, pos_sha256=np.array(sha), edges=sp["edges"],
                        counts=sp["counts"], k_mean=sp["k_mean"], p_cdm=sp["p_cdm"],
                        pnu_half=r["pnu_half"], ratio=r["ratio"],
                        pm_half_now=r["pm_half_now"], particle_index=pidx, acc=acc,
                        node_index=nidx, grid=gs)
    print(f"wrote {OUT} ({os.path.getsize(OUT) / 1e3:.0f} kB)", flush=True)


if __name__ == "__main__":
    main()
