"""The seeded input generators (CPU): determinism, ranges, amplitude, particle order."""
import numpy as np

from synth import CONFIGS, batched_lattices, log_spaced_nodes, morton_codes, zeldovich_lattice
from synth.history import growth


def test_lattice_is_seeded_in_range_and_has_the_requested_rms():
    a = zeldovich_lattice(16, 64.0, 0.3, seed=5, order="c")
    b = zeldovich_lattice(16, 64.0, 0.3, seed=5, order="c")
    assert a.dtype == np.float32 and a.shape == (4096, 3) and np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() < 64.0
    g = (np.arange(16) + 0.5) * 4.0
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    d = (a.astype(np.float64) - q + 32.0) % 64.0 - 32.0
    assert abs(np.sqrt(np.mean(np.sum(d * d, axis=1))) / 4.0 - 0.3) < 1e-5


def test_morton_order_is_a_permutation_of_c_order():
    c = zeldovich_lattice(8, 32.0, 0.2, seed=2, order="c")
    m = zeldovich_lattice(8, 32.0, 0.2, seed=2)
    codes = morton_codes(8)
    assert sorted(codes.tolist()) == list(range(512))
    assert np.array_equal(m[codes.astype(np.int64)], c)
    # the first 64 Morton entries are the lattice block [0,4)^3
    assert np.all(m[:64] < 4 * 4.0 + 1.0)


def test_batched_masses_and_seeds():
    cfg = dict(CONFIGS["batch64x64"], n_boxes=3, n_side=8, n_mesh=8)
    pos, masses = batched_lattices(cfg)
    assert pos.shape == (3, 512, 3)
    assert np.all((masses >= 0.05) & (masses <= 0.6))
    assert not np.array_equal(pos[0], pos[1])


def test_growth_factor_matter_era_and_rate():
    d, f = growth(np.array([1e-3, 2e-3, 1.0]), 0.3)
    assert abs(d[1] / d[0] - 2.0) < 2e-3          # D ~ a deep in matter domination
    assert abs(f[0] - 1.0) < 1e-3
    assert abs(f[2] - 0.3 ** 0.55) < 0.01        # f ~ Omega_M^0.55 today


def test_log_spaced_nodes():
    a = log_spaced_nodes(0.01, 1.0, 200)
    assert a[0] == 0.01 and abs(a[-1] - 1.0) < 1e-15 and np.allclose(np.diff(np.log(a)),
                                                                       np.log(100) / 199)
