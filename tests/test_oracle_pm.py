"""Pins of the oracle's particle-mesh stages (CPU): invariants, brute force, linear theory
and a direct Ewald sum."""
import itertools

import numpy as np
import pytest
from scipy.special import erfc

from oracle import background as bg
from oracle import pm, step
from synth import zeldovich_lattice


def _lattice(n, box, offset=0.5):
    g = (np.arange(n) + offset) * (box / n)
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)


# ------------------------------------------------------------------ deposit ----
def test_cic_conserves_mass():
    rng = np.random.default_rng(1)
    pos = rng.uniform(0, 100.0, size=(5000, 3)).astype(np.float32)
    rho = pm.cic_deposit(pos, 16, 100.0)
    assert rho.sum() == pytest.approx(5000.0, rel=1e-13)
    assert rho.min() >= 0.0


@pytest.mark.parametrize("offset", [0.5, 0.0])
def test_uniform_lattice_has_zero_overdensity(offset):
    pos = _lattice(8, 64.0, offset)
    delta = pm.overdensity(pm.cic_deposit(pos, 8, 64.0), len(pos))
    assert np.abs(delta).max() < 1e-13


def test_single_particle_weights_by_hand():
    # spacing 2: x = 2.5 -> u = 1.25, nodes 1 (0.75) and 2 (0.25);
    # y = 5.0 -> u = 2.5, nodes 2, 3 (0.5 each); z = 7.5 -> u = 3.75, nodes 3 (0.25), 4 (0.75)
    rho = pm.cic_deposit(np.array([[2.5, 5.0, 7.5]]), 8, 16.0)
    expect = {}
    for (ix, wx), (iy, wy), (iz, wz) in itertools.product(
            [(1, 0.75), (2, 0.25)], [(2, 0.5), (3, 0.5)], [(3, 0.25), (4, 0.75)]):
        expect[(ix, iy, iz)] = wx * wy * wz
    for idx, w in expect.items():
        assert rho[idx] == pytest.approx(w, abs=1e-15)
    assert np.count_nonzero(rho) == 8


def test_particle_on_node_and_periodic_wrap():
    rho = pm.cic_deposit(np.array([[4.0, 0.0, 14.0]]), 8, 16.0)   # exactly on node (2, 0, 7)
    assert rho[2, 0, 7] == 1.0 and np.count_nonzero(rho) == 1
    rho = pm.cic_deposit(np.array([[15.0, 1.0, 1.0]]), 8, 16.0)   # u_x = 7.5 -> nodes 7 and 0
    assert rho[7, 0, 0] == pytest.approx(0.125) and rho[0, 0, 0] == pytest.approx(0.125)


def test_translation_by_one_cell_rolls_the_grid():
    rng = np.random.default_rng(2)
    pos = rng.uniform(0, 32.0, size=(300, 3))
    rho = pm.cic_deposit(pos, 16, 32.0)
    moved = np.mod(pos + np.array([2.0, 0.0, -4.0]), 32.0)
    assert np.allclose(pm.cic_deposit(moved, 16, 32.0),
                       np.roll(rho, (1, 0, -2), axis=(0, 1, 2)), atol=1e-12)


def test_interpolation_of_linear_field_is_exact_between_nodes():
    # CIC interpolation reproduces a field that is linear inside the cell
    n, box = 8, 8.0
    g = np.zeros((1, n, n, n))
    g[0] = np.arange(n)[:, None, None] * 1.0 + 2.0 * np.arange(n)[None, :, None]
    p = np.array([[2.3, 4.6, 1.1]])
    assert pm.cic_interpolate(p, g, box)[0, 0] == pytest.approx(2.3 + 2 * 4.6, abs=1e-12)


# ----------------------------------------------------------------------- FFT ----
def test_forward_fft_equals_brute_force_dft():
    n = 8
    rng = np.random.default_rng(3)
    f = rng.standard_normal((n, n, n))
    x = np.arange(n)
    ref = np.zeros((n, n, n // 2 + 1), dtype=complex)
    for kx in range(n):
        for ky in range(n):
            for kz in range(n // 2 + 1):
                ph = np.exp(-2j * np.pi * (kx * x[:, None, None] + ky * x[None, :, None]
                                           + kz * x[None, None, :]) / n)
                ref[kx, ky, kz] = np.sum(f * ph)
    assert np.allclose(pm.forward_modes(f), ref, atol=1e-11)


def test_inverse_fft_equals_brute_force_sum():
    n = 8
    rng = np.random.default_rng(4)
    f = rng.standard_normal((n, n, n))
    full = np.fft.fftn(f)
    x = np.arange(n)
    got = pm.inverse_real(pm.forward_modes(f), n)
    ref = np.zeros((n, n, n))
    for kx, ky, kz in itertools.product(range(n), repeat=3):
        ref += np.real(full[kx, ky, kz] * np.exp(2j * np.pi * (
            kx * x[:, None, None] + ky * x[None, :, None] + kz * x[None, None, :]) / n))
    assert np.allclose(got, ref / n ** 3, atol=1e-12)


# -------------------------------------------------------------------- k-bins ----
@pytest.mark.parametrize("n,nb", [(8, 6), (16, 10), (32, 32)])
def test_bin_counts_equal_brute_force(n, nb):
    edges, counts, k_mean = pm.bin_geometry(n, 100.0, nb)
    brute = np.zeros(nb)
    ksum = np.zeros(nb)
    half = n // 2
    for i, j, l in itertools.product(range(-half, half), range(-half, half), range(-half, half)):
        n2 = i * i + j * j + l * l
        if n2 == 0:
            continue
        b = max(bb for bb in range(nb) if edges[bb] <= n2) if n2 < edges[-1] else nb - 1
        brute[b] += 1
        ksum[b] += 2 * np.pi / 100.0 * np.sqrt(n2)
    assert np.array_equal(counts, brute)                # half-spectrum weights = full count
    assert counts.sum() == n ** 3 - 1
    ok = counts > 0
    assert np.allclose(k_mean[ok], ksum[ok] / brute[ok], rtol=1e-13)


def test_bin_edges_are_log_spaced_integers():
    edges = pm.bin_edges_n2(256, 64)
    assert edges[0] == 1 and edges[-1] == 3 * 256 * 256 // 4
    assert np.all(np.diff(edges) >= 0)
    r = np.log(edges[1:].astype(float)) / np.log(3 * 256 * 256 / 4.0)
    assert np.all(np.abs(r - np.arange(1, 65) / 64.0) < 0.5)


def test_plane_wave_power_lands_in_its_bin_with_right_normalisation():
    n, box, nb, m, amp = 16, 50.0, 12, 3, 0.01
    x = np.arange(n) * box / n
    delta = np.broadcast_to(amp * np.cos(2 * np.pi * m * x / box)[:, None, None], (n, n, n))
    p = pm.binned_power(pm.forward_modes(delta), n, box, nb)
    edges, counts, _ = pm.bin_geometry(n, box, nb)
    b = pm.bin_of_n2(np.array([m * m]), edges)[0]
    assert np.count_nonzero(p > 1e-20) == 1
    # variance amp^2/2 = (1/L^3) sum over modes of P  ->  C_b P_b = L^3 amp^2 / 2
    assert counts[b] * p[b] == pytest.approx(box ** 3 * amp ** 2 / 2, rel=1e-12)


def test_parseval_of_binned_power():
    rng = np.random.default_rng(5)
    n, box = 16, 80.0
    delta = rng.standard_normal((n, n, n))
    p = pm.binned_power(pm.forward_modes(delta), n, box, 9)
    _, counts, _ = pm.bin_geometry(n, box, 9)
    assert np.sum(counts * p) / box ** 3 == pytest.approx(np.var(delta), rel=1e-12)


# ------------------------------------------------------------------ forces ----
@pytest.mark.parametrize("m,tol", [(1, 2e-4), (2, 4e-4), (4, 3e-3)])
def test_zeldovich_plane_wave_force(m, tol):
    """delta = -div(psi) for a small displacement psi; the linear force is C psi."""
    n, box, a_now, om = 32, 128.0, 0.5, 0.3
    q = _lattice(n, box)
    amp = 1e-3 * box / n
    psi = amp * np.sin(2 * np.pi * m * q[:, 0] / box)
    pos = q.copy()
    pos[:, 0] = np.mod(q[:, 0] + psi, box)
    sp = step.spectrum(pos, n, box, 8)
    acc = step.forces(pos, sp["delta_k"], n, box, sp["k_mean"], sp["counts"],
                      np.ones(8), 0.0, a_now, om)
    c = 1.5 * om * bg.H0 ** 2 / a_now
    err = np.abs(acc[:, 0] - c * psi).max() / (c * amp)
    assert err < tol
    assert np.abs(acc[:, 1:]).max() < 1e-10 * c * amp


def test_neutrino_rescale_on_plane_wave():
    """With R(k) = r0 everywhere, delta_M = (1 - f + f r0) delta_cdm, so the force scales."""
    n, box, a_now, om = 16, 64.0, 0.5, 0.3
    q = _lattice(n, box)
    amp = 1e-3 * box / n
    psi = amp * np.sin(2 * np.pi * q[:, 1] / box)
    pos = q.copy()
    pos[:, 1] = np.mod(q[:, 1] + psi, box)
    sp = step.spectrum(pos, n, box, 8)
    base = step.forces(pos, sp["delta_k"], n, box, sp["k_mean"], sp["counts"], np.ones(8),
                       0.0, a_now, om)
    f, r0 = 0.05, 0.3
    got = step.forces(pos, sp["delta_k"], n, box, sp["k_mean"], sp["counts"],
                      np.full(8, r0), f, a_now, om)
    assert np.allclose(got, base * (1 - f + f * r0), rtol=1e-12, atol=1e-20)


def test_zero_neutrino_fraction_is_plain_pm():
    pos = zeldovich_lattice(16, 64.0, 0.3, seed=7).astype(np.float64)
    sp = step.spectrum(pos, 16, 64.0, 8)
    a = step.forces(pos, sp["delta_k"], 16, 64.0, sp["k_mean"], sp["counts"],
                    np.linspace(0.1, 1, 8), 0.0, 0.5, 0.3)
    b = step.forces(pos, sp["delta_k"], 16, 64.0, sp["k_mean"], sp["counts"],
                    np.ones(8), 0.0, 0.5, 0.3)
    assert np.array_equal(a, b)


def test_momentum_conservation():
    rng = np.random.default_rng(8)
    pos = rng.uniform(0, 64.0, size=(2000, 3))
    sp = step.spectrum(pos, 16, 64.0, 8)
    acc = step.forces(pos, sp["delta_k"], 16, 64.0, sp["k_mean"], sp["counts"],
                      np.full(8, 0.5), 0.02, 0.5, 0.3)
    assert np.abs(acc.sum(axis=0)).max() < 1e-11 * np.sqrt((acc ** 2).sum())


def _ewald_acc(r, box, strength, alpha=None, nreal=3, nk=8):
    """Acceleration at separation r from one periodic point mass with a uniform
    neutralising background (Ewald summation), strength S: phi = -S / |r| near the mass."""
    alpha = 2.0 / box if alpha is None else alpha
    acc = np.zeros(3)
    for nv in itertools.product(range(-nreal, nreal + 1), repeat=3):
        rn = r + box * np.array(nv)
        d = np.linalg.norm(rn)
        acc -= strength * rn / d ** 3 * (erfc(alpha * d)
                                          + 2 * alpha * d / np.sqrt(np.pi) * np.exp(-(alpha * d) ** 2))
    for kv in itertools.product(range(-nk, nk + 1), repeat=3):
        if kv == (0, 0, 0):
            continue
        k = 2 * np.pi * np.array(kv) / box
        k2 = k @ k
        acc -= strength * 4 * np.pi / box ** 3 * k / k2 * np.exp(-k2 / (4 * alpha ** 2)) * np.sin(k @ r)
    return acc


@pytest.mark.parametrize("sep_cells", [6.0, 8.0, 12.0])
@pytest.mark.parametrize("p0", [(20.3, 31.1, 30.7), (5.5, 5.5, 5.5), (10.0, 12.25, 3.1)])
def test_pair_force_matches_ewald_sum(sep_cells, p0):
    """Physics sanity of sign, units and normalisation: the PM pair force of two particles
    against the periodic point-mass force, S = C L^3 / (4 pi N_p).

    Without deconvolution: dividing by W^2 amplifies the aliased near-Nyquist power of a
    point-like source (errors of order one at a few cells), while it is what makes smooth
    fields accurate (the plane-wave test above). The normalisation at low k is the same."""
    n, box, a_now, om = 32, 64.0, 0.5, 0.3
    cell = box / n
    p0 = np.array(p0)
    p1 = p0 + np.array([sep_cells * cell * 0.8, sep_cells * cell * 0.6, 0.0])
    pos = np.mod(np.stack([p0, p1]), box)
    sp = step.spectrum(pos, n, box, 8)
    acc = step.forces(pos, sp["delta_k"], n, box, sp["k_mean"], sp["counts"], np.ones(8),
                      0.0, a_now, om, deconvolve=False)
    c = 1.5 * om * bg.H0 ** 2 / a_now
    ref = _ewald_acc(p1 - p0, box, c * box ** 3 / (4 * np.pi * 2))
    assert np.linalg.norm(acc[1] - ref) / np.linalg.norm(ref) < 0.025
    assert acc[1] @ (p0 - p1) > 0          # attractive


# ----------------------------------- R(|k|) on every mode (eq. (phases), Sec. 4.3 (iv)) ----
def _modes_lnk(n, box):
    n2, _ = pm.mode_n2_and_weight(n)
    with np.errstate(divide="ignore"):
        return n2, np.log((2.0 * np.pi / box) * np.sqrt(n2.astype(np.float64)))


@pytest.mark.parametrize("n,nb,n_empty", [(32, 32, 4), (64, 48, 6), (16, 8, 0)])
def test_ratio_linear_in_ln_k_comes_back_on_every_mode(n, nb, n_empty):
    """A bin ratio linear in ln k (R_b = alpha + beta ln kbar_b) is reproduced exactly on
    every mode between the first and last non-empty bin means by interpolation in ln k
    (not in k), and held at the end values outside them. Empty bins carry a huge value in
    R, which must not reach any mode."""
    box = 128.0
    _, counts, kmean = pm.bin_geometry(n, box, nb)
    ok = counts > 0
    assert int((~ok).sum()) == n_empty
    alpha, beta = 0.7, -0.15
    lnkb = np.log(np.where(ok, kmean, 1.0))
    ratio = np.where(ok, alpha + beta * lnkb, 1e6)
    got = pm.ratio_on_modes(n, box, kmean, counts, ratio)
    n2, lnk = _modes_lnk(n, box)
    lo, hi = lnkb[ok][0], lnkb[ok][-1]
    expect = alpha + beta * np.minimum(np.maximum(lnk, lo), hi)
    nz = n2 > 0
    assert np.abs(got[nz] - expect[nz]).max() < 1e-14
    assert np.all(np.abs(got) < 2.0)                 # nothing from the empty bins
    # modes above the last bin mean exist and take its value exactly
    above = nz & (lnk > hi)
    assert above.any() and np.all(got[above] == ratio[ok][-1])


def test_ratio_on_modes_hand_computed_8_cubed():
    """N = 8, L = 2 pi (so |k| = |n|), 8 bins. Counting the modes by hand:
    bin 0 holds |n|^2 = 1 (6 modes), bin 1 |n|^2 = 2 (12), bin 2 |n|^2 = 3 (8) and 4 (6),
    bin 3 |n|^2 = 5 (24) and 6 (24). Bin means: 1, sqrt 2, (8 sqrt 3 + 6*2)/14,
    (sqrt 5 + sqrt 6)/2. The top mode |n|^2 = 48 lies above the last bin mean."""
    n, box, nb = 8, 2.0 * np.pi, 8
    edges, counts, kmean = pm.bin_geometry(n, box, nb)
    assert list(edges[:5]) == [1, 2, 3, 5, 7]
    assert list(counts[:4]) == [6, 12, 14, 48]
    kb = np.array([1.0, np.sqrt(2.0), (8 * np.sqrt(3.0) + 12.0) / 14.0,
                   (np.sqrt(5.0) + np.sqrt(6.0)) / 2.0])
    assert np.allclose(kmean[:4], kb, rtol=1e-15)
    ratio = np.array([1.0, 0.5, 0.25, 0.2, 0.15, 0.1, 0.08, 0.05])
    got = pm.ratio_on_modes(n, box, kmean, counts, ratio)
    nx, ny, nz = pm.mode_indices(n)
    n2 = nx * nx + ny * ny + nz * nz
    # single-shell bins: the modes sit exactly at the bin mean
    assert np.all(got[n2 == 1] == 1.0) and np.all(got[n2 == 2] == 0.5)
    # |k| = sqrt 3 between the means of bins 1 and 2
    t3 = np.log(np.sqrt(3.0) / np.sqrt(2.0)) / np.log(kb[2] / np.sqrt(2.0))
    assert np.allclose(got[n2 == 3], 0.5 + t3 * (0.25 - 0.5), rtol=0, atol=1e-15)
    # |k| = 2 between the means of bins 2 and 3
    t4 = np.log(2.0 / kb[2]) / np.log(kb[3] / kb[2])
    assert 0.0 < t4 < 1.0
    assert np.allclose(got[n2 == 4], 0.25 + t4 * (0.2 - 0.25), rtol=0, atol=1e-15)
    # above the last mean: the last bin's value
    assert kmean[-1] < np.sqrt(48.0)
    assert np.all(got[n2 == 48] == 0.05)


def test_ratio_between_bins_is_monotone_and_bounded():
    """Between two neighbouring non-empty bin means the interpolant stays between their
    values, for any R_b (a property of piecewise-linear interpolation)."""
    n, box, nb = 32, 128.0, 32
    _, counts, kmean = pm.bin_geometry(n, box, nb)
    ok = counts > 0
    rng = np.random.default_rng(5)
    ratio = np.where(ok, rng.uniform(0.1, 1.0, nb), -1.0)
    got = pm.ratio_on_modes(n, box, kmean, counts, ratio)
    n2, lnk = _modes_lnk(n, box)
    lnkb, rb = np.log(kmean[ok]), ratio[ok]
    for i in range(len(lnkb) - 1):
        sel = (n2 > 0) & (lnk >= lnkb[i]) & (lnk <= lnkb[i + 1])
        lo, hi = min(rb[i], rb[i + 1]), max(rb[i], rb[i + 1])
        assert np.all((got[sel] >= lo - 1e-15) & (got[sel] <= hi + 1e-15))


def test_undisplaced_lattice_gives_zero_force_with_neutrinos():
    """A lattice at cell centres deposits exactly one unit per node: delta = 0, every bin has
    P_cdm = 0, and the force must be exactly zero even though the history gives P_nu != 0
    (R of a bin without CDM power reads 0, not P_nu/0)."""
    from oracle import step as ostep
    from synth import log_spaced_nodes, synthetic_history
    n, box, nb = 16, 64.0, 8
    q = _lattice(n, box)
    sp = ostep.spectrum(q, n, box, nb)
    assert np.all(sp["p_cdm"] == 0.0)
    nodes = log_spaced_nodes(0.01, 0.5, 10)
    hist = synthetic_history(sp["k_mean"], np.ones(nb), nodes, 0.3)
    r = ostep.full_step(q, n, box, nb, hist, 0.5, 0.3)
    ok = r["counts"] > 0
    assert np.all(r["pnu_half"][ok] > 0)
    assert np.all(r["ratio"] == 0.0)
    assert np.all(r["acc"] == 0.0)
