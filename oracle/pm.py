"""Particle-mesh stages of the step, FP64, one box at a time.

Mesh: N^3 nodes, node (i, j, l) at ((i, j, l) * L/N); arrays are indexed [i, j, l] and
position component 0 belongs to axis i. Fourier modes follow numpy.fft.rfftn: integer
indices n_x, n_y in [-N/2, N/2) and n_z in [0, N/2], k = 2 pi n / L.

The paper builds these stages inside Gadget-3's PM solver (Sec. 4.3) and does not spell
them out; the choices below (cloud-in-cell assignment, log-spaced integer-edge k-bins,
CIC deconvolution, spectral gradient) are stated where they are made.
"""
import numpy as np

from .background import H0


# ---------------------------------------------------------------- cloud-in-cell ----
def _cic_corners(pos, n_mesh, box):
    """Per particle and axis: lower node index (wrapped) and the weight d of the upper node.

    u = x / (L/N); i0 = floor(u); d = u - i0. The lower node (i0 mod N) gets 1 - d, the
    upper node ((i0 + 1) mod N) gets d. A coordinate exactly on a node puts all of its
    weight on that node.
    """
    u = np.asarray(pos, dtype=np.float64) / (box / n_mesh)
    i0 = np.floor(u)
    d = u - i0
    i0 = np.mod(i0.astype(np.int64), n_mesh)
    return i0, d


def cic_deposit(pos, n_mesh, box):
    """Mass density on the mesh, one unit of mass per particle (sum = number of particles)."""
    i0, d = _cic_corners(pos, n_mesh, box)
    n = n_mesh
    rho = np.zeros(n * n * n, dtype=np.float64)
    for cx in (0, 1):
        wx = d[:, 0] if cx else 1.0 - d[:, 0]
        ix = (i0[:, 0] + cx) % n
        for cy in (0, 1):
            wy = d[:, 1] if cy else 1.0 - d[:, 1]
            iy = (i0[:, 1] + cy) % n
            for cz in (0, 1):
                wz = d[:, 2] if cz else 1.0 - d[:, 2]
                iz = (i0[:, 2] + cz) % n
                rho += np.bincount((ix * n + iy) * n + iz, weights=wx * wy * wz,
                                   minlength=n * n * n)
    return rho.reshape(n, n, n)


def overdensity(rho, n_particles):
    """delta = rho / rho_bar - 1 with rho_bar = N_p / N^3."""
    return rho * (rho.size / float(n_particles)) - 1.0


def cic_interpolate(pos, grids, box):
    """Cloud-in-cell gather of each grid in ``grids`` (shape (C, N, N, N)) at the particles."""
    grids = np.asarray(grids, dtype=np.float64)
    n = grids.shape[-1]
    i0, d = _cic_corners(pos, n, box)
    flat = grids.reshape(grids.shape[0], -1)
    out = np.zeros((pos.shape[0], grids.shape[0]), dtype=np.float64)
    for cx in (0, 1):
        wx = d[:, 0] if cx else 1.0 - d[:, 0]
        ix = (i0[:, 0] + cx) % n
        for cy in (0, 1):
            wy = d[:, 1] if cy else 1.0 - d[:, 1]
            iy = (i0[:, 1] + cy) % n
            for cz in (0, 1):
                wz = d[:, 2] if cz else 1.0 - d[:, 2]
                iz = (i0[:, 2] + cz) % n
                idx = (ix * n + iy) * n + iz
                w = wx * wy * wz
                for c in range(flat.shape[0]):
                    out[:, c] += w * flat[c, idx]
    return out


# ------------------------------------------------------------------ Fourier modes ----
def forward_modes(delta):
    """delta_k = sum_x delta(x) exp(-2 pi i n.x / N), unnormalised, half spectrum (rfftn)."""
    return np.fft.rfftn(np.asarray(delta, dtype=np.float64))


def mode_indices(n_mesh):
    """Integer mode indices (n_x, n_y, n_z) broadcastable to the rfftn half spectrum."""
    full = np.fft.fftfreq(n_mesh, d=1.0 / n_mesh).astype(np.int64)
    half = np.arange(n_mesh // 2 + 1, dtype=np.int64)
    return full[:, None, None], full[None, :, None], half[None, None, :]


def mode_n2_and_weight(n_mesh):
    """|n|^2 (integer) and the half-spectrum multiplicity w (1 on the n_z = 0, N/2 planes, else 2)."""
    nx, ny, nz = mode_indices(n_mesh)
    n2 = nx * nx + ny * ny + nz * nz
    w = np.where((nz == 0) | (nz == n_mesh // 2), 1, 2) * np.ones_like(n2)
    return n2, w


# -------------------------------------------------------------------------- k-bins ----
def bin_edges_n2(n_mesh, n_bins):
    """Integer |n|^2 edges of B log-spaced bins over [k_f, sqrt(3) k_Nyq].

    In units of the fundamental mode the range is |n| in [1, sqrt(3) N/2], i.e.
    |n|^2 in [1, r2] with r2 = 3 N^2 / 4. Edge b is ceil(r2^(b/B)), edge 0 is 1, and a
    mode belongs to bin b when E_b <= |n|^2 < E_{b+1} (the last bin also takes |n|^2 = r2).
    """
    r2 = 3.0 * n_mesh * n_mesh / 4.0
    b = np.arange(n_bins + 1, dtype=np.float64)
    edges = np.ceil(r2 ** (b / n_bins)).astype(np.int64)
    edges[0] = 1
    return edges


def bin_of_n2(n2, edges):
    """Bin index of each |n|^2 (-1 for the DC mode)."""
    b = np.searchsorted(edges, n2, side="right") - 1
    b = np.minimum(b, len(edges) - 2)
    return np.where(n2 == 0, -1, b)


def bin_geometry(n_mesh, box, n_bins):
    """Per bin: mode count C_b (with half-spectrum weights) and mean |k| (h/Mpc)."""
    n2, w = mode_n2_and_weight(n_mesh)
    edges = bin_edges_n2(n_mesh, n_bins)
    b = bin_of_n2(n2, edges)
    keep = b >= 0
    kmag = (2.0 * np.pi / box) * np.sqrt(n2.astype(np.float64))
    counts = np.bincount(b[keep], weights=w[keep].astype(np.float64), minlength=n_bins)
    ksum = np.bincount(b[keep], weights=(w * kmag)[keep], minlength=n_bins)
    k_mean = np.where(counts > 0, ksum / np.where(counts > 0, counts, 1.0), 0.0)
    return edges, counts, k_mean


def binned_power(delta_k, n_mesh, box, n_bins):
    """P_cdm(k_b) = (L^3 / N^6) sum_b w |delta_k|^2 / C_b, FP64; 0 for empty bins.

    This is the mode summation the paper names as the costliest part of its Fourier
    calculation (Sec. 5.4); the DC mode is excluded.
    """
    n2, w = mode_n2_and_weight(n_mesh)
    edges = bin_edges_n2(n_mesh, n_bins)
    b = bin_of_n2(n2, edges)
    keep = b >= 0
    power = (np.abs(delta_k) ** 2) * w
    s = np.bincount(b[keep], weights=power[keep], minlength=n_bins)
    _, counts, _ = bin_geometry(n_mesh, box, n_bins)
    norm = box ** 3 / float(n_mesh) ** 6
    return np.where(counts > 0, norm * s / np.where(counts > 0, counts, 1.0), 0.0)


# ---------------------------------------------------- rescale, Green, gradient ----
def ratio_on_modes(n_mesh, box, k_mean, counts, ratio):
    """R(|k|) on every mode: linear interpolation in ln k of R_b over the non-empty bins,
    held at the end values outside them."""
    n2, _ = mode_n2_and_weight(n_mesh)
    ok = counts > 0
    lnk_b = np.log(k_mean[ok])
    with np.errstate(divide="ignore"):
        lnk = np.log((2.0 * np.pi / box) * np.sqrt(n2.astype(np.float64)))
    lnk = np.where(n2 == 0, lnk_b[0], lnk)
    return np.interp(lnk, lnk_b, ratio[ok])


def total_matter_modes(delta_k, f_nu, ratio_modes):
    """delta_M(k) = (1 - f_nu) delta_cdm(k) + f_nu delta_nu(k), with the neutrino field in
    phase with the CDM, delta_nu = (P_nu/P_cdm)^{1/2} delta_cdm (eq. (phases), Sec. 4.3 (iv))."""
    out = ((1.0 - f_nu) + f_nu * ratio_modes) * delta_k
    out = np.array(out, dtype=np.complex128)
    out[0, 0, 0] = 0.0
    return out


def cic_window(n_mesh):
    """W(n) = prod_a sinc^2(pi n_a / N), the Fourier transform of the CIC assignment."""
    nx, ny, nz = mode_indices(n_mesh)
    w = 1.0
    for na in (nx, ny, nz):
        w = w * np.sinc(na / float(n_mesh)) ** 2      # np.sinc(t) = sin(pi t)/(pi t)
    return w


def potential_modes(delta_m_k, n_mesh, box, a_now, omega_m, deconvolve=True):
    """Poisson's equation, eq. (Poisson): k^2 phi = -(3/2) H0^2 Omega_M delta_M / a.

    With CIC deconvolution the assignment and interpolation windows are divided out once
    each (1/W^2). The DC mode is set to zero.
    """
    nx, ny, nz = mode_indices(n_mesh)
    k2 = (2.0 * np.pi / box) ** 2 * (nx * nx + ny * ny + nz * nz).astype(np.float64)
    c = 1.5 * omega_m * H0 * H0 / a_now
    den = k2 * (cic_window(n_mesh) ** 2 if deconvolve else 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(k2 > 0, -c * delta_m_k / np.where(k2 > 0, den, 1.0), 0.0)
    return phi


def gradient_modes(phi_k, n_mesh, box):
    """g_a(k) = -i k_a phi(k), the acceleration -grad(phi) in Fourier space, per axis a.

    The Nyquist index of axis a (n_x or n_y = -N/2, n_z = N/2) has no sign and is zeroed
    in component a.
    """
    out = []
    for na in mode_indices(n_mesh):
        ka = (2.0 * np.pi / box) * na.astype(np.float64)
        ga = -1j * ka * phi_k
        ga = np.where(np.abs(na) == n_mesh // 2, 0.0, ga)
        out.append(ga)
    return out


def inverse_real(g_k, n_mesh):
    """g(x) = (1/N^3) sum_n g(n) exp(+2 pi i n.x / N) (irfftn)."""
    return np.fft.irfftn(g_k, s=(n_mesh,) * 3, axes=(0, 1, 2))
