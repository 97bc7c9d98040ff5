"""Zel'dovich-displaced particle lattices with a power-law spectrum (seeded, FP64 -> FP32).

The paper's runs start from Boltzmann-code transfer functions and a 2LPT generator, which
are not available here. A power-law Gaussian field displaced with the Zel'dovich
approximation stands in for them: it has the same structure (a lattice perturbed by a
smooth, curl-free displacement) and a controlled amplitude.

Recipe (all in FP64 with ``numpy.random.default_rng(seed)``):
  1. white noise on the n^3 lattice;
  2. forward real FFT, multiplied by sqrt(P(k)) with P(k) ~ k^spectral_index, k != 0;
  3. the DC mode and every mode with a Nyquist index on any axis are zeroed;
  4. displacement psi_k = i k delta_k / k^2 (so that delta = -div psi), back to real space;
  5. psi is rescaled so that its 3-D RMS equals ``sigma_cells`` mesh cells;
  6. positions q = (i + 1/2) * spacing + psi, wrapped into [0, L), rounded to FP32.

The lattice sits at cell centres: a lattice on the mesh nodes makes the cloud-in-cell
density of the unperturbed lattice non-smooth at first order in psi.

Particle order: ``order="morton"`` (default) lists the particles along the Morton (Z-order)
curve of their lattice index, the way a TreePM code keeps its particles sorted along a
space-filling curve for domain decomposition; ``order="c"`` gives C order of the lattice
index (i, j, l) -> (i*n + j)*n + l. Position component 0 belongs to lattice axis i.
"""
import numpy as np

# The workloads, by name. Sizes follow the measurement plan of the method's PM step.
CONFIGS = {
    # 32^3 particles on a 32^3 mesh in a 128 Mpc/h box; small enough for the oracle.
    "tiny32": dict(n_side=32, n_mesh=32, box=128.0, sigma_cells=0.2, m_nu=(0.3,),
                   n_kbins=32, n_hist=16, a_lo=0.01, a_now=0.5, substeps=8,
                   seeds=(0, 1, 2, 3, 4), n_boxes=1),
    # 256^3 particles on a 256^3 mesh, 512 Mpc/h: the headline single-box workload.
    "pm256": dict(n_side=256, n_mesh=256, box=512.0, sigma_cells=0.3,
                  m_nu=(0.15, 0.3, 0.6), n_kbins=64, n_hist=200, a_lo=0.01,
                  a_now=1.0, substeps=8, seeds=(256, 257, 258), n_boxes=1),
    # 512^3 particles on a 512^3 mesh, 1000 Mpc/h (cell 1.953125 Mpc/h, exact in binary).
    "pm512": dict(n_side=512, n_mesh=512, box=1000.0, sigma_cells=0.3, m_nu=(0.3,),
                  n_kbins=128, n_hist=400, a_lo=0.01, a_now=1.0, substeps=8,
                  seeds=(512,), n_boxes=1),
    # 64 independent boxes of 64^3 particles on 64^3 meshes, 256 Mpc/h each.
    "batch64x64": dict(n_side=64, n_mesh=64, box=256.0, sigma_cells=0.3, m_nu=None,
                       m_nu_range=(0.05, 0.6), m_nu_seed=999, n_kbins=48, n_hist=100,
                       a_lo=0.01, a_now=1.0, substeps=8, seeds=None, seed0=1000,
                       n_boxes=64),
}


def morton_codes(n_side):
    """Morton code of every lattice site, in C order of (i, j, l); bits of i are the most
    significant of each triple."""
    p = int(n_side).bit_length() - 1
    idx = np.arange(n_side, dtype=np.uint64)
    spread = np.zeros(n_side, dtype=np.uint64)
    for b in range(p):
        spread |= ((idx >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return ((spread[:, None, None] << np.uint64(2)) | (spread[None, :, None] << np.uint64(1))
            | spread[None, None, :]).reshape(-1)


def zeldovich_lattice(n_side, box, sigma_cells, seed, spectral_index=-2.0, order="morton",
                      return_displacement=False):
    """Return FP32 positions, shape (n_side**3, 3), in [0, box); with return_displacement
    also the FP64 displacement of every particle (same order)."""
    n = int(n_side)
    if n < 2 or n & (n - 1):
        raise ValueError("n_side must be a power of two >= 2")
    spacing = box / n
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n, n))
    dk = np.fft.rfftn(noise)
    del noise
    ix = np.fft.fftfreq(n, d=1.0 / n)            # integer mode index, [-n/2, n/2)
    iz = np.arange(n // 2 + 1, dtype=np.float64)
    nx = ix[:, None, None]
    ny = ix[None, :, None]
    nz = iz[None, None, :]
    n2 = nx * nx + ny * ny + nz * nz
    amp = np.zeros_like(n2)
    nz0 = n2 > 0
    amp[nz0] = n2[nz0] ** (0.25 * spectral_index)   # sqrt(P) with P ~ |n|^index
    nyq = (np.abs(nx) == n // 2) | (np.abs(ny) == n // 2) | (nz == n // 2)
    amp = np.where(nyq, 0.0, amp)
    dk *= amp
    del amp
    inv_n2 = np.zeros_like(n2)
    inv_n2[nz0] = 1.0 / n2[nz0]
    psi = np.empty((n, n, n, 3), dtype=np.float64)
    for axis, na in enumerate((nx, ny, nz)):
        comp = 1j * na * inv_n2 * dk                  # unit-free: rescaled below
        psi[..., axis] = np.fft.irfftn(comp, s=(n, n, n), axes=(0, 1, 2))
    del dk
    rms = np.sqrt(np.mean(np.sum(psi * psi, axis=-1)))
    psi *= (sigma_cells * spacing) / rms
    disp = psi.reshape(-1, 3).copy() if return_displacement else None
    grid = (np.arange(n, dtype=np.float64) + 0.5) * spacing
    psi[..., 0] += grid[:, None, None]
    psi[..., 1] += grid[None, :, None]
    psi[..., 2] += grid[None, None, :]
    pos = np.mod(psi.reshape(-1, 3), box).astype(np.float32)
    pos[pos >= np.float32(box)] = np.float32(0.0)  # an FP32 round-up to L wraps to 0
    pos[pos < 0] = np.float32(0.0)
    if order == "morton":
        codes = morton_codes(n).astype(np.int64)
        out = np.empty_like(pos)
        out[codes] = pos
        pos = out
        if disp is not None:
            d = np.empty_like(disp)
            d[codes] = disp
            disp = d
    elif order != "c":
        raise ValueError("order must be 'morton' or 'c'")
    if return_displacement:
        return np.ascontiguousarray(pos), disp
    return np.ascontiguousarray(pos)


def second_order_displacement(psi1, box):
    """The second-order Lagrangian displacement of a first-order one on an n^3 lattice.

    psi1 (n, n, n, 3): the first-order displacement in length units, psi1 = -grad phi1.
    Second-order Lagrangian perturbation theory (Scoccimarro 1998) adds psi2 = D2 grad phi2
    with lap phi2 = sum_{i<j} (phi1_ii phi1_jj - phi1_ij^2) and D2 = -(3/7) D1^2 (the
    matter-era value); in terms of psi1 (already multiplied by D1) this is
    psi2 = -(3/7) grad phi2[phi1]. Derivatives are spectral; returns psi2 (n, n, n, 3).
    """
    n = psi1.shape[0]
    k1 = 2 * np.pi / box * np.fft.fftfreq(n, d=1.0 / n)
    kz = 2 * np.pi / box * np.arange(n // 2 + 1, dtype=np.float64)
    kv = (k1[:, None, None], k1[None, :, None], kz[None, None, :])
    pk = [np.fft.rfftn(psi1[..., i]) for i in range(3)]

    def deriv(i, j):                          # d psi1_i / d q_j = -phi1_ij
        return np.fft.irfftn(1j * kv[j] * pk[i], s=(n, n, n), axes=(0, 1, 2))

    m = {(i, j): deriv(i, j) for i in range(3) for j in range(i, 3)}
    src = (m[0, 0] * m[1, 1] - m[0, 1] ** 2 + m[0, 0] * m[2, 2] - m[0, 2] ** 2
           + m[1, 1] * m[2, 2] - m[1, 2] ** 2)
    del m, pk
    k2 = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
    inv_k2 = np.zeros_like(k2)
    inv_k2[k2 > 0] = 1.0 / k2[k2 > 0]
    phi2_k = -np.fft.rfftn(src) * inv_k2      # lap phi2 = src
    psi2 = np.empty_like(psi1)
    for i in range(3):
        psi2[..., i] = -(3.0 / 7.0) * np.fft.irfftn(1j * kv[i] * phi2_k, s=(n, n, n),
                                                     axes=(0, 1, 2))
    return psi2


def zeldovich_ics(n_side, box, sigma_cells, seed, a, omega_m=0.3, spectral_index=-2.0,
                  order="morton", second_order=False):
    """Positions and growing-mode velocities at scale factor a, both FP32 (n_side**3, 3).

    The lattice is displaced by psi (RMS sigma_cells cells); in the Zel'dovich growing mode
    x = q + (D/D(a)) psi, so the velocity in superconformal time s (ds = dt/a^2) is
    u = dx/ds = a^2 dx/dt = a^2 H(a) f(a) psi, with H and f = dln D/dln a of a flat
    matter + Lambda background. With second_order the second-order displacement psi2
    (second_order_displacement, scaled by Omega_M(a)^(-1/143)) is added, moving with
    f2 = 2 Omega_M(a)^(6/11): u = a^2 H (f psi + f2 psi2).
    """
    from .history import growth, hubble_rate
    pos, disp = zeldovich_lattice(n_side, box, sigma_cells, seed, spectral_index, order,
                                  return_displacement=True)
    _, f = growth(np.array([a]), omega_m)
    ah = a * a * hubble_rate(a, omega_m)
    vel = (ah * f[0]) * disp
    if second_order:
        n = int(n_side)
        codes = morton_codes(n).astype(np.int64) if order == "morton" else None
        psi1 = disp if codes is None else disp[codes]              # back to C order
        psi2 = second_order_displacement(psi1.reshape(n, n, n, 3), box).reshape(-1, 3)
        om_a = omega_m / (omega_m + (1.0 - omega_m) * a ** 3)
        psi2 *= om_a ** (-1.0 / 143.0)
        grid = (np.arange(n, dtype=np.float64) + 0.5) * (box / n)
        q = np.stack(np.meshgrid(grid, grid, grid, indexing="ij"), -1).reshape(-1, 3)
        x = np.mod(q + psi1 + psi2, box).astype(np.float32)
        x[x >= np.float32(box)] = np.float32(0.0)                  # FP32 round-up wraps to 0
        v2 = (ah * 2.0 * om_a ** (6.0 / 11.0)) * psi2
        if codes is not None:
            pos = np.empty_like(x)
            pos[codes] = x
            tmp = np.empty_like(v2)
            tmp[codes] = v2
            v2 = tmp
        else:
            pos = x
        vel = vel + v2
    return pos, np.ascontiguousarray(vel.astype(np.float32))


def batched_lattices(cfg, order="morton"):
    """Positions (n_boxes, n_side**3, 3) FP32 and per-box total neutrino masses [eV]."""
    nb = cfg["n_boxes"]
    if cfg.get("m_nu") is not None:
        masses = np.resize(np.asarray(cfg["m_nu"], dtype=np.float64), nb)
    else:
        lo, hi = cfg["m_nu_range"]
        masses = np.random.default_rng(cfg["m_nu_seed"]).uniform(lo, hi, size=nb)
    seeds = cfg.get("seeds") or tuple(cfg["seed0"] + b for b in range(nb))
    pos = np.stack([zeldovich_lattice(cfg["n_side"], cfg["box"], cfg["sigma_cells"],
                                      seeds[b % len(seeds)], order=order) for b in range(nb)])
    return pos, masses
