"""One PM + linear-response-neutrino step in the order of Sec. 4.3 (ii)-(iv), and the loop
that repeats it, FP64.

  (ii)  CDM density by cloud-in-cell, its Fourier transform and binned power spectrum
  (iii) P_nu^{1/2} from eq. (P-final) over the stored history (one iteration by default)
  (iv)  delta_nu = (P_nu/P_cdm)^{1/2} delta_cdm (eq. (phases)), delta_M = (1-f_nu) delta_cdm
        + f_nu delta_nu, then Poisson's equation and the force back at the particles;
        the new total-matter amplitude is what gets stored for later steps.
"""
import numpy as np

from . import background as bgmod
from . import pm, response


def spectrum(pos, n_mesh, box, n_bins):
    """Stage (ii): density, modes and binned CDM power of one box."""
    pos = np.asarray(pos, dtype=np.float64)
    rho = pm.cic_deposit(pos, n_mesh, box)
    delta = pm.overdensity(rho, pos.shape[0])
    delta_k = pm.forward_modes(delta)
    edges, counts, k_mean = pm.bin_geometry(n_mesh, box, n_bins)
    p_cdm = pm.binned_power(delta_k, n_mesh, box, n_bins)
    return dict(rho=rho, delta_k=delta_k, edges=edges, counts=counts, k_mean=k_mean,
                p_cdm=p_cdm)


def forces(pos, delta_k, n_mesh, box, k_mean, counts, ratio, f_nu, a_now, omega_m,
           deconvolve=True, return_grids=False):
    """Stage (iv): total-matter modes, potential, gradient, inverse FFT, interpolation."""
    pos = np.asarray(pos, dtype=np.float64)
    rm = pm.ratio_on_modes(n_mesh, box, k_mean, counts, ratio)
    dm = pm.total_matter_modes(delta_k, f_nu, rm)
    phi = pm.potential_modes(dm, n_mesh, box, a_now, omega_m, deconvolve)
    grids = np.stack([pm.inverse_real(g, n_mesh) for g in pm.gradient_modes(phi, n_mesh, box)])
    acc = pm.cic_interpolate(pos, grids, box)
    if return_grids:
        return acc, grids
    return acc


def full_step(pos, n_mesh, box, n_bins, history, a_now, m_nu_total, omega_m=0.3,
              hubble=0.7, substeps=8, iterations=1, deconvolve=True, n_species=3,
              return_grids=False, species=None, relativistic=False, kernel="fit"):
    """Whole step for one box. ``history`` is a dict with keys a, pm_half, pnu_half,
    pnu_half_init, theta_over_delta_init (as produced by synth.synthetic_history);
    relativistic selects the background of Sec. 4.4 for the time grid; kernel "fit" or
    "series" the form of I(x) (Appendix C)."""
    sp = spectrum(pos, n_mesh, box, n_bins)
    pcdm_half = np.sqrt(sp["p_cdm"])
    r = response.nu_amplitude(sp["k_mean"], sp["counts"], pcdm_half, history["a"],
                              history["pm_half"], history["pnu_half"][-1],
                              history["pnu_half_init"], history["theta_over_delta_init"],
                              a_now, m_nu_total, omega_m, hubble, substeps,
                              iterations=iterations, n_species=n_species, species=species,
                              relativistic=relativistic, kernel=kernel)
    out = forces(pos, sp["delta_k"], n_mesh, box, sp["k_mean"], sp["counts"], r["ratio"],
                 r["f_nu"], a_now, omega_m, deconvolve, return_grids)
    if return_grids:
        acc, grids = out
        sp["grids"] = grids
    else:
        acc = out
    sp.update(r)
    sp["acc"] = acc
    return sp


def advance(pos, vel, acc, history, a_steps, n_mesh, box, n_bins, m_nu_total, omega_m=0.3,
            hubble=0.7, substeps=8, iterations=1, deconvolve=True, n_species=3, species=None,
            relativistic=False, kernel="fit"):
    """Repeat steps (ii)-(iv) of Sec. 4.3 along a_steps with kick-drift-kick leapfrog steps in
    the superconformal time s (ds = dt/a^2, Sec. 3.2), in which comoving positions obey
    d^2x/ds^2 = a^2 g with g the force of full_step (g = -grad phi, phi ~ 1/a).

    Reading (the paper's N-body code is Gadget-3, whose integrator it does not restate):
    within one step a0 -> a1, with a_m = sqrt(a0 a1), a g is held at its value at the
    start (end) of each half: u += a0 g(a0) int_{a0}^{a_m} da/(a^2 H); x += u (s(a1) - s(a0));
    g(a1) from full_step at a1, which also stores the node a1; u += a1 g(a1) int_{a_m}^{a1}
    da/(a^2 H). Positions wrap into [0, box).

    pos, vel, acc (N, 3): positions, u = dx/ds and the force at a_steps[0]. Returns the
    positions, velocities and force at a_steps[-1] (FP64) and the extended history.
    """
    masses = (np.asarray(species, dtype=np.float64) if species is not None
              else np.full(n_species, m_nu_total / n_species))
    bg = bgmod.Background(omega_m, hubble, masses) if relativistic else None
    x = np.asarray(pos, dtype=np.float64).copy()
    u = np.asarray(vel, dtype=np.float64).copy()
    g = np.asarray(acc, dtype=np.float64).copy()
    hist = {k: np.array(v, dtype=np.float64, copy=True) for k, v in history.items()}
    for a0, a1 in zip(a_steps[:-1], a_steps[1:]):
        am = np.sqrt(a0 * a1)
        u += a0 * bgmod.kick_interval(a0, am, omega_m, bg) * g
        x = np.mod(x + bgmod.superconformal_interval(a0, a1, omega_m, bg) * u, box)
        r = full_step(x, n_mesh, box, n_bins, hist, a1, m_nu_total, omega_m, hubble, substeps,
                      iterations, deconvolve, n_species, species=species,
                      relativistic=relativistic, kernel=kernel)
        g = r["acc"]
        u += a1 * bgmod.kick_interval(am, a1, omega_m, bg) * g
        hist["a"] = np.append(hist["a"], a1)
        hist["pm_half"] = np.vstack([hist["pm_half"], r["pm_half_now"][None, :]])
        hist["pnu_half"] = np.vstack([hist["pnu_half"], r["pnu_half"][None, :]])
    return x, u, g, hist
