"""Linear theory of the stepped model (FP64): one Fourier mode of infinitesimal amplitude.

Test infrastructure. It is the expectation that the suppression of the total matter power
measured from the particle loop is compared with (the paper compares its simulations with
linear theory the same way). The model is the particle loop's, linearised:

  d^2 delta_cdm / ds^2 = (3/2) H0^2 Omega_M a delta_M,          ds = dt / a^2 (Sec. 3.2),
  delta_M = (1 - f_nu) delta_cdm + f_nu delta_nu,                 (Sec. 4.3 (iv))
  delta_nu(k, a) from eq. (P-final) over the stored delta_M history (response.nu_amplitude),

(the first line is the divergence of d^2x/ds^2 = a^2 g with grad^2 phi = (3/2) H0^2
Omega_M delta_M / a). It is integrated with kick-drift-kick steps in s on a scale-factor grid
much finer than a particle run's, holding delta_M fixed over each half kick as the particle
loop holds a g fixed, and stores a node per step as the loop does.
"""
import numpy as np

from . import background as bgmod
from . import response


def linear_modes(k, a_steps, m_nu_total, nu_ratio_init, theta_over_delta_init,
                 growth_rate_init, omega_m=0.3, hubble=0.7, substeps=8, n_species=3,
                 species=None, relativistic=False, kernel="fit"):
    """delta_cdm, delta_nu, delta_M at every a_steps node for modes k (B,), with
    delta_cdm(a_steps[0]) = 1, d delta_cdm/ds = growth_rate_init a^2 H delta_cdm there, and
    delta_nu(a_steps[0]) = nu_ratio_init (B,) with [theta/delta]_i = theta_over_delta_init.

    Returns dict of arrays (n_steps + 1, B): d_cdm, d_nu, d_m.
    """
    k = np.asarray(k, dtype=np.float64)
    B = len(k)
    a_steps = np.asarray(a_steps, dtype=np.float64)
    masses = (np.asarray(species, dtype=np.float64) if species is not None
              else np.full(n_species, m_nu_total / n_species))
    m_tot = float(masses.sum())
    fn = bgmod.f_nu(m_tot, omega_m, hubble)
    bg = bgmod.Background(omega_m, hubble, masses) if relativistic else None
    c_src = 1.5 * bgmod.H0 ** 2 * omega_m
    nu0 = np.asarray(nu_ratio_init, dtype=np.float64) * np.ones(B)
    a0 = a_steps[0]
    d_c = np.ones(B)
    v = growth_rate_init * a0 * a0 * float(bgmod.hubble_rate(a0, omega_m, bg)) * d_c
    d_nu = nu0.copy() if m_tot > 0 else np.zeros(B)
    d_m = (1.0 - fn) * d_c + fn * d_nu
    out_c, out_nu, out_m = [d_c.copy()], [d_nu.copy()], [d_m.copy()]
    hist_a, hist_m = [a0], [d_m.copy()]
    kw = dict(n_species=n_species, species=species, relativistic=relativistic, kernel=kernel)
    for a_lo, a_hi in zip(a_steps[:-1], a_steps[1:]):
        am = np.sqrt(a_lo * a_hi)
        v = v + c_src * d_m * bgmod.kick_interval(a_lo, am, omega_m, bg)
        d_c = d_c + v * bgmod.superconformal_interval(a_lo, a_hi, omega_m, bg)
        if m_tot > 0:
            r = response.nu_amplitude(k, np.ones(B), d_c, np.array(hist_a), np.array(hist_m),
                                      d_nu, nu0, theta_over_delta_init, a_hi, m_tot, omega_m,
                                      hubble, substeps, **kw)
            d_nu = r["pnu_half"]
        d_m = (1.0 - fn) * d_c + fn * d_nu
        v = v + c_src * d_m * bgmod.kick_interval(am, a_hi, omega_m, bg)
        hist_a.append(a_hi)
        hist_m.append(d_m.copy())
        out_c.append(d_c.copy())
        out_nu.append(d_nu.copy())
        out_m.append(d_m.copy())
    return dict(d_cdm=np.array(out_c), d_nu=np.array(out_nu), d_m=np.array(out_m))
