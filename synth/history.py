"""Smooth synthetic power-spectrum histories, as a simulation would have stored them.

The method keeps, per k-bin, the square root of the total matter power spectrum at every
earlier step, plus the initial neutrino amplitude and velocity-to-density ratio. A single
PM step needs that history as input. Here it is built in closed form from linear theory:

  * CDM amplitude at node j: D(a_j) / D(a_now) times the amplitude measured now;
  * neutrino amplitude: the CDM amplitude times 1 / (1 + k / k_fs(a_j))^2 (the simple
    all-scale approximation of the paper's Appendix A);
  * stored total: (1 - f_nu) * CDM + f_nu * neutrino, the total-matter amplitude of
    Sec. 4.3 (iv) and Appendix B;
  * initial neutrino velocity/density ratio: the growing mode, theta/delta = -f a H.

D(a) and f = dlnD/dlna are the flat matter + Lambda growth factor and rate.
None of this is the method's own integral; it only supplies plausible inputs.
"""
import numpy as np
from scipy import integrate

_C_KMS = 299792.458
_H0 = 100.0 / _C_KMS          # H0 in h/Mpc with c = 1
_T_NU0_EV = 1.95 * 8.617333262e-5
_ZETA3 = 1.2020569031595942


def log_spaced_nodes(a_lo, a_hi, n):
    """n scale factors log-spaced on [a_lo, a_hi] (both ends included)."""
    j = np.arange(n, dtype=np.float64)
    return a_lo * (a_hi / a_lo) ** (j / (n - 1))


def _e(a, om):
    return np.sqrt(om / a ** 3 + 1.0 - om)


def hubble_rate(a, om):
    """H(a) [h/Mpc] of a flat matter + Lambda background (input recipes only)."""
    return _H0 * _e(a, om)


def _growth_integral(a, om):
    val, _ = integrate.quad(lambda x: 1.0 / (x * _e(x, om)) ** 3, 0.0, a,
                            epsabs=0.0, epsrel=1e-12, limit=200)
    return val


def growth(a, om):
    """Unnormalised linear growth D(a) and its log-derivative f(a)."""
    a = np.atleast_1d(np.asarray(a, dtype=np.float64))
    d = np.empty_like(a)
    f = np.empty_like(a)
    for i, ai in enumerate(a):
        ig = _growth_integral(ai, om)
        e = _e(ai, om)
        d[i] = 2.5 * om * e * ig
        f[i] = -1.5 * om / (ai ** 3 * e * e) + 1.0 / (ai * ai * e ** 3 * ig)
    return d, f


def free_streaming_k(a, m_nu_single, om):
    """k_fs(a) in h/Mpc for one neutrino species of mass m [eV] (paper Sec. 2.3)."""
    e = _e(a, om)
    om_a = om / (a ** 3 * e * e)
    v2 = (2.0 * np.log(2.0) / (3.0 * _ZETA3)) * (m_nu_single * a / _T_NU0_EV) ** 2
    return np.sqrt(1.5 * om_a * v2) * a * _H0 * e


def growth_history(pcdm_half_now, a_nodes, omega_m=0.3):
    """CDM amplitudes at every node (J, B): D(a_j) / D(a_now) times the amplitude now
    (a_now = a_nodes[-1]), and the growing-mode [theta/delta]_i at a_nodes[0] (h/Mpc).

    These are the CDM rows a self-consistent history is replayed from: the stored total
    at each node is then computed by the method itself, node by node."""
    amp_now = np.asarray(pcdm_half_now, dtype=np.float64)
    a = np.asarray(a_nodes, dtype=np.float64)
    d, f = growth(a, omega_m)
    cdm = (d / d[-1])[:, None] * amp_now[None, :]
    theta = -f[0] * a[0] * _H0 * _e(a[0], omega_m)
    return np.ascontiguousarray(cdm), np.full(amp_now.shape, theta)


def free_streaming_ic(k_mean, cdm_half_init, a_init, m_nu_total, omega_m=0.3, n_species=3):
    """Initial neutrino amplitude: the CDM amplitude at a_init times Appendix A's simple
    all-scale approximation 1 / (1 + k / k_fs(a_init))^2 (0 without neutrinos)."""
    k = np.asarray(k_mean, dtype=np.float64)
    m1 = m_nu_total / n_species
    if m1 <= 0:
        return np.zeros_like(k)
    kfs = free_streaming_k(np.float64(a_init), m1, omega_m)
    return np.asarray(cdm_half_init, dtype=np.float64) / (1.0 + k / kfs) ** 2


def synthetic_history(k_mean, pcdm_half_now, a_nodes, m_nu_total, omega_m=0.3,
                      hubble=0.7, n_species=3):
    """History for the nodes ``a_nodes[:-1]``; ``a_nodes[-1]`` is the current step.

    Returns a dict with
      a              (J-1,)    stored node scale factors
      pm_half        (J-1, B)  stored total-matter amplitudes P_M^{1/2}
      pnu_half       (J-1, B)  neutrino amplitudes at those nodes
      pnu_half_init  (B,)      P_nu^{1/2} at a_nodes[0]
      theta_over_delta_init (B,)  [theta/delta]_i in h/Mpc (conformal time, c = 1)
    Empty bins (amplitude 0) stay 0.
    """
    k = np.asarray(k_mean, dtype=np.float64)
    amp_now = np.asarray(pcdm_half_now, dtype=np.float64)
    a = np.asarray(a_nodes, dtype=np.float64)
    f_nu = m_nu_total / (93.14 * omega_m * hubble * hubble)
    m1 = m_nu_total / n_species
    d, f = growth(a, omega_m)
    a_hist = a[:-1]
    cdm = (d[:-1] / d[-1])[:, None] * amp_now[None, :]
    if m1 > 0:
        kfs = free_streaming_k(a_hist, m1, omega_m)[:, None]
        nu = cdm / (1.0 + k[None, :] / kfs) ** 2
    else:
        nu = np.zeros_like(cdm)
    pm = (1.0 - f_nu) * cdm + f_nu * nu
    theta = -f[0] * a[0] * _H0 * _e(a[0], omega_m)
    return dict(a=a_hist.copy(), pm_half=np.ascontiguousarray(pm),
                pnu_half=np.ascontiguousarray(nu), pnu_half_init=nu[0].copy(),
                theta_over_delta_init=np.full(k.shape, theta))
