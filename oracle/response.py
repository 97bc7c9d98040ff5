"""The neutrino amplitude of eq. (P-final), by quadrature over the stored history (FP64).

For each k-bin, with s the superconformal time (Sec. 3.2) and I_{s',s} = I(k (s - s') T_nu0 / m):

  P_nu^{1/2}(k, tau) = I_{s_i,s} P_nu^{1/2}(k, tau_i) {1 - (s - s_i) a_i [theta/delta]_i(k)}
                     + (3/2) Omega_M H0^2 int_{tau_i}^{tau} I_{s',s} P_M^{1/2}(k, tau') (s - s') dtau'

(the initial-condition term is eq. (deltaI-nu) under the phase assumptions of Sec. 4.2).

Discretisation (the paper integrates "interpolating over our tables of stored power
spectra", Sec. 4.3 (iii), and gives no rule):
  * the stored nodes a_0 < ... < a_{n-1} and the current a_n split [a_0, a_n]; every
    interval is cut into Q equal steps in ln a;
  * dtau' = d ln a' / (a' H(a')); the integral is the trapezoid rule in ln a over the
    sub-nodes;
  * P_M^{1/2} at a sub-node is linear in ln a between the two bracketing nodes;
  * the current node is not known yet (the equation is implicit, Sec. 4.3 (iii)): the first
    iteration uses P_M^{1/2}(a_n) = (1 - f_nu) P_cdm^{1/2}(a_n) + f_nu P_nu^{1/2}(a_{n-1}),
    i.e. P_nu(tau) ~ P_nu(tau - dtau); iteration i+1 uses the P_nu^{1/2} of iteration i
    (Appendix B).
"""
import numpy as np

from .background import (H0, T_NU0, Background, f_nu as f_nu_of, hubble_rate,
                         superconformal_interval)
from .kernel import I_fit, I_series

_DS_CACHE = {}


def _ds_piece(a1, a2, omega_m, background=None):
    key = (float(a1), float(a2), float(omega_m), None if background is None else background.key)
    v = _DS_CACHE.get(key)
    if v is None:
        v = superconformal_interval(a1, a2, omega_m, background)
        _DS_CACHE[key] = v
    return v


def sub_grid(a_nodes, substeps, omega_m, background=None):
    """Sub-nodes of the quadrature over nodes a_0..a_n (a_n = current step); the background
    (default flat matter + Lambda) sets s.

    Returns a dict of per-sub-node arrays: a, trapezoid weight in ln a, bracketing node j,
    interpolation fraction t (amplitude = (1-t) A_j + t A_{j+1}), and s_n - s_q.
    """
    lna = np.log(np.asarray(a_nodes, dtype=np.float64))
    n = len(lna) - 1
    q_lna, q_j, q_t, q_w = [], [], [], []
    for j in range(n):
        h = (lna[j + 1] - lna[j]) / substeps
        for r in range(substeps):
            q_lna.append(lna[j] + r * h)
            q_j.append(j)
            q_t.append(r / substeps)
            q_w.append(h if r > 0 else 0.5 * h)
        if j > 0:
            q_w[j * substeps] += 0.5 * (lna[j] - lna[j - 1]) / substeps
    # final sub-node: the current step itself
    q_lna.append(lna[n])
    q_j.append(n - 1 if n > 0 else 0)
    q_t.append(1.0 if n > 0 else 0.0)
    q_w.append(0.5 * (lna[n] - lna[n - 1]) / substeps if n > 0 else 0.0)
    a_sub = np.exp(np.array(q_lna))
    a_sub[-1] = a_nodes[-1]
    for j in range(n):                      # sub-nodes that coincide with nodes are exact
        a_sub[j * substeps] = a_nodes[j]
    # s_n - s_q, summed backwards over the sub-intervals (each an accurate quadrature)
    ds = np.zeros(len(a_sub))
    for q in range(len(a_sub) - 2, -1, -1):
        ds[q] = ds[q + 1] + _ds_piece(a_sub[q], a_sub[q + 1], omega_m, background)
    return dict(a=a_sub, w=np.array(q_w), j=np.array(q_j), t=np.array(q_t), ds=ds)


def nu_amplitude(k_mean, counts, pcdm_half, hist_a, hist_pm_half, pnu_half_prev,
                 pnu_half_init, theta_over_delta_init, a_now, m_nu_total, omega_m,
                 hubble, substeps, iterations=1, n_species=3, f_nu=None, species=None,
                 pnu_half_init_species=None, relativistic=False, kernel="fit"):
    """P_nu^{1/2}(k_b, a_now) for every bin, eq. (P-final).

    hist_a (n,), hist_pm_half (n, B): stored nodes strictly before a_now (hist_a[0] = a_i).
    pnu_half_prev (B,): P_nu^{1/2} at the last stored node (the first-iteration guess).
    Returns dict: pnu_half, ratio = P_nu^{1/2}/P_cdm^{1/2}, pm_half_now (the node to store),
    f_nu. Empty bins (counts == 0) give 0 everywhere; a bin with P_cdm = 0 (no CDM mode to
    put the neutrinos in phase with, eq. (phases)) has R = 0. Without massive neutrinos
    (m_nu_total = 0, so f_nu = 0) the neutrino term of Sec. 4.3 (iv) drops out: P_nu^{1/2}
    and R are reported as 0 and the stored node is P_cdm^{1/2}.

    species: masses of individual species [eV] (mass hierarchy, Sec. 6.2); by default
    n_species equal masses m_nu_total / n_species. Each species free-streams with its own
    kernel I(k (s - s') T_nu0 / m_s) and the neutrino density contrast is the mean over
    species weighted by their share of the neutrino density, m_s / M_nu (non-relativistic);
    a massless species adds nothing. pnu_half_init_species (n_species, B): initial
    amplitude of each species (default: pnu_half_init for all).

    relativistic: take s and dtau from the background of Sec. 4.4 (radiation, massless
    species, and the massive species' energy density of eq. (relativistic)); f_nu and the
    source (3/2) Omega_M H0^2 keep the non-relativistic matter density.

    kernel: "fit" (eq. (fit), the method's choice) or "series" (the exact function of
    Appendix C).
    """
    k = np.asarray(k_mean, dtype=np.float64)
    ok = np.asarray(counts) > 0
    pcdm_half = np.asarray(pcdm_half, dtype=np.float64)
    if species is None:
        masses = np.full(n_species, m_nu_total / n_species)
    else:
        masses = np.asarray(species, dtype=np.float64)
        m_nu_total = masses.sum()
    fn = f_nu_of(m_nu_total, omega_m, hubble) if f_nu is None else f_nu
    if m_nu_total <= 0.0:
        zero = np.zeros_like(k)
        return dict(pnu_half=zero, ratio=zero.copy(),
                    pm_half_now=np.where(ok, pcdm_half, 0.0), f_nu=0.0)
    nodes = np.append(np.asarray(hist_a, dtype=np.float64), a_now)
    bg = Background(omega_m, hubble, masses) if relativistic else None
    g = sub_grid(nodes, substeps, omega_m, bg)
    pref = 1.5 * omega_m * H0 * H0
    measure = g["w"] / (g["a"] * hubble_rate(g["a"], omega_m, bg))  # d ln a / (a H)
    hist = np.asarray(hist_pm_half, dtype=np.float64)
    if species is None:
        # equal masses: one kernel
        groups = [(1.0, masses[0], np.asarray(pnu_half_init))]
    else:
        ics = (np.asarray(pnu_half_init_species, dtype=np.float64)
               if pnu_half_init_species is not None
               else np.tile(np.asarray(pnu_half_init, dtype=np.float64), (len(masses), 1)))
        groups = [(m / m_nu_total, m, ics[i]) for i, m in enumerate(masses) if m > 0.0]

    if kernel == "fit":
        I = I_fit
    elif kernel == "series":
        def I(x):
            x = np.asarray(x, dtype=np.float64)
            return I_series(x.reshape(-1)).reshape(x.shape)
    else:
        raise ValueError(f"kernel must be 'fit' or 'series', not {kernel!r}")

    # initial-condition term: I(x_i) P_nu^{1/2}(a_i) {1 - (s - s_i) a_i [theta/delta]_i}
    phase = 1.0 - g["ds"][0] * nodes[0] * np.asarray(theta_over_delta_init)
    ic = sum(w * I(k * g["ds"][0] * T_NU0 / m) * p0 for w, m, p0 in groups) * phase

    kern = sum(w * I(np.outer(g["ds"] * T_NU0 / m, k)) for w, m, _ in groups)
    kern = kern * g["ds"][:, None]                                     # (q, B)

    pnu_guess = np.asarray(pnu_half_prev, dtype=np.float64)
    for _ in range(max(1, iterations)):
        a_cur = (1.0 - fn) * pcdm_half + fn * pnu_guess
        table = np.vstack([hist, a_cur[None, :]])                     # (n+1, B)
        amp = ((1.0 - g["t"])[:, None] * table[g["j"]]
               + g["t"][:, None] * table[np.minimum(g["j"] + 1, len(table) - 1)])
        integral = pref * np.sum(measure[:, None] * kern * amp, axis=0)
        pnu = ic + integral
        pnu_guess = pnu
    pnu = np.where(ok, pnu, 0.0)
    # R_b carries the neutrino amplitude on the CDM modes of the bin (eq. (phases)); a bin
    # whose CDM modes are all zero has no phase to carry it, and R_b reads 0 there
    has_cdm = ok & (pcdm_half > 0.0)
    ratio = np.where(has_cdm, pnu / np.where(has_cdm, pcdm_half, 1.0), 0.0)
    pm_now = np.where(ok, (1.0 - fn) * pcdm_half + fn * pnu, 0.0)
    return dict(pnu_half=pnu, ratio=ratio, pm_half_now=pm_now, f_nu=fn)


def replay_history(k_mean, counts, cdm_half, a_nodes, pnu_half_init,
                   theta_over_delta_init, m_nu_total, omega_m, hubble, substeps,
                   n_species=3, f_nu=None, species=None, relativistic=False):
    """A self-consistent stored history: the neutrino amplitude at every node computed by
    eq. (P-final) from the earlier nodes, as the step-by-step loop of Sec. 4.3 would.

    cdm_half (n_nodes, B): CDM amplitudes at every node a_nodes[j].
    Returns pm_half (n_nodes, B) and pnu_half (n_nodes, B).
    """
    if species is not None:
        m_nu_total = float(np.sum(species))
    fn = f_nu_of(m_nu_total, omega_m, hubble) if f_nu is None else f_nu
    n = len(a_nodes)
    B = len(k_mean)
    pm = np.zeros((n, B))
    pnu = np.zeros((n, B))
    pnu[0] = pnu_half_init
    pm[0] = (1.0 - fn) * cdm_half[0] + fn * pnu[0]
    for j in range(1, n):
        r = nu_amplitude(k_mean, counts, cdm_half[j], a_nodes[:j], pm[:j], pnu[j - 1],
                         pnu_half_init, theta_over_delta_init, a_nodes[j], m_nu_total,
                         omega_m, hubble, substeps, n_species=n_species, f_nu=fn,
                         species=species, relativistic=relativistic)
        pnu[j] = r["pnu_half"]
        pm[j] = r["pm_half_now"]
    return pm, pnu
