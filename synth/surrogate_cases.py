"""Random stored histories for the surrogate network's training set.

Each case is one box at the current node a_j of a fixed log-spaced node grid: a total
neutrino mass, a linear power-law amplitude with a random tilt, a non-linear change of
the CDM amplitude that grows with time, and a smooth departure from linear growth of its
own in every k-bin,

    A_cdm(k, a_i) = g_i k^(-1 + tilt) (1 + eps(k) g_i^p) exp(delta_k (1 - g_i^q)),
    g_i = D(a_i)/D(a_j),  eps(k) = e0 (k/k0)^s / (1 + (k/k0)^s),

with e0 uniform in [-0.4, 0] (suppression, as below the mesh scale) for one case in five
and log-uniform in [0.02, 8] (enhancement, up to the several-fold growth of the
amplitude beyond the mesh Nyquist frequency late in a run) otherwise, k0 log-uniform in
[0.05, 1] h/Mpc, s in [1, 3], p in [0.5, 4], q in [0.5, 3] and delta_k
normal with a scale drawn from [0, 0.05] per case, independent between bins (a particle
run's measured amplitudes depart from D(a) by a few per cent at low k, differently in
each bin, from mode coupling and its start-up transients). The neutrino amplitude
follows the linear CDM one times 1/(1 + k/k_fs)^2 and the stored total is
(1 - f_nu) CDM + f_nu neutrino, as in synth.history. None of this is the method's
integral; it only spans the inputs the network will see.
"""
import numpy as np

from .history import _H0, _e, free_streaming_k, growth


def surrogate_batch(k_mean, a_nodes, j, n_boxes, rng, omega_m=0.3, hubble=0.7,
                    m_range=(0.03, 0.7), n_species=3, growth_nodes=None):
    """n_boxes random cases sharing the current node a_nodes[j].

    growth_nodes: optional (D, f) at every node (computed here when not given).
    Returns (masses [n_boxes], histories (list of dicts for nodes 0..j-1), p_cdm
    [n_boxes][B]) ready for pm_nu_set_history / pm_nu_set_power.
    """
    k = np.asarray(k_mean, dtype=np.float64)
    kk = np.where(k > 0, k, 1.0)
    a = np.asarray(a_nodes[: j + 1], dtype=np.float64)
    if growth_nodes is None:
        d, f = growth(a, omega_m)
    else:
        d, f = growth_nodes[0][: j + 1], growth_nodes[1][: j + 1]
    g = d / d[-1]
    theta = -f[0] * a[0] * _H0 * _e(a[0], omega_m)
    masses = rng.uniform(m_range[0], m_range[1], size=n_boxes)
    hists, powers = [], []
    for m in masses:
        tilt = rng.uniform(-0.5, 0.5)
        e0 = rng.uniform(-0.4, 0.0) if rng.random() < 0.2 else \
            float(np.exp(rng.uniform(np.log(0.02), np.log(8.0))))
        k0 = np.exp(rng.uniform(np.log(0.05), np.log(1.0)))
        s = rng.uniform(1.0, 3.0)
        p = rng.uniform(0.5, 4.0)
        q = rng.uniform(0.5, 3.0)
        delta = rng.normal(size=k.shape) * rng.uniform(0.0, 0.05)
        eps = e0 * (kk / k0) ** s / (1.0 + (kk / k0) ** s)
        lin = g[:, None] * kk[None, :] ** (-1.0 + tilt)
        cdm = lin * (1.0 + eps[None, :] * g[:, None] ** p) \
            * np.exp(delta[None, :] * (1.0 - g[:, None] ** q))
        f_nu = m / (93.14 * omega_m * hubble * hubble)
        kfs = free_streaming_k(a, m / n_species, omega_m)[:, None]
        nu = lin / (1.0 + kk[None, :] / kfs) ** 2
        pm = (1.0 - f_nu) * cdm + f_nu * nu
        empty = k <= 0
        pm[:, empty] = 0.0
        nu[:, empty] = 0.0
        hists.append(dict(a=a[:-1].copy(), pm_half=np.ascontiguousarray(pm[:-1]),
                          pnu_half=np.ascontiguousarray(nu[:-1]), pnu_half_init=nu[0].copy(),
                          theta_over_delta_init=np.full(k.shape, theta)))
        powers.append(np.where(empty, 0.0, cdm[-1] ** 2))
    return masses, hists, np.asarray(powers)
