"""Pins of the oracle's neutrino response, eq. (P-final) (CPU).

* Appendix A: in a matter-dominated universe with delta_M ~ a and no initial neutrino
  perturbation, P_nu^{1/2}/delta_M has a closed form F_fin(k); the quadrature must converge
  to it at second order in the history spacing.
* Sec. 3.3.1: for k -> 0 the neutrinos follow the pressureless fluid solution, so with a
  growing-mode history and initial conditions P_nu^{1/2} -> P_M^{1/2}.
* Sec. 3.3.2 / Appendix A: for k >> k_fs, delta_nu -> (k_fs/k)^2 delta_M, and at all k
  F ~ 1/(1 + k/k_fs)^2 to within 12%.
* Appendix B / Sec. 4.3 (iii): one iteration is converged to ~1e-4.
"""
import json
import os
import numpy as np
import pytest
from scipy import integrate

from oracle import background as bg
from oracle import kernel, response
from synth import log_spaced_nodes, synthetic_history
from synth.history import growth

# the paper's printed figures, each with its citation and the tolerance applied
with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as _f:
    GOLD = json.load(_f)


def _eds_response(k, m, a0, an, J, Q=8, kern="fit"):
    nodes = log_spaced_nodes(a0, an, J)
    B = len(k)
    r = response.nu_amplitude(k, np.ones(B), an * np.ones(B), nodes[:-1],
                              nodes[:-1, None] * np.ones((1, B)), np.zeros(B), np.zeros(B),
                              np.zeros(B), an, 3 * m, 1.0, 0.7, Q, f_nu=0.0, kernel=kern)
    return r["pnu_half"] / an


def _eds_closed_form(k, m, a0, an, I=kernel.I_fit):
    """F_fin = (6/x_k^2) int_0^{x_max} x I(x) / (1 + x/x_k)^4 dx (Appendix A), with
    x_k = 2 k T/(m a^2 H) and x_max = k (s - s_i) T / m, s = -2/(H0 sqrt(a)) in EdS."""
    T = bg.T_NU0
    h = bg.H0 * an ** -1.5
    xk = 2 * k * T / (m * an ** 2 * h)
    xmax = k * (2.0 / bg.H0) * (a0 ** -0.5 - an ** -0.5) * T / m
    val = integrate.quad(lambda x: x * float(np.asarray(I(x)).reshape(-1)[0]) / (1 + x / xk) ** 4,
                         0, xmax, limit=500, epsrel=1e-12)[0]
    return 6.0 / xk ** 2 * val


def test_eds_closed_form_second_order_convergence():
    k = np.array([0.01, 0.1, 0.3, 1.0])
    m, a0, an = 0.1, 0.01, 0.5
    ref = np.array([_eds_closed_form(kk, m, a0, an) for kk in k])
    errs = []
    for J in (100, 200, 400):
        errs.append(np.abs(_eds_response(k, m, a0, an, J) / ref - 1.0))
    errs = np.array(errs)
    assert np.all(errs[-1] < 2e-5)
    ratio = errs[:-1] / errs[1:]
    assert np.all((ratio > 3.6) & (ratio < 4.4))


def test_eds_closed_form_with_the_exact_kernel():
    """Appendix A's closed form holds for any I: with the exact series of Appendix C in both
    the closed form and the quadrature."""
    k = np.array([0.02, 0.2, 1.0])
    m, a0, an = 0.1, 0.01, 0.5
    ref = np.array([_eds_closed_form(kk, m, a0, an, kernel.I_series) for kk in k])
    got = _eds_response(k, m, a0, an, 400, kern="series")
    assert np.allclose(got, ref, rtol=2e-5)
    # and the fit's response stays within the fit's own accuracy of the exact one (App. C)
    fit = _eds_response(k, m, a0, an, 400)
    assert np.all(np.abs(fit / got - 1) < GOLD["fit_rel_err_all_x"]["tol"])
    assert np.abs(fit / got - 1).max() > 1e-5          # but they are different kernels


def test_eds_closed_form_other_mass():
    k = np.array([0.05, 0.5])
    m, a0, an = 0.05, 0.02, 1.0
    ref = np.array([_eds_closed_form(kk, m, a0, an) for kk in k])
    got = _eds_response(k, m, a0, an, 600)
    assert np.allclose(got, ref, rtol=2e-5)


def test_large_scale_fluid_limit():
    """k -> 0 in LCDM: history ~ D(a), growing-mode initial conditions -> R -> 1, with an
    error that falls at second order in the node spacing."""
    om = 0.3
    errs = []
    for J in (32, 64, 128):
        nodes = log_spaced_nodes(0.01, 1.0, J)
        d, f = growth(nodes, om)
        amp = d / d[-1]
        k = np.array([1e-5])
        theta = -f[0] * nodes[0] * bg.hubble_rate(nodes[0], om)
        r = response.nu_amplitude(k, [1], [1.0], nodes[:-1], amp[:-1, None], [amp[-2]],
                                  [amp[0]], [theta], 1.0, 0.3, om, 0.7, 1)
        errs.append(abs(1.0 - r["ratio"][0]))
    assert errs[-1] < 1e-4
    assert 3.5 < errs[0] / errs[1] < 4.6 and 3.5 < errs[1] / errs[2] < 4.6


def test_initial_condition_term_alone():
    """With no source (P_M = 0) and k -> 0, P_nu^{1/2} = P_nu,i^{1/2}{1 - (s - s_i) a_i [theta/delta]_i}."""
    om, a0, an = 0.3, 0.05, 0.4
    nodes = log_spaced_nodes(a0, an, 20)
    theta = -3.7e-4
    r = response.nu_amplitude([1e-7], [1], [1e-300], nodes[:-1], np.zeros((19, 1)), [0.0],
                              [2.0], [theta], an, 0.3, om, 0.7, 4, f_nu=0.0)
    ds = integrate.quad(lambda a: 1.0 / (a ** 3 * bg.hubble_rate(a, om)), a0, an,
                        epsrel=1e-13)[0]
    assert r["pnu_half"][0] == pytest.approx(2.0 * (1.0 - ds * a0 * theta), rel=1e-10)


def test_small_scale_limit_and_appendix_a_fit():
    """EdS, history ~ a: R (k/k_fs)^2 -> 1 for k >> k_fs; R ~ 1/(1+k/k_fs)^2 within 12%."""
    m, a0, an = 0.1, 1e-3, 1.0
    kfs = np.sqrt(1.5 * bg.mean_inverse_v2(an, m)) * an * bg.hubble_rate(an, 1.0)
    k = kfs * np.array([0.3, 1.0, 3.0, 10.0, 30.0, 100.0])
    r = _eds_response(k, m, a0, an, 600)
    approx = 1.0 / (1.0 + k / kfs) ** 2
    assert np.all(np.abs(r / approx - 1.0) < GOLD["app_a_approx_rel_err"]["tol"])
    lim = r * (k / kfs) ** 2
    assert lim[-1] == pytest.approx(1.0, abs=0.05)
    assert np.all(np.diff(lim[2:]) > 0)


def test_trapezoid_weights_integrate_ln_a():
    nodes = np.array([0.01, 0.02, 0.05, 0.07, 0.2])
    g = response.sub_grid(nodes, 5, 0.3)
    assert g["w"].sum() == pytest.approx(np.log(0.2 / 0.01), rel=1e-14)
    assert g["ds"][-1] == 0.0 and np.all(np.diff(g["ds"]) < 0)
    full = integrate.quad(lambda a: 1.0 / (a ** 3 * bg.hubble_rate(a, 0.3)), 0.01, 0.2,
                          epsrel=1e-13)[0]
    assert g["ds"][0] == pytest.approx(full, rel=1e-11)


def test_single_iteration_is_converged():
    """Sec. 4.3 (iii): iterating again changes P_nu^{1/2} by ~1e-4 (Appendix B: O(f_nu (H dt)^2))."""
    om = 0.3
    nodes = log_spaced_nodes(0.01, 1.0, 200)
    k = np.geomspace(0.0123, 2.7, 24)
    pcdm = 30.0 / k
    h = synthetic_history(k, pcdm, nodes, 0.6, om)
    kw = dict(k_mean=k, counts=np.ones(24), pcdm_half=pcdm, hist_a=h["a"],
              hist_pm_half=h["pm_half"], pnu_half_prev=h["pnu_half"][-1],
              pnu_half_init=h["pnu_half_init"], theta_over_delta_init=h["theta_over_delta_init"],
              a_now=1.0, m_nu_total=0.6, omega_m=om, hubble=0.7, substeps=8)
    one = response.nu_amplitude(iterations=1, **kw)["pnu_half"]
    two = response.nu_amplitude(iterations=2, **kw)["pnu_half"]
    three = response.nu_amplitude(iterations=3, **kw)["pnu_half"]
    d12 = np.abs(two / one - 1.0)
    assert d12.max() < GOLD["iteration_change"]["tol"]
    assert np.abs(three / two - 1.0).max() < 1e-2 * d12.max() + 1e-15


def test_massless_neutrinos_drop_out():
    """M_nu = 0: f_nu = 0, no neutrino term (Sec. 4.3 (iv)); the stored node is P_cdm^{1/2}."""
    nodes = log_spaced_nodes(0.01, 0.5, 8)
    k = np.array([0.05, 0.5])
    r = response.nu_amplitude(k, [1, 1], [2.0, 3.0], nodes[:-1], np.ones((7, 2)), [1, 1],
                              [1, 1], [0, 0], 0.5, 0.0, 0.3, 0.7, 4)
    assert r["f_nu"] == 0.0 and np.all(r["pnu_half"] == 0) and np.all(r["ratio"] == 0)
    assert np.array_equal(r["pm_half_now"], [2.0, 3.0])


# ---- mass hierarchy (Sec. 6.2): species with their own masses -------------------------------

def _eds_species(k, masses, a0, an, J, Q=8):
    nodes = log_spaced_nodes(a0, an, J)
    B = len(k)
    r = response.nu_amplitude(k, np.ones(B), an * np.ones(B), nodes[:-1],
                              nodes[:-1, None] * np.ones((1, B)), np.zeros(B), np.zeros(B),
                              np.zeros(B), an, 0.0, 1.0, 0.7, Q, f_nu=0.0, species=masses)
    return r["pnu_half"] / an


@pytest.mark.parametrize("which", ["hierarchy_normal_eV", "hierarchy_inverted_eV"])
def test_hierarchy_eds_is_the_mass_weighted_closed_form(which):
    """EdS with delta_M ~ a: each species follows Appendix A's closed form with its own mass,
    and the neutrino contrast is their mean weighted by m_s / M_nu (a massless species adds
    nothing). The paper's normal and inverted hierarchies of M_nu = 0.1 eV."""
    masses = GOLD[which]["value"]
    M = sum(masses)
    k = np.array([0.01, 0.1, 0.5])
    a0, an = 0.01, 0.5
    ref = sum(m / M * np.array([_eds_closed_form(kk, m, a0, an) for kk in k])
              for m in masses if m > 0)
    got = _eds_species(k, masses, a0, an, 400)
    assert np.allclose(got, ref, rtol=2e-5)


def test_hierarchy_reduces_to_the_degenerate_and_single_species_cases():
    """Equal masses give the default degenerate computation; one massive species among
    massless ones gives a single species of that mass."""
    om = 0.3
    nodes = log_spaced_nodes(0.01, 1.0, 40)
    k = np.geomspace(0.0123, 2.7, 12)
    pcdm = 30.0 / k
    h = synthetic_history(k, pcdm, nodes, 0.3, om)
    kw = dict(k_mean=k, counts=np.ones(12), pcdm_half=pcdm, hist_a=h["a"],
              hist_pm_half=h["pm_half"], pnu_half_prev=h["pnu_half"][-1],
              pnu_half_init=h["pnu_half_init"], theta_over_delta_init=h["theta_over_delta_init"],
              a_now=1.0, omega_m=om, hubble=0.7, substeps=4)
    degenerate = response.nu_amplitude(m_nu_total=0.3, n_species=3, **kw)["pnu_half"]
    three = response.nu_amplitude(m_nu_total=0.0, species=[0.1, 0.1, 0.1], **kw)["pnu_half"]
    assert np.allclose(three, degenerate, rtol=1e-13, atol=0.0)
    one = response.nu_amplitude(m_nu_total=0.3, n_species=1, **kw)["pnu_half"]
    lone = response.nu_amplitude(m_nu_total=0.0, species=[0.0, 0.3, 0.0], **kw)["pnu_half"]
    assert np.allclose(lone, one, rtol=1e-13, atol=0.0)


def test_hierarchy_species_initial_amplitudes_enter_with_their_weights():
    """With no source term the neutrino amplitude is the weighted sum of each species'
    initial-condition term I(x_i,s) P_s {1 - (s - s_i) a_i theta} (eq. (deltaI-nu))."""
    nodes = np.array([0.01, 0.02])
    k = np.array([0.05, 0.3])
    masses = [0.02, 0.08]
    ics = np.array([[1.0, 2.0], [3.0, 5.0]])
    theta = np.array([-0.4, -0.4])
    with np.errstate(divide="ignore", invalid="ignore"):     # P_cdm = 0: R is undefined
        r = response.nu_amplitude(k, [1, 1], [0.0, 0.0], nodes[:-1], np.zeros((1, 2)),
                                  [0.0, 0.0], [0.0, 0.0], theta, nodes[-1], 0.0, 0.3, 0.7, 2,
                                  f_nu=0.0, species=masses, pnu_half_init_species=ics)
    ds = integrate.quad(lambda a: 1.0 / (a ** 3 * bg.hubble_rate(a, 0.3)), 0.01, 0.02,
                        epsrel=1e-13)[0]
    want = sum(m / 0.1 * kernel.I_fit(k * ds * bg.T_NU0 / m) * ics[i]
               for i, m in enumerate(masses)) * (1.0 - ds * 0.01 * theta)
    assert np.allclose(r["pnu_half"], want, rtol=1e-10)


def test_response_at_the_first_node_is_the_initial_amplitude():
    """At tau = tau_i eq. (P-final) has no interval to integrate and I(0) = 1."""
    k = np.array([0.01, 0.3, 2.0])
    init = np.array([0.7, 0.4, 0.05])
    r = response.nu_amplitude(k, np.ones(3), np.ones(3), np.zeros(0), np.zeros((0, 3)),
                              np.zeros(3), init, np.full(3, -3e-4), 0.02, 0.3, 0.3, 0.7, 8)
    assert np.array_equal(r["pnu_half"], init)


# ------------------------------------- self-consistent stored histories (Sec. 4.3) ----
def _eds_replay(k, m, a0, an, J):
    nodes = log_spaced_nodes(a0, an, J)
    cdm = nodes[:, None] * np.ones((1, len(k)))
    B = len(k)
    pm, pnu = response.replay_history(k, np.ones(B), cdm, nodes, np.zeros(B), np.zeros(B),
                                      3 * m, 1.0, 0.7, 8, f_nu=0.0)
    return nodes, pm, pnu


def test_replayed_history_matches_the_eds_closed_form_at_every_node():
    """Appendix A at every stored node: in EdS with delta_M ~ a and no initial neutrino
    perturbation, the node j of a replayed history is F_fin(k, a_j) a_j, and its error falls
    at second order in the node spacing at the same a (J - 1 = 98 -> 196 intervals)."""
    k = np.array([0.01, 0.1, 0.3, 1.0])
    m, a0, an = 0.1, 0.01, 0.5
    errs = {}
    for J in (99, 197):
        nodes, pm, pnu = _eds_replay(k, m, a0, an, J)
        assert np.array_equal(pm, nodes[:, None] * np.ones((1, len(k))))   # f_nu = 0
        step = (J - 1) // 49
        rows = []
        for j in (1, 6, 12, 24, 49):
            a_j = nodes[j * step]
            ref = np.array([_eds_closed_form(kk, m, a0, a_j) for kk in k])
            rows.append(np.abs(pnu[j * step] / a_j / ref - 1.0))
        errs[J] = np.array(rows)
    assert errs[197][-1].max() < 1e-4
    ratio = errs[99] / errs[197]
    assert np.all((ratio > 3.5) & (ratio < 4.5))


def test_replayed_node_depends_only_on_earlier_nodes():
    """Causality of the loop: the node a_j of a replay over J nodes equals the last node of
    a replay over the first j + 1 nodes only, for every j."""
    om = 0.3
    nodes = log_spaced_nodes(0.02, 1.0, 12)
    k = np.array([0.005, 0.05, 0.5, 2.0])
    d, f = growth(nodes, om)
    cdm = (d / d[-1])[:, None] * np.array([3.0, 2.0, 1.0, 0.5])[None, :]
    theta = np.full(4, -f[0] * nodes[0] * bg.hubble_rate(nodes[0], om))
    ic = cdm[0] / (1.0 + k / 0.1) ** 2
    pm, pnu = response.replay_history(k, np.ones(4), cdm, nodes, ic, theta, 0.3, om, 0.7, 4)
    for j in range(1, len(nodes)):
        pm_j, pnu_j = response.replay_history(k, np.ones(4), cdm[:j + 1], nodes[:j + 1], ic,
                                              theta, 0.3, om, 0.7, 4)
        assert np.array_equal(pm_j[-1], pm[j]) and np.array_equal(pnu_j[-1], pnu[j])


def test_replayed_history_limits_of_the_total_matter_node():
    """What each stored node holds, P_M^{1/2} = (1 - f_nu) P_cdm^{1/2} + f_nu P_nu^{1/2}, from
    the two limits of Sec. 3.3: for k -> 0 the neutrinos follow the CDM (growing mode, so
    P_M -> P_cdm and P_nu -> P_cdm at every node), for k >> k_fs they do not cluster
    (P_nu^{1/2} < (k_fs/k)^2 P_cdm^{1/2}, so P_M^{1/2} -> (1 - f_nu) P_cdm^{1/2})."""
    om, m_tot = 0.3, 0.6
    nodes = log_spaced_nodes(0.01, 1.0, 120)
    d, f = growth(nodes, om)
    k = np.array([1e-5, 50.0])
    cdm = (d / d[-1])[:, None] * np.ones((1, 2))
    theta = np.full(2, -f[0] * nodes[0] * bg.hubble_rate(nodes[0], om))
    ic = np.array([cdm[0, 0], 0.0])
    pm, pnu = response.replay_history(k, np.ones(2), cdm, nodes, ic, theta, m_tot, om, 0.7, 8)
    fn = bg.f_nu(m_tot, om, 0.7)
    assert fn > 0.04
    assert np.all(np.abs(pnu[1:, 0] / cdm[1:, 0] - 1.0) < 1e-3)
    assert np.all(np.abs(pm[1:, 0] / cdm[1:, 0] - 1.0) < 1e-3 * fn)
    kfs = np.array([np.sqrt(1.5 * bg.mean_inverse_v2(a, m_tot / 3)) * a * bg.hubble_rate(a, om)
                    for a in nodes[1:]])
    bound = (kfs / k[1]) ** 2
    assert np.all(pnu[1:, 1] / cdm[1:, 1] < bound)
    assert np.all(np.abs(pm[1:, 1] / ((1.0 - fn) * cdm[1:, 1]) - 1.0) < fn * bound / (1.0 - fn))


def test_replay_with_all_matter_in_neutrinos_is_the_fluid_growing_mode():
    """f_nu = 1 (all matter in neutrinos, the CDM rows then carry weight 1 - f_nu = 0): for
    k -> 0 the neutrinos are the pressureless fluid of Sec. 3.3.1 and, started on the
    growing mode, follow D(a) at every node, which needs every stored node to be the
    replayed neutrino amplitude itself (the CDM rows here are deliberately wrong)."""
    om = 0.3
    nodes = log_spaced_nodes(0.01, 1.0, 150)
    d, f = growth(nodes, om)
    amp = d / d[-1]
    k = np.array([1e-5])
    theta = np.array([-f[0] * nodes[0] * bg.hubble_rate(nodes[0], om)])
    wrong_cdm = 5.0 * amp[:, None] + 1.0
    pm, pnu = response.replay_history(k, [1], wrong_cdm, nodes, [amp[0]], theta, 0.3, om,
                                      0.7, 8, f_nu=1.0)
    assert np.array_equal(pm, pnu)
    assert np.all(np.abs(pnu[:, 0] / amp - 1.0) < 2e-4)
