"""Pins of the oracle's relativistic background, eq. (relativistic) and Sec. 4.4 (CPU).

* The energy of a Fermi-Dirac gas of mass m over its rest mass has closed-form limits: the
  radiation one (7 pi^4/120 over 3 zeta(3)/2 in units of T/(m a)) and the non-relativistic
  expansion 1 + 15 zeta(5)/(2 zeta(3)) (T/ma)^2 - ... .
* Photons against one neutrino species: (8/7)(11/4)^{4/3} (Stefan-Boltzmann); their
  density against the critical density from the physical constants.
* Flatness today, and the superconformal time of a matter + radiation universe in closed
  form.
* The response consumes the background through s and dtau: the k -> 0 source integral and
  the initial-condition term against adaptive quadratures of the same background.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import background as bg
from oracle import response

ZETA3 = 1.2020569031595942


def _fd_moment(n):
    """int_0^inf x^n / (e^x + 1) dx = (1 - 2^-n) n! zeta(n + 1)."""
    return (1.0 - 2.0 ** -n) * math.factorial(n) * special.zeta(n + 1)


def test_energy_ratio_non_relativistic_expansion():
    """E/E_rest - 1 = sum_j binom(1/2, j) M_{2j+2} / (M_2 y^{2j}), y = m a / T, from
    sqrt(1 + x^2/y^2) expanded under the Fermi-Dirac moments M_n (an asymptotic series; four
    terms leave < 1e-7 of the correction at y >= 50)."""
    for y in (50.0, 100.0, 1000.0):
        m = y * bg.T_NU0                       # at a = 1
        got = bg.nu_energy_over_rest(1.0, m) - 1.0
        series = sum(special.binom(0.5, j) * _fd_moment(2 * j + 2) / (_fd_moment(2) * y ** (2 * j))
                     for j in range(1, 5))
        assert got == pytest.approx(series, rel=1e-6)
    assert _fd_moment(2) == pytest.approx(1.5 * ZETA3, rel=1e-15)


def test_energy_ratio_radiation_limit():
    """y -> 0: E = M_3 + (y^2 / 2) M_1 + O(y^4 ln y), so E/E_rest y -> (7 pi^4/120) / (3 zeta3/2)
    (every species as radiation), M_3 = 7 pi^4 / 120, M_1 = pi^2 / 12."""
    for y in (1e-2, 1e-3, 1e-4):
        m = 0.06
        a = y * bg.T_NU0 / m
        got = bg.nu_energy_over_rest(a, m) * y
        lead = 7 * np.pi ** 4 / 120 + 0.5 * y * y * np.pi ** 2 / 12
        assert got == pytest.approx(lead / (1.5 * ZETA3), rel=1e-11 + y ** 4)


def test_photons_against_one_neutrino_species():
    assert bg.photon_omega_h2() / bg.massless_omega_h2() == pytest.approx(
        (8.0 / 7.0) * (11.0 / 4.0) ** (4.0 / 3.0), rel=1e-11)


def test_photon_density_from_physical_constants():
    """Omega_gamma h^2 = (pi^2/15) T_gamma^4 / (3 H0^2 / 8 pi G) with CODATA constants. The
    oracle goes through the 93.14 eV conversion of Sec. 2.1, which belongs to a slightly
    colder neutrino background than 1.95 K (93.40 eV at 1.95 K): 0.3% apart."""
    G, mpc, c = 6.67430e-11, 3.0856775814913673e22, 299792458.0
    ev, hbarc = 1.602176634e-19, 197.3269804e-9                      # J, eV m
    rho_crit = 3 * (1e5 / mpc) ** 2 / (8 * np.pi * G) * c ** 2 / ev * hbarc ** 3   # eV^4/h^2
    t_gamma = (11.0 / 4.0) ** (1.0 / 3.0) * bg.T_NU0
    assert bg.photon_omega_h2() == pytest.approx(np.pi ** 2 / 15 * t_gamma ** 4 / rho_crit,
                                                 rel=5e-3)


@pytest.mark.parametrize("masses", [(0.1, 0.1, 0.1), (0.0, 0.049, 0.051), (0.0, 0.0, 0.0)])
def test_flat_today_and_matter_at_late_times(masses):
    b = bg.Background(0.3, 0.7, masses)
    assert float(bg.hubble_rate(1.0, 0.3, b)) == pytest.approx(bg.H0, rel=1e-14)
    # the cold matter and the neutrino rest mass add up to Omega_M
    assert b.omega_cb + sum(b.omega_rest) == pytest.approx(0.3, rel=1e-15)
    # radiation: photons and every massless species
    n0 = sum(1 for m in masses if m == 0.0)
    assert b.omega_rad * 0.49 == pytest.approx(bg.photon_omega_h2() + n0 * bg.massless_omega_h2(),
                                               rel=1e-14)


def test_superconformal_time_matter_plus_radiation_closed_form():
    """Three massless species and Omega_M = 1 - Omega_r (no Lambda): H = H0 sqrt(Om a^-3 +
    Or a^-4), and s(a2) - s(a1) = [ln((u - sqrt Or)/(u + sqrt Or))] / (H0 sqrt Or),
    u = sqrt(Om a + Or)."""
    h = 0.7
    o_r = (bg.photon_omega_h2() + 3 * bg.massless_omega_h2()) / h ** 2
    b = bg.Background(1.0 - o_r, h, (0.0, 0.0, 0.0))
    assert abs(b.omega_lambda) < 1e-15
    om = 1.0 - o_r

    def s(a):
        u = np.sqrt(om * a + o_r)
        return np.log((u - np.sqrt(o_r)) / (u + np.sqrt(o_r))) / (bg.H0 * np.sqrt(o_r))

    for a1, a2 in ((1e-5, 1e-4), (1e-3, 0.02), (0.02, 1.0)):
        got = bg.superconformal_interval(a1, a2, om, b)
        assert got == pytest.approx(s(a2) - s(a1), rel=1e-11)


def test_early_universe_is_radiation_dominated():
    """At a = 1e-6 every species is relativistic: (H/H0)^2 a^4 -> photons + 3 species."""
    b = bg.Background(0.3, 0.7, (0.1, 0.1, 0.1))
    a = 1e-6
    e2a4 = (float(bg.hubble_rate(a, 0.3, b)) / bg.H0) ** 2 * a ** 4
    rad = (bg.photon_omega_h2() + 3 * bg.massless_omega_h2()) / 0.49
    assert e2a4 == pytest.approx(rad, rel=2e-2)            # cold matter adds O(a / a_eq)
    e2a4_cold_removed = e2a4 - b.omega_cb * a
    assert e2a4_cold_removed == pytest.approx(rad, rel=1e-6)


def _source_integral(a_i, a_n, om, b):
    """int_{tau_i}^{tau_n} (s_n - s') dtau' = int_{s_i}^{s_n} (tau - tau_i) ds (exchange the
    order of integration), as an ODE in a: d tau/da = 1/(a^2 H), dI/da = (tau - tau_i)/(a^3 H)."""
    def rhs(a, y):
        h = float(bg.hubble_rate(a, om, b))
        return [1.0 / (a * a * h), y[0] / (a ** 3 * h)]
    sol = integrate.solve_ivp(rhs, (a_i, a_n), [0.0, 0.0], method="DOP853", rtol=1e-12,
                              atol=1e-30)
    return sol.y[1, -1]


def test_response_source_term_uses_the_background():
    """k -> 0 (I = 1), constant P_M = 1, no initial amplitude: P_nu^{1/2} = (3/2) Om H0^2
    int (s - s') dtau', second order in the node spacing towards an ODE solution."""
    om, a_i, a_n = 0.3, 0.01, 0.1
    masses = (0.0, 0.049, 0.051)
    b = bg.Background(om, 0.7, masses)
    ref = 1.5 * om * bg.H0 ** 2 * _source_integral(a_i, a_n, om, b)
    flat = 1.5 * om * bg.H0 ** 2 * _source_integral(a_i, a_n, om, None)
    assert abs(ref / flat - 1) > 3e-3                        # radiation matters at these a
    errs = []
    for J in (16, 32):
        nodes = np.geomspace(a_i, a_n, J)
        r = response.nu_amplitude([1e-9], [1], [1.0], nodes[:-1], np.ones((J - 1, 1)), [1.0],
                                  [0.0], [0.0], a_n, 0.1, om, 0.7, 4, f_nu=0.0,
                                  species=masses, relativistic=True)
        errs.append(abs(r["pnu_half"][0] / ref - 1))
    assert errs[-1] < 2e-5
    assert 3.8 < errs[0] / errs[1] < 4.5


def test_response_initial_condition_term_uses_the_background():
    om, a0, an = 0.3, 0.02, 0.2
    masses = (0.1, 0.1, 0.1)
    b = bg.Background(om, 0.7, masses)
    nodes = np.geomspace(a0, an, 12)
    theta = -2.1e-3
    r = response.nu_amplitude([1e-9], [1], [1e-300], nodes[:-1], np.zeros((11, 1)), [0.0],
                              [2.0], [theta], an, 0.3, om, 0.7, 4, f_nu=0.0,
                              relativistic=True)
    ds = integrate.quad(lambda a: 1.0 / (a ** 3 * float(bg.hubble_rate(a, om, b))), a0, an,
                        epsabs=0.0, epsrel=1e-12)[0]
    assert r["pnu_half"][0] == pytest.approx(2.0 * (1.0 - ds * a0 * theta), rel=1e-10)
