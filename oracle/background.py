"""Background cosmology for the oracle (FP64).

Units (paper Sec. 2.1): c = G = k_B = 1, comoving lengths in Mpc/h, wavenumbers in h/Mpc,
so H0 = 100 h km/s/Mpc = 1/2997.92458 h/Mpc and time is measured in Mpc/h.

Two flat backgrounds: matter + Lambda with the neutrinos counted as matter (the default),
and the one of Sec. 4.4 (`Background`), in which the massive neutrinos carry the energy
density of eq. (relativistic) and photons and massless neutrinos add radiation.
"""
import functools

import numpy as np
from scipy import integrate

C_KMS = 299792.458                  # speed of light [km/s]
H0 = 100.0 / C_KMS                  # [h/Mpc]
KB_EV_PER_K = 8.617333262e-5        # Boltzmann constant [eV/K]
T_NU0 = 1.95 * KB_EV_PER_K          # neutrino temperature today [eV], Sec. 2.1
ZETA3 = 1.2020569031595942
ZETA5 = 1.0369277551433699


def f_nu(m_nu_total, omega_m, hubble):
    """Neutrino fraction of matter, Omega_nu/Omega_M = sum(m)/(93.14 eV Omega_M h^2), Sec. 2.1."""
    return m_nu_total / (93.14 * omega_m * hubble * hubble)


def _momentum_integral(g):
    """int_0^inf g(q) dq for a smooth g decaying like a thermal tail (q in eV)."""
    edges = np.array([0.0, 1.0, 4.0, 12.0, 40.0, 120.0]) * T_NU0
    return sum(integrate.quad(g, lo, hi, epsabs=0.0, epsrel=1e-13, limit=200)[0]
               for lo, hi in zip(edges[:-1], edges[1:]))


def fermi_dirac(q):
    """Relic neutrino occupation f_0(q) at temperature T_nu0 (the constant g/(2 pi)^3 of the
    phase-space density cancels in every ratio below)."""
    return 1.0 / (np.exp(q / T_NU0) + 1.0)


@functools.lru_cache(maxsize=None)
def _number_integral():
    return _momentum_integral(lambda q: q * q * fermi_dirac(q))


def nu_energy_over_rest(a, m):
    """rho_nu(a) / (rest-mass density at a) for one species of mass m [eV], eq. (relativistic):
    a^-3 int eps(q, a) f_0 4 pi q^2 dq over a^-3 m int f_0 4 pi q^2 dq, eps = sqrt(m^2 + q^2/a^2)."""
    num = _momentum_integral(lambda q: np.sqrt(m * m + (q / a) ** 2) * q * q * fermi_dirac(q))
    return num / (m * _number_integral())


def massless_omega_h2():
    """Omega h^2 a^4 of one massless species: the m -> 0 limit of
    (m / 93.14 eV) a^-3 nu_energy_over_rest(a, m), i.e. int q^3 f_0 / int q^2 f_0 / 93.14 eV."""
    return _momentum_integral(lambda q: q ** 3 * fermi_dirac(q)) / _number_integral() / 93.14


def photon_omega_h2():
    """Omega_gamma h^2 a^4: photons at T_gamma = (11/4)^{1/3} T_nu0 (two polarisations,
    Bose-Einstein) against one neutrino species (neutrino + antineutrino, Fermi-Dirac)."""
    t_gamma = (11.0 / 4.0) ** (1.0 / 3.0) * T_NU0
    bose = integrate.quad(lambda q: q ** 3 / np.expm1(q / t_gamma), 0.0, 200.0 * t_gamma,
                          epsabs=0.0, epsrel=1e-13, limit=200)[0]
    fermi = _momentum_integral(lambda q: q ** 3 * fermi_dirac(q))
    return massless_omega_h2() * bose / fermi


class Background:
    """Flat background of Sec. 4.4 with the neutrino energy density of eq. (relativistic).

    masses: every neutrino species [eV] (massless ones included). Densities in units of
    today's critical density: a species of mass m has Omega h^2 = m / 93.14 eV once
    non-relativistic (Sec. 2.1) and Omega(a) = (m / 93.14 eV h^2) a^-3 nu_energy_over_rest;
    massless species and photons are radiation; cold matter is Omega_M minus the neutrino
    rest mass, so that Omega_M counts all matter; Lambda closes the budget today.
    """

    def __init__(self, omega_m, hubble, masses):
        self.omega_m = float(omega_m)
        self.hubble = float(hubble)
        self.masses = tuple(float(m) for m in masses)
        h2 = self.hubble ** 2
        self.massive = tuple(m for m in self.masses if m > 0.0)
        n_massless = len(self.masses) - len(self.massive)
        self.omega_rest = tuple(m / (93.14 * h2) for m in self.massive)
        self.omega_cb = self.omega_m - sum(self.omega_rest)
        self.omega_rad = (photon_omega_h2() + n_massless * massless_omega_h2()) / h2
        nu_today = sum(o * nu_energy_over_rest(1.0, m)
                       for o, m in zip(self.omega_rest, self.massive))
        self.omega_lambda = 1.0 - self.omega_cb - self.omega_rad - nu_today
        self.key = ("relativistic", self.omega_m, self.hubble, self.masses)

    def e2(self, a):
        """(H(a) / H0)^2 at one scale factor."""
        nu = sum(o * nu_energy_over_rest(a, m) for o, m in zip(self.omega_rest, self.massive))
        return (self.omega_cb + nu) / a ** 3 + self.omega_rad / a ** 4 + self.omega_lambda


def hubble_rate(a, omega_m, background=None):
    """H(a) [h/Mpc]: flat matter + Lambda, or the given Background (Sec. 4.4)."""
    a = np.asarray(a, dtype=np.float64)
    if background is None:
        return H0 * np.sqrt(omega_m / a ** 3 + 1.0 - omega_m)
    e2 = np.vectorize(background.e2, otypes=[np.float64])(a)
    return H0 * np.sqrt(e2)


def _ds_da(a, omega_m, background):
    # s = int dtau / a and dtau = da / (a^2 H)  =>  ds = da / (a^3 H)
    return 1.0 / (a ** 3 * float(hubble_rate(a, omega_m, background)))


def kick_interval(a1, a2, omega_m, background=None):
    """int_{a1}^{a2} da / (a^2 H(a)) [Mpc/h]: with ds = da/(a^3 H) and d^2x/ds^2 = a^2 g,
    g = -grad phi ~ 1/a, a kick holding a g fixed changes dx/ds by (a g) times this."""
    if a1 == a2:
        return 0.0
    val, _ = integrate.quad(lambda a: 1.0 / (a * a * float(hubble_rate(a, omega_m, background))),
                            a1, a2, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


def superconformal_interval(a1, a2, omega_m, background=None):
    """s(a2) - s(a1) = int_{a1}^{a2} da / (a^3 H(a))  [Mpc/h], Sec. 3.2."""
    if a1 == a2:
        return 0.0
    val, _ = integrate.quad(_ds_da, a1, a2, args=(omega_m, background), epsabs=0.0,
                            epsrel=1e-13, limit=200)
    return val


def omega_m_of_a(a, omega_m):
    """Matter fraction of the total density at scale factor a."""
    e2 = omega_m / a ** 3 + 1.0 - omega_m
    return omega_m / (a ** 3 * e2)


def mean_inverse_v2(a, m_nu_single):
    """Mean inverse squared velocity of relic neutrinos, eq. (v2) (c = 1, dimensionless)."""
    return (2.0 * np.log(2.0) / (3.0 * ZETA3)) * (m_nu_single * a / T_NU0) ** 2


def k_free_streaming(a, m_nu_single, omega_m):
    """k_fs(a) = sqrt(3/2 Omega_M(a) <v^-2>) a H  [h/Mpc], eq. (kfs-formal)."""
    return (np.sqrt(1.5 * omega_m_of_a(a, omega_m) * mean_inverse_v2(a, m_nu_single))
            * a * hubble_rate(a, omega_m))
