"""Background cosmology for the oracle (FP64).

Units (paper Sec. 2.1): c = G = k_B = 1, comoving lengths in Mpc/h, wavenumbers in h/Mpc,
so H0 = 100 h km/s/Mpc = 1/2997.92458 h/Mpc and time is measured in Mpc/h.

The background is flat matter + Lambda with the neutrinos counted as matter (the paper's
relativistic neutrino background, eq. (relativistic), is not part of this step).
"""
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


def hubble_rate(a, omega_m):
    """H(a) [h/Mpc] for a flat matter + Lambda universe."""
    a = np.asarray(a, dtype=np.float64)
    return H0 * np.sqrt(omega_m / a ** 3 + 1.0 - omega_m)


def _ds_da(a, omega_m):
    # s = int dtau / a and dtau = da / (a^2 H)  =>  ds = da / (a^3 H)
    return 1.0 / (a ** 3 * float(hubble_rate(a, omega_m)))


def superconformal_interval(a1, a2, omega_m):
    """s(a2) - s(a1) = int_{a1}^{a2} da / (a^3 H(a))  [Mpc/h], Sec. 3.2."""
    if a1 == a2:
        return 0.0
    val, _ = integrate.quad(_ds_da, a1, a2, args=(omega_m,), epsabs=0.0,
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
