"""Pins of the oracle's linear theory of the stepped model (CPU).

* No neutrinos, flat Lambda-CDM: delta = D(a)/D(a_i) with D ~ H int da/(a H)^3, at second
  order in the step.
* Einstein-de Sitter with massive neutrinos that do not cluster (k -> infinity, no initial
  neutrino perturbation): delta_cdm ~ a^p, p = (sqrt(25 - 24 f_nu) - 1)/4 (the growing root of
  p(p + 1/2) = (3/2)(1 - f_nu) for delta'' + (3/2a) delta' = (3/(2a^2))(1 - f_nu) delta).
* Einstein-de Sitter, k -> 0 with neutrinos following the matter (equal initial perturbation,
  growing-mode velocity): every component grows as a.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import background as bg
from oracle import linear


def _lcdm_growth(a, om):
    e = lambda x: np.sqrt(om / x ** 3 + 1 - om)
    i = integrate.quad(lambda x: 1.0 / (x * e(x)) ** 3, 0.0, a, epsabs=0, epsrel=1e-12)[0]
    d = e(a) * i
    dlne = -1.5 * om / (a ** 3 * e(a) ** 2)
    f = dlne + 1.0 / (a * a * e(a) ** 3 * i)
    return d, f


def test_lcdm_growth_factor_at_second_order():
    om, a0, a1 = 0.3, 0.02, 1.0
    d0, f0 = _lcdm_growth(a0, om)
    d1, _ = _lcdm_growth(a1, om)
    errs = []
    for n in (100, 200, 400):
        r = linear.linear_modes([0.1], np.geomspace(a0, a1, n + 1), 0.0, [0.0], [0.0], f0,
                                omega_m=om)
        errs.append(abs(r["d_cdm"][-1, 0] / (d1 / d0) - 1))
    assert errs[-1] < 3e-5
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_eds_non_clustering_neutrinos_power_law():
    m_tot, a0, a1 = 0.3, 0.05, 1.0
    fn = bg.f_nu(m_tot, 1.0, 0.7)
    p = (np.sqrt(25 - 24 * fn) - 1) / 4
    r = linear.linear_modes([300.0], np.geomspace(a0, a1, 401), m_tot, [0.0], [0.0], p,
                            omega_m=1.0, substeps=4)
    got = r["d_cdm"][-1, 0]
    assert got == pytest.approx((a1 / a0) ** p, rel=3e-5)
    assert abs(r["d_nu"][-1, 0]) < 1e-3 * got          # (k_fs/k)^2 of the matter
    assert (a1 / a0) ** p < 0.99 * (a1 / a0)            # really suppressed against a


def test_eds_large_scales_follow_the_matter():
    m_tot, a0, a1 = 0.3, 0.05, 1.0
    theta = -a0 * float(bg.hubble_rate(a0, 1.0))        # growing mode, f = 1
    r = linear.linear_modes([1e-6], np.geomspace(a0, a1, 401), m_tot, [1.0], [theta], 1.0,
                            omega_m=1.0, substeps=4)
    for key in ("d_cdm", "d_nu", "d_m"):
        assert r[key][-1, 0] == pytest.approx(a1 / a0, rel=2e-5), key
