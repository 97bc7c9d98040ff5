// Expansion history used by the time grid of eq. (P-final): the superconformal time
// s = int da / (a^3 H) and the measure dtau = d ln a / (a H).
//
// Two flat backgrounds:
//  * matter + Lambda, the neutrinos counted as matter (the default);
//  * the relativistic one of Sec. 4.4: every massive species carries the energy density of
//    eq. (relativistic), rho_nu(a) = a^-3 int sqrt(m^2 + q^2/a^2) f_0(q) 4 pi q^2 dq, which
//    goes over from radiation to matter; photons and massless species are radiation;
//    Lambda closes the budget today.
// Densities are in units of today's critical density. A species of mass m has
// Omega_nu h^2 = m / 93.14 eV once non-relativistic (Sec. 2.1); the same conversion at
// m -> 0 gives a massless species, and photons are (8/7)(11/4)^{4/3} times that.
#pragma once

#include <vector>

#include "host_consts.hpp"

namespace pmnu {

struct Background {
  bool relativistic = false;
  double om_m = 0.3;              // all matter today, neutrino rest mass included
  double om_cb = 0.3;             // cold matter: om_m minus the neutrino rest mass
  double om_lambda = 0.7;
  double om_rad = 0.0;            // photons + massless species (a^-4)
  int n_nu = 0;                   // massive species with distinct masses
  double om_nu[kMaxSpecies] = {}; // their non-relativistic Omega (sum of equal masses)
  double m_over_t[kMaxSpecies] = {};  // m / T_nu0
};

// masses: the massive species [eV] as the response kernel sees them (equal masses: one
// entry with mass m and multiplicity n_equal); n_massless species add radiation.
Background make_background(bool relativistic, double omega_m, double hubble,
                           const std::vector<double>& masses, int n_equal, int n_massless);

// H(a) in h/Mpc (c = 1, lengths in Mpc/h).
double hubble_of(const Background& bg, double a);

// s(a2) - s(a1) over a short interval (16-point Gauss-Legendre in ln a).
double ds_of(const Background& bg, double a1, double a2);

// int_{a1}^{a2} da / (a^2 H) over a short interval (the kick factor of the leapfrog in s:
// du/ds = a^2 acc with a acc held fixed, Delta u = (a acc) int da / (a^2 H)).
double kick_of(const Background& bg, double a1, double a2);

// E(y) = int_0^inf sqrt(x^2 + y^2) x^2 / (e^x + 1) dx, y = m a / T_nu0: the energy
// integral of eq. (relativistic) in units of T_nu0^4/a^4 (up to the Fermi-Dirac prefactor).
double fd_energy(double y);

}  // namespace pmnu
