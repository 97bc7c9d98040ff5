// Flat expansion histories for the time grid of eq. (P-final), with the relativistic
// neutrino energy density of eq. (relativistic) as an option (Sec. 4.4).
#include "background.hpp"

#include <cmath>
#include <vector>

namespace pmnu {

namespace {

constexpr double kZeta3 = 1.2020569031595942;
constexpr double kEvPerOmegaH2 = 93.14;   // m_nu = 93.14 eV Omega_nu h^2 (Sec. 2.1)

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
struct GaussLegendre {
  std::vector<double> x, w;
  explicit GaussLegendre(int n) : x(n), w(n) {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      double q0 = 1.0, q1 = z;
      for (int k = 2; k <= n; ++k) {
        const double q2 = ((2.0 * k - 1.0) * z * q1 - (k - 1.0) * q0) / k;
        q0 = q1;
        q1 = q2;
      }
      const double d = n * (z * q1 - q0) / (z * z - 1.0);
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * d * d);
    }
  }
};

const GaussLegendre& gl16() {
  static const GaussLegendre g(16);
  return g;
}

// E(y) and dE/dy by quadrature. With x = y sinh t the square root becomes y cosh t and the
// integrand y^4 sinh^2 t cosh^2 t / (e^{y sinh t} + 1) is analytic on the real axis, its
// nearest poles pi/2 away (small y) or at the Fermi-Dirac poles scaled by 1/y (large y);
// 16 equal panels over x in [0, 64] (e^-64 truncation) of 16 Gauss points each.
void fd_energy_direct(double y, double* e, double* de) {
  const GaussLegendre& g = gl16();
  const int panels = 16;
  const double t_end = std::asinh(64.0 / y);
  const double hw = 0.5 * t_end / panels;
  double se = 0.0, sd = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double mid = (2 * p + 1) * hw;
    for (size_t i = 0; i < g.x.size(); ++i) {
      const double t = mid + hw * g.x[i];
      const double sh = std::sinh(t), ch = std::cosh(t);
      const double fd = 1.0 / (std::exp(y * sh) + 1.0);
      se += g.w[i] * sh * sh * ch * ch * fd;
      sd += g.w[i] * sh * sh * fd;
    }
  }
  const double y3 = y * y * y;
  *e = y3 * y * se * hw;
  *de = y3 * sd * hw;   // dE/dy = int y x^2 f / sqrt(x^2 + y^2) dx
}

// E(e^u) tabulated with its u-derivative; cubic Hermite between nodes.
struct FdTable {
  static constexpr int kN = 8192;
  double u0, du;
  std::vector<double> g, dg;
  FdTable() : u0(std::log(1e-3)), du((std::log(1e6) - std::log(1e-3)) / (kN - 1)), g(kN), dg(kN) {
    for (int i = 0; i < kN; ++i) {
      const double y = std::exp(u0 + i * du);
      double e, de;
      fd_energy_direct(y, &e, &de);
      g[i] = e;
      dg[i] = y * de;
    }
  }
  bool covers(double y) const { return y >= 1e-3 && y < 1e6; }
  double operator()(double y) const {
    const double u = (std::log(y) - u0) / du;
    int i = static_cast<int>(u);
    if (i > kN - 2) i = kN - 2;
    const double t = u - i, t2 = t * t, t3 = t2 * t;
    return (2 * t3 - 3 * t2 + 1) * g[i] + (t3 - 2 * t2 + t) * du * dg[i] +
           (-2 * t3 + 3 * t2) * g[i + 1] + (t3 - t2) * du * dg[i + 1];
  }
};

const FdTable& fd_table() {
  static const FdTable t;
  return t;
}

// Energy density of one massive species today relative to its rest mass density:
// r(y) = E(y) / (E_rest y), E_rest = int x^2 / (e^x + 1) dx = 3 zeta(3) / 2.
double energy_over_rest(double y) { return fd_energy(y) / (1.5 * kZeta3 * y); }

}  // namespace

double fd_energy(double y) {
  if (!(y > 0.0)) return 7.0 * kPi * kPi * kPi * kPi / 120.0;   // massless: 7 pi^4 / 120
  const FdTable& t = fd_table();
  if (t.covers(y)) return t(y);
  double e, de;
  fd_energy_direct(y, &e, &de);
  return e;
}

Background make_background(bool relativistic, double omega_m, double hubble,
                           const std::vector<double>& masses, int n_equal, int n_massless) {
  Background bg;
  bg.relativistic = relativistic;
  bg.om_m = omega_m;
  bg.om_cb = omega_m;
  bg.om_lambda = 1.0 - omega_m;
  if (!relativistic) return bg;
  const double h2 = hubble * hubble;
  double om_nu_today = 0.0;
  bg.n_nu = 0;
  for (double m : masses) {
    if (!(m > 0.0) || bg.n_nu >= kMaxSpecies) continue;
    const double om_rest = n_equal * m / (kEvPerOmegaH2 * h2);
    bg.om_nu[bg.n_nu] = om_rest;
    bg.m_over_t[bg.n_nu] = m / kTnu0;
    bg.om_cb -= om_rest;
    om_nu_today += om_rest * energy_over_rest(m / kTnu0);
    ++bg.n_nu;
  }
  // one massless species: the m -> 0 limit of om_rest * r(m a / T) / a^3, times a^4
  const double om_one = (kTnu0 / (kEvPerOmegaH2 * h2)) * fd_energy(0.0) / (1.5 * kZeta3);
  const double photons = (8.0 / 7.0) * std::pow(11.0 / 4.0, 4.0 / 3.0);
  bg.om_rad = (photons + n_massless) * om_one;
  bg.om_lambda = 1.0 - bg.om_cb - bg.om_rad - om_nu_today;
  return bg;
}

double hubble_of(const Background& bg, double a) {
  const double a3 = a * a * a;
  if (!bg.relativistic) return kH0 * std::sqrt(bg.om_m / a3 + bg.om_lambda);
  double e2 = bg.om_cb / a3 + bg.om_rad / (a3 * a) + bg.om_lambda;
  for (int s = 0; s < bg.n_nu; ++s)
    e2 += bg.om_nu[s] * energy_over_rest(bg.m_over_t[s] * a) / a3;
  return kH0 * std::sqrt(e2);
}

double ds_of(const Background& bg, double a1, double a2) {
  const GaussLegendre& g = gl16();
  const double u1 = std::log(a1), u2 = std::log(a2);
  const double hw = 0.5 * (u2 - u1), mid = 0.5 * (u1 + u2);
  double s = 0.0;
  for (size_t i = 0; i < g.x.size(); ++i) {
    const double a = std::exp(mid + hw * g.x[i]);
    s += g.w[i] / (a * a * hubble_of(bg, a));
  }
  return s * hw;
}

double kick_of(const Background& bg, double a1, double a2) {
  const GaussLegendre& g = gl16();
  const double u1 = std::log(a1), u2 = std::log(a2);
  const double hw = 0.5 * (u2 - u1), mid = 0.5 * (u1 + u2);
  double s = 0.0;
  for (size_t i = 0; i < g.x.size(); ++i) {
    const double a = std::exp(mid + hw * g.x[i]);
    s += g.w[i] / (a * hubble_of(bg, a));
  }
  return s * hw;
}

}  // namespace pmnu
