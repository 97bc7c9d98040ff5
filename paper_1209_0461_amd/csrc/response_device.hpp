// Device pieces of the neutrino response shared by the exact and the surrogate kernels
// (FP64, one workgroup of NT threads per (k-bin, box): RT = 256 when there are few
// (bin, box) pairs to spread over the chip, one wave when there are many).
#pragma once
#include "pm_nu_internal.hpp"

namespace pmnu {

constexpr int RT = 256;

// Rational fit of the free-streaming kernel I(x), the paper's Appendix C eq. (fit).
// x^4.1811 is taken as x^4 2^(0.1811 log2 x): FP64 to a few ulp, and cheaper than pow,
// whose extra-precision logarithm the small fractional exponent does not need.
__device__ __forceinline__ double i_fit_l2(double x, double l2x) {   // l2x = log2 x
  const double x2 = x * x, x4 = x2 * x2;
  const double num = 1.0 + 0.0168 * x2 + 0.0407 * x4;
  const double xp = x > 0.0 ? x4 * exp2(0.1811 * l2x) : 0.0;
  const double den = 1.0 + 2.1734 * x2 + 1.6787 * xp + 0.1467 * x4 * x4;
  return num / den;
}
__device__ __forceinline__ double i_fit(double x) {
  return i_fit_l2(x, x > 0.0 ? log2(x) : 0.0);
}

// The exact kernel of Appendix C, I(x) = 4/(3 zeta(3)) sum_{n>=1} (-1)^{n+1} n/(n^2+x^2)^2,
// summed with the alternating-series acceleration of Cohen, Rodriguez Villegas and Zagier
// (Experimental Math. 9 (2000) 3, their Algorithm 1): sum_{k>=0} (-1)^k a_k ~ sum_k c_k a_k/d
// over n terms. It applies because a_k = (k+1)/((k+1)^2+x^2)^2 = int_0^1 t^k w(t) dt with
// w(e^-u) = u sin(xu)/(2x), and the error is below 2 int|w| / (3+sqrt 8)^n: with n = 32 the
// relative error stays below ~1e-15 x^3, i.e. at rounding level up to x ~ 1e3 (where I is
// already ~3e-13) and below 1e-12 up to x ~ 1e4.
constexpr int kSeriesTerms = 32;
struct SeriesWeights {
  double w[kSeriesTerms];   // c_k / d times 4/(3 zeta(3)), signs included
};
constexpr SeriesWeights series_weights() {
  SeriesWeights s{};
  const int n = kSeriesTerms;
  // d = ((3+sqrt 8)^n + (3-sqrt 8)^n) / 2 = u_n / 2 with u_0 = 2, u_1 = 6, u_n = 6u_{n-1} - u_{n-2}
  double u0 = 2.0, u1 = 6.0;
  for (int i = 1; i < n; ++i) {
    const double u2 = 6.0 * u1 - u0;
    u0 = u1;
    u1 = u2;
  }
  const double d = 0.5 * u1;
  double b = -1.0, c = -d;
  for (int k = 0; k < n; ++k) {
    c = b - c;
    s.w[k] = c / d * (4.0 / (3.0 * 1.2020569031595942));
    b = (k + n) * (k - n) * b / ((k + 0.5) * (k + 1.0));
  }
  return s;
}

__device__ __forceinline__ double i_series(double x) {
  constexpr SeriesWeights W = series_weights();
  const double x2 = x * x;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kSeriesTerms; ++k) {
    const double n = k + 1.0;
    const double r = 1.0 / (n * n + x2);
    s += W.w[k] * n * r * r;
  }
  return s;
}

template <bool SERIES>
__device__ __forceinline__ double i_kernel(double x) {
  if constexpr (SERIES) return i_series(x);
  else return i_fit(x);
}
// the same with log2 x known (the fit then needs no logarithm; the series ignores it)
template <bool SERIES>
__device__ __forceinline__ double i_kernel_l2(double x, double l2x) {
  if constexpr (SERIES) return i_series(x);
  else return i_fit_l2(x, l2x);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup (NT threads); every thread gets the result.
template <int NT = RT>
__device__ __forceinline__ double block_sum_d(double v, double* red) {
  v = wave_sum_d(v);
  if constexpr (NT == 64) return v;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// Two sums over the workgroup at once; every thread gets both.
template <int NT = RT>
__device__ __forceinline__ double2 block_sum_d2(double2 v, double* red) {
  v.x = wave_sum_d(v.x);
  v.y = wave_sum_d(v.y);
  if constexpr (NT == 64) return v;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    red[2 * wave] = v.x;
    red[2 * wave + 1] = v.y;
  }
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    s.x += red[2 * w];
    s.y += red[2 * w + 1];
  }
  return s;
}

// sum over the per-workgroup partial mode sums of bin b ([box][bin][workgroup]):
// sum w |delta_k|^2
template <int NT = RT>
__device__ __forceinline__ double bin_mode_sum(const double* partial, int n_partial, int nbins,
                                               int box, int b, double* red) {
  // Each thread reads per = ceil(n_partial / NT) values at i = tid + NT u (coalesced for
  // every u), in as few rounds of at most U loads in flight as cover them, split evenly, so
  // that no round is a nearly empty one that would cost a memory latency of its own.
  constexpr int U = 16;
  const double* pp = partial + (static_cast<size_t>(box) * nbins + b) * n_partial;
  const int per = (n_partial + NT - 1) / NT;
  const int rounds = (per + U - 1) / U;
  const int chunk = rounds > 0 ? (per + rounds - 1) / rounds : 0;
  double s = 0.0;
  for (int u0 = 0; u0 < per; u0 += chunk) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = threadIdx.x + (u0 + u) * NT;
      v[u] = (u < chunk && i < n_partial) ? pp[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  return block_sum_d<NT>(s, red);
}

// eq. (P-final) for one bin: the initial-condition term plus the trapezoid sum over the
// sub-nodes, iterated `iterations` times on the current node (every thread gets it). With
// several species (mass hierarchy) each free-streams with its own kernel and the result is
// their mean weighted by m_s / M_nu; the source term is the common P_M^{1/2} history, so
// the quadrature uses the weighted sum of the kernels. ic_pnu: [kMaxSpecies][nbins] initial
// amplitudes of this box.
//
// The sum is linear in the unknown current node A_n = (1 - f_nu) P_cdm^{1/2} + f_nu P_nu^{1/2}
// (it enters only the last stored interval), so one pass gathers the part from the stored
// nodes and the coefficient of A_n; each iteration of Appendix B is then a scalar update
// and the kernel is evaluated once whatever the number of iterations. The initial-condition
// term is evaluated by the first wave only and enters the sum through thread 0. Each
// thread takes ceil(nq / NT) sub-nodes q = tid + NT u, in as few rounds of at most U
// whose loads go out together as cover them.
// red: 2 * NT / 64 doubles.
template <int NSP, bool SERIES, int NT>   // species: 1 (equal masses) or kMaxSpecies
__device__ __forceinline__ double exact_pnu_n(const RespBox& bx, double k, double pcdm_half,
                                              double pnu_prev, const double* ic_pnu,
                                              double ic_theta, const double* hpm, int nbins,
                                              int b, const double* ds, const double* l2ds,
                                              const double* w, int q_sub, int iterations,
                                              double* red) {
  const double inv_q = 1.0 / q_sub;
  // log2(k T/m_s) of each species: with log2(ds) per sub-node (host FP64) it gives the
  // fit's log2 x without a logarithm per sub-node
  double l2k[NSP];
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp)
    l2k[sp] = (SERIES || !(sp < bx.n_sp) || !(k * bx.tm_sp[sp] > 0.0)) ? 0.0
                                                                       : log2(k * bx.tm_sp[sp]);
  double known = 0.0, coef = 0.0;
  if (threadIdx.x < 64) {                    // wave-uniform
    double ic = 0.0;
#pragma unroll
    for (int sp = 0; sp < NSP; ++sp)         // constant bound: the arrays stay in registers
      if (sp < bx.n_sp)
        ic += bx.w_sp[sp] * i_kernel<SERIES>(k * bx.tm_sp[sp] * bx.ds_ic) *
              ic_pnu[sp * nbins + b];
    ic *= 1.0 - bx.ds_ic * bx.a_i * ic_theta;
    if (threadIdx.x == 0) known = ic;
  }
  constexpr int U = NT == 64 ? 5 : 8;        // one wave: keep registers for occupancy
  const int per = (bx.nq + NT - 1) / NT;
  const int rounds = (per + U - 1) / U;
  const int chunk = rounds > 0 ? (per + rounds - 1) / rounds : 0;
  for (int u0 = 0; u0 < per; u0 += chunk) {
    double d[U], l2d[U], wq[U], a0[U], a1[U];
    bool c0[U], c1[U];                       // the bracketing node is the current one
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = threadIdx.x + (u0 + u) * NT;
      const int j = q / q_sub;
      const bool in = u < chunk && q < bx.nq;
      d[u] = in ? ds[q] : 0.0;
      l2d[u] = (in && !SERIES) ? l2ds[q] : 0.0;
      wq[u] = in ? w[q] : 0.0;
      c0[u] = !(j < bx.n_cur);
      c1[u] = !(j + 1 < bx.n_cur);
      a0[u] = (in && !c0[u]) ? hpm[static_cast<size_t>(j) * nbins + b] : 0.0;
      a1[u] = (in && !c1[u]) ? hpm[static_cast<size_t>(j + 1) * nbins + b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = threadIdx.x + (u0 + u) * NT;
      if (u >= chunk || q >= bx.nq) continue;
      const int j = q / q_sub, r = q - j * q_sub;
      const double t = r * inv_q;
      // amplitude = (1 - t) A_j + t A_{j+1}, with A_n split off
      const double amp = (r != 0) ? (1.0 - t) * a0[u] + t * a1[u] : a0[u];
      const double cur = (c0[u] ? (r != 0 ? 1.0 - t : 1.0) : 0.0) +
                         ((r != 0 && c1[u]) ? t : 0.0);
      double kern = 0.0;
#pragma unroll
      for (int sp = 0; sp < NSP; ++sp)
        if (sp < bx.n_sp)
          kern += bx.w_sp[sp] * i_kernel_l2<SERIES>(k * bx.tm_sp[sp] * d[u], l2k[sp] + l2d[u]);
      const double g = wq[u] * kern * d[u];
      known += g * amp;
      coef += g * cur;
    }
  }
  const double2 sums = block_sum_d2<NT>(make_double2(known, coef), red);
  double pnu_guess = pnu_prev, pnu = 0.0;
  for (int it = 0; it < iterations; ++it) {
    const double a_cur = (1.0 - bx.f_nu) * pcdm_half + bx.f_nu * pnu_guess;
    pnu = sums.x + sums.y * a_cur;
    pnu_guess = pnu;
  }
  return pnu;
}

// One kernel form (I(x) series or fit, one or several species): a kernel that takes only
// this form needs the registers of this form alone.
template <int NT, bool SERIES, int NSP>
__device__ __forceinline__ double exact_pnu_form(const RespBox& bx, double k, double pcdm_half,
                                                 double pnu_prev, const double* ic_pnu,
                                                 double ic_theta, const double* hpm, int nbins,
                                                 int b, const double* ds, const double* l2ds,
                                                 const double* w, int q_sub, int iterations,
                                                 double* red) {
  if (bx.n_sp <= 0) return 0.0;          // no massive neutrinos: the term drops out
  return exact_pnu_n<NSP, SERIES, NT>(bx, k, pcdm_half, pnu_prev, ic_pnu, ic_theta, hpm, nbins,
                                      b, ds, l2ds, w, q_sub, iterations, red);
}

template <int NT = RT>
__device__ __forceinline__ double exact_pnu(const RespBox& bx, double k, double pcdm_half,
                                            double pnu_prev, const double* ic_pnu,
                                            double ic_theta, const double* hpm, int nbins,
                                            int b, const double* ds, const double* l2ds,
                                            const double* w, int q_sub, int iterations,
                                            double* red) {
  if (bx.n_sp <= 0) return 0.0;          // no massive neutrinos: the term drops out
#define PMNU_EXACT_PNU(NSP, SERIES)                                                        \
  exact_pnu_n<NSP, SERIES, NT>(bx, k, pcdm_half, pnu_prev, ic_pnu, ic_theta, hpm, nbins, b, ds, \
                               l2ds, w, q_sub, iterations, red)
  if (bx.series) {
    if (bx.n_sp == 1) return PMNU_EXACT_PNU(1, true);
    return PMNU_EXACT_PNU(kMaxSpecies, true);
  }
  if (bx.n_sp == 1) return PMNU_EXACT_PNU(1, false);
  return PMNU_EXACT_PNU(kMaxSpecies, false);
#undef PMNU_EXACT_PNU
}

}  // namespace pmnu
