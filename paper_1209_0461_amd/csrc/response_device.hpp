// Device pieces of the neutrino response shared by the exact and the surrogate kernels
// (FP64, one workgroup of RT threads per (k-bin, box)).
#pragma once
#include "pm_nu_internal.hpp"

namespace pmnu {

constexpr int RT = 256;

// Rational fit of the free-streaming kernel I(x), the paper's Appendix C eq. (fit).
__device__ __forceinline__ double i_fit(double x) {
  const double x2 = x * x, x4 = x2 * x2;
  const double num = 1.0 + 0.0168 * x2 + 0.0407 * x4;
  const double den = 1.0 + 2.1734 * x2 + 1.6787 * pow(x, 4.1811) + 0.1467 * x4 * x4;
  return num / den;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup (RT threads); every thread gets the result.
__device__ __forceinline__ double block_sum_d(double v, double* red) {
  v = wave_sum_d(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < RT / 64; ++w) s += red[w];
  return s;
}

// sum over the per-workgroup partial mode sums of bin b ([box][bin][workgroup]):
// sum w |delta_k|^2
__device__ __forceinline__ double bin_mode_sum(const double* partial, int n_partial, int nbins,
                                               int box, int b, double* red) {
  constexpr int U = 8;                       // loads in flight per thread
  double s = 0.0;
  const double* pp = partial + (static_cast<size_t>(box) * nbins + b) * n_partial;
  for (int i0 = 0; i0 < n_partial; i0 += U * RT) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + threadIdx.x + u * RT;
      v[u] = i < n_partial ? pp[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  return block_sum_d(s, red);
}

// eq. (P-final) for one bin: the initial-condition term plus the trapezoid sum over the
// sub-nodes, iterated `iterations` times on the current node (every thread gets it). With
// several species (mass hierarchy) each free-streams with its own kernel and the result is
// their mean weighted by m_s / M_nu; the source term is the common P_M^{1/2} history, so
// the quadrature uses the weighted sum of the kernels. ic_pnu: [kMaxSpecies][nbins] initial
// amplitudes of this box.
template <int NSP>   // species evaluated: 1 (equal masses) or kMaxSpecies (a hierarchy)
__device__ __forceinline__ double exact_pnu_n(const RespBox& bx, double k, double pcdm_half,
                                              double pnu_prev, const double* ic_pnu,
                                              double ic_theta, const double* hpm, int nbins,
                                              int b, const double* ds, const double* w,
                                              int q_sub, int iterations, double* red) {
  const double inv_q = 1.0 / q_sub;
  double ic = 0.0;
#pragma unroll
  for (int sp = 0; sp < NSP; ++sp)           // constant bound: the arrays stay in registers
    if (sp < bx.n_sp)
      ic += bx.w_sp[sp] * i_fit(k * bx.tm_sp[sp] * bx.ds_ic) * ic_pnu[sp * nbins + b];
  ic *= 1.0 - bx.ds_ic * bx.a_i * ic_theta;
  double pnu_guess = pnu_prev, pnu = 0.0;
  for (int it = 0; it < iterations; ++it) {
    const double a_cur = (1.0 - bx.f_nu) * pcdm_half + bx.f_nu * pnu_guess;
    double acc = 0.0;
    constexpr int U = 4;                     // sub-nodes per thread whose loads go out together
    for (int q0 = 0; q0 < bx.nq; q0 += U * RT) {
      double d[U], wq[U], a0[U], a1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + threadIdx.x + u * RT;
        const int j = q / q_sub;
        const bool in = q < bx.nq;
        d[u] = in ? ds[q] : 0.0;
        wq[u] = in ? w[q] : 0.0;
        a0[u] = (in && j < bx.n_cur) ? hpm[static_cast<size_t>(j) * nbins + b] : a_cur;
        a1[u] = (in && j + 1 < bx.n_cur) ? hpm[static_cast<size_t>(j + 1) * nbins + b] : a_cur;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + threadIdx.x + u * RT;
        if (q >= bx.nq) continue;
        const int j = q / q_sub, r = q - j * q_sub;
        double amp = a0[u];
        if (r != 0) {
          const double t = r * inv_q;
          amp = (1.0 - t) * a0[u] + t * a1[u];
        }
        double kern = 0.0;
#pragma unroll
        for (int sp = 0; sp < NSP; ++sp)
          if (sp < bx.n_sp) kern += bx.w_sp[sp] * i_fit(k * bx.tm_sp[sp] * d[u]);
        acc += wq[u] * kern * d[u] * amp;
      }
    }
    pnu = ic + block_sum_d(acc, red);
    pnu_guess = pnu;
  }
  return pnu;
}

__device__ __forceinline__ double exact_pnu(const RespBox& bx, double k, double pcdm_half,
                                            double pnu_prev, const double* ic_pnu,
                                            double ic_theta, const double* hpm, int nbins,
                                            int b, const double* ds, const double* w,
                                            int q_sub, int iterations, double* red) {
  if (bx.n_sp <= 0) return 0.0;          // no massive neutrinos: the term drops out
  if (bx.n_sp == 1)
    return exact_pnu_n<1>(bx, k, pcdm_half, pnu_prev, ic_pnu, ic_theta, hpm, nbins, b, ds, w,
                          q_sub, iterations, red);
  return exact_pnu_n<kMaxSpecies>(bx, k, pcdm_half, pnu_prev, ic_pnu, ic_theta, hpm, nbins, b,
                                  ds, w, q_sub, iterations, red);
}

}  // namespace pmnu
