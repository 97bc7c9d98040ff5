// Neutrino response of the step, FP64 (gfx950).
//
// response_kernel: one workgroup per (bin b, box). It
//   1. sums the per-workgroup partial mode sums of the forward FFT for bin b and forms
//      P_cdm(k_b) = (L^3/N^6) sum w |delta_k|^2 / C_b;
//   2. evaluates eq. (P-final) for P_nu^{1/2}(k_b, a_now):
//        I(x_i) P_nu,i^{1/2} {1 - (s - s_i) a_i [theta/delta]_i}
//        + sum_q W_q I(k_b ds_q T/m) ds_q A_q
//      where ds_q = s(a_now) - s(a_q), W_q = (3/2) Omega_M H0^2 * (trapezoid weight in
//      ln a) / (a_q H(a_q)) and A_q is the stored P_M^{1/2}, linear in ln a between the
//      two bracketing nodes (Q sub-nodes per interval). The current node uses
//      (1 - f_nu) P_cdm^{1/2} + f_nu P_nu^{1/2}(previous node) on the first iteration
//      and the previous iteration's P_nu^{1/2} after that;
//   3. writes P_nu^{1/2}, R = P_nu^{1/2}/P_cdm^{1/2} (0 where P_cdm = 0), and the new
//      history row.
// Lanes stride over the sub-nodes; sums are reduced across the wave and the workgroup
// in FP64 in a fixed order. The sum is gathered as a part from the stored nodes plus a
// coefficient of the current node, so iterations do not evaluate the kernel again.
//
// I(x) is the rational fit of the paper's Appendix C, eq. (fit), or (per box) the exact
// alternating series of the same appendix, accelerated.
//
// ratio_index_kernel (once per geometry): for every integer n^2 in [0, 3N^2/4] the lower of
// the two non-empty bins whose means bracket ln(k_f |n|) and the weight of the upper one,
// packed in 32 bits, so that R(|k|) is linear in ln k between the means of the non-empty
// bins and held at the end values outside them; the first inverse pass turns it and the
// step's R into T(n^2) = (1 - f_nu) + f_nu R(|k|) (eq. (phases)).
#include "response_device.hpp"

namespace pmnu {
namespace {

// FORM: 0 fit with one species per box, 1 fit with a mass hierarchy, 2 and 3 the same with
// the exact series (the host takes the form the boxes need)
template <int NT, int FORM>
__global__ __launch_bounds__(NT) void response_kernel(
    const RespBox* __restrict__ boxes, const double* __restrict__ partial, int n_partial,
    const double* __restrict__ counts, const double* __restrict__ kmean,
    double* __restrict__ hist_pm, double* __restrict__ hist_pnu,
    const double* __restrict__ ic_pnu, const double* __restrict__ ic_theta,
    const double* __restrict__ tg_ds, const double* __restrict__ tg_l2,
    const double* __restrict__ tg_w, int nbins, int jcap,
    int qcap, int q_sub, int iterations, double norm, double* __restrict__ pcdm_out,
    double* __restrict__ pnu_out, double* __restrict__ ratio_out) {
  __shared__ double red[2 * NT / 64];
  const int b = blockIdx.x, box = blockIdx.y;
  const RespBox bx = boxes[box];
  const size_t ob = static_cast<size_t>(box) * nbins + b;
  double* hpm = hist_pm + static_cast<size_t>(box) * jcap * nbins;
  double* hpn = hist_pnu + static_cast<size_t>(box) * jcap * nbins;

  // 1. binned CDM power
  const double s = bin_mode_sum<NT>(partial, n_partial, nbins, box, b, red);
  const double cb = counts[b];
  if (!(cb > 0.0)) {
    if (threadIdx.x == 0) {
      pcdm_out[ob] = 0.0;
      pnu_out[ob] = 0.0;
      ratio_out[ob] = 0.0;
      hpm[static_cast<size_t>(bx.n_cur) * nbins + b] = 0.0;
      hpn[static_cast<size_t>(bx.n_cur) * nbins + b] = 0.0;
    }
    return;
  }
  const double pcdm = norm * s / cb;
  const double pcdm_half = sqrt(pcdm);

  // 2. history integral
  constexpr bool SERIES = FORM >= 2;
  constexpr int NSP = (FORM & 1) ? kMaxSpecies : 1;
  const double pnu = exact_pnu_form<NT, SERIES, NSP>(bx, kmean[b], pcdm_half,
                               (bx.n_cur > 0 ? hpn[static_cast<size_t>(bx.n_cur - 1) * nbins + b] : 0.0),
                               ic_pnu + static_cast<size_t>(box) * kMaxSpecies * nbins,
                               ic_theta[ob], hpm, nbins, b, tg_ds + static_cast<size_t>(box) * qcap,
                               tg_l2 + static_cast<size_t>(box) * qcap,
                               tg_w + static_cast<size_t>(box) * qcap, q_sub, iterations, red);
  if (threadIdx.x == 0) {
    pcdm_out[ob] = pcdm;
    pnu_out[ob] = pnu;
    // a bin without CDM power has no phase to carry the neutrinos (eq. (phases)): R = 0
    ratio_out[ob] = pcdm_half > 0.0 ? pnu / pcdm_half : 0.0;
    hpm[static_cast<size_t>(bx.n_cur) * nbins + b] = (1.0 - bx.f_nu) * pcdm_half + bx.f_nu * pnu;
    hpn[static_cast<size_t>(bx.n_cur) * nbins + b] = pnu;
  }
}

// The exact response for many (bin, box) pairs with the fit and one species per box (the
// batched boxes): one workgroup of RT threads per (group of G bins, box). The box's time
// grid (s differences, their log2, weights) and the group's stored history rows are staged
// in LDS with one round of loads, since every bin of the box reads the same grid; then
// WPB = 4 / G waves share each bin's sub-nodes (wave h of a bin takes the lanes' sub-nodes
// q = 64 (WPB i + h) + lane), sum them over the wave, and the bin's first wave adds the
// others' sums from LDS. Dynamic LDS: 3 nq + n_cur G doubles.
template <int G>
__global__ __launch_bounds__(RT) void response_group_kernel(
    const RespBox* __restrict__ boxes, const double* __restrict__ partial, int n_partial,
    const double* __restrict__ counts, const double* __restrict__ kmean,
    double* __restrict__ hist_pm, double* __restrict__ hist_pnu,
    const double* __restrict__ ic_pnu, const double* __restrict__ ic_theta,
    const double* __restrict__ tg_ds, const double* __restrict__ tg_l2,
    const double* __restrict__ tg_w, int nbins, int jcap, int qcap, int q_sub, int iterations,
    double norm, double* __restrict__ pcdm_out, double* __restrict__ pnu_out,
    double* __restrict__ ratio_out) {
  constexpr int WPB = (RT / 64) / G;                 // waves per bin
  static_assert(G * WPB == RT / 64, "the waves cover the bins evenly");
  extern __shared__ double sm[];
  __shared__ double s_red[RT / 64][2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gv = wave / WPB, h = wave % WPB;         // this wave's bin in the group, its share
  const int box = blockIdx.y, b0 = blockIdx.x * G, b = b0 + gv;
  const bool bin_on = b < nbins;
  const RespBox bx = boxes[box];
  const int nq = bx.nq, ncur = bx.n_cur;
  double* hpm = hist_pm + static_cast<size_t>(box) * jcap * nbins;
  double* hpn = hist_pnu + static_cast<size_t>(box) * jcap * nbins;
  const double* ds = tg_ds + static_cast<size_t>(box) * qcap;
  const double* l2 = tg_l2 + static_cast<size_t>(box) * qcap;
  const double* wt = tg_w + static_cast<size_t>(box) * qcap;
  double* s_ds = sm;
  double* s_l2 = sm + nq;
  double* s_w = sm + 2 * nq;
  double* s_h = sm + 3 * nq;                         // [j][g], j < n_cur
  // the bin's partial sums (its first wave; loads before the staging's stores)
  double psum = 0.0;
  if (bin_on && h == 0) {
    constexpr int UP = 4;                            // loads in flight per lane
    const double* pp = partial + (static_cast<size_t>(box) * nbins + b) * n_partial;
    for (int i0 = lane; i0 < n_partial; i0 += UP * 64) {
      double x[UP];
#pragma unroll
      for (int u = 0; u < UP; ++u) x[u] = i0 + u * 64 < n_partial ? pp[i0 + u * 64] : 0.0;
#pragma unroll
      for (int u = 0; u < UP; ++u) psum += x[u];
    }
  }
  {
    constexpr int UB = 12;                           // one round at 100 nodes, Q = 8
    const int nst = 3 * nq + ncur * G;
    for (int i0 = tid; i0 < nst; i0 += UB * RT) {
      double val[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int i = i0 + u * RT;
        double x = 0.0;
        if (i < nq) x = ds[i];
        else if (i < 2 * nq) x = l2[i - nq];
        else if (i < 3 * nq) x = wt[i - 2 * nq];
        else if (i < nst) {
          const int k = i - 3 * nq, j = k / G, g = k - j * G;
          if (b0 + g < nbins) x = hpm[static_cast<size_t>(j) * nbins + b0 + g];
        }
        val[u] = x;
      }
#pragma unroll
      for (int u = 0; u < UB; ++u)
        if (i0 + u * RT < nst) sm[i0 + u * RT] = val[u];
    }
  }
  __syncthreads();
  const bool massive = bx.n_sp > 0;
  const double tm = bx.tm_sp[0], wsp = bx.w_sp[0], inv_q = 1.0 / q_sub;
  const double kb = kmean[bin_on ? b : nbins - 1];
  const double l2k = massive && kb * tm > 0.0 ? log2(kb * tm) : 0.0;
  double known = 0.0, coef = 0.0;
  if (massive && bin_on) {
    for (int q = 64 * h + lane; q < nq; q += 64 * WPB) {
      const double d = s_ds[q], l2d = s_l2[q], wq = s_w[q];
      const int j = q / q_sub, r = q - j * q_sub;
      const double t = r * inv_q;
      const bool c0 = !(j < ncur), c1 = !(j + 1 < ncur);
      const double cur = (c0 ? (r != 0 ? 1.0 - t : 1.0) : 0.0) + ((r != 0 && c1) ? t : 0.0);
      const double a0 = c0 ? 0.0 : s_h[j * G + gv];
      const double a1 = c1 ? 0.0 : s_h[(j + 1) * G + gv];
      const double amp = (r != 0) ? (1.0 - t) * a0 + t * a1 : a0;
      const double gq = wq * (wsp * i_fit_l2(kb * tm * d, l2k + l2d)) * d;
      known += gq * amp;
      coef += gq * cur;
    }
  }
  known = wave_sum_d(known);
  coef = wave_sum_d(coef);
  psum = wave_sum_d(psum);
  if (WPB > 1) {
    if (lane == 0) {
      s_red[wave][0] = known;
      s_red[wave][1] = coef;
    }
    __syncthreads();
    if (h == 0) {
#pragma unroll
      for (int o = 1; o < WPB; ++o) {                // fixed order over the bin's waves
        known += s_red[wave + o][0];
        coef += s_red[wave + o][1];
      }
    }
  }
  if (h != 0 || lane != 0 || !bin_on) return;
  const size_t ob = static_cast<size_t>(box) * nbins + b;
  const size_t row = static_cast<size_t>(ncur) * nbins + b;
  const double cb = counts[b];
  if (!(cb > 0.0)) {
    pcdm_out[ob] = pnu_out[ob] = ratio_out[ob] = 0.0;
    hpm[row] = hpn[row] = 0.0;
    return;
  }
  const double pcdm = norm * psum / cb;
  const double ph = sqrt(pcdm);
  double pnu = 0.0;
  if (massive) {
    double ic = wsp * i_fit(kb * tm * bx.ds_ic) *
                ic_pnu[static_cast<size_t>(box) * kMaxSpecies * nbins + b];   // species 0
    ic *= 1.0 - bx.ds_ic * bx.a_i * ic_theta[ob];
    double guess = ncur > 0 ? hpn[row - nbins] : 0.0;
    for (int it = 0; it < iterations; ++it) {
      const double a_cur = (1.0 - bx.f_nu) * ph + bx.f_nu * guess;
      pnu = ic + known + coef * a_cur;
      guess = pnu;
    }
  }
  pcdm_out[ob] = pcdm;
  pnu_out[ob] = pnu;
  ratio_out[ob] = ph > 0.0 ? pnu / ph : 0.0;       // no CDM power in the bin: R = 0
  hpm[row] = (1.0 - bx.f_nu) * ph + bx.f_nu * pnu;
  hpn[row] = pnu;
}

// P_cdm(k_b) from the deposit's partial sums alone (for reading the spectrum before a
// response): one workgroup per (bin, box).
__global__ __launch_bounds__(RT) void bin_power_kernel(const double* __restrict__ partial,
                                                      int n_partial,
                                                      const double* __restrict__ counts,
                                                      int nbins, double norm,
                                                      double* __restrict__ pcdm_out) {
  __shared__ double red[RT / 64];
  const int b = blockIdx.x, box = blockIdx.y;
  const double s = bin_mode_sum(partial, n_partial, nbins, box, b, red);
  if (threadIdx.x == 0)
    pcdm_out[static_cast<size_t>(box) * nbins + b] = counts[b] > 0.0 ? norm * s / counts[b] : 0.0;
}

__global__ __launch_bounds__(256) void ratio_index_kernel(const double* __restrict__ lnk,
                                                          const int* __restrict__ nonempty,
                                                          int n_nonempty, int n2max, double kf,
                                                          uint32_t* __restrict__ out) {
  // ln k of the non-empty bins, staged once per workgroup (the search runs in LDS)
  __shared__ double s_lk[kMaxBins];
  __shared__ int s_bin[kMaxBins];
  for (int i = threadIdx.x; i < n_nonempty; i += blockDim.x) {
    s_bin[i] = nonempty[i];
    s_lk[i] = lnk[nonempty[i]];
  }
  __syncthreads();
  const int n2 = blockIdx.x * blockDim.x + threadIdx.x;
  if (n2 > n2max) return;
  int a = 0, z = 0;
  double t = 0.0;
  if (n2 > 0) {
    const double lk = log(kf * sqrt(static_cast<double>(n2)));
    if (lk >= s_lk[n_nonempty - 1]) {
      a = z = n_nonempty - 1;
    } else if (lk > s_lk[0]) {
      z = n_nonempty - 1;                 // s_lk[a] <= lk < s_lk[z]
      while (z - a > 1) {
        const int mid = (a + z) >> 1;
        if (s_lk[mid] <= lk) a = mid; else z = mid;
      }
      t = (lk - s_lk[a]) / (s_lk[z] - s_lk[a]);
    }
  }
  // t in units of 2^-22 (error <= 2^-23, far below the FP32 rounding of T); a weight that
  // rounds to 1 is the upper bin itself
  uint32_t q = static_cast<uint32_t>(rint(t * 4194304.0));
  if (q >= (1u << 22)) {
    a = z;
    q = 0;
  }
  out[n2] = static_cast<uint32_t>(s_bin[a]) | (q << kRatioBinBits);
}

// I(x) at n points, the fit or the exact series (a diagnostic of the device kernels).
__global__ __launch_bounds__(256) void kernel_values_kernel(const double* __restrict__ x,
                                                            int64_t n, int series,
                                                            double* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = series ? i_series(x[i]) : i_fit(x[i]);
}

}  // namespace

hipError_t launch_kernel_values(const double* x, int64_t n, int series, double* out,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(kernel_values_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0,
                     s, x, n, series, out);
  return hipGetLastError();
}

hipError_t launch_response(const RespBox* boxes, const double* partial, int n_partial,
                           const double* counts, const double* kmean, const double* hist_pm,
                           const double* hist_pnu, const double* ic_pnu,
                           const double* ic_theta, const double* tg_ds, const double* tg_l2,
                           const double* tg_w,
                           int nbins, int jcap, int qcap, int q_sub, int iterations,
                           double norm, int nbox, double* pcdm, double* pnu, double* ratio,
                           hipStream_t s, int threads, bool series, bool hierarchy) {
#define PMNU_LAUNCH_RESPONSE(NT, FORM)                                                       \
  hipLaunchKernelGGL((response_kernel<NT, FORM>), dim3(nbins, nbox), dim3(NT), 0, s, boxes,  \
                     partial,                                                                \
                     n_partial, counts, kmean, const_cast<double*>(hist_pm),                 \
                     const_cast<double*>(hist_pnu), ic_pnu, ic_theta, tg_ds, tg_l2, tg_w,    \
                     nbins,                                                                  \
                     jcap, qcap, q_sub, iterations, norm, pcdm, pnu, ratio)
  const int form = (series ? 2 : 0) + (hierarchy ? 1 : 0);
  constexpr int G = 4;                             // bins per workgroup of the grouped form
  const size_t group_lds = (3 * static_cast<size_t>(qcap) + static_cast<size_t>(jcap) * G) *
                           sizeof(double);
  if (threads == 64 && form == 0 && group_lds <= 64 * 1024) {
    hipLaunchKernelGGL((response_group_kernel<G>), dim3((nbins + G - 1) / G, nbox), dim3(RT),
                       group_lds, s, boxes, partial, n_partial, counts, kmean,
                       const_cast<double*>(hist_pm), const_cast<double*>(hist_pnu), ic_pnu,
                       ic_theta, tg_ds, tg_l2, tg_w, nbins, jcap, qcap, q_sub, iterations, norm,
                       pcdm, pnu, ratio);
  } else if (threads == 64) {
    switch (form) {
      case 0: PMNU_LAUNCH_RESPONSE(64, 0); break;
      case 1: PMNU_LAUNCH_RESPONSE(64, 1); break;
      case 2: PMNU_LAUNCH_RESPONSE(64, 2); break;
      default: PMNU_LAUNCH_RESPONSE(64, 3); break;
    }
  } else {
    switch (form) {
      case 0: PMNU_LAUNCH_RESPONSE(RT, 0); break;
      case 1: PMNU_LAUNCH_RESPONSE(RT, 1); break;
      case 2: PMNU_LAUNCH_RESPONSE(RT, 2); break;
      default: PMNU_LAUNCH_RESPONSE(RT, 3); break;
    }
  }
#undef PMNU_LAUNCH_RESPONSE
  return hipGetLastError();
}

int response_threads(int nbins, int nbox) {
  // one wave per (bin, box) once the pairs alone fill the chip's SIMDs several times over
  // (the batched boxes); a full workgroup per pair otherwise, to spread its sub-nodes
  return static_cast<int64_t>(nbins) * nbox >= 1024 ? 64 : RT;
}

hipError_t launch_bin_power(const double* partial, int n_partial, const double* counts,
                            int nbins, double norm, int nbox, double* pcdm, hipStream_t s) {
  hipLaunchKernelGGL(bin_power_kernel, dim3(nbins, nbox), dim3(RT), 0, s, partial, n_partial,
                     counts, nbins, norm, pcdm);
  return hipGetLastError();
}

hipError_t launch_ratio_index(const double* lnk, const int* nonempty, int n_nonempty,
                              int n2max, double kf, uint32_t* out, hipStream_t s) {
  if (n_nonempty < 1 || n_nonempty > kMaxBins) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ratio_index_kernel, dim3((n2max + 1 + 255) / 256), dim3(256), 0, s, lnk,
                     nonempty, n_nonempty, n2max, kf, out);
  return hipGetLastError();
}

}  // namespace pmnu
