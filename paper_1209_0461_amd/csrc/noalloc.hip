// Stage (ii) of the step for one box without any device allocation: the CIC deposit, the
// forward real FFT and the binned P_cdm(k_b) of pm_nu_deposit + pm_nu_get_spectrum, with
// every intermediate in one file-scope device array (`scratch`) instead of a context's
// buffers. For callers that cannot allocate: code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc.
//
// The same kernels as the context's step do the work (LDS-privatised fixed-point deposit,
// the three forward transform passes with the FP64 bin sums of the last one, the bin power
// reduction). What a context computes once on the host at init (bin table, mode counts,
// twiddles) is rebuilt here on every call by one setup workgroup, from edges and twiddles
// passed by value, so the call needs no host-to-device copy either.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "pm_nu_internal.hpp"

namespace pmnu {
namespace {

constexpr int kStaticMaxMesh = 64;     // largest N
constexpr int kStaticMaxBins = 256;    // largest B
constexpr int64_t kStaticBytes = 5 << 20;   // 5 MiB; the N = 64, B = 256 layout needs 4.3 MiB
constexpr int kMaxDevices = 64;

// The scratch of every call on this device (each device holds its own copy). In host code
// this name is not a device address: the address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};   // per device: the address of `scratch` on that device

struct StaticTables {
  int edges[kStaticMaxBins + 1];      // integer |n|^2 edges of the bins
  float2 tw[kStaticMaxMesh];          // exp(-2 pi i m / N)
};

// Bin of every integer |n|^2 (as the context's host table), the twiddles, and the full-sphere
// mode count of every bin (exact integer counts over the triples of [-N/2, N/2)^3).
__global__ __launch_bounds__(1024) void static_setup_kernel(StaticTables t, int n, int nbins,
                                                            int n2max, uint16_t* __restrict__ bin_of_n2,
                                                            float2* __restrict__ tw,
                                                            double* __restrict__ counts) {
  __shared__ uint16_t s_bin[3 * kStaticMaxMesh * kStaticMaxMesh / 4 + 1];
  __shared__ int s_cnt[kStaticMaxBins];
  const int tid = threadIdx.x;
  for (int b = tid; b < nbins; b += blockDim.x) s_cnt[b] = 0;
  for (int m = tid; m < n; m += blockDim.x) tw[m] = t.tw[m];
  for (int n2 = tid; n2 <= n2max; n2 += blockDim.x) {
    int lo = 0, hi = nbins - 1;        // the last b with edges[b] <= n2, at most nbins - 1
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (t.edges[mid] <= n2) lo = mid; else hi = mid - 1;
    }
    const uint16_t b = static_cast<uint16_t>(n2 == 0 ? 0 : lo);
    s_bin[n2] = b;
    bin_of_n2[n2] = b;
  }
  __syncthreads();
  const int h = n / 2, m3 = n * n * n;
  for (int t3 = tid; t3 < m3; t3 += blockDim.x) {
    const int i = t3 / (n * n) - h, j = (t3 / n) % n - h, l = t3 % n - h;
    const int n2 = i * i + j * j + l * l;
    if (n2 > 0) atomicAdd(&s_cnt[s_bin[n2]], 1);
  }
  __syncthreads();
  for (int b = tid; b < nbins; b += blockDim.x) counts[b] = static_cast<double>(s_cnt[b]);
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// The address of `scratch` on the current device, looked up once per device.
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(PM_NU_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(PM_NU_ENODEV, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(PM_NU_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return PM_NU_OK;
}

}  // namespace
}  // namespace pmnu

using namespace pmnu;

extern "C" int pm_nu_binned_power_noalloc(const float* pos, int64_t n_particles, int n_mesh,
                                          double box_size, int n_kbins, double* p_cdm,
                                          void* stream) {
  const int n = n_mesh;
  if (n < 8 || n > kStaticMaxMesh || (n & (n - 1)))
    return set_error(PM_NU_EINVAL, "n_mesh %d: the no-allocation call takes powers of two "
                                   "from 8 to %d", n, kStaticMaxMesh);
  if (n_kbins < 1 || n_kbins > kStaticMaxBins)
    return set_error(PM_NU_EINVAL, "n_kbins %d: the no-allocation call takes 1 to %d bins",
                     n_kbins, kStaticMaxBins);
  if (n_particles < 1 || !pos || !p_cdm)
    return set_error(PM_NU_EINVAL, "need n_particles >= 1, pos and p_cdm");
  if (!(box_size > 0.0) || !std::isfinite(box_size))
    return set_error(PM_NU_EINVAL, "box_size must be finite and > 0");

  // layout of the scratch for this call
  const int64_t M = static_cast<int64_t>(n) * n * n;
  const int64_t MH = static_cast<int64_t>(n) * n * (n / 2 + 1);
  const int n2max = 3 * n * n / 4;
  const int n_partial = fwd_x_partials(n);
  size_t off = 0;
  const size_t o_rho = off;     off = align256(off + M * sizeof(unsigned long long));
  const size_t o_ca = off;      off = align256(off + MH * sizeof(float2));
  const size_t o_cb = off;      off = align256(off + MH * sizeof(float2));
  const size_t o_part = off;    off = align256(off + static_cast<size_t>(n_partial) * n_kbins * sizeof(double));
  const size_t o_counts = off;  off = align256(off + n_kbins * sizeof(double));
  const size_t o_bins = off;    off = align256(off + (n2max + 1) * sizeof(uint16_t));
  const size_t o_tw = off;      off = align256(off + n * sizeof(float2));
  const size_t o_flags = off;   off = align256(off + sizeof(int));
  if (n_partial <= 0 || off > static_cast<size_t>(kStaticBytes))
    return set_error(PM_NU_EINVAL, "n_mesh %d with %d bins needs %zu bytes of scratch (%lld held)",
                     n, n_kbins, off, static_cast<long long>(kStaticBytes));

  void* base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  unsigned char* s = static_cast<unsigned char*>(base);
  auto* rho = reinterpret_cast<unsigned long long*>(s + o_rho);
  auto* ca = reinterpret_cast<float2*>(s + o_ca);
  auto* cb = reinterpret_cast<float2*>(s + o_cb);
  auto* part = reinterpret_cast<double*>(s + o_part);
  auto* counts = reinterpret_cast<double*>(s + o_counts);
  auto* bins = reinterpret_cast<uint16_t*>(s + o_bins);
  auto* tw = reinterpret_cast<float2*>(s + o_tw);
  auto* flags = reinterpret_cast<int*>(s + o_flags);

  // bin edges and twiddles exactly as a context computes them
  StaticTables t{};
  const double r2 = 3.0 * n * n / 4.0;
  for (int b = 0; b <= n_kbins; ++b)
    t.edges[b] = static_cast<int>(std::ceil(std::pow(r2, static_cast<double>(b) / n_kbins)));
  t.edges[0] = 1;
  for (int m = 0; m < n; ++m) {
    const double ph = -2.0 * kPi * m / n;
    t.tw[m] = make_float2(static_cast<float>(std::cos(ph)), static_cast<float>(std::sin(ph)));
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(static_setup_kernel, dim3(1), dim3(1024), 0, st, t, n, n_kbins, n2max, bins,
                     tw, counts);
  hipError_t e = hipGetLastError();
  const double scale = static_cast<double>(M) / static_cast<double>(n_particles) / kFixScale;
  const double norm = std::pow(box_size, 3) / (static_cast<double>(M) * M);
  e = e ? e : launch_fill_zero(rho, M * static_cast<int64_t>(sizeof(unsigned long long)), st);
  e = e ? e : launch_fill_zero(flags, sizeof(int), st);
  e = e ? e : launch_deposit(pos, rho, n_particles, 1, n, n / box_size, flags, 4, 256, st);
  e = e ? e : launch_fwd_z(n, rho, nullptr, nullptr, nullptr, 0, ca, tw, scale, 1, st);
  e = e ? e : launch_fwd_y(n, ca, cb, tw, 1, st);
  e = e ? e : launch_fwd_x_bin(n, cb, tw, bins, part, n_kbins, 1, st);
  e = e ? e : launch_bin_power(part, n_partial, counts, n_kbins, norm, 1, p_cdm, st);
  if (e != hipSuccess)
    return set_error(PM_NU_EHIP, "no-allocation spectrum launch failed: %s", hipGetErrorString(e));
  return PM_NU_OK;
}
