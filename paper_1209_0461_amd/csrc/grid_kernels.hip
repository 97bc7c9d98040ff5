// Cloud-in-cell mass assignment and force interpolation (gfx950).
//
// Mesh node (i, j, l) of box b sits at (i, j, l) L/N and lives at
// grid[b N^3 + (i N + j) N + l]; particle component 0 is axis i. Per axis the particle
// coordinate u = x N / L is split in FP64 into the lower node floor(u) (mod N) and the
// fraction d = u - floor(u): the lower node gets 1 - d and the upper node d. The eight
// corner weights are the products over the axes.
//
// The deposit accumulates in 64-bit fixed point (weight * 2^40, rounded, summed with
// integer atomics). Rounding O(1) cell sums to FP32 leaves a white-noise floor of ~6e-8
// per cell, which swamps the corner-of-the-cube modes whose power is ~1e-4 of the low-k
// power and so limits the binned spectrum there to ~1e-6; integer sums are exact, so the
// density is bitwise reproducible and only delta is rounded to FP32 (in the FFT's load).
// The interpolation weights are rounded to FP32.
#include "pm_nu_internal.hpp"

namespace pmnu {
namespace {

struct Corner {
  int lo[3], hi[3];
  float w[3][2];
};


__device__ __forceinline__ void cic_axis64(float x, double inv_cell, int nmask, int& lo,
                                           int& hi, double& w0, double& w1) {
  const double u = static_cast<double>(x) * inv_cell;
  const double f = floor(u);
  const double d = u - f;
  const int i = static_cast<int>(static_cast<long long>(f) & nmask);
  lo = i;
  hi = (i + 1) & nmask;
  w0 = 1.0 - d;
  w1 = d;
}

__device__ __forceinline__ void cic_axis(float x, double inv_cell, int nmask, int& lo,
                                         int& hi, float& w0, float& w1) {
  const double u = static_cast<double>(x) * inv_cell;
  const double f = floor(u);
  const float d = static_cast<float>(u - f);
  const int i = static_cast<int>(static_cast<long long>(f) & nmask);
  lo = i;
  hi = (i + 1) & nmask;
  w0 = 1.0f - d;
  w1 = d;
}

__global__ void fill_zero_kernel(float4* __restrict__ p, int64_t n4) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n4;
       i += stride)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void fill_zero_tail_kernel(float* __restrict__ p, int64_t start, int64_t n) {
  const int64_t i = start + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

__global__ __launch_bounds__(1024) void deposit_kernel(const float* __restrict__ pos,
                                                       unsigned long long* __restrict__ rho,
                                                       int64_t np,
                                                       int nbox, int n, double inv_cell,
                                                       int* __restrict__ flags) {
  const int64_t total = np * nbox;
  const int64_t m = static_cast<int64_t>(n) * n * n;
  const int nmask = n - 1;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += stride) {
    const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
      atomicOr(flags, 1);
      continue;
    }
    int lo[3], hi[3];
    double w[3][2];
    cic_axis64(x, inv_cell, nmask, lo[0], hi[0], w[0][0], w[0][1]);
    cic_axis64(y, inv_cell, nmask, lo[1], hi[1], w[1][0], w[1][1]);
    cic_axis64(z, inv_cell, nmask, lo[2], hi[2], w[2][0], w[2][1]);
    unsigned long long* g = rho + (i / np) * m;
#pragma unroll
    for (int cx = 0; cx < 2; ++cx) {
      const int ix = cx ? hi[0] : lo[0];
#pragma unroll
      for (int cy = 0; cy < 2; ++cy) {
        const int iy = cy ? hi[1] : lo[1];
        const double wxy = w[0][cx] * w[1][cy] * kFixScale;
        const int64_t row = (static_cast<int64_t>(ix) * n + iy) * n;
        atomicAdd(g + row + lo[2], static_cast<unsigned long long>(__double2ll_rn(wxy * w[2][0])));
        atomicAdd(g + row + hi[2], static_cast<unsigned long long>(__double2ll_rn(wxy * w[2][1])));
      }
    }
  }
}

__global__ __launch_bounds__(1024) void interp_kernel(const float* __restrict__ pos,
                                                      const float* __restrict__ force,
                                                      float* __restrict__ acc, int64_t np,
                                                      int nbox, int n, double inv_cell) {
  const int64_t total = np * nbox;
  const int64_t m = static_cast<int64_t>(n) * n * n;
  const int64_t comp_stride = m * nbox;
  const int nmask = n - 1;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += stride) {
    const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    if (isfinite(x) && isfinite(y) && isfinite(z)) {
      Corner c;
      cic_axis(x, inv_cell, nmask, c.lo[0], c.hi[0], c.w[0][0], c.w[0][1]);
      cic_axis(y, inv_cell, nmask, c.lo[1], c.hi[1], c.w[1][0], c.w[1][1]);
      cic_axis(z, inv_cell, nmask, c.lo[2], c.hi[2], c.w[2][0], c.w[2][1]);
      const float* g = force + (i / np) * m;
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        const int ix = cx ? c.hi[0] : c.lo[0];
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          const int iy = cy ? c.hi[1] : c.lo[1];
          const float wxy = c.w[0][cx] * c.w[1][cy];
          const int64_t row = (static_cast<int64_t>(ix) * n + iy) * n;
#pragma unroll
          for (int cz = 0; cz < 2; ++cz) {
            const int64_t idx = row + (cz ? c.hi[2] : c.lo[2]);
            const float w = wxy * c.w[2][cz];
            a0 += w * g[idx];
            a1 += w * g[comp_stride + idx];
            a2 += w * g[2 * comp_stride + idx];
          }
        }
      }
    }
    acc[3 * i] = a0;
    acc[3 * i + 1] = a1;
    acc[3 * i + 2] = a2;
  }
}

__global__ void fixed_to_float_kernel(const unsigned long long* __restrict__ src,
                                      float* __restrict__ dst, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    dst[i] = static_cast<float>(static_cast<double>(src[i]) / kFixScale);
}

int grid_blocks(int64_t work, int block, int ppt) {
  int64_t b = (work + static_cast<int64_t>(block) * ppt - 1) / (static_cast<int64_t>(block) * ppt);
  if (b < 1) b = 1;
  if (b > (1 << 30)) b = 1 << 30;
  return static_cast<int>(b);
}

}  // namespace

hipError_t launch_fill_zero(void* ptr, int64_t bytes, hipStream_t s) {
  float* p = static_cast<float*>(ptr);
  const int64_t n = bytes / 4;
  const int64_t n4 = n / 4;
  if (n4 > 0) {
    int blocks = static_cast<int>(std::min<int64_t>((n4 + 255) / 256, 8192));
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<float4*>(p), n4);
  }
  if (n4 * 4 < n)
    hipLaunchKernelGGL(fill_zero_tail_kernel, dim3(1), dim3(4), 0, s, p, n4 * 4, n);
  return hipGetLastError();
}

hipError_t launch_fixed_to_float(const unsigned long long* src, float* dst, int64_t n,
                                 hipStream_t s) {
  int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(fixed_to_float_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_deposit(const float* pos, unsigned long long* rho, int64_t np, int nbox, int n,
                          double inv_cell, int* flags, int block, int ppt, hipStream_t s) {
  hipLaunchKernelGGL(deposit_kernel, dim3(grid_blocks(np * nbox, block, ppt)), dim3(block), 0,
                     s, pos, rho, np, nbox, n, inv_cell, flags);
  return hipGetLastError();
}

hipError_t launch_interp(const float* pos, const float* force, float* acc, int64_t np,
                         int nbox, int n, double inv_cell, int block, int ppt,
                         hipStream_t s) {
  hipLaunchKernelGGL(interp_kernel, dim3(grid_blocks(np * nbox, block, ppt)), dim3(block), 0,
                     s, pos, force, acc, np, nbox, n, inv_cell);
  return hipGetLastError();
}

}  // namespace pmnu
