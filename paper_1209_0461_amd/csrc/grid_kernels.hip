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
//
// deposit_tiled_kernel privatises the accumulation in LDS: a workgroup takes CH
// consecutive particles, finds the bounding box of their cells (periodic, relative to the
// first particle's cell), and if the box plus its upper neighbours fits in CAP cells it
// sums the chunk's weights there with 64-bit LDS atomics and then adds every non-zero
// cell to HBM with one coalesced global atomic. Chunks that are not spatially compact
// (particles in arbitrary order) take the per-particle global-atomic path instead, so
// the result does not depend on the order; the speed does. Particles kept along a
// space-filling curve (as tree codes keep them) give compact chunks.
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

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ int cell_of(float x, double inv_cell, int nmask) {
  return static_cast<int>(static_cast<long long>(floor(static_cast<double>(x) * inv_cell)) & nmask);
}

// 8 global atomics for one particle
__device__ __forceinline__ void deposit_global(unsigned long long* g, float x, float y, float z,
                                               int n, double inv_cell, int nmask) {
  int lo[3], hi[3];
  double w[3][2];
  cic_axis64(x, inv_cell, nmask, lo[0], hi[0], w[0][0], w[0][1]);
  cic_axis64(y, inv_cell, nmask, lo[1], hi[1], w[1][0], w[1][1]);
  cic_axis64(z, inv_cell, nmask, lo[2], hi[2], w[2][0], w[2][1]);
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

template <int CH, int CAP>
__global__ __launch_bounds__(256) void deposit_tiled_kernel(const float* __restrict__ pos,
                                                            unsigned long long* __restrict__ rho,
                                                            int64_t np, int n, double inv_cell,
                                                            int* __restrict__ flags,
                                                            int64_t chunks_per_box) {
  constexpr int NT = 256, NW = NT / 64;
  __shared__ unsigned long long tile[CAP];
  __shared__ int red[6][NW];
  __shared__ int ref_s[3];
  const int tid = threadIdx.x;
  const int64_t box = blockIdx.x / chunks_per_box;
  const int64_t c0 = (blockIdx.x - box * chunks_per_box) * CH;
  const int cnt = static_cast<int>(min(static_cast<int64_t>(CH), np - c0));
  const float* p = pos + (box * np + c0) * 3;
  const int nmask = n - 1, half = n / 2;
  unsigned long long* g = rho + box * static_cast<int64_t>(n) * n * n;
  if (tid == 0) {
    const float x = p[0], y = p[1], z = p[2];
    const bool ok = isfinite(x) && isfinite(y) && isfinite(z);
    ref_s[0] = ok ? cell_of(x, inv_cell, nmask) : 0;
    ref_s[1] = ok ? cell_of(y, inv_cell, nmask) : 0;
    ref_s[2] = ok ? cell_of(z, inv_cell, nmask) : 0;
  }
  __syncthreads();
  const int r0 = ref_s[0], r1 = ref_s[1], r2 = ref_s[2];
  int mn0 = 1 << 30, mn1 = 1 << 30, mn2 = 1 << 30, mx0 = -(1 << 30), mx1 = -(1 << 30),
      mx2 = -(1 << 30);
  bool bad = false;
  for (int j = tid; j < cnt; j += NT) {
    const float x = p[3 * j], y = p[3 * j + 1], z = p[3 * j + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
      bad = true;
      continue;
    }
    const int a = ((cell_of(x, inv_cell, nmask) - r0 + half) & nmask) - half;
    const int b = ((cell_of(y, inv_cell, nmask) - r1 + half) & nmask) - half;
    const int c = ((cell_of(z, inv_cell, nmask) - r2 + half) & nmask) - half;
    mn0 = min(mn0, a); mx0 = max(mx0, a);
    mn1 = min(mn1, b); mx1 = max(mx1, b);
    mn2 = min(mn2, c); mx2 = max(mx2, c);
  }
  if (bad) atomicOr(flags, 1);
  mn0 = wave_min(mn0); mn1 = wave_min(mn1); mn2 = wave_min(mn2);
  mx0 = wave_max(mx0); mx1 = wave_max(mx1); mx2 = wave_max(mx2);
  const int lane = tid & 63, wv = tid >> 6;
  if (lane == 0) {
    red[0][wv] = mn0; red[1][wv] = mn1; red[2][wv] = mn2;
    red[3][wv] = mx0; red[4][wv] = mx1; red[5][wv] = mx2;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    mn0 = min(mn0, red[0][w]); mn1 = min(mn1, red[1][w]); mn2 = min(mn2, red[2][w]);
    mx0 = max(mx0, red[3][w]); mx1 = max(mx1, red[4][w]); mx2 = max(mx2, red[5][w]);
  }
  if (mn0 > mx0) return;   // no finite particle in the chunk
  const int ex = mx0 - mn0 + 2, ey = mx1 - mn1 + 2, ez = mx2 - mn2 + 2;
  const int64_t vol = static_cast<int64_t>(ex) * ey * ez;
  if (vol <= CAP) {
    for (int t = tid; t < vol; t += NT) tile[t] = 0ull;
    __syncthreads();
    for (int j = tid; j < cnt; j += NT) {
      const float x = p[3 * j], y = p[3 * j + 1], z = p[3 * j + 2];
      if (!(isfinite(x) && isfinite(y) && isfinite(z))) continue;
      int lo[3], hi[3];
      double w[3][2];
      cic_axis64(x, inv_cell, nmask, lo[0], hi[0], w[0][0], w[0][1]);
      cic_axis64(y, inv_cell, nmask, lo[1], hi[1], w[1][0], w[1][1]);
      cic_axis64(z, inv_cell, nmask, lo[2], hi[2], w[2][0], w[2][1]);
      const int a = ((lo[0] - r0 + half) & nmask) - half - mn0;
      const int b = ((lo[1] - r1 + half) & nmask) - half - mn1;
      const int c = ((lo[2] - r2 + half) & nmask) - half - mn2;
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          const double wxy = w[0][cx] * w[1][cy] * kFixScale;
          const int base = ((a + cx) * ey + (b + cy)) * ez + c;
          atomicAdd(&tile[base], static_cast<unsigned long long>(__double2ll_rn(wxy * w[2][0])));
          atomicAdd(&tile[base + 1],
                    static_cast<unsigned long long>(__double2ll_rn(wxy * w[2][1])));
        }
      }
    }
    __syncthreads();
    const int gx0 = r0 + mn0, gy0 = r1 + mn1, gz0 = r2 + mn2;
    for (int t = tid; t < vol; t += NT) {
      const unsigned long long v = tile[t];
      if (v == 0ull) continue;
      const int tz = t % ez, txy = t / ez, ty = txy % ey, tx = txy / ey;
      const int gx = (gx0 + tx) & nmask, gy = (gy0 + ty) & nmask, gz = (gz0 + tz) & nmask;
      atomicAdd(g + (static_cast<int64_t>(gx) * n + gy) * n + gz, v);
    }
  } else {
    for (int j = tid; j < cnt; j += NT) {
      const float x = p[3 * j], y = p[3 * j + 1], z = p[3 * j + 2];
      if (!(isfinite(x) && isfinite(y) && isfinite(z))) continue;
      deposit_global(g, x, y, z, n, inv_cell, nmask);
    }
  }
}

__global__ __launch_bounds__(1024) void interp_kernel(const float* __restrict__ pos,
                                                      const float* __restrict__ force,
                                                      float* __restrict__ acc, int64_t np,
                                                      int nbox, int n, double inv_cell) {
  const int64_t total = np * nbox;
  const int64_t m = static_cast<int64_t>(n) * n * n;
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
      const float* g = force + (i / np) * m * 3;   // [x][y][z][3] per box
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
            const float* v = g + 3 * (row + (cz ? c.hi[2] : c.lo[2]));
            const float w = wxy * c.w[2][cz];
            a0 += w * v[0];
            a1 += w * v[1];
            a2 += w * v[2];
          }
        }
      }
    }
    acc[3 * i] = a0;
    acc[3 * i + 1] = a1;
    acc[3 * i + 2] = a2;
  }
}

// Interpolation with the chunk's bounding-box tile of the acceleration grid staged in LDS
// (rows of 3*ez consecutive floats, coalesced), PPT = CH / 256 particles per thread kept
// in registers; chunks whose box does not fit gather straight from HBM.
template <int CH, int CAP>
__global__ __launch_bounds__(256) void interp_tiled_kernel(const float* __restrict__ pos,
                                                           const float* __restrict__ force,
                                                           float* __restrict__ acc, int64_t np,
                                                           int n, double inv_cell,
                                                           int64_t chunks_per_box) {
  constexpr int NT = 256, NW = NT / 64, PPT = CH / NT;
  __shared__ float tile[CAP * 3];
  __shared__ int red[6][NW];
  __shared__ int ref_s[3];
  const int tid = threadIdx.x;
  const int64_t box = blockIdx.x / chunks_per_box;
  const int64_t c0 = (blockIdx.x - box * chunks_per_box) * CH;
  const int cnt = static_cast<int>(min(static_cast<int64_t>(CH), np - c0));
  const float* p = pos + (box * np + c0) * 3;
  float* a_out = acc + (box * np + c0) * 3;
  const int nmask = n - 1, half = n / 2;
  const float* g = force + box * static_cast<int64_t>(n) * n * n * 3;
  float px[PPT], py[PPT], pz[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int j = tid + q * NT;
    if (j < cnt) {
      px[q] = p[3 * j];
      py[q] = p[3 * j + 1];
      pz[q] = p[3 * j + 2];
    } else {
      px[q] = py[q] = pz[q] = __builtin_nanf("");
    }
  }
  if (tid == 0) {
    const bool ok = isfinite(px[0]) && isfinite(py[0]) && isfinite(pz[0]);
    ref_s[0] = ok ? cell_of(px[0], inv_cell, nmask) : 0;
    ref_s[1] = ok ? cell_of(py[0], inv_cell, nmask) : 0;
    ref_s[2] = ok ? cell_of(pz[0], inv_cell, nmask) : 0;
  }
  __syncthreads();
  const int r0 = ref_s[0], r1 = ref_s[1], r2 = ref_s[2];
  int mn0 = 1 << 30, mn1 = 1 << 30, mn2 = 1 << 30, mx0 = -(1 << 30), mx1 = -(1 << 30),
      mx2 = -(1 << 30);
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    if (!(isfinite(px[q]) && isfinite(py[q]) && isfinite(pz[q]))) continue;
    const int a = ((cell_of(px[q], inv_cell, nmask) - r0 + half) & nmask) - half;
    const int b = ((cell_of(py[q], inv_cell, nmask) - r1 + half) & nmask) - half;
    const int c = ((cell_of(pz[q], inv_cell, nmask) - r2 + half) & nmask) - half;
    mn0 = min(mn0, a); mx0 = max(mx0, a);
    mn1 = min(mn1, b); mx1 = max(mx1, b);
    mn2 = min(mn2, c); mx2 = max(mx2, c);
  }
  mn0 = wave_min(mn0); mn1 = wave_min(mn1); mn2 = wave_min(mn2);
  mx0 = wave_max(mx0); mx1 = wave_max(mx1); mx2 = wave_max(mx2);
  const int lane = tid & 63, wv = tid >> 6;
  if (lane == 0) {
    red[0][wv] = mn0; red[1][wv] = mn1; red[2][wv] = mn2;
    red[3][wv] = mx0; red[4][wv] = mx1; red[5][wv] = mx2;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    mn0 = min(mn0, red[0][w]); mn1 = min(mn1, red[1][w]); mn2 = min(mn2, red[2][w]);
    mx0 = max(mx0, red[3][w]); mx1 = max(mx1, red[4][w]); mx2 = max(mx2, red[5][w]);
  }
  const bool any = mn0 <= mx0;
  const int ex = any ? mx0 - mn0 + 2 : 0, ey = any ? mx1 - mn1 + 2 : 0,
            ez = any ? mx2 - mn2 + 2 : 0;
  const int64_t vol = static_cast<int64_t>(ex) * ey * ez;
  const bool use_tile = any && vol <= CAP;
  if (use_tile) {
    const int gx0 = r0 + mn0, gy0 = r1 + mn1, gz0 = r2 + mn2;
    const int row3 = 3 * ez;
    for (int t = tid; t < vol * 3; t += NT) {
      const int row = t / row3, w = t - row * row3;
      const int tz = w / 3, comp = w - tz * 3;
      const int ty = row % ey, tx = row / ey;
      const int gx = (gx0 + tx) & nmask, gy = (gy0 + ty) & nmask, gz = (gz0 + tz) & nmask;
      tile[t] = g[((static_cast<int64_t>(gx) * n + gy) * n + gz) * 3 + comp];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int j = tid + q * NT;
    if (j >= cnt) continue;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    if (isfinite(px[q]) && isfinite(py[q]) && isfinite(pz[q])) {
      Corner c;
      cic_axis(px[q], inv_cell, nmask, c.lo[0], c.hi[0], c.w[0][0], c.w[0][1]);
      cic_axis(py[q], inv_cell, nmask, c.lo[1], c.hi[1], c.w[1][0], c.w[1][1]);
      cic_axis(pz[q], inv_cell, nmask, c.lo[2], c.hi[2], c.w[2][0], c.w[2][1]);
      if (use_tile) {
        const int ta = ((c.lo[0] - r0 + half) & nmask) - half - mn0;
        const int tb = ((c.lo[1] - r1 + half) & nmask) - half - mn1;
        const int tc = ((c.lo[2] - r2 + half) & nmask) - half - mn2;
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
#pragma unroll
          for (int cy = 0; cy < 2; ++cy) {
            const float wxy = c.w[0][cx] * c.w[1][cy];
            const float* v = tile + 3 * (((ta + cx) * ey + (tb + cy)) * ez + tc);
            a0 += wxy * (c.w[2][0] * v[0] + c.w[2][1] * v[3]);
            a1 += wxy * (c.w[2][0] * v[1] + c.w[2][1] * v[4]);
            a2 += wxy * (c.w[2][0] * v[2] + c.w[2][1] * v[5]);
          }
        }
      } else {
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
              const float* v = g + 3 * (row + (cz ? c.hi[2] : c.lo[2]));
              const float w = wxy * c.w[2][cz];
              a0 += w * v[0];
              a1 += w * v[1];
              a2 += w * v[2];
            }
          }
        }
      }
    }
    a_out[3 * j] = a0;
    a_out[3 * j + 1] = a1;
    a_out[3 * j + 2] = a2;
  }
}

__global__ void fixed_to_float_kernel(const unsigned long long* __restrict__ src,
                                      float* __restrict__ dst, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    dst[i] = static_cast<float>(static_cast<double>(src[i]) / kFixScale);
}

__global__ void extract_component_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                         int64_t n, int comp) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    dst[i] = src[3 * i + comp];
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

hipError_t launch_extract_component(const float* src, float* dst, int64_t n, int comp,
                                   hipStream_t s) {
  int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(extract_component_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n, comp);
  return hipGetLastError();
}

hipError_t launch_fixed_to_float(const unsigned long long* src, float* dst, int64_t n,
                                 hipStream_t s) {
  int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(fixed_to_float_kernel, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

template <int CH, int CAP>
hipError_t launch_tiled(const float* pos, unsigned long long* rho, int64_t np, int nbox, int n,
                        double inv_cell, int* flags, hipStream_t s) {
  const int64_t chunks = (np + CH - 1) / CH;
  hipLaunchKernelGGL((deposit_tiled_kernel<CH, CAP>), dim3(static_cast<unsigned>(chunks * nbox)),
                     dim3(256), 0, s, pos, rho, np, n, inv_cell, flags, chunks);
  return hipGetLastError();
}

hipError_t launch_deposit(const float* pos, unsigned long long* rho, int64_t np, int nbox, int n,
                          double inv_cell, int* flags, int mode, int block, hipStream_t s) {
  switch (mode) {
    case 1: return launch_tiled<1024, 2560>(pos, rho, np, nbox, n, inv_cell, flags, s);
    case 2: return launch_tiled<2048, 4608>(pos, rho, np, nbox, n, inv_cell, flags, s);
    case 3: return launch_tiled<4096, 8192>(pos, rho, np, nbox, n, inv_cell, flags, s);
    default:
      hipLaunchKernelGGL(deposit_kernel, dim3(grid_blocks(np * nbox, block, 1)), dim3(block), 0,
                         s, pos, rho, np, nbox, n, inv_cell, flags);
      return hipGetLastError();
  }
}

template <int CH, int CAP>
hipError_t launch_interp_tiled(const float* pos, const float* force, float* acc, int64_t np,
                               int nbox, int n, double inv_cell, hipStream_t s) {
  const int64_t chunks = (np + CH - 1) / CH;
  hipLaunchKernelGGL((interp_tiled_kernel<CH, CAP>), dim3(static_cast<unsigned>(chunks * nbox)),
                     dim3(256), 0, s, pos, force, acc, np, n, inv_cell, chunks);
  return hipGetLastError();
}

hipError_t launch_interp(const float* pos, const float* force, float* acc, int64_t np,
                         int nbox, int n, double inv_cell, int mode, int block, hipStream_t s) {
  switch (mode) {
    case 1: return launch_interp_tiled<1024, 2560>(pos, force, acc, np, nbox, n, inv_cell, s);
    case 2: return launch_interp_tiled<2048, 4608>(pos, force, acc, np, nbox, n, inv_cell, s);
    case 3: return launch_interp_tiled<4096, 8192>(pos, force, acc, np, nbox, n, inv_cell, s);
    default:
      hipLaunchKernelGGL(interp_kernel, dim3(grid_blocks(np * nbox, block, 1)), dim3(block), 0,
                         s, pos, force, acc, np, nbox, n, inv_cell);
      return hipGetLastError();
  }
}

}  // namespace pmnu
