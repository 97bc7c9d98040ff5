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
#include "patch_device.hpp"

namespace pmnu {
namespace {

// Per axis: lower node (mod N) and the fraction beyond it, in FP64 (u = x N / L is exact
// for an FP32 coordinate times an FP64 inverse cell size up to the product's rounding).
// The node index comes from adding 1.5 * 2^52, which leaves floor(u) in two's complement
// in the low bits for |u| < 2^51; the mask keeps any index in range.
__device__ __forceinline__ void axis64(float x, double inv_cell, int nmask, int& i, double& d) {
  const double u = static_cast<double>(x) * inv_cell;
  const double f = floor(u);
  d = u - f;
  i = static_cast<int>(__double2loint(f + 6755399441055744.0)) & nmask;
}

// Round-to-nearest-even of 0 <= v < 2^52 as an integer: adding 2^52 leaves the rounded
// value in the low mantissa bits (same result as __double2ll_rn, far fewer instructions).
__device__ __forceinline__ unsigned long long fix_rn(double v) {
  return static_cast<unsigned long long>(__double_as_longlong(v + 4503599627370496.0)) -
         0x4330000000000000ull;
}

__device__ __forceinline__ bool finite3(float x, float y, float z) {
  return isfinite(x) && isfinite(y) && isfinite(z);
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

// The eight fixed-point contributions of one particle, added straight to HBM.
__device__ __forceinline__ void deposit_global(unsigned long long* g, int n, const int (&i)[3],
                                               const double (&d)[3], int nmask) {
  const double wx[2] = {(1.0 - d[0]) * kFixScale, d[0] * kFixScale};
  const double wy[2] = {1.0 - d[1], d[1]};
  const int iz0 = i[2], iz1 = (i[2] + 1) & nmask;
#pragma unroll
  for (int cx = 0; cx < 2; ++cx) {
    const int ix = (i[0] + cx) & nmask;
#pragma unroll
    for (int cy = 0; cy < 2; ++cy) {
      const int iy = (i[1] + cy) & nmask;
      const double wxy = wx[cx] * wy[cy];
      const unsigned row = (static_cast<unsigned>(ix) * n + iy) * n;
      atomicAdd(g + row + iz0, fix_rn(wxy * (1.0 - d[2])));
      atomicAdd(g + row + iz1, fix_rn(wxy * d[2]));
    }
  }
}

__global__ __launch_bounds__(1024) void deposit_kernel(const float* __restrict__ pos,
                                                      unsigned long long* __restrict__ rho,
                                                      int64_t np, int nbox, int n,
                                                      double inv_cell, int* __restrict__ flags) {
  const int64_t total = np * nbox;
  const int64_t m = static_cast<int64_t>(n) * n * n;
  const int nmask = n - 1;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  bool bad = false;
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < total;
       k += stride) {
    const float x = pos[3 * k], y = pos[3 * k + 1], z = pos[3 * k + 2];
    if (!finite3(x, y, z)) {
      bad = true;
      continue;
    }
    int i[3];
    double d[3];
    axis64(x, inv_cell, nmask, i[0], d[0]);
    axis64(y, inv_cell, nmask, i[1], d[1]);
    axis64(z, inv_cell, nmask, i[2], d[2]);
    deposit_global(rho + (k / np) * m, n, i, d, nmask);
  }
  if (bad) atomicOr(flags, 1);
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

// Chunk of PPT * 256 consecutive particles held in registers (lower node and fraction per
// axis) and the periodic bounding box of their lower nodes relative to the first particle's
// node. Every thread computes the same reference node, so no barrier is needed for it.
// With KEEP the lower node (relative to r, three 10-bit fields offset by 512) and the FP32
// fraction of every particle are kept, so users need not find them again.
template <int PPT>
struct Chunk {
  float p[PPT][3];
  bool ok[PPT];
  int rel[PPT];
  float f[PPT][3];
  int r[3];
  int mn[3], ext[3];   // box origin (relative to r) and extent in nodes, upper neighbours included
  bool any;
};

template <int PPT, int NT = 256, bool KEEP = false>
__device__ __forceinline__ void load_chunk(Chunk<PPT>& c, const float* p, int cnt, double inv_cell,
                                           int nmask, int (*red)[NT / 64], bool& bad) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, half = (nmask + 1) / 2;
  {
    const float x = p[0], y = p[1], z = p[2];
    const bool ok0 = finite3(x, y, z);
    double dd;
    axis64(ok0 ? x : 0.f, inv_cell, nmask, c.r[0], dd);
    axis64(ok0 ? y : 0.f, inv_cell, nmask, c.r[1], dd);
    axis64(ok0 ? z : 0.f, inv_cell, nmask, c.r[2], dd);
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int j = tid + q * NT;
    c.p[q][0] = c.p[q][1] = c.p[q][2] = 0.f;
    if (j < cnt) {
      c.p[q][0] = p[3 * j];
      c.p[q][1] = p[3 * j + 1];
      c.p[q][2] = p[3 * j + 2];
    }
  }
  int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int j = tid + q * NT;
    c.ok[q] = j < cnt && finite3(c.p[q][0], c.p[q][1], c.p[q][2]);
    bad |= (j < cnt) && !c.ok[q];
    if (KEEP) c.rel[q] = 0;
    if (c.ok[q]) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        int i;
        double d;
        axis64(c.p[q][a], inv_cell, nmask, i, d);
        const int rel = ((i - c.r[a] + half) & nmask) - half;
        mn[a] = min(mn[a], rel);
        mx[a] = max(mx[a], rel);
        if (KEEP) {
          c.rel[q] |= (rel + 512) << (10 * a);      // -256 <= rel < 256
          c.f[q][a] = static_cast<float>(d);
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mn[a] = wave_min(mn[a]);
    mx[a] = wave_max(mx[a]);
  }
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      red[a][wv] = mn[a];
      red[3 + a][wv] = mx[a];
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      mn[a] = min(mn[a], red[a][w]);
      mx[a] = max(mx[a], red[3 + a][w]);
    }
  }
  // the box is the same for the whole workgroup: keep it in scalar registers
  c.any = __builtin_amdgcn_readfirstlane(mn[0] <= mx[0] ? 1 : 0) != 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c.r[a] = __builtin_amdgcn_readfirstlane(c.r[a]);
    c.mn[a] = __builtin_amdgcn_readfirstlane(mn[a]);
    c.ext[a] = c.any ? __builtin_amdgcn_readfirstlane(mx[a] - mn[a] + 2) : 0;
  }
}

// Walks the rows (tx, ty) of an ex x ey x ez box with the lanes of a wave spread over
// (row, z): lane l takes z = l mod ez of row l / ez, so short rows keep the wave busy
// without a division per node. Calls f(tx, ty, tz, linear index).
template <int NT = 256, typename F>
__device__ __forceinline__ void for_box_nodes(int ex, int ey, int ez, F f) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (ez <= 64) {
    const int rpi = 64 / ez, dr = lane / ez, tz = lane - dr * ez;
    if (dr >= rpi) return;
    const int step = NW * rpi;
    int r = wv * rpi + dr;
    int tx = r / ey, ty = r - tx * ey;
    while (tx < ex) {
      f(tx, ty, tz, r * ez + tz);
      r += step;
      ty += step;
      while (ty >= ey) {
        ty -= ey;
        ++tx;
      }
    }
  } else {
    for (int r = wv; r < ex * ey; r += NW) {
      const int tx = r / ey, ty = r - tx * ey;
      for (int tz = lane; tz < ez; tz += 64) f(tx, ty, tz, r * ez + tz);
    }
  }
}

// Deposit with the accumulation privatised in LDS: a workgroup takes CH consecutive
// particles; if their box (upper neighbours included) fits in CAP nodes, it sums the
// chunk's fixed-point weights there with 64-bit LDS atomics and adds every non-zero node
// to HBM with one global atomic. Chunks that are not spatially compact (particles in
// arbitrary order) take the per-particle global-atomic path, so the result does not depend
// on the order; the speed does. Particles kept along a space-filling curve (as tree codes
// keep them) give compact chunks.
template <int CH, int CAP, int NT>
__global__ __launch_bounds__(NT) void deposit_tiled_kernel(const float* __restrict__ pos,
                                                           unsigned long long* __restrict__ rho,
                                                           int64_t np, int n, double inv_cell,
                                                           int* __restrict__ flags,
                                                           int64_t chunks_per_box) {
  constexpr int PPT = CH / NT;
  __shared__ unsigned long long tile[CAP];
  __shared__ int red[6][NT / 64];
  const int tid = threadIdx.x;
  const int64_t box = blockIdx.x / chunks_per_box;
  const int64_t c0 = (blockIdx.x - box * chunks_per_box) * CH;
  const int cnt = static_cast<int>(min(static_cast<int64_t>(CH), np - c0));
  const int nmask = n - 1;
  unsigned long long* g = rho + box * static_cast<int64_t>(n) * n * n;
  Chunk<PPT> c;
  bool bad = false;
  load_chunk<PPT, NT>(c, pos + (box * np + c0) * 3, cnt, inv_cell, nmask, red, bad);
  if (bad) atomicOr(flags, 1);
  const int ex = c.ext[0], ey = c.ext[1], ez = c.ext[2];
  // Tile strides padded so that a wave's 16-lane groups of particles along the curve
  // (2 x 2 x 4 blocks of nodes for lattice-ordered chunks) hit 16 distinct 8-byte bank
  // slots: z stride = 4 (mod 8), y stride = 2 (mod 4). Unpadded if the padding does not fit.
  int sz = ez + ((12 - ez % 8) % 8), sy = ey + ((6 - ey % 4) % 4);
  if (ex * sy * sz > CAP) {
    sz = ez;
    sy = ey;
  }
  const int vol = ex * sy * sz;
  if (c.any && vol <= CAP && ex <= n && ey <= n && ez <= n) {
    for (int t = tid; t < vol; t += NT) tile[t] = 0ull;
    __syncthreads();
    const int half = n / 2;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      if (!c.ok[q]) continue;
      int t[3];
      double d[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        int i;
        axis64(c.p[q][a], inv_cell, nmask, i, d[a]);
        t[a] = ((i - c.r[a] + half) & nmask) - half - c.mn[a];
      }
      const double wx[2] = {(1.0 - d[0]) * kFixScale, d[0] * kFixScale};
      const double wy[2] = {1.0 - d[1], d[1]};
      const double wz0 = 1.0 - d[2], wz1 = d[2];
      const int base = (t[0] * sy + t[1]) * sz + t[2];
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          const double wxy = wx[cx] * wy[cy];
          const int o = base + (cx * sy + cy) * sz;
          atomicAdd(&tile[o], fix_rn(wxy * wz0));
          atomicAdd(&tile[o + 1], fix_rn(wxy * wz1));
        }
      }
    }
    __syncthreads();
    const int gx0 = c.r[0] + c.mn[0], gy0 = c.r[1] + c.mn[1], gz0 = c.r[2] + c.mn[2];
    for_box_nodes<NT>(ex, ey, ez, [&](int tx, int ty, int tz, int) {
      const unsigned long long v = tile[(tx * sy + ty) * sz + tz];
      if (v == 0ull) return;
      const unsigned gx = (gx0 + tx) & nmask, gy = (gy0 + ty) & nmask, gz = (gz0 + tz) & nmask;
      atomicAdd(g + (gx * n + gy) * n + gz, v);
    });
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      if (!c.ok[q]) continue;
      int i[3];
      double d[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) axis64(c.p[q][a], inv_cell, nmask, i[a], d[a]);
      deposit_global(g, n, i, d, nmask);
    }
  }
}

// ---------------------------------------------------------------- patch deposit ----
// Deposit without global atomics. D1: each chunk sums its particles in an LDS tile as
// above, writes the tile (its box, unpadded) to its own patch slot with plain stores and
// registers the patch in every coarse cell (CB^3 nodes) that the box overlaps; a registry
// entry carries everything D2 needs (chunk, box origin, extents). D2: one workgroup per
// slab of a coarse cell adds up the registered patches in exact integers and writes
// delta = rho / rho_bar - 1 once, rounded to FP32. Weights that cannot go through a patch
// (a box too large: the whole chunk; a coarse cell whose list is full: the box's part in
// that cell) are added with global atomics to a side grid kept at zero, which D2 folds in
// (and clears) only when something was added to it.

__device__ __forceinline__ int ceil_div_pow2(int a, int lg) { return (a + (1 << lg) - 1) >> lg; }

template <int CH, int CAP, int NT>
__global__ __launch_bounds__(NT) void deposit_patch_kernel(
    const float* __restrict__ pos, unsigned long long* __restrict__ patches,
    int* __restrict__ reg_count, int4* __restrict__ reg_list,
    unsigned long long* __restrict__ rho_fb, int* __restrict__ n_fb,
    int64_t np, int n, double inv_cell, int* __restrict__ flags, int64_t chunks_per_box,
    int cb_lg) {
  constexpr int PPT = CH / NT;
  __shared__ unsigned long long tile[CAP];
  __shared__ int red[6][NT / 64];
  __shared__ unsigned s_over;          // bit t: registry cell t of the box was full
  const int tid = threadIdx.x;
  const int64_t chunk = blockIdx.x;
  // grid sizes stay below 2^31 blocks: a 32-bit division suffices
  const int64_t box = static_cast<uint32_t>(chunk) / static_cast<uint32_t>(chunks_per_box);
  const int64_t c0 = (chunk - box * chunks_per_box) * CH;
  const int cnt = static_cast<int>(min(static_cast<int64_t>(CH), np - c0));
  const int nmask = n - 1;
  const int64_t m = static_cast<int64_t>(n) * n * n;
  unsigned long long* fb = rho_fb + box * m;
  if (tid == 0) s_over = 0u;
  Chunk<PPT> c;
  bool bad = false;
  load_chunk<PPT, NT>(c, pos + (box * np + c0) * 3, cnt, inv_cell, nmask, red, bad);
  if (bad) atomicOr(flags, 1);
  const int ex = c.ext[0], ey = c.ext[1], ez = c.ext[2];
  int sz = ez + ((12 - ez % 8) % 8), sy = ey + ((6 - ey % 4) % 4);
  if (ex * sy * sz > CAP) {
    sz = ez;
    sy = ey;
  }
  const int vol = ex * sy * sz;
  const int gx0 = (c.r[0] + c.mn[0]) & nmask, gy0 = (c.r[1] + c.mn[1]) & nmask,
            gz0 = (c.r[2] + c.mn[2]) & nmask;
  const int nc = n >> cb_lg;
  const int rx = min(nc, ceil_div_pow2((gx0 & ((1 << cb_lg) - 1)) + ex, cb_lg));
  const int ry = min(nc, ceil_div_pow2((gy0 & ((1 << cb_lg) - 1)) + ey, cb_lg));
  const int rz = min(nc, ceil_div_pow2((gz0 & ((1 << cb_lg) - 1)) + ez, cb_lg));
  const bool fits = c.any && vol <= CAP && ex <= n && ey <= n && ez <= n &&
                    rx * ry * rz <= kPatchRegMax;
  if (fits) {
    // register the patch in the coarse cells its box overlaps (origin and extents < 1024)
    const int64_t cells = static_cast<int64_t>(nc) * nc * nc;
    const int fx = gx0 >> cb_lg, fy = gy0 >> cb_lg, fz = gz0 >> cb_lg;
    const int4 entry = make_int4(static_cast<int>(chunk), gx0 | (gy0 << 10) | (gz0 << 20),
                                 ex | (ey << 10) | (ez << 20), 0);
    for (int t = tid; t < rx * ry * rz; t += NT) {
      const int iz = t % rz, ixy = t / rz, iy = ixy % ry, ix = ixy / ry;
      const int64_t cell = box * cells +
                           ((static_cast<int64_t>((fx + ix) % nc) * nc + (fy + iy) % nc) * nc +
                            (fz + iz) % nc);
      const int slot = atomicAdd(reg_count + cell, 1);
      if (slot < kPatchList)
        reg_list[cell * kPatchList + slot] = entry;
      else
        atomicOr(&s_over, 1u << t);             // t < kPatchRegMax <= 32
    }
    for (int t = tid; t < vol; t += NT) tile[t] = 0ull;
    __syncthreads();
    const int half = n / 2;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      if (!c.ok[q]) continue;
      int t[3];
      double d[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        int i;
        axis64(c.p[q][a], inv_cell, nmask, i, d[a]);
        t[a] = ((i - c.r[a] + half) & nmask) - half - c.mn[a];
      }
      const double wx[2] = {(1.0 - d[0]) * kFixScale, d[0] * kFixScale};
      const double wy[2] = {1.0 - d[1], d[1]};
      const double wz0 = 1.0 - d[2], wz1 = d[2];
      const int base = (t[0] * sy + t[1]) * sz + t[2];
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
          const double wxy = wx[cx] * wy[cy];
          const int o = base + (cx * sy + cy) * sz;
          atomicAdd(&tile[o], fix_rn(wxy * wz0));
          atomicAdd(&tile[o + 1], fix_rn(wxy * wz1));
        }
      }
    }
    __syncthreads();
    // the patch (the box unpadded): consecutive lanes at consecutive nodes, four nodes per
    // thread per round with their LDS reads ahead of the stores. Node li of the box is
    // (tx, ty, tz) = (li / (ey ez), li / ez % ey, li % ez); the FP32 quotients are exact
    // (li < 2^14 and the fractional part of (li + 1/2) / e is at least 1 / (2e)).
    unsigned long long* pat = patches + chunk * kPatchCap;     // stored patch stride
    {
      const int volp = ex * ey * ez;
      const float inv_ez = 1.0f / static_cast<float>(ez), inv_ey = 1.0f / static_cast<float>(ey);
      for (int l0 = tid; l0 < volp; l0 += 4 * NT) {
        unsigned long long val[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int li = l0 + u * NT;
          val[u] = 0ull;
          if (li < volp) {
            const int t = static_cast<int>((static_cast<float>(li) + 0.5f) * inv_ez);
            const int tz = li - t * ez;
            const int tx = static_cast<int>((static_cast<float>(t) + 0.5f) * inv_ey);
            const int ty = t - tx * ey;
            val[u] = tile[(tx * sy + ty) * sz + tz];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (l0 + u * NT < volp) pat[l0 + u * NT] = val[u];
      }
    }
    const unsigned over = s_over;
    if (over == 0u) return;
    // coarse cells whose list was full: the box's part in them goes to the side grid
    const int cbm = (1 << cb_lg) - 1;
    for_box_nodes<NT>(ex, ey, ez, [&](int tx, int ty, int tz, int) {
      int ix = ((gx0 & cbm) + tx) >> cb_lg, iy = ((gy0 & cbm) + ty) >> cb_lg,
          iz = ((gz0 & cbm) + tz) >> cb_lg;
      ix -= ix >= nc ? nc : 0;                  // a box as wide as the mesh wraps onto fx
      iy -= iy >= nc ? nc : 0;
      iz -= iz >= nc ? nc : 0;
      if (!((over >> ((ix * ry + iy) * rz + iz)) & 1u)) return;
      const unsigned long long v = tile[(tx * sy + ty) * sz + tz];
      if (v == 0ull) return;
      const unsigned gx = (gx0 + tx) & nmask, gy = (gy0 + ty) & nmask, gz = (gz0 + tz) & nmask;
      atomicAdd(fb + (gx * n + gy) * n + gz, v);
    });
  } else {
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      if (!c.ok[q]) continue;
      int i[3];
      double d[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) axis64(c.p[q][a], inv_cell, nmask, i[a], d[a]);
      deposit_global(fb, n, i, d, nmask);
    }
  }
  if (tid == 0) atomicAdd(n_fb, 1);
}

// D2: one workgroup of 256 threads per (slab of XD x-planes of a coarse cell, box), CB =
// 1 << cb_lg <= 16, XD <= CB (halving the slab halves the LDS copy and doubles the
// workgroups, which hides more of the load latency). A cell is mostly covered by one patch
// (the chunk whose block it is) and touched by a few others in thin layers (their halos).
// The largest overlap goes through registers: thread (iy, iz) owns the slab's column
// x = 0..XD-1 and loads it from that patch. Every other overlap is cut into boxes (up to
// two periodic pieces per axis), which wave 0 lists once in LDS with their item offsets,
// sizes and source and destination bases; all threads then stride over the flat item list,
// find an item's box by bisection and add the node into an LDS copy of the slab with
// 64-bit LDS atomics. Every thread issues all of its loads (its column and up to kBatch
// list items) before it uses any, so each workgroup waits on few load latencies. The sums
// are exact integers.
template <int XD>
__global__ __launch_bounds__(256) void patch_reduce_kernel(
    const unsigned long long* __restrict__ patches, int pcap, const int* __restrict__ reg_count,
    const int4* __restrict__ reg_list, unsigned long long* __restrict__ rho_fb,
    const int* __restrict__ n_fb, float* __restrict__ delta, int n, int cb_lg, double scale) {
  constexpr int CBM = 16, kBatch = 8, kPieces = kPatchList * 8;
  const int tid = threadIdx.x;
  const int cb = 1 << cb_lg, nc = n >> cb_lg;
  const int slabs = cb / XD;
  const int64_t cells = static_cast<int64_t>(nc) * nc * nc;
  const int64_t box = blockIdx.y;
  // workgroups go to the 8 XCDs in turn: each XCD takes a contiguous run of slabs instead,
  // so that neighbouring cells (which read the same patches' halo lines) share an L2; a
  // ragged tail keeps its own index
  const int nb = gridDim.x, per = nb / 8;
  const int bid = static_cast<int>(blockIdx.x) < per * 8
                      ? static_cast<int>(blockIdx.x % 8) * per + static_cast<int>(blockIdx.x / 8)
                      : static_cast<int>(blockIdx.x);
  const int cix = bid / slabs;
  const int64_t cell = box * cells + cix;
  const int ccz = (cix % nc) << cb_lg, ccy = ((cix / nc) % nc) << cb_lg,
            ccx = ((cix / (nc * nc)) << cb_lg) + (bid - cix * slabs) * XD;  // slab's x0
  const int iy = tid >> cb_lg, iz = tid & (cb - 1);
  const bool on = tid < cb * cb;
  const int vol_cell = XD * cb * cb;
  __shared__ unsigned long long s_acc[XD * CBM * CBM];    // [x][y][z] of the slab
  // the piece list: item offset (INT_MAX past the end), Lz | Ly << 8, source base
  // (patch element of the piece's first node), strides ez | (ey ez) << 10, LDS base
  __shared__ int p_off[kPieces + 1];
  __shared__ int p_dim[kPieces];
  __shared__ long long p_src[kPieces];
  __shared__ int p_str[kPieces];
  __shared__ int p_dst[kPieces];
  __shared__ int4 s_home;                  // home patch: chunk, origin, extents; chunk < 0: none
  __shared__ int s_total;                  // items in the piece list
  for (int i = tid; i < vol_cell; i += 256) s_acc[i] = 0ull;
  if (tid < 64) {
    // wave 0: the cell's patches (list row and count fetched together), their overlap
    // pieces, the home patch and the piece list of the others
    const int cnt_raw = reg_count[cell];
    const int4 listed =
        tid < kPatchList ? reg_list[cell * kPatchList + tid] : make_int4(-1, 0, 0, 0);
    const bool mine = tid < min(cnt_raw, kPatchList);
    const int gx = listed.y & 1023, gy = (listed.y >> 10) & 1023, gz = listed.y >> 20;
    const int ex = listed.z & 1023, ey = (listed.z >> 10) & 1023, ez = listed.z >> 20;
    Pieces px, py, pz;
    px.cnt = py.cnt = pz.cnt = 0;
    int vol = -1;
    if (mine) {
      px = overlap(gx, ex, ccx, XD, n);
      py = overlap(gy, ey, ccy, cb, n);
      pz = overlap(gz, ez, ccz, cb, n);
      int lx = 0, ly = 0, lz = 0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {           // constant bounds: no indexed scratch
        lx += q < px.cnt ? px.len[q] : 0;
        ly += q < py.cnt ? py.len[q] : 0;
        lz += q < pz.cnt ? pz.len[q] : 0;
      }
      vol = lx * ly * lz;
    }
    // home: the largest volume, ties to the lowest index
    int key = vol > 0 ? (vol << 6) | (63 - tid) : -1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) key = max(key, __shfl_xor(key, off, 64));
    const int home = key >= 0 ? 63 - (key & 63) : -1;
    if (tid == 0) s_home = make_int4(-1, 0, 0, 0);
    if (tid == home) s_home = listed;
    // exclusive prefixes of the others' piece counts and volumes
    const bool other = vol > 0 && tid != home;
    const int np_mine = other ? px.cnt * py.cnt * pz.cnt : 0;
    int inc_p = np_mine, inc_v = other ? vol : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int tp = __shfl_up(inc_p, off, 64), tv = __shfl_up(inc_v, off, 64);
      if (tid >= off) {
        inc_p += tp;
        inc_v += tv;
      }
    }
    const int n_pieces = __shfl(inc_p, 63, 64);
    if (tid == 63) s_total = inc_v;
    int slot = inc_p - np_mine;
    int item = inc_v - (other ? vol : 0);
    if (other) {
      const long long src0 = static_cast<long long>(listed.x) * pcap;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            if (a >= px.cnt || b >= py.cnt || c >= pz.cnt) continue;
            const int Lx = px.len[a], Ly = py.len[b], Lz = pz.len[c];
            p_off[slot] = item;
            p_dim[slot] = Lz | (Ly << 8);
            p_src[slot] = src0 + (px.pl[a] * ey + py.pl[b]) * ez + pz.pl[c];
            p_str[slot] = ez | ((ey * ez) << 10);
            p_dst[slot] = (px.cl[a] * cb + py.cl[b]) * cb + pz.cl[c];
            item += Lx * Ly * Lz;
            ++slot;
          }
    }
    for (int i = n_pieces + tid; i <= kPieces; i += 64) p_off[i] = 0x7fffffff;
  }
  __syncthreads();
  const int total = s_total;
  // the home patch's column loads go out first
  unsigned long long acc[XD];
#pragma unroll
  for (int x = 0; x < XD; ++x) acc[x] = 0ull;
  const int4 hl = s_home;
  if (hl.x >= 0) {
    const int hx = hl.y & 1023, hy = (hl.y >> 10) & 1023, hz = hl.y >> 20;
    const int ex = hl.z & 1023, ey = (hl.z >> 10) & 1023, ez = hl.z >> 20;
    const Pieces px = overlap(hx, ex, ccx, XD, n), py = overlap(hy, ey, ccy, cb, n),
                 pz = overlap(hz, ez, ccz, cb, n);
    int ly = -1, lz = -1;                       // this thread's row (y, z) inside the patch
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q < py.cnt && iy >= py.cl[q] && iy < py.cl[q] + py.len[q]) ly = py.pl[q] + iy - py.cl[q];
      if (q < pz.cnt && iz >= pz.cl[q] && iz < pz.cl[q] + pz.len[q]) lz = pz.pl[q] + iz - pz.cl[q];
    }
    const bool lane_in = on && ly >= 0 && lz >= 0;
    const unsigned long long* row =
        patches + static_cast<int64_t>(hl.x) * pcap + (lane_in ? ly * ez + lz : 0);
    const int xs = ey * ez;                     // patch stride along x
#pragma unroll
    for (int x = 0; x < XD; ++x) {
      int lx = -1;                              // patch-local x of slab-local x (uniform)
      if (px.cnt > 0 && x >= px.cl[0] && x < px.cl[0] + px.len[0]) lx = px.pl[0] + x - px.cl[0];
      if (px.cnt > 1 && x >= px.cl[1] && x < px.cl[1] + px.len[1]) lx = px.pl[1] + x - px.cl[1];
      acc[x] = (lx >= 0 && lane_in) ? row[lx * xs] : 0ull;
    }
  }
  // the other overlaps: kBatch items per thread per round, all loads before the adds
  for (int base = 0; base < total; base += kBatch * 256) {
    unsigned long long v[kBatch];
    int li[kBatch];
#pragma unroll
    for (int r = 0; r < kBatch; ++r) {
      const int i = base + r * 256 + tid;
      li[r] = -1;
      v[r] = 0ull;
      if (i < total) {
        int e = 0;                              // the piece: last offset <= i
#pragma unroll
        for (int step = kPieces / 2; step > 0; step >>= 1)
          if (p_off[e + step] <= i) e += step;
        const int rem = i - p_off[e];
        const int dim = p_dim[e], str = p_str[e];
        const int Lz = dim & 255, Ly = dim >> 8;
        // exact: rem < 4096 and the divisors are at most 16
        const int t = static_cast<int>((rem + 0.5f) * (1.0f / Lz));
        const int z = rem - t * Lz;
        const int x = static_cast<int>((t + 0.5f) * (1.0f / Ly));
        const int y = t - x * Ly;
        v[r] = patches[p_src[e] + x * (str >> 10) + y * (str & 1023) + z];
        li[r] = p_dst[e] + (x * cb + y) * cb + z;
      }
    }
#pragma unroll
    for (int r = 0; r < kBatch; ++r)
      if (li[r] >= 0) atomicAdd(&s_acc[li[r]], v[r]);
  }
  __syncthreads();
  const bool fold = *n_fb > 0;
  if (on) {
    const int64_t m = static_cast<int64_t>(n) * n * n;
    const int64_t col = box * m + static_cast<int64_t>(ccy + iy) * n + ccz + iz;
#pragma unroll
    for (int x = 0; x < XD; ++x) {
      const int64_t node = col + static_cast<int64_t>(ccx + x) * n * n;
      unsigned long long val = acc[x] + s_acc[(x * cb + iy) * cb + iz];
      if (fold) {
        val += rho_fb[node];
        rho_fb[node] = 0ull;
      }
      // exact integer sum, rounded once: delta = rho / rho_bar - 1
      delta[node] = static_cast<float>(static_cast<double>(val) * scale - 1.0);
    }
  }
  // reg_count is cleared by the next kernel (the first forward FFT pass): the other slabs of
  // this cell may still read it
}

__global__ void delta_to_density_kernel(const float* __restrict__ delta, float* __restrict__ out,
                                        int64_t n, float rho_bar) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride)
    out[i] = (delta[i] + 1.0f) * rho_bar;
}

// FP32 corner weights of one particle (the fraction rounded once to FP32).
struct Corner {
  int i[3];
  float w[3][2];
};

__device__ __forceinline__ void corner_of(float x, float y, float z, double inv_cell, int nmask,
                                          Corner& c) {
  double d;
  axis64(x, inv_cell, nmask, c.i[0], d);
  c.w[0][1] = static_cast<float>(d);
  c.w[0][0] = 1.0f - c.w[0][1];
  axis64(y, inv_cell, nmask, c.i[1], d);
  c.w[1][1] = static_cast<float>(d);
  c.w[1][0] = 1.0f - c.w[1][1];
  axis64(z, inv_cell, nmask, c.i[2], d);
  c.w[2][1] = static_cast<float>(d);
  c.w[2][0] = 1.0f - c.w[2][1];
}

// Gather of the interleaved acceleration grid ([x][y][z][3] per box) at the 8 corners.
__device__ __forceinline__ void gather_global(const float* g, int n, int nmask, const Corner& c,
                                              float& a0, float& a1, float& a2) {
  const int iz0 = c.i[2], iz1 = (c.i[2] + 1) & nmask;
#pragma unroll
  for (int cx = 0; cx < 2; ++cx) {
    const int ix = (c.i[0] + cx) & nmask;
#pragma unroll
    for (int cy = 0; cy < 2; ++cy) {
      const int iy = (c.i[1] + cy) & nmask;
      const float wxy = c.w[0][cx] * c.w[1][cy];
      const unsigned row = (static_cast<unsigned>(ix) * n + iy) * n;
#pragma unroll
      for (int cz = 0; cz < 2; ++cz) {
        const float* v = g + 3 * (row + (cz ? iz1 : iz0));
        const float w = wxy * c.w[2][cz];
        a0 += w * v[0];
        a1 += w * v[1];
        a2 += w * v[2];
      }
    }
  }
}

// Workgroups are handed to the XCDs in turn; remapping the block index gives each XCD one
// contiguous run of chunks, so neighbouring chunks (which share grid lines) hit the same L2.
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t nblocks) {
  constexpr int kXcd = 8;
  const int64_t per = (nblocks + kXcd - 1) / kXcd;
  return (b % kXcd) * per + b / kXcd;
}

// Direct interpolation: PPT particles per thread (strided by the block size inside a
// contiguous chunk), gathering from HBM through the caches.
// The end of the interpolation for particle gi (global index) at position (x, y, z): store
// the acceleration, or apply the leapfrog of pm_nu_advance (u += K acc; x += D u).
template <bool LEAP>
__device__ __forceinline__ void finish_particle(const Leap& lp, float* __restrict__ acc,
                                                int64_t gi, float x, float y, float z,
                                                float a0, float a1, float a2, float kk,
                                                float dd) {
  if (!LEAP || lp.store_acc) {
    acc[3 * gi] = a0;
    acc[3 * gi + 1] = a1;
    acc[3 * gi + 2] = a2;
  }
  if (!LEAP) return;
  float* u = lp.vel + 3 * gi;
  const float u0 = u[0] + kk * a0, u1 = u[1] + kk * a1, u2 = u[2] + kk * a2;
  u[0] = u0;
  u[1] = u1;
  u[2] = u2;
  if (lp.pos) {
    float* px = lp.pos + 3 * gi;
    px[0] = wrap_box(x + dd * u0, lp.box);
    px[1] = wrap_box(y + dd * u1, lp.box);
    px[2] = wrap_box(z + dd * u2, lp.box);
  }
}

template <int PPT, bool LEAP>
__global__ __launch_bounds__(256) void interp_kernel(const float* pos,
                                                     const float* __restrict__ force,
                                                     float* __restrict__ acc, int64_t np, int n,
                                                     double inv_cell, int64_t chunks_per_box,
                                                     int64_t nchunks, Leap lp) {
  constexpr int NT = 256, CH = NT * PPT;
  const int64_t chunk = xcd_chunk(blockIdx.x, gridDim.x);
  if (chunk >= nchunks) return;
  // grid sizes stay below 2^31 blocks: a 32-bit division suffices
  const int64_t box = static_cast<uint32_t>(chunk) / static_cast<uint32_t>(chunks_per_box);
  const int64_t c0 = (chunk - box * chunks_per_box) * CH;
  const int cnt = static_cast<int>(min(static_cast<int64_t>(CH), np - c0));
  const float* p = pos + (box * np + c0) * 3;
  const float* g = force + box * static_cast<int64_t>(n) * n * n * 3;
  const int nmask = n - 1;
  float kk = 0.f, dd = 0.f;
  if (LEAP) {
    kk = static_cast<float>(lp.kd[2 * box]);
    dd = static_cast<float>(lp.kd[2 * box + 1]);
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int j = threadIdx.x + q * NT;
    if (j >= cnt) break;
    const float x = p[3 * j], y = p[3 * j + 1], z = p[3 * j + 2];
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    if (finite3(x, y, z)) {
      Corner c;
      corner_of(x, y, z, inv_cell, nmask, c);
      gather_global(g, n, nmask, c, a0, a1, a2);
    }
    finish_particle<LEAP>(lp, acc, box * np + c0 + j, x, y, z, a0, a1, a2, kk, dd);
  }
}

// Interpolation with the chunk's box of the acceleration grid staged in LDS (rows of
// 3 * ez consecutive floats); chunks whose box does not fit gather straight from HBM.
template <int CH, int CAP, bool LEAP>
__global__ __launch_bounds__(256) void interp_tiled_kernel(const float* pos,
                                                           const float* __restrict__ force,
                                                           float* __restrict__ acc, int64_t np,
                                                           int n, double inv_cell,
                                                           int64_t chunks_per_box,
                                                           int64_t nchunks, Leap lp) {
  constexpr int NT = 256, PPT = CH / NT;
  __shared__ float tile[CAP * 3];
  __shared__ int red[6][256 / 64];
  const int tid = threadIdx.x;
  const int64_t chunk = xcd_chunk(blockIdx.x, gridDim.x);
  if (chunk >= nchunks) return;
  // grid sizes stay below 2^31 blocks: a 32-bit division suffices
  const int64_t box = static_cast<uint32_t>(chunk) / static_cast<uint32_t>(chunks_per_box);
  const int64_t c0 = (chunk - box * chunks_per_box) * CH;
  const int cnt = static_cast<int>(min(static_cast<int64_t>(CH), np - c0));
  const int nmask = n - 1;
  const float* g = force + box * static_cast<int64_t>(n) * n * n * 3;
  float kk = 0.f, dd = 0.f;
  if (LEAP) {
    kk = static_cast<float>(lp.kd[2 * box]);
    dd = static_cast<float>(lp.kd[2 * box + 1]);
  }
  Chunk<PPT> c;
  bool bad = false;
  load_chunk<PPT, 256, true>(c, pos + (box * np + c0) * 3, cnt, inv_cell, nmask, red, bad);
  const int ex = c.ext[0], ey = c.ext[1], ez = c.ext[2];
  const int vol = ex * ey * ez;
  const bool use_tile = c.any && vol <= CAP && ex <= n && ey <= n && ez <= n;
  if (use_tile) {
    const int gx0 = c.r[0] + c.mn[0], gy0 = c.r[1] + c.mn[1], gz0 = c.r[2] + c.mn[2];
    constexpr int RMAX = 32;                 // rows per wave held in registers
    const int rows = ex * ey;
    if (3 * ez <= 64 && rows <= 4 * RMAX) {
      // one row (3 ez consecutive floats, contiguous in HBM unless z wraps) per wave and
      // step; all of a wave's row loads are in flight before the LDS stores
      const int lane = tid & 63;
      const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: scalar row walk
      const int tz = lane / 3, comp = lane - 3 * tz;
      const bool on = lane < 3 * ez;
      const unsigned lane_off = 3 * ((gz0 + tz) & nmask) + comp;
      float vals[RMAX];
      int tx = wv / ey, ty = wv - (wv / ey) * ey;
#pragma unroll
      for (int i = 0; i < RMAX; ++i) {
        if (wv + 4 * i < rows) {
          const unsigned gx = (gx0 + tx) & nmask, gy = (gy0 + ty) & nmask;
          const float* rowp = g + 3 * static_cast<size_t>((gx * n + gy) * n);
          if (on) vals[i] = rowp[lane_off];
        }
        ty += 4;
        while (ty >= ey) {
          ty -= ey;
          ++tx;
        }
      }
#pragma unroll
      for (int i = 0; i < RMAX; ++i)
        if (on && wv + 4 * i < rows) tile[(wv + 4 * i) * 3 * ez + lane] = vals[i];
    } else {
      for_box_nodes(ex, ey, ez, [&](int tx, int ty, int tz, int li) {
        const unsigned gx = (gx0 + tx) & nmask, gy = (gy0 + ty) & nmask,
                       gz = (gz0 + tz) & nmask;
        const float* v = g + 3 * ((gx * n + gy) * n + gz);
        tile[3 * li] = v[0];
        tile[3 * li + 1] = v[1];
        tile[3 * li + 2] = v[2];
      });
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int j = tid + q * NT;
    if (j >= cnt) continue;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    if (c.ok[q]) {
      Corner k;                                  // from the node and fraction kept above
      int rel[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        rel[a] = ((c.rel[q] >> (10 * a)) & 1023) - 512;
        k.w[a][1] = c.f[q][a];
        k.w[a][0] = 1.0f - k.w[a][1];
      }
      if (use_tile) {
        int t[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) t[a] = rel[a] - c.mn[a];
        const int base = (t[0] * ey + t[1]) * ez + t[2];
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
#pragma unroll
          for (int cy = 0; cy < 2; ++cy) {
            const float wxy = k.w[0][cx] * k.w[1][cy];
            const float* v = tile + 3 * (base + (cx * ey + cy) * ez);
#pragma unroll
            for (int cz = 0; cz < 2; ++cz) {
              const float w = wxy * k.w[2][cz];
              a0 += w * v[3 * cz];
              a1 += w * v[3 * cz + 1];
              a2 += w * v[3 * cz + 2];
            }
          }
        }
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) k.i[a] = (c.r[a] + rel[a]) & nmask;
        gather_global(g, n, nmask, k, a0, a1, a2);
      }
    }
    finish_particle<LEAP>(lp, acc, box * np + c0 + j, c.p[q][0], c.p[q][1], c.p[q][2], a0, a1,
                          a2, kk, dd);
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

template <int CH, int CAP, int NT>
hipError_t launch_tiled(const float* pos, unsigned long long* rho, int64_t np, int nbox, int n,
                        double inv_cell, int* flags, hipStream_t s) {
  const int64_t chunks = (np + CH - 1) / CH;
  hipLaunchKernelGGL((deposit_tiled_kernel<CH, CAP, NT>),
                     dim3(static_cast<unsigned>(chunks * nbox)), dim3(NT), 0, s, pos, rho, np, n,
                     inv_cell, flags, chunks);
  return hipGetLastError();
}

// mode 0: one thread per particle, global atomics (`block` threads per workgroup);
// modes 1-5: LDS-privatised chunks of 1024 / 2048 / 4096 particles with 256 threads, 4096
// with 512 threads, 8192 with 1024 threads.
hipError_t launch_deposit(const float* pos, unsigned long long* rho, int64_t np, int nbox, int n,
                          double inv_cell, int* flags, int mode, int block, hipStream_t s) {
  switch (mode) {
    case 1: return launch_tiled<1024, 3328, 256>(pos, rho, np, nbox, n, inv_cell, flags, s);
    case 2: return launch_tiled<2048, 5120, 256>(pos, rho, np, nbox, n, inv_cell, flags, s);
    case 3: return launch_tiled<4096, 9216, 256>(pos, rho, np, nbox, n, inv_cell, flags, s);
    case 4: return launch_tiled<4096, 9216, 512>(pos, rho, np, nbox, n, inv_cell, flags, s);
    case 5: return launch_tiled<8192, 18432, 1024>(pos, rho, np, nbox, n, inv_cell, flags, s);
    default:
      hipLaunchKernelGGL(deposit_kernel, dim3(grid_blocks(np * nbox, block, 1)), dim3(block), 0,
                         s, pos, rho, np, nbox, n, inv_cell, flags);
      return hipGetLastError();
  }
}

int patch_cb_log2(int n) { return n >= 16 ? 4 : 3; }
int64_t patch_coarse_cells(int n) {
  const int64_t nc = n >> patch_cb_log2(n);
  return nc * nc * nc;
}
int64_t patch_chunks(int64_t np) { return (np + kPatchCH - 1) / kPatchCH; }

hipError_t launch_deposit_patch(const float* pos, unsigned long long* patches, int* reg_count,
                                int4* reg_list, unsigned long long* rho_fb, int* n_fb,
                                int64_t np, int nbox, int n, double inv_cell, int* flags,
                                bool big_tile, hipStream_t s) {
  if (n > 1024) return hipErrorInvalidValue;     // registry entries pack indices in 10 bits
  const int64_t chunks = patch_chunks(np);
  const dim3 grid(static_cast<unsigned>(chunks * nbox));
  if (big_tile)
    hipLaunchKernelGGL((deposit_patch_kernel<kPatchCH, kPatchCap, kPatchNT>), grid,
                       dim3(kPatchNT), 0, s, pos, patches, reg_count, reg_list, rho_fb, n_fb,
                       np, n, inv_cell, flags, chunks, patch_cb_log2(n));
  else
    hipLaunchKernelGGL((deposit_patch_kernel<kPatchCH, kPatchTile, kPatchNT>), grid,
                       dim3(kPatchNT), 0, s, pos, patches, reg_count, reg_list, rho_fb, n_fb,
                       np, n, inv_cell, flags, chunks, patch_cb_log2(n));
  return hipGetLastError();
}

hipError_t launch_patch_reduce(const unsigned long long* patches, const int* reg_count,
                               const int4* reg_list, unsigned long long* rho_fb,
                               const int* n_fb, float* delta, int nbox, int n, double scale,
                               hipStream_t s) {
  // slabs of 8 x-planes: half a 16^3 cell (a whole 8^3 one)
  const int slabs = (1 << patch_cb_log2(n)) / 8;
  hipLaunchKernelGGL(patch_reduce_kernel<8>,
                     dim3(static_cast<unsigned>(patch_coarse_cells(n) * slabs), nbox), dim3(256),
                     0, s, patches, kPatchCap, reg_count, reg_list, rho_fb, n_fb, delta, n,
                     patch_cb_log2(n), scale);
  return hipGetLastError();
}

hipError_t launch_delta_to_density(const float* delta, float* out, int64_t n, float rho_bar,
                                   hipStream_t s) {
  int blocks = static_cast<int>(std::min<int64_t>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(delta_to_density_kernel, dim3(blocks), dim3(256), 0, s, delta, out, n,
                     rho_bar);
  return hipGetLastError();
}

// Blocks rounded up to whole XCD rounds; the extra blocks exit at once.
int xcd_blocks(int64_t nchunks) { return static_cast<int>((nchunks + 7) / 8 * 8); }

template <int CH, int CAP>
hipError_t launch_interp_tiled(const float* pos, const float* force, float* acc, int64_t np,
                               int nbox, int n, double inv_cell, const Leap* lp, hipStream_t s) {
  const int64_t chunks = (np + CH - 1) / CH;
  const dim3 grid(xcd_blocks(chunks * nbox));
  if (lp)
    hipLaunchKernelGGL((interp_tiled_kernel<CH, CAP, true>), grid, dim3(256), 0, s, pos, force,
                       acc, np, n, inv_cell, chunks, chunks * nbox, *lp);
  else
    hipLaunchKernelGGL((interp_tiled_kernel<CH, CAP, false>), grid, dim3(256), 0, s, pos, force,
                       acc, np, n, inv_cell, chunks, chunks * nbox, Leap());
  return hipGetLastError();
}

template <int PPT>
hipError_t launch_interp_direct(const float* pos, const float* force, float* acc, int64_t np,
                                int nbox, int n, double inv_cell, const Leap* lp,
                                hipStream_t s) {
  const int64_t chunks = (np + 256 * PPT - 1) / (256 * PPT);
  const dim3 grid(xcd_blocks(chunks * nbox));
  if (lp)
    hipLaunchKernelGGL((interp_kernel<PPT, true>), grid, dim3(256), 0, s, pos, force, acc, np, n,
                       inv_cell, chunks, chunks * nbox, *lp);
  else
    hipLaunchKernelGGL((interp_kernel<PPT, false>), grid, dim3(256), 0, s, pos, force, acc, np,
                       n, inv_cell, chunks, chunks * nbox, Leap());
  return hipGetLastError();
}

// mode 0: direct gather, `block` = particles per workgroup (256, 512 or 1024);
// modes 1-3: LDS-staged boxes of 1024 / 2048 / 4096 particles (mode 1's tile of 2048 nodes,
// 24 KB, leaves room for six workgroups per CU). lp (may be NULL): the leapfrog applied
// with each acceleration.
hipError_t launch_interp(const float* pos, const float* force, float* acc, int64_t np,
                         int nbox, int n, double inv_cell, int mode, int block, hipStream_t s,
                         const Leap* lp) {
  switch (mode) {
    case 1: return launch_interp_tiled<1024, 2048>(pos, force, acc, np, nbox, n, inv_cell, lp, s);
    case 2: return launch_interp_tiled<2048, 4608>(pos, force, acc, np, nbox, n, inv_cell, lp, s);
    case 3: return launch_interp_tiled<4096, 8192>(pos, force, acc, np, nbox, n, inv_cell, lp, s);
    default:
      if (block >= 1024)
        return launch_interp_direct<4>(pos, force, acc, np, nbox, n, inv_cell, lp, s);
      if (block >= 512)
        return launch_interp_direct<2>(pos, force, acc, np, nbox, n, inv_cell, lp, s);
      return launch_interp_direct<1>(pos, force, acc, np, nbox, n, inv_cell, lp, s);
  }
}

}  // namespace pmnu
