// 3-D real FFT passes of the PM step, with the k-binning fused into the last forward pass
// and the neutrino rescale, Green's function and first gradient factor fused into the
// first inverse pass (gfx950, FP32 data, FP64 bin sums).
//
// Layouts (per box b):
//   real grid      [b][x][y][z]                 (z contiguous)
//   y-side fields  [b][kz][x][ky], kz in [0, N/2], x, ky in [0, N)   (ky contiguous)
//   z-side fields  [b][x][kz][ky]               (the planes next to the real grid)
// Every row is a power of two long and aligned. The passes along z work inside one
// contiguous x-slab of the z-side layout; the passes along y move whole rows between the
// two complex layouts (transposing [x][kz] <-> [kz][x] at row granularity); the passes
// along x work inside one contiguous kz-slab. numpy's rfftn order [kx][ky][kz] is
// produced only by launch_copy_modes.
//
// Forward:  fwd_z   delta (from the fixed-point density, or given in FP32), real rows
//                   along z -> half spectra (two rows per complex FFT), written as
//                   [x][kz][y]
//           fwd_y   complex FFT of every contiguous y row, written to [kz][x][ky]
//           fwd_x   complex FFT along x (tile of N x TX) in LDS and the FP64 mode sums
//                   per k-bin: sum w |delta_k|^2, w = 1 on the kz = 0, N/2 planes, else 2;
//                   the transformed tile is not stored (the inverse pass redoes it,
//                   which costs arithmetic but saves writing the whole field)
// Inverse:  inv_x   FFT along x again, delta_M = T(|n|^2) delta_cdm,
//                   phi = -C delta_M/(k^2 W^2), and the two fields F1 = phi,
//                   F2 = -i k_x phi, inverse FFT along kx
//           inv_y   G1 = IFFT_y F1, G2 = IFFT_y(-i k_y F1), G3 = IFFT_y F2, written to
//                   [x][kz][y]
//           inv_z   complex-to-real along z of -i k_z G1, G2, G3 (two rows per complex
//                   FFT), transposed back to [x][y][z] with the three acceleration
//                   components (g_x, g_y, g_z) interleaved per node
// Since the derivative along an axis commutes with the transforms along the other axes,
// this needs 2 + 3 intermediate fields instead of 3 + 3 + 3.
// Where a plane or slab fits the LDS, two passes run as one kernel with the same arithmetic:
// fwd_zy (N <= 128, per x-plane), inv_xy (N <= 64, per kz-slab) and inv_yz (N <= 64, per
// x-plane, after inv_x); patch_fwd_z does the patch deposit's sums and fwd_z in one kernel.
#include <type_traits>

#include "fft_lds.hpp"
#include "patch_device.hpp"

namespace pmnu {
namespace {

constexpr int NT = 256;

template <int N> struct Shape {
  static constexpr int NK = N / 2 + 1;
  static constexpr int FZ_TY = N <= 32 ? N : (N <= 256 ? 32 : 16);   // real rows per WG
  static constexpr int FY_NL = N <= 256 ? (N < 16 ? N : 16) : 8;      // rows per WG
  static constexpr int FX_TX = N < 16 ? N : (N <= 256 ? 16 : 8);      // ky columns per WG
  static constexpr int IX_TX = N < 16 ? N : 8;
  static constexpr int IY_NL = N < 8 ? N : 4;
  static constexpr int IZ_TY = N < 16 ? N : (N <= 256 ? 16 : 8);
};

// Tile candidates of every pass for the autotuner: [0] is Shape's default, [1] and [2] the
// alternatives (below N = 64 the tiles stay fixed). All fit the LDS of one CU and give each
// transform line the same arithmetic, so every candidate computes the same result.
template <int N> struct Tiles {
  static constexpr bool kFixed = N < 64;
  static constexpr int alt(int d, int a) { return kFixed ? d : a; }
  static constexpr int FZ[3] = {Shape<N>::FZ_TY, alt(Shape<N>::FZ_TY, Shape<N>::FZ_TY / 2),
                                alt(Shape<N>::FZ_TY, Shape<N>::FZ_TY * 2)};
  static constexpr int FY[3] = {Shape<N>::FY_NL, alt(Shape<N>::FY_NL, Shape<N>::FY_NL / 2),
                                alt(Shape<N>::FY_NL, Shape<N>::FY_NL < 16 ? Shape<N>::FY_NL * 2
                                                                          : Shape<N>::FY_NL / 4)};
  static constexpr int FX[3] = {Shape<N>::FX_TX, alt(Shape<N>::FX_TX, Shape<N>::FX_TX == 16 ? 8 : 16),
                                alt(Shape<N>::FX_TX, Shape<N>::FX_TX == 16 ? 32 : 4)};
  static constexpr int IX[3] = {Shape<N>::IX_TX, alt(Shape<N>::IX_TX, 4), alt(Shape<N>::IX_TX, 16)};
  static constexpr int IY[3] = {Shape<N>::IY_NL, alt(Shape<N>::IY_NL, 2), alt(Shape<N>::IY_NL, 8)};
  static constexpr int IZ[3] = {Shape<N>::IZ_TY, alt(Shape<N>::IZ_TY, Shape<N>::IZ_TY == 16 ? 8 : 16),
                                alt(Shape<N>::IZ_TY, Shape<N>::IZ_TY == 16 ? 32 : 4)};
};

__device__ __forceinline__ int signed_index(int i, int n) { return i < n / 2 ? i : i - n; }

// ------------------------------------------------------------------------ forward ----
// Input: the fixed-point density (DELTA = false; delta = rho / rho_bar - 1 is formed here
// from the exact sum and rounded once to FP32) or delta already in FP32 (DELTA = true;
// then thread 0 of the first workgroup also moves the side-grid counter of the patch
// deposit, whose last reader ran before this kernel, into its running total).
template <int N, bool DELTA, int TY>
__global__ __launch_bounds__(NT) void fwd_z_kernel(const void* __restrict__ in,
                                                   float2* __restrict__ out,
                                                   const float2* __restrict__ twg,
                                                   double scale, int* __restrict__ reset,
                                                   int* __restrict__ clear, int n_clear) {
  constexpr int NL = TY / 2, ES = NL + 1, NK = Shape<N>::NK;
  __shared__ float2 lds[N * ES];
  __shared__ float2 tw[N];
  const int y0 = blockIdx.x * TY, x = blockIdx.y, box = blockIdx.z;
  load_twiddles<N, NT>(tw, twg);
  const size_t off = ((static_cast<size_t>(box) * N + x) * N + y0) * N;
  float* ldsf = reinterpret_cast<float*>(lds);
  if constexpr (DELTA) {
    if (reset && threadIdx.x == 0 && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0) {
      reset[1] += reset[0];
      reset[0] = 0;
    }
    // the patch registry's counts, read for the last time by the reduce before this kernel
    const int64_t gid =
        ((static_cast<int64_t>(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) *
            NT + threadIdx.x;
    if (clear && gid < n_clear) clear[gid] = 0;
    const float4* src = reinterpret_cast<const float4*>(static_cast<const float*>(in) + off);
    constexpr int IT = (TY * N / 4 + NT - 1) / NT;
    float4 v[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = threadIdx.x + i * NT;
      if (t < TY * N / 4) v[i] = src[t];
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = threadIdx.x + i * NT;
      if (t >= TY * N / 4) break;
      const int row = (4 * t) / N, e = (4 * t) % N, sl = row & 1, p = row >> 1;
      ldsf[(e * ES + p) * 2 + sl] = v[i].x;
      ldsf[((e + 1) * ES + p) * 2 + sl] = v[i].y;
      ldsf[((e + 2) * ES + p) * 2 + sl] = v[i].z;
      ldsf[((e + 3) * ES + p) * 2 + sl] = v[i].w;
    }
  } else {
    const ulonglong2* src =
        reinterpret_cast<const ulonglong2*>(static_cast<const unsigned long long*>(in) + off);
    for (int t = threadIdx.x; t < TY * N / 2; t += NT) {
      const int row = (2 * t) / N, e = (2 * t) % N;
      const ulonglong2 v = src[t];
      // delta = rho / rho_bar - 1 from the exact fixed-point sum, rounded once to FP32
      ldsf[(e * ES + (row >> 1)) * 2 + (row & 1)] =
          static_cast<float>(static_cast<double>(v.x) * scale - 1.0);
      ldsf[((e + 1) * ES + (row >> 1)) * 2 + (row & 1)] =
          static_cast<float>(static_cast<double>(v.y) * scale - 1.0);
    }
  }
  __syncthreads();
  fft_lines<N, NL, NT, -1>(lds, tw);
  for (int t = threadIdx.x; t < NK * TY; t += NT) {
    const int row = t % TY, k = t / TY, p = row >> 1;
    const float2 zk = lds[k * ES + p];
    const float2 zn = cconj(lds[((N - k) & (N - 1)) * ES + p]);
    float2 r;
    if ((row & 1) == 0) {
      r = cscale(cadd(zk, zn), 0.5f);                       // A = (Z_k + conj Z_{N-k})/2
    } else {
      const float2 d = csub(zk, zn);                        // B = (Z_k - conj Z_{N-k})/(2i)
      r = make_float2(0.5f * d.y, -0.5f * d.x);
    }
    out[((static_cast<size_t>(box) * N + x) * NK + k) * N + y0 + row] = r;
  }
}

// The patch deposit's second half and the first forward pass in one kernel (deposit modes
// 8 and 9): the per-patch fixed-point sums are added up for a slab of the mesh and
// transformed along z before delta ever reaches HBM. One workgroup per (x-plane, group of
// CB = 16 y-rows, box): its slab is one x-plane of a column of N / CB coarse cells.
//   1. Every cell's registry count and list row are loaded together (a half-wave per cell,
//      all cells in one round); per cell the patch with the largest overlap of the slab
//      (its "home") is chosen, and every other overlap is counted in boxes (up to two
//      periodic pieces per axis) and nodes, kept per list entry in LDS.
//   2. Each thread loads the CB z-nodes of its (row, cell) runs from their home patches into
//      registers; meanwhile one workgroup-wide scan turns the entries' piece and node
//      counts into offsets, the entries write their pieces into one flat list, and every
//      thread walks that list's nodes (a bisection finds a node's piece), all of its loads
//      issued before any add, into an LDS copy of the slab with 64-bit LDS atomics. The
//      list holds kPieces; a slab with more (crowded registries) takes several windows of
//      whole entries.
//   3. Registers + LDS (+ the side grid when anything went there, which is then cleared) give
//      the exact integer sum of each node, rounded once to delta = rho / rho_bar - 1 in FP32;
//      the slab's 16 rows become 8 complex lines (rows 2p and 2p + 1 as real and imaginary
//      parts) over the LDS the sums used, and the z transform and the split into the two real
//      rows' half spectra follow as in fwd_z_kernel. The output is that of
//      patch_reduce_kernel + fwd_z_kernel bit for bit.
// With delta_out the slab's delta is also stored (only for reading the density back).
// The registry counts and the side-grid count are reset by the next pass (fwd_y): the other
// x-planes of a cell read them until this kernel ends. Workgroups of one cell column (the
// 16 x-planes that read the same patches) run on one XCD, so its L2 serves their halos.
constexpr int kPatchFwdNT = 512;   // threads per workgroup of patch_fwd_z_kernel
template <int N>
__global__ __launch_bounds__(kPatchFwdNT) void patch_fwd_z_kernel(
    const unsigned long long* __restrict__ patches, int pcap, const int* __restrict__ reg_count,
    const int4* __restrict__ reg_list, unsigned long long* __restrict__ rho_fb,
    const int* __restrict__ n_fb, float2* __restrict__ out, const float2* __restrict__ twg,
    double scale, float* __restrict__ delta_out) {
  constexpr int NT = kPatchFwdNT;                  // this kernel's workgroup size
  constexpr int CB = 16, NC = N / CB, TY = CB, NL = TY / 2, ES = NL + 1, NK = Shape<N>::NK;
  constexpr int RUNS = TY * NC;                    // (row, cell) runs of CB z-nodes
  constexpr int RG = NT / CB;                      // runs a workgroup covers at once
  constexpr int JPT = RUNS / RG;                   // nodes per thread: z = tid % CB of runs
                                                   // r = tid / CB + RG j, j < JPT
  constexpr int NE = NC * kPatchList;              // list entries of the column's cells
  constexpr int EPT = (NE + NT - 1) / NT;          // entries per thread in the scan
  constexpr int kPieces = 256, kBatch = 8;         // piece list capacity (power of two)
  static_assert(NC >= 2 && RUNS % RG == 0, "runs cover the threads evenly");
  static_assert(NE % NT == 0 || NE < NT, "entries cover the threads evenly");
  static_assert(N * ES * sizeof(float2) <= TY * N * sizeof(unsigned long long),
                "the complex lines fit over the sums");
  __shared__ unsigned long long s_acc[TY * N];     // [y][z]; later the complex lines
  __shared__ float2 tw[N];
  __shared__ int4 s_home[NC];                      // chunk < 0: no patch
  __shared__ int4 s_ent[NE];                       // list entries (chunk < 0: none)
  __shared__ int s_np[NE + 1], s_ni[NE + 1];       // their pieces and nodes -> offsets
  __shared__ int p_off[kPieces + 1];
  __shared__ int p_dim[kPieces];
  __shared__ long long p_src[kPieces];
  __shared__ int p_dst[kPieces];
  __shared__ int s_wsum[2][NT / 64];
  __shared__ int s_win[2];                         // current window: first, end entry
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // block -> (box, cell column, x within the column, y group): consecutive dispatch ids go
  // to the 8 XCDs in turn, so each XCD takes a contiguous run of virtual ids instead
  const int nb = gridDim.x, per = nb / 8;
  const int vid = static_cast<int>(blockIdx.x) < per * 8
                      ? static_cast<int>(blockIdx.x % 8) * per + static_cast<int>(blockIdx.x / 8)
                      : static_cast<int>(blockIdx.x);
  const int xi = vid % CB, col = vid / CB;         // col = (cx, cy) of the cell column
  const int cy = col % NC, cx = col / NC;
  const int64_t box = blockIdx.y;
  const int x = cx * CB + xi, y0 = cy * CB;
  const int64_t cells = static_cast<int64_t>(NC) * NC * NC;
  const int64_t cell0 = box * cells + (static_cast<int64_t>(cx) * NC + cy) * NC;  // cz = 0
  // overlap of a registry entry with the slab's part of cell c
  auto pieces_of = [&](const int4& en, int c, Pieces& px, Pieces& py, Pieces& pz) {
    px = overlap(en.y & 1023, en.z & 1023, x, 1, N);
    py = overlap((en.y >> 10) & 1023, (en.z >> 10) & 1023, y0, CB, N);
    pz = overlap(en.y >> 20, en.z >> 20, c * CB, CB, N);
  };
  load_twiddles<N, NT>(tw, twg);
  for (int i = tid; i < TY * N; i += NT) s_acc[i] = 0ull;
  // 1. every cell's count and list row in one round: half-wave h of wave w takes the cells
  //    c = 2 w + h + 2 (NT / 64) i
  {
    constexpr int CPR = 2 * (NT / 64);             // cells per round
    constexpr int ROUNDS = (NC + CPR - 1) / CPR;
    int cnt[ROUNDS];
    int4 listed[ROUNDS];
#pragma unroll
    for (int i = 0; i < ROUNDS; ++i) {
      const int c = 2 * wave + (lane >> 5) + CPR * i;
      cnt[i] = 0;
      listed[i] = make_int4(-1, 0, 0, 0);
      if (c < NC) {
        cnt[i] = reg_count[cell0 + c];
        listed[i] = reg_list[(cell0 + c) * kPatchList + (lane & 31)];
      }
    }
#pragma unroll
    for (int i = 0; i < ROUNDS; ++i) {
      const int c = 2 * wave + (lane >> 5) + CPR * i, e = lane & 31;
      const bool mine = c < NC && e < min(cnt[i], kPatchList);
      int vol = 0, np = 0;
      if (mine) {
        Pieces px, py, pz;
        pieces_of(listed[i], c, px, py, pz);
        int lx = 0, ly = 0, lz = 0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          lx += q < px.cnt ? px.len[q] : 0;
          ly += q < py.cnt ? py.len[q] : 0;
          lz += q < pz.cnt ? pz.len[q] : 0;
        }
        vol = lx * ly * lz;
        np = px.cnt * py.cnt * pz.cnt;
      }
      // home: the largest volume, ties to the lowest lane
      int key = vol > 0 ? (vol << 6) | (63 - lane) : -1;
#pragma unroll
      for (int off = 16; off > 0; off >>= 1) key = max(key, __shfl_xor(key, off, 64));
      const bool home = key >= 0 && lane == 63 - (key & 63);
      if (c < NC) {
        if (e == 0 && key < 0) s_home[c] = make_int4(-1, 0, 0, 0);
        if (home) s_home[c] = listed[i];
        const int slot = c * kPatchList + e;
        const bool other = mine && vol > 0 && !home;
        s_ent[slot] = other ? listed[i] : make_int4(-1, 0, 0, 0);
        s_np[slot] = other ? np : 0;
        s_ni[slot] = other ? vol : 0;
      }
    }
  }
  __syncthreads();
  // 2a. the home patches' loads go out first: run r = cell * TY + row; lanes of a wave
  //     take consecutive z of four runs (rows of one cell: neighbouring patch rows)
  const int zt = tid % CB;
  unsigned long long hv[JPT];
#pragma unroll
  for (int j = 0; j < JPT; ++j) {
    const int r = tid / CB + RG * j, c = r / TY, row = r % TY;
    hv[j] = 0ull;
    const int4 hl = s_home[c];
    if (hl.x < 0) continue;
    const int ey = (hl.z >> 10) & 1023, ez = hl.z >> 20;
    Pieces px, py, pz;
    pieces_of(hl, c, px, py, pz);
    int lx = -1, ly = -1, lz = -1;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k < px.cnt && px.cl[k] == 0) lx = px.pl[k];
      if (k < py.cnt && row >= py.cl[k] && row < py.cl[k] + py.len[k])
        ly = py.pl[k] + row - py.cl[k];
      if (k < pz.cnt && zt >= pz.cl[k] && zt < pz.cl[k] + pz.len[k]) lz = pz.pl[k] + zt - pz.cl[k];
    }
    if (lx >= 0 && ly >= 0 && lz >= 0)
      hv[j] = patches[static_cast<int64_t>(hl.x) * pcap +
                      (static_cast<int64_t>(lx) * ey + ly) * ez + lz];
  }
  // 2b. exclusive scan of the entries' piece and node counts (thread t: EPT consecutive
  //     entries), s_np / s_ni become offsets, [NE] the totals
  {
    int lp[EPT], li[EPT], sp = 0, si = 0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int en = tid * EPT + k;
      lp[k] = en < NE ? s_np[en] : 0;
      li[k] = en < NE ? s_ni[en] : 0;
      sp += lp[k];
      si += li[k];
    }
    int ip = sp, ii = si;                          // inclusive scan over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int tp = __shfl_up(ip, off, 64), ti = __shfl_up(ii, off, 64);
      if (lane >= off) {
        ip += tp;
        ii += ti;
      }
    }
    if (lane == 63) {
      s_wsum[0][wave] = ip;
      s_wsum[1][wave] = ii;
    }
    __syncthreads();
    int bp = 0, bi = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
      if (w < wave) {
        bp += s_wsum[0][w];
        bi += s_wsum[1][w];
      }
    }
    int op = bp + ip - sp, oi = bi + ii - si;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int en = tid * EPT + k;
      if (en < NE) {
        s_np[en] = op;
        s_ni[en] = oi;
      }
      op += lp[k];
      oi += li[k];
    }
    if (tid == NT - 1) {
      s_np[NE] = op;
      s_ni[NE] = oi;
    }
    if (tid == 0) s_win[1] = 0;
  }
  __syncthreads();
  // 2c. windows of whole entries whose pieces fit the list (one window unless crowded)
  while (true) {
    if (tid == 0) {
      // the last entry boundary e1 with pieces [e0, e1) <= kPieces (offsets are monotone)
      const int e0 = s_win[1], lim = s_np[e0] + kPieces;
      int e1 = NE;
      if (s_np[NE] > lim) {
        int lo = e0, hi = NE;                    // s_np[lo] <= lim < s_np[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_np[mid] <= lim) lo = mid;
          else hi = mid;
        }
        e1 = lo;
      }
      s_win[0] = e0;
      s_win[1] = e1;
    }
    __syncthreads();
    const int e0 = s_win[0], e1 = s_win[1];
    if (e0 >= NE) break;
    const int pbase = s_np[e0], ibase = s_ni[e0];
    const int n_pieces = s_np[e1] - pbase, total = s_ni[e1] - ibase;
    for (int en = e0 + tid; en < e1; en += NT) {
      const int4 en4 = s_ent[en];
      if (en4.x < 0) continue;
      const int c = en / kPatchList;
      Pieces px, py, pz;
      pieces_of(en4, c, px, py, pz);
      const int ey = (en4.z >> 10) & 1023, ez = en4.z >> 20;
      const long long src0 = static_cast<long long>(en4.x) * pcap;
      int slot = s_np[en] - pbase, item = s_ni[en] - ibase;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int cc = 0; cc < 2; ++cc) {
            if (a >= px.cnt || b >= py.cnt || cc >= pz.cnt) continue;
            const int Ly = py.len[b], Lz = pz.len[cc];   // Lx = 1: the slab is one plane
            p_off[slot] = item;
            p_dim[slot] = Lz | (ez << 8);
            p_src[slot] = src0 + (static_cast<long long>(px.pl[a]) * ey + py.pl[b]) * ez + pz.pl[cc];
            // LDS node (y, z) of the piece's first node
            p_dst[slot] = py.cl[b] * N + c * CB + pz.cl[cc];
            item += Ly * Lz;
            ++slot;
          }
    }
    for (int i = n_pieces + tid; i <= kPieces; i += NT) p_off[i] = 0x7fffffff;
    __syncthreads();
    for (int base = 0; base < total; base += kBatch * NT) {
      unsigned long long v[kBatch];
      int li[kBatch];
#pragma unroll
      for (int r = 0; r < kBatch; ++r) {
        const int i = base + r * NT + tid;
        li[r] = -1;
        v[r] = 0ull;
        if (i < total) {
          int pe = 0;                             // the piece: last offset <= i
#pragma unroll
          for (int step = kPieces / 2; step > 0; step >>= 1)
            if (p_off[pe + step] <= i) pe += step;
          const int rem = i - p_off[pe];
          const int dim = p_dim[pe], Lz = dim & 255, ez = dim >> 8;
          // exact: rem < 256 and Lz <= 16 (x is one plane, so rem = y Lz + z)
          const int y = static_cast<int>((rem + 0.5f) * (1.0f / Lz));
          const int z = rem - y * Lz;
          v[r] = patches[p_src[pe] + y * ez + z];
          li[r] = p_dst[pe] + y * N + z;
        }
      }
#pragma unroll
      for (int r = 0; r < kBatch; ++r)
        if (li[r] >= 0) atomicAdd(&s_acc[li[r]], v[r]);
    }
    __syncthreads();                               // before the next window's list
  }
  // 3. exact sums -> delta, then the z transform over the same LDS
  const bool fold = *n_fb > 0;
  const int64_t m = static_cast<int64_t>(N) * N * N;
  float dv[JPT];
#pragma unroll
  for (int j = 0; j < JPT; ++j) {
    const int r = tid / CB + RG * j, c = r / TY, row = r % TY;
    unsigned long long val = hv[j] + s_acc[row * N + c * CB + zt];
    const int64_t node = box * m + (static_cast<int64_t>(x) * N + y0 + row) * N + c * CB + zt;
    if (fold) {
      val += rho_fb[node];
      rho_fb[node] = 0ull;
    }
    dv[j] = static_cast<float>(static_cast<double>(val) * scale - 1.0);
    if (delta_out) delta_out[node] = dv[j];        // kept for reading the density back
  }
  __syncthreads();
  float2* lds = reinterpret_cast<float2*>(s_acc);
  float* ldsf = reinterpret_cast<float*>(s_acc);
#pragma unroll
  for (int j = 0; j < JPT; ++j) {
    const int r = tid / CB + RG * j, c = r / TY, row = r % TY;
    ldsf[((c * CB + zt) * ES + (row >> 1)) * 2 + (row & 1)] = dv[j];
  }
  __syncthreads();
  fft_lines<N, NL, NT, -1>(lds, tw);
  for (int t = tid; t < NK * TY; t += NT) {
    const int row = t % TY, k = t / TY, p = row >> 1;
    const float2 zk = lds[k * ES + p];
    const float2 zn = cconj(lds[((N - k) & (N - 1)) * ES + p]);
    float2 rr;
    if ((row & 1) == 0) {
      rr = cscale(cadd(zk, zn), 0.5f);
    } else {
      const float2 d = csub(zk, zn);
      rr = make_float2(0.5f * d.y, -0.5f * d.x);
    }
    out[((box * N + x) * NK + k) * N + y0 + row] = rr;
  }
}

// After the fused patch pass (patch_fwd_z_kernel) it also does the patch registry's
// end-of-step work that fwd_z does otherwise: reset (n_fb: this step's side-grid count
// into the running total) and clear (the registry counts), when given.
template <int N, int NL>
__global__ __launch_bounds__(NT) void fwd_y_kernel(const float2* __restrict__ in,
                                                   float2* __restrict__ out,
                                                   const float2* __restrict__ twg,
                                                   int* __restrict__ reset,
                                                   int* __restrict__ clear, int n_clear) {
  constexpr int ES = NL + 1, NK = Shape<N>::NK;
  __shared__ float2 lds[N * ES];
  __shared__ float2 tw[N];
  if (reset && threadIdx.x == 0 && blockIdx.x == 0) {
    reset[1] += reset[0];
    reset[0] = 0;
  }
  if (clear) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
    if (gid < n_clear) clear[gid] = 0;
  }
  load_twiddles<N, NT>(tw, twg);
  const size_t r0 = static_cast<size_t>(blockIdx.x) * NL;
  const float4* src = reinterpret_cast<const float4*>(in + r0 * N);
  // all of a thread's loads in flight before the LDS stores
  constexpr int IT = (NL * N / 2 + NT - 1) / NT;
  float4 v[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t < NL * N / 2) v[i] = src[t];
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t < NL * N / 2) {
      const int e = (2 * t) % N, l = (2 * t) / N;
      lds[e * ES + l] = make_float2(v[i].x, v[i].y);
      lds[(e + 1) * ES + l] = make_float2(v[i].z, v[i].w);
    }
  }
  __syncthreads();
  fft_lines<N, NL, NT, -1>(lds, tw);
  for (int t = threadIdx.x; t < NL * N / 2; t += NT) {
    const int e = (2 * t) % N, l = (2 * t) / N;
    const size_t r = r0 + l;
    const size_t box = r / (static_cast<size_t>(N) * NK), rem = r % (static_cast<size_t>(N) * NK);
    const size_t x = rem / NK, kz = rem % NK;
    const float2 a = lds[e * ES + l], b = lds[(e + 1) * ES + l];
    *reinterpret_cast<float4*>(out + ((box * NK + kz) * N + x) * N + e) =
        make_float4(a.x, a.y, b.x, b.y);
  }
}

// For N <= 128 the first two forward passes in one kernel, one workgroup per (x-plane, box):
// the plane (N rows of y by N z) fits the LDS. Its rows are transformed along z as in
// fwd_z_kernel (rows 2p and 2p + 1 as one complex line, then split into the two real rows'
// half spectra), the half spectra go through registers to lines along y (one per k_z), are
// transformed as in fwd_y_kernel and written to [box][k_z][x][k_y]. The same arithmetic in the
// same order as the two passes, so the same modes bit for bit; the z-transformed plane never
// reaches HBM. With DELTA it also does fwd_z_kernel's registry work (reset, clear).
constexpr int kFwdZYNT = 256;   // threads per workgroup of fwd_zy_kernel
template <int N, bool DELTA>
__global__ __launch_bounds__(kFwdZYNT) void fwd_zy_kernel(const void* __restrict__ in,
                                                          float2* __restrict__ out,
                                                          const float2* __restrict__ twg,
                                                          double scale, int* __restrict__ reset,
                                                          int* __restrict__ clear, int n_clear) {
  constexpr int NT = kFwdZYNT;                     // this kernel's workgroup size
  constexpr int NL = N / 2, ES = NL + 1, NK = Shape<N>::NK, ES2 = NK + 1;
  constexpr int LDS_N = N * (ES > ES2 ? ES : ES2);
  constexpr int PER = (NK * N + NT - 1) / NT;      // half-spectrum values per thread
  static_assert(N <= 128, "the plane must fit the LDS");
  __shared__ float2 lds[LDS_N];
  __shared__ float2 tw[N];
  const int x = blockIdx.x, box = blockIdx.y, tid = threadIdx.x;
  load_twiddles<N, NT>(tw, twg);
  const size_t off = (static_cast<size_t>(box) * N + x) * N * N;   // the plane, [y][z]
  float* ldsf = reinterpret_cast<float*>(lds);
  if constexpr (DELTA) {
    if (reset && tid == 0 && blockIdx.x == 0 && blockIdx.y == 0) {
      reset[1] += reset[0];
      reset[0] = 0;
    }
    // the patch registry's counts, read for the last time by the reduce before this kernel
    const int64_t gid = (static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * NT + tid;
    if (clear && gid < n_clear) clear[gid] = 0;
    const float4* src = reinterpret_cast<const float4*>(static_cast<const float*>(in) + off);
    constexpr int IT = (N * N / 4 + NT - 1) / NT;
    float4 v[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * NT;
      if (t < N * N / 4) v[i] = src[t];
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * NT;
      if (t >= N * N / 4) break;
      const int row = (4 * t) / N, e = (4 * t) % N, sl = row & 1, p = row >> 1;
      ldsf[(e * ES + p) * 2 + sl] = v[i].x;
      ldsf[((e + 1) * ES + p) * 2 + sl] = v[i].y;
      ldsf[((e + 2) * ES + p) * 2 + sl] = v[i].z;
      ldsf[((e + 3) * ES + p) * 2 + sl] = v[i].w;
    }
  } else {
    const ulonglong2* src =
        reinterpret_cast<const ulonglong2*>(static_cast<const unsigned long long*>(in) + off);
    for (int t = tid; t < N * N / 2; t += NT) {
      const int row = (2 * t) / N, e = (2 * t) % N;
      const ulonglong2 v = src[t];
      // delta = rho / rho_bar - 1 from the exact fixed-point sum, rounded once to FP32
      ldsf[(e * ES + (row >> 1)) * 2 + (row & 1)] =
          static_cast<float>(static_cast<double>(v.x) * scale - 1.0);
      ldsf[((e + 1) * ES + (row >> 1)) * 2 + (row & 1)] =
          static_cast<float>(static_cast<double>(v.y) * scale - 1.0);
    }
  }
  __syncthreads();
  fft_lines<N, NL, NT, -1>(lds, tw);
  // the two rows' half spectra, value t = (k_z, y) held in registers
  float2 h[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int t = tid + i * NT;
    h[i] = make_float2(0.f, 0.f);
    if (t < NK * N) {
      const int row = t % N, k = t / N, p = row >> 1;
      const float2 zk = lds[k * ES + p];
      const float2 zn = cconj(lds[((N - k) & (N - 1)) * ES + p]);
      if ((row & 1) == 0) {
        h[i] = cscale(cadd(zk, zn), 0.5f);               // A = (Z_k + conj Z_{N-k})/2
      } else {
        const float2 d = csub(zk, zn);                   // B = (Z_k - conj Z_{N-k})/(2i)
        h[i] = make_float2(0.5f * d.y, -0.5f * d.x);
      }
    }
  }
  __syncthreads();
  // line k_z, element y
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int t = tid + i * NT;
    if (t < NK * N) lds[(t % N) * ES2 + t / N] = h[i];
  }
  __syncthreads();
  fft_lines<N, NK, NT, -1, ES2>(lds, tw);
  for (int t = tid; t < NK * N / 2; t += NT) {
    const int kz = t / (N / 2), e = 2 * (t % (N / 2));
    const float2 a = lds[e * ES2 + kz], b = lds[(e + 1) * ES2 + kz];
    *reinterpret_cast<float4*>(out + ((static_cast<size_t>(box) * NK + kz) * N + x) * N + e) =
        make_float4(a.x, a.y, b.x, b.y);
  }
}

// STORE: write the transformed tile back (only for reading the modes out); BIN: the mode
// sums per k-bin (the step bins without storing; the inverse pass redoes the x transform).
template <int N, bool STORE, bool BIN, int TX>
__global__ __launch_bounds__(NT) void fwd_x_bin_kernel(float2* __restrict__ data,
                                                       const float2* __restrict__ twg,
                                                       const uint16_t* __restrict__ bin_of_n2,
                                                       double* __restrict__ partial, int nbins) {
  constexpr int ES = TX + 1, NK = Shape<N>::NK;
  __shared__ float2 lds[N * ES];
  __shared__ float2 tw[N];
  extern __shared__ double bins[];
  // workgroups go to the 8 XCDs in turn; the remap gives each XCD a contiguous run of
  // (k_y block, k_z) tiles of a box, so that the workgroups reading the two halves of a
  // 128-byte line (TX = 8) share one L2
  constexpr int NYB = N / TX;
  const int per = static_cast<int>(gridDim.x) / 8, lid = static_cast<int>(blockIdx.x);
  const int tile = (lid % 8) * per + lid / 8;
  if (tile >= NYB * NK) return;
  const int y0 = (tile % NYB) * TX, kz = tile / NYB, box = blockIdx.y;
  load_twiddles<N, NT>(tw, twg);
  if constexpr (BIN)
    for (int b = threadIdx.x; b < nbins; b += NT) bins[b] = 0.0;
  // binning: thread t walks a run of RUN consecutive k_x at k_y = y0 + t % TX, where |n|^2
  // changes slowly; the run's bin indices are fetched here so that their latency hides
  // behind the loads and the transform (-1: no mode)
  constexpr int RUNS = NT / TX;                        // runs per k_y column
  constexpr int RUN = (N + RUNS - 1) / RUNS;           // k_x values per run
  static_assert(TX * RUNS == NT, "one run per thread");
  [[maybe_unused]] const int by = threadIdx.x % TX, bx0 = (threadIdx.x / TX) * RUN;
  [[maybe_unused]] int bk[RUN];
  if constexpr (BIN) {
    const int ny = signed_index(y0 + by, N);
#pragma unroll
    for (int u = 0; u < RUN; ++u) {
      const int nx = signed_index(bx0 + u, N);
      const int n2 = nx * nx + ny * ny + kz * kz;
      bk[u] = (bx0 + u < N && n2 > 0) ? static_cast<int>(bin_of_n2[n2]) : -1;
    }
  }
  float2* base = data + ((static_cast<size_t>(box) * NK + kz) * N) * N + y0;
  // float4 = two consecutive k_y; all loads in flight before the LDS stores
  constexpr int P = TX / 2, IT = (N * P + NT - 1) / NT;
  static_assert(TX % 2 == 0 && NT % P == 0, "k_y pairs");
  const int py = 2 * (threadIdx.x % P);
  float4 v[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int x = (threadIdx.x + i * NT) / P;
    if (x < N) v[i] = *reinterpret_cast<const float4*>(base + static_cast<size_t>(x) * N + py);
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int x = (threadIdx.x + i * NT) / P;
    if (x < N) {
      lds[x * ES + py] = make_float2(v[i].x, v[i].y);
      lds[x * ES + py + 1] = make_float2(v[i].z, v[i].w);
    }
  }
  __syncthreads();
  fft_lines<N, TX, NT, -1>(lds, tw);
  const double w = (kz == 0 || kz == N / 2) ? 1.0 : 2.0;
  // store the tile back, then bin it, adding to the LDS bin only when the bin changes
  if constexpr (STORE) {
    for (int t = threadIdx.x; t < N * P; t += NT) {
      const int x = t / P, y = 2 * (t % P);
      const float2 a = lds[x * ES + y], b = lds[x * ES + y + 1];
      *reinterpret_cast<float4*>(base + static_cast<size_t>(x) * N + y) =
          make_float4(a.x, a.y, b.x, b.y);
    }
  }
  if constexpr (!BIN) return;
  {
    int cur = -1;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < RUN; ++u) {
      const int b = bk[u];
      if (b < 0) continue;
      const float2 v = lds[(bx0 + u) * ES + by];
      const double p = w * (static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y);
      if (b != cur) {
        if (cur >= 0) atomicAdd(&bins[cur], acc);
        cur = b;
        acc = 0.0;
      }
      acc += p;
    }
    if (cur >= 0) atomicAdd(&bins[cur], acc);
  }
  __syncthreads();
  // partial sums stored bin-major, [box][bin][workgroup], for contiguous reads per bin
  const int wg = tile;
  const size_t n_wg = static_cast<size_t>(NYB) * NK;
  double* dst = partial + static_cast<size_t>(box) * nbins * n_wg + wg;
  for (int b = threadIdx.x; b < nbins; b += NT) dst[b * n_wg] = bins[b];
}

// ------------------------------------------------------------------------ inverse ----
// The neutrino factor of eq. (phases), T(n^2) = (1 - f_nu) + f_nu R(|k|), with R linear in
// ln k between the bracketing non-empty bins: e packs the lower bin lo and the weight t of
// the upper one, next(lo) (both fixed by the geometry); the step's per-bin R and next are
// staged in LDS (dynamic: nbins doubles, then nbins ints), with independent loads.
__device__ __forceinline__ void stage_ratio(double* s_r, const double* ratio, const int* next,
                                            int nbins, int tid, int nt) {
  int* s_next = reinterpret_cast<int*>(s_r + nbins);
  for (int b = tid; b < nbins; b += nt) {
    s_r[b] = ratio[b];
    s_next[b] = next[b];
  }
}
__device__ __forceinline__ float neutrino_factor(uint32_t e, const double* s_r, int nbins,
                                                 double f) {
  const int lo = static_cast<int>(e & ((1u << kRatioBinBits) - 1));
  const int hi = reinterpret_cast<const int*>(s_r + nbins)[lo];
  const double t = static_cast<double>(e >> kRatioBinBits) * kRatioUnit;
  const double r = s_r[lo] + t * (s_r[hi] - s_r[lo]);
  return static_cast<float>((1.0 - f) + f * r);
}

// Threads per workgroup of inv_x_kernel: at N = 512 its LDS tile (N x 2 TX values, 75 KB)
// leaves two workgroups per CU, and 512 threads keep twice the waves in flight (587 -> 510 us
// at 512^3; no gain at 256^3, where four workgroups fit).
template <int N> constexpr int kInvXNT = N >= 512 ? 512 : 256;
template <int N, int TX>
__global__ __launch_bounds__(kInvXNT<N>) void inv_x_kernel(const float2* __restrict__ dk,
                                                   float2* __restrict__ f1,
                                                   float2* __restrict__ f2,
                                                   const float2* __restrict__ twg,
                                                   const uint32_t* __restrict__ ridx,
                                                   const int* __restrict__ next,
                                                   const double* __restrict__ ratio,
                                                   const RespBox* __restrict__ boxes, int nbins,
                                                   const float* __restrict__ inv_w2,
                                                   float c, float kf, int nbox) {
  constexpr int NT = kInvXNT<N>;                   // this kernel's workgroup size
  constexpr int NL = 2 * TX, ES = NL + 1, NK = Shape<N>::NK;
  constexpr int NYB = N / TX;
  __shared__ float2 lds[N * ES];
  __shared__ float2 tw[N];
  __shared__ float s_iw[N];
  extern __shared__ double s_r[];                  // R and next of this box (dynamic)
  // Workgroups go to the 8 XCDs in turn; the remap gives each XCD a contiguous run of
  // (k_y block, k_z) tiles, so the two workgroups writing the halves of a 128-byte line
  // (TX = 8 complex values = 64 bytes per row) share one L2 instead of each fetching it.
  const int total = NYB * NK * nbox, per = static_cast<int>(gridDim.x) / 8;
  const int lid = static_cast<int>(blockIdx.x);
  const int logical = (lid % 8) * per + lid / 8;
  if (logical >= total) return;
  const int y0 = (logical % NYB) * TX, kz = (logical / NYB) % NK, box = logical / (NYB * NK);
  load_twiddles<N, NT>(tw, twg);
  for (int m = threadIdx.x; m < N; m += NT) s_iw[m] = inv_w2[m];
  stage_ratio(s_r, ratio + static_cast<size_t>(box) * nbins, next, nbins, threadIdx.x, NT);
  const size_t off = ((static_cast<size_t>(box) * NK + kz) * N) * N + y0;
  const float wz = inv_w2[kz];
  const double fnu = boxes[box].f_nu;
  // where n^2 of this thread's Green's-function modes falls among the bins, fetched before
  // the tile so that the gathers' latency hides behind its loads
  constexpr int GI = (N * TX + NT - 1) / NT;
  uint32_t ri[GI];
#pragma unroll
  for (int i = 0; i < GI; ++i) {
    const int t = threadIdx.x + i * NT;
    const int y = t % TX, x = t / TX;
    const int nx = signed_index(x, N), ny = signed_index(y0 + y, N);
    const int n2 = nx * nx + ny * ny + kz * kz;
    ri[i] = ridx[t < N * TX ? n2 : 0];
  }
  // the tile holds x (real space) by k_y: forward transform along x first (lines 0..TX-1)
  constexpr int P = TX / 2, IT = (N * P + NT - 1) / NT;
  static_assert(TX % 2 == 0 && NT % P == 0, "k_y pairs");
  const int py = 2 * (threadIdx.x % P);
  float4 v[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int x = (threadIdx.x + i * NT) / P;
    if (x < N) v[i] = *reinterpret_cast<const float4*>(dk + off + static_cast<size_t>(x) * N + py);
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int x = (threadIdx.x + i * NT) / P;
    if (x < N) {
      lds[x * ES + py] = make_float2(v[i].x, v[i].y);
      lds[x * ES + py + 1] = make_float2(v[i].z, v[i].w);
    }
  }
  __syncthreads();
  float tv[GI];                                    // T(n^2) (unused at the k = 0 mode)
#pragma unroll
  for (int i = 0; i < GI; ++i) tv[i] = neutrino_factor(ri[i], s_r, nbins, fnu);
  fft_lines<N, TX, NT, -1, ES>(lds, tw);
  // delta_M -> phi and -i k_x phi, in place on the (k_x, k_y) tile
#pragma unroll
  for (int i = 0; i < GI; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t >= N * TX) break;
    const int y = t % TX, x = t / TX;
    const int nx = signed_index(x, N), ny = signed_index(y0 + y, N);
    const int n2 = nx * nx + ny * ny + kz * kz;
    float2 phi = make_float2(0.f, 0.f);
    if (n2 > 0) {
      // phi = -C T(n^2) delta / (k^2 W^2), k^2 = kf^2 n^2
      const float g = -c * tv[i] * s_iw[x] * s_iw[y0 + y] * wz /
                      (kf * kf * static_cast<float>(n2));
      phi = cscale(lds[x * ES + y], g);
    }
    const float kx = (x == N / 2) ? 0.f : kf * static_cast<float>(nx);
    lds[x * ES + y] = phi;
    lds[x * ES + TX + y] = make_float2(kx * phi.y, -kx * phi.x);     // -i k_x phi
  }
  __syncthreads();
  fft_lines<N, NL, NT, +1>(lds, tw);
  for (int t = threadIdx.x; t < N * P; t += NT) {
    const int x = t / P, y = 2 * (t % P);
    const size_t o = off + static_cast<size_t>(x) * N + y;
    float2 a = lds[x * ES + y], b = lds[x * ES + y + 1];
    *reinterpret_cast<float4*>(f1 + o) = make_float4(a.x, a.y, b.x, b.y);
    a = lds[x * ES + TX + y];
    b = lds[x * ES + TX + y + 1];
    *reinterpret_cast<float4*>(f2 + o) = make_float4(a.x, a.y, b.x, b.y);
  }
}

// For N <= 64 the first two inverse passes in one kernel, one workgroup per (k_z, box): the
// whole k_z slab (N x N modes, [x][k_y]) fits the LDS, so F1 = phi and F2 = -i k_x phi never
// go to HBM. As inv_x_kernel with all k_y at once: forward transform along x, the Green's
// function with the neutrino factor T(n^2) and the deconvolution, -i k_x, inverse along x;
// then the slab is transposed through registers (each thread holds 2 N^2 / NT values) to
// lines along k_y, and as inv_y_kernel G1 = F1 and G3 = F2 are transformed along y and
// written to [box][x][k_z][y], then G2 = -i k_y F1 from the registers. The same arithmetic
// as the two passes in the same order, so the same result bit for bit.
constexpr int kInvXYNT = 512;   // threads per workgroup of inv_xy_kernel
template <int N>
__global__ __launch_bounds__(kInvXYNT) void inv_xy_kernel(const float2* __restrict__ dk,
                                                    float2* __restrict__ g1,
                                                    float2* __restrict__ g2,
                                                    float2* __restrict__ g3,
                                                    const float2* __restrict__ twg,
                                                    const uint32_t* __restrict__ ridx,
                                                    const int* __restrict__ next,
                                                    const double* __restrict__ ratio,
                                                    const RespBox* __restrict__ boxes, int nbins,
                                                    const float* __restrict__ inv_w2, float c,
                                                    float kf) {
  constexpr int NT = kInvXYNT;                     // this kernel's workgroup size
  constexpr int NK = Shape<N>::NK, NL = 2 * N, ES = NL + 1;
  constexpr int PER = (2 * N * N + NT - 1) / NT;    // F1, F2 values each thread holds
  constexpr int GI = (N * N + NT - 1) / NT;         // Green's-function modes per thread
  static_assert(N <= 64, "the slab must fit the LDS");
  __shared__ float2 lds[N * ES];
  __shared__ float2 tw[N];
  __shared__ float s_iw[N];
  extern __shared__ double s_r[];                  // R and next of this box (dynamic)
  const int tid = threadIdx.x;
  const int kz = static_cast<int>(blockIdx.x) % NK, box = static_cast<int>(blockIdx.x) / NK;
  load_twiddles<N, NT>(tw, twg);
  for (int m = tid; m < N; m += NT) s_iw[m] = inv_w2[m];
  stage_ratio(s_r, ratio + static_cast<size_t>(box) * nbins, next, nbins, tid, NT);
  const size_t off = (static_cast<size_t>(box) * NK + kz) * N * N;   // the slab, [x][k_y]
  const float wz = inv_w2[kz];
  const double fnu = boxes[box].f_nu;
  // where n^2 of this thread's modes falls among the bins, fetched before the slab so that
  // the gathers' latency hides behind its loads
  uint32_t ri[GI];
#pragma unroll
  for (int i = 0; i < GI; ++i) {
    const int t = tid + i * NT;
    const int y = t % N, x = t / N;
    const int nx = signed_index(x, N), ny = signed_index(y, N);
    const int n2 = nx * nx + ny * ny + kz * kz;
    ri[i] = ridx[t < N * N ? n2 : 0];
  }
  // the slab: element x of line k_y at lds[x ES + k_y]
  {
    constexpr int IT = (N * N / 2 + NT - 1) / NT;
    float4 v[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * NT;
      if (t < N * N / 2) v[i] = *reinterpret_cast<const float4*>(dk + off + 2 * t);
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * NT;
      if (t >= N * N / 2) break;
      const int x = (2 * t) / N, y = (2 * t) % N;
      lds[x * ES + y] = make_float2(v[i].x, v[i].y);
      lds[x * ES + y + 1] = make_float2(v[i].z, v[i].w);
    }
  }
  __syncthreads();
  float tv[GI];                                    // T(n^2) (unused at the k = 0 mode)
#pragma unroll
  for (int i = 0; i < GI; ++i) tv[i] = neutrino_factor(ri[i], s_r, nbins, fnu);
  fft_lines<N, N, NT, -1, ES>(lds, tw);
  // delta_M -> phi (lines 0..N-1) and -i k_x phi (lines N..2N-1)
#pragma unroll
  for (int i = 0; i < GI; ++i) {
    const int t = tid + i * NT;
    if (t >= N * N) break;
    const int y = t % N, x = t / N;
    const int nx = signed_index(x, N), ny = signed_index(y, N);
    const int n2 = nx * nx + ny * ny + kz * kz;
    float2 phi = make_float2(0.f, 0.f);
    if (n2 > 0) {
      const float g = -c * tv[i] * s_iw[x] * s_iw[y] * wz / (kf * kf * static_cast<float>(n2));
      phi = cscale(lds[x * ES + y], g);
    }
    const float kx = (x == N / 2) ? 0.f : kf * static_cast<float>(nx);
    lds[x * ES + y] = phi;
    lds[x * ES + N + y] = make_float2(kx * phi.y, -kx * phi.x);
  }
  __syncthreads();
  fft_lines<N, NL, NT, +1, ES>(lds, tw);
  // transpose through registers: value idx = (x, l), l < N: F1(x, k_y = l), else F2
  float2 f[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = tid + i * NT;
    f[i] = idx < 2 * N * N ? lds[(idx / NL) * ES + idx % NL] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  // G1 (lines x) and G3 (lines N + x), element k_y
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = tid + i * NT;
    if (idx >= 2 * N * N) break;
    const int x = idx / NL, l = idx % NL;
    if (l < N) lds[l * ES + x] = f[i];
    else lds[(l - N) * ES + N + x] = f[i];
  }
  __syncthreads();
  fft_lines<N, NL, NT, +1, ES>(lds, tw);
  auto store = [&](float2* g, int line0) {
    for (int t = tid; t < N * N / 2; t += NT) {
      const int x = (2 * t) / N, e = (2 * t) % N;
      const size_t o = ((static_cast<size_t>(box) * N + x) * NK + kz) * N + e;
      const float2 a = lds[e * ES + line0 + x], b = lds[(e + 1) * ES + line0 + x];
      *reinterpret_cast<float4*>(g + o) = make_float4(a.x, a.y, b.x, b.y);
    }
  };
  store(g1, 0);
  store(g3, N);
  __syncthreads();
  // G2 = -i k_y F1
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = tid + i * NT;
    if (idx >= 2 * N * N) break;
    const int x = idx / NL, l = idx % NL;
    if (l < N) {
      const float ky = (l == N / 2) ? 0.f : kf * static_cast<float>(signed_index(l, N));
      lds[l * ES + x] = make_float2(ky * f[i].y, -ky * f[i].x);
    }
  }
  __syncthreads();
  fft_lines<N, N, NT, +1, ES>(lds, tw);
  store(g2, 0);
}

// in: rows of [box][kz][x] (flattened); out: G1, G2, G3 rows at [box][x][kz].
template <int N, int NLR>
__global__ __launch_bounds__(NT) void inv_y_kernel(const float2* __restrict__ f1,
                                                   const float2* __restrict__ f2,
                                                   float2* __restrict__ g1,
                                                   float2* __restrict__ g2,
                                                   float2* __restrict__ g3,
                                                   const float2* __restrict__ twg, float kf) {
  constexpr int NL = 3 * NLR, ES = NL + 1;
  __shared__ float2 lds[N * ES];
  __shared__ float2 tw[N];
  load_twiddles<N, NT>(tw, twg);
  const size_t off = static_cast<size_t>(blockIdx.x) * NLR * N;
  const float4* f1v = reinterpret_cast<const float4*>(f1 + off);
  const float4* f2v = reinterpret_cast<const float4*>(f2 + off);
  // all of a thread's loads in flight before the LDS stores
  constexpr int IT = (NLR * N / 2 + NT - 1) / NT;
  float4 va[IT], vb[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t < NLR * N / 2) {
      va[i] = f1v[t];
      vb[i] = f2v[t];
    }
  }
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t >= NLR * N / 2) continue;
    const int l = (2 * t) / N, e0 = (2 * t) % N;
    const float4 a4 = va[i], b4 = vb[i];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = e0 + h;
      const float2 a = h ? make_float2(a4.z, a4.w) : make_float2(a4.x, a4.y);
      lds[e * ES + l] = a;
      const float ky = (e == N / 2) ? 0.f : kf * static_cast<float>(signed_index(e, N));
      lds[e * ES + NLR + l] = make_float2(ky * a.y, -ky * a.x);        // -i k_y F1
      lds[e * ES + 2 * NLR + l] = h ? make_float2(b4.z, b4.w) : make_float2(b4.x, b4.y);
    }
  }
  __syncthreads();
  fft_lines<N, NL, NT, +1>(lds, tw);
  constexpr int NK = Shape<N>::NK;
  for (int t = threadIdx.x; t < NLR * N / 2; t += NT) {
    const int l = (2 * t) / N, e = (2 * t) % N;
    const size_t r = static_cast<size_t>(blockIdx.x) * NLR + l;
    const size_t box = r / (static_cast<size_t>(NK) * N), rem = r % (static_cast<size_t>(NK) * N);
    const size_t kz = rem / N, x = rem % N;
    const size_t o = ((box * N + x) * NK + kz) * N + e;
    float2 a = lds[e * ES + l], b = lds[(e + 1) * ES + l];
    *reinterpret_cast<float4*>(g1 + o) = make_float4(a.x, a.y, b.x, b.y);
    a = lds[e * ES + NLR + l];
    b = lds[(e + 1) * ES + NLR + l];
    *reinterpret_cast<float4*>(g2 + o) = make_float4(a.x, a.y, b.x, b.y);
    a = lds[e * ES + 2 * NLR + l];
    b = lds[(e + 1) * ES + 2 * NLR + l];
    *reinterpret_cast<float4*>(g3 + o) = make_float4(a.x, a.y, b.x, b.y);
  }
}

// out: [nbox][x][y][z][3] with component 0 = g_x (from G3), 1 = g_y (G2), 2 = g_z (G1).
// 512 threads per workgroup: the LDS tile limits a CU to a few workgroups, and twice the
// waves of 256 keep more of the transform's LDS traffic in flight (88.5 -> 82.6 us at 256^3).
constexpr int kInvZNT = 512;
template <int N, int TY>
__global__ __launch_bounds__(kInvZNT) void inv_z_kernel(const float2* __restrict__ g1,
                                                        const float2* __restrict__ g2,
                                                        const float2* __restrict__ g3,
                                                        float* __restrict__ out,
                                                        const float2* __restrict__ twg, float kf,
                                                        int nbox) {
  constexpr int NT = kInvZNT;                      // this kernel's workgroup size
  constexpr int ROWS = 3 * TY, NL = ROWS / 2, ES = NL + 1;
  constexpr int NK = Shape<N>::NK;
  static_assert(TY % 2 == 0 && NT % (TY / 2) == 0, "row pairs per float4");
  // Loads: float4 = the values of one k at two consecutive y (a row pair), for the three
  // fields; all issued before any LDS store so that many are in flight per thread.
  constexpr int PAIRS = TY / 2, PER_COMP = NK * PAIRS, TOTAL = 3 * PER_COMP;
  constexpr int IT = (TOTAL + NT - 1) / NT;
  __shared__ float2 lds[N * ES];
  __shared__ float2 tw[N];
  const int y0 = blockIdx.x * TY, x = blockIdx.y, box = blockIdx.z;
  load_twiddles<N, NT>(tw, twg);
  const size_t plane = ((static_cast<size_t>(box) * N + x) * NK) * N + y0;   // (k = 0, y0)
  const int pr = threadIdx.x % PAIRS;                 // row pair within the field
  float4 v[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    const int comp = t / PER_COMP, k = (t - comp * PER_COMP) / PAIRS;
    const float2* src = comp == 0 ? g3 : (comp == 1 ? g2 : g1);
    if (t < TOTAL)
      v[i] = *reinterpret_cast<const float4*>(src + plane + static_cast<size_t>(k) * N + 2 * pr);
  }
  float* ldsf = reinterpret_cast<float*>(lds);
  // Half spectra of row pair p: A[k] at slot k and B[k] at slot N-k for 0 < k < N/2;
  // the real parts of A and B at k = 0 and k = N/2 share slots 0 and N/2.
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NT;
    if (t >= TOTAL) break;
    const int comp = t / PER_COMP, k = (t - comp * PER_COMP) / PAIRS;
    float2 a = make_float2(v[i].x, v[i].y), b = make_float2(v[i].z, v[i].w);
    if (comp == 2) {                                   // -i k_z G1
      const float kz = (k == N / 2) ? 0.f : kf * static_cast<float>(k);
      a = make_float2(kz * a.y, -kz * a.x);
      b = make_float2(kz * b.y, -kz * b.x);
    }
    const int p = comp * PAIRS + pr;                   // rows 2p (A) and 2p + 1 (B)
    if (k == 0 || k == N / 2) {
      ldsf[(k * ES + p) * 2] = a.x;
      ldsf[(k * ES + p) * 2 + 1] = b.x;
    } else {
      lds[k * ES + p] = a;
      lds[(N - k) * ES + p] = b;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < (N / 2 - 1) * NL; t += NT) {
    const int p = t % NL, k = 1 + t / NL;
    const float2 a = lds[k * ES + p], b = lds[(N - k) * ES + p];
    lds[k * ES + p] = make_float2(a.x - b.y, a.y + b.x);                // A + iB
    lds[(N - k) * ES + p] = make_float2(a.x + b.y, b.x - a.y);          // conj A + i conj B
  }
  __syncthreads();
  fft_lines<N, NL, NT, +1>(lds, tw);
  // interleaved output: (g_x, g_y, g_z) of node (x, y, z) are 3 consecutive floats. One
  // lane per node, consecutive lanes at consecutive z: the LDS reads of a wave then fall in
  // distinct banks (four nodes per lane, as float4 stores, put a wave's reads on 8 banks)
  float* dst = out + ((static_cast<size_t>(box) * N + x) * N + y0) * N * 3;
  constexpr int NODES = TY * N;
  for (int n = threadIdx.x; n < NODES; n += NT) {
    const int y = n / N, z = n % N;
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      const int row = comp * TY + y;
      dst[3 * n + comp] = ldsf[(z * ES + (row >> 1)) * 2 + (row & 1)];
    }
  }
}

// For N <= 64 the last two inverse passes in one kernel, one workgroup per (x-plane, box):
// F1 and F2 of the plane (all k_z, all k_y: 2 N (N/2 + 1) modes) fit the LDS. As
// inv_y_kernel, G1 = F1, G2 = -i k_y F1 and G3 = F2 are transformed along y (one line per
// k_z each); the G values go through registers to the layout of inv_z_kernel (rows comp N + y,
// two rows per complex line as A + iB, -i k_z on G1) and are transformed along z into the
// plane's interleaved accelerations. The same arithmetic in the same order as the two passes,
// so the same forces bit for bit; G1..G3 never reach HBM.
constexpr int kInvYZNT = 512;   // threads per workgroup of inv_yz_kernel
template <int N>
__global__ __launch_bounds__(kInvYZNT) void inv_yz_kernel(const float2* __restrict__ f1,
                                                          const float2* __restrict__ f2,
                                                          float* __restrict__ out,
                                                          const float2* __restrict__ twg,
                                                          float kf) {
  constexpr int NT = kInvYZNT;                     // this kernel's workgroup size
  constexpr int NK = Shape<N>::NK;
  constexpr int NL1 = 3 * NK, ES1 = NL1 + 1;       // y lines: F1, -i k_y F1, F2 per k_z
  constexpr int NL2 = 3 * N / 2, ES2 = NL2 + 1;    // z lines: row pairs of rows comp N + y
  constexpr int LDS_N = N * (ES1 > ES2 ? ES1 : ES2);
  constexpr int NG = 3 * NK * N;                   // G values of the plane
  constexpr int PER = (NG + NT - 1) / NT;
  static_assert(N <= 64, "the plane's modes must fit the LDS");
  __shared__ float2 lds[LDS_N];
  __shared__ float2 tw[N];
  const int x = blockIdx.x, box = blockIdx.y, tid = threadIdx.x;
  load_twiddles<N, NT>(tw, twg);
  // 1. F1, F2 of the plane: the k_z rows of [box][k_z][x][k_y], two values per float4
  {
    constexpr int IT = (NK * N / 2 + NT - 1) / NT;
    float4 va[IT], vb[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * NT;
      if (t < NK * N / 2) {
        const int kz = t / (N / 2), e0 = 2 * (t % (N / 2));
        const size_t o = ((static_cast<size_t>(box) * NK + kz) * N + x) * N + e0;
        va[i] = *reinterpret_cast<const float4*>(f1 + o);
        vb[i] = *reinterpret_cast<const float4*>(f2 + o);
      }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = tid + i * NT;
      if (t >= NK * N / 2) continue;
      const int kz = t / (N / 2), e0 = 2 * (t % (N / 2));
      const float4 a4 = va[i], b4 = vb[i];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = e0 + h;
        const float2 a = h ? make_float2(a4.z, a4.w) : make_float2(a4.x, a4.y);
        lds[e * ES1 + kz] = a;
        const float ky = (e == N / 2) ? 0.f : kf * static_cast<float>(signed_index(e, N));
        lds[e * ES1 + NK + kz] = make_float2(ky * a.y, -ky * a.x);     // -i k_y F1
        lds[e * ES1 + 2 * NK + kz] = h ? make_float2(b4.z, b4.w) : make_float2(b4.x, b4.y);
      }
    }
  }
  __syncthreads();
  fft_lines<N, NL1, NT, +1, ES1>(lds, tw);
  // 2. value t = (field f, k_z, y): G1 (f = 0) is g_z, G2 g_y, G3 g_x
  float2 g[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int t = tid + i * NT;
    g[i] = make_float2(0.f, 0.f);
    if (t < NG) {
      const int y = t % N, r = t / N, kz = r % NK, f = r / NK;
      g[i] = lds[y * ES1 + f * NK + kz];
    }
  }
  __syncthreads();
  // 3. half spectra of row pair p: A[k] at slot k and B[k] at slot N-k for 0 < k < N/2; the
  //    real parts of A and B at k = 0 and k = N/2 share slots 0 and N/2
  float* ldsf = reinterpret_cast<float*>(lds);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int t = tid + i * NT;
    if (t >= NG) break;
    const int y = t % N, r = t / N, k = r % NK, f = r / NK;
    const int comp = 2 - f;
    float2 a = g[i];
    if (comp == 2) {                                 // -i k_z G1
      const float kz = (k == N / 2) ? 0.f : kf * static_cast<float>(k);
      a = make_float2(kz * a.y, -kz * a.x);
    }
    const int row = comp * N + y, p = row >> 1;
    if (k == 0 || k == N / 2)
      ldsf[(k * ES2 + p) * 2 + (row & 1)] = a.x;
    else if ((row & 1) == 0)
      lds[k * ES2 + p] = a;
    else
      lds[(N - k) * ES2 + p] = a;
  }
  __syncthreads();
  for (int t = tid; t < (N / 2 - 1) * NL2; t += NT) {
    const int p = t % NL2, k = 1 + t / NL2;
    const float2 a = lds[k * ES2 + p], b = lds[(N - k) * ES2 + p];
    lds[k * ES2 + p] = make_float2(a.x - b.y, a.y + b.x);                // A + iB
    lds[(N - k) * ES2 + p] = make_float2(a.x + b.y, b.x - a.y);          // conj A + i conj B
  }
  __syncthreads();
  fft_lines<N, NL2, NT, +1, ES2>(lds, tw);
  // interleaved output of the plane, one lane per node as in inv_z_kernel
  float* dst = out + (static_cast<size_t>(box) * N + x) * N * N * 3;
  for (int n = tid; n < N * N; n += NT) {
    const int y = n / N, z = n % N;
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
      const int row = comp * N + y;
      dst[3 * n + comp] = ldsf[(z * ES2 + (row >> 1)) * 2 + (row & 1)];
    }
  }
}

template <int N>
__global__ void copy_modes_kernel(const float2* __restrict__ ck, float2* __restrict__ out,
                                  int box) {
  constexpr int NK = N / 2 + 1;
  const int64_t total = static_cast<int64_t>(N) * N * NK;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int kz = static_cast<int>(i % NK);
    const int ky = static_cast<int>((i / NK) % N);
    const int kx = static_cast<int>(i / (static_cast<int64_t>(NK) * N));
    out[i] = ck[((static_cast<size_t>(box) * NK + kz) * N + kx) * N + ky];
  }
}

// ------------------------------------------------------------------ dispatchers ----
// Call go(std::integral_constant<int, tile>) with tile candidate v of a pass (v outside 1..2:
// the default, candidate 0).
template <int T0, int T1, int T2, typename F>
hipError_t with_tile(F&& go, int v) {
  switch (v) {
    case 1: return go(std::integral_constant<int, T1>{});
    case 2: return go(std::integral_constant<int, T2>{});
    default: return go(std::integral_constant<int, T0>{});
  }
}
#define PMNU_TILES(ARR) Tiles<N>::ARR[0], Tiles<N>::ARR[1], Tiles<N>::ARR[2]
template <template <int> class F, typename... A>
hipError_t dispatch_n(int n, A... args) {
  switch (n) {
    case 8: return F<8>::run(args...);
    case 16: return F<16>::run(args...);
    case 32: return F<32>::run(args...);
    case 64: return F<64>::run(args...);
    case 128: return F<128>::run(args...);
    case 256: return F<256>::run(args...);
    case 512: return F<512>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

template <int N> struct FwdZ {
  static hipError_t run(const unsigned long long* rho, const float* delta, int* reset,
                        int* clear, int n_clear, float2* out, const float2* tw, double scale,
                        int nbox, hipStream_t s, int v) {
    auto go = [&](auto ty) -> hipError_t {
      constexpr int TY = decltype(ty)::value;
      dim3 grid(N / TY, N, nbox);
      if (static_cast<int64_t>(grid.x) * grid.y * grid.z * NT < n_clear)
        return hipErrorInvalidValue;               // every count needs a thread to clear it
      if (delta)
        hipLaunchKernelGGL((fwd_z_kernel<N, true, TY>), grid, dim3(NT), 0, s, delta, out, tw,
                           scale, reset, clear, n_clear);
      else
        hipLaunchKernelGGL((fwd_z_kernel<N, false, TY>), grid, dim3(NT), 0, s, rho, out, tw,
                           scale, reset, clear, n_clear);
      return hipGetLastError();
    };
    return with_tile<PMNU_TILES(FZ)>(go, v);
  }
};
template <int N> struct FwdY {
  static hipError_t run(const float2* in, float2* out, const float2* tw, int nbox,
                        hipStream_t s, int v, int* reset, int* clear, int n_clear) {
    auto go = [&](auto nl) -> hipError_t {
      constexpr int NL = decltype(nl)::value;
      dim3 grid(static_cast<unsigned>(static_cast<int64_t>(nbox) * Shape<N>::NK * N / NL));
      if (static_cast<int64_t>(grid.x) * NT < n_clear)
        return hipErrorInvalidValue;               // every count needs a thread to clear it
      hipLaunchKernelGGL((fwd_y_kernel<N, NL>), grid, dim3(NT), 0, s, in, out, tw, reset, clear,
                         n_clear);
      return hipGetLastError();
    };
    return with_tile<PMNU_TILES(FY)>(go, v);
  }
};
template <int N> struct FwdZY {
  static hipError_t run(const unsigned long long* rho, const float* delta, int* reset,
                        int* clear, int n_clear, float2* out, const float2* tw, double scale,
                        int nbox, hipStream_t s) {
    if constexpr (N > 128) {
      return hipErrorInvalidValue;                 // the plane does not fit the LDS
    } else {
      dim3 grid(N, nbox);
      if (static_cast<int64_t>(grid.x) * grid.y * kFwdZYNT < n_clear)
        return hipErrorInvalidValue;               // every count needs a thread to clear it
      if (delta)
        hipLaunchKernelGGL((fwd_zy_kernel<N, true>), grid, dim3(kFwdZYNT), 0, s, delta, out, tw,
                           scale, reset, clear, n_clear);
      else
        hipLaunchKernelGGL((fwd_zy_kernel<N, false>), grid, dim3(kFwdZYNT), 0, s, rho, out, tw,
                           scale, reset, clear, n_clear);
      return hipGetLastError();
    }
  }
};
template <int N> struct FwdX {
  // partial != NULL: bin without storing (the step); NULL: store the modes, no binning
  static hipError_t run(float2* data, const float2* tw, const uint16_t* bins, double* partial,
                        int nbins, int nbox, hipStream_t s, int v) {
    auto go = [&](auto tx) -> hipError_t {
      constexpr int TX = decltype(tx)::value;
      const int tiles = N / TX * Shape<N>::NK;
      dim3 grid((tiles + 7) / 8 * 8, nbox);          // whole rounds over the 8 XCDs
      if (partial)
        hipLaunchKernelGGL((fwd_x_bin_kernel<N, false, true, TX>), grid, dim3(NT),
                           nbins * sizeof(double), s, data, tw, bins, partial, nbins);
      else
        hipLaunchKernelGGL((fwd_x_bin_kernel<N, true, false, TX>), grid, dim3(NT), 0, s, data,
                           tw, bins, partial, nbins);
      return hipGetLastError();
    };
    return with_tile<PMNU_TILES(FX)>(go, v);
  }
};
template <int N> struct InvX {
  static hipError_t run(const float2* dk, float2* f1, float2* f2, const float2* tw,
                        const uint32_t* ridx, const int* next, const double* ratio,
                        const RespBox* boxes, int nbins, const float* iw, float cfac, float kf,
                        int nbox,
                        hipStream_t s, int v) {
    auto go = [&](auto txv) -> hipError_t {
      constexpr int TX = decltype(txv)::value;
      const int total = N / TX * Shape<N>::NK * nbox;
      dim3 grid((total + 7) / 8 * 8);   // whole rounds over the 8 XCDs; extra blocks exit
      const size_t lds_ratio = nbins * (sizeof(double) + sizeof(int));   // R and next
      hipLaunchKernelGGL((inv_x_kernel<N, TX>), grid, dim3(kInvXNT<N>), lds_ratio, s, dk, f1,
                         f2, tw, ridx, next, ratio, boxes, nbins, iw, cfac, kf, nbox);
      return hipGetLastError();
    };
    return with_tile<PMNU_TILES(IX)>(go, v);
  }
};
template <int N> struct InvY {
  static hipError_t run(const float2* f1, const float2* f2, float2* g1, float2* g2, float2* g3,
                        const float2* tw, float kf, int nbox, hipStream_t s, int v) {
    auto go = [&](auto nl) -> hipError_t {
      constexpr int NLR = decltype(nl)::value;
      dim3 grid(static_cast<unsigned>(static_cast<int64_t>(nbox) * Shape<N>::NK * N / NLR));
      hipLaunchKernelGGL((inv_y_kernel<N, NLR>), grid, dim3(NT), 0, s, f1, f2, g1, g2, g3, tw,
                         kf);
      return hipGetLastError();
    };
    return with_tile<PMNU_TILES(IY)>(go, v);
  }
};
template <int N> struct InvXY {
  static hipError_t run(const float2* dk, float2* g1, float2* g2, float2* g3, const float2* tw,
                        const uint32_t* ridx, const int* next, const double* ratio,
                        const RespBox* boxes, int nbins, const float* iw, float cfac, float kf,
                        int nbox,
                        hipStream_t s) {
    if constexpr (N > 64) {
      return hipErrorInvalidValue;                 // the k_z slab does not fit the LDS
    } else {
      hipLaunchKernelGGL(inv_xy_kernel<N>, dim3(static_cast<unsigned>(Shape<N>::NK * nbox)),
                         dim3(kInvXYNT), nbins * (sizeof(double) + sizeof(int)), s, dk, g1, g2,
                         g3, tw, ridx, next, ratio, boxes, nbins, iw, cfac, kf);
      return hipGetLastError();
    }
  }
};
template <int N> struct InvYZ {
  static hipError_t run(const float2* f1, const float2* f2, float* out, const float2* tw, float kf,
                        int nbox, hipStream_t s) {
    if constexpr (N > 64) {
      return hipErrorInvalidValue;                 // the plane's modes do not fit the LDS
    } else {
      hipLaunchKernelGGL(inv_yz_kernel<N>, dim3(N, nbox), dim3(kInvYZNT), 0, s, f1, f2, out, tw,
                         kf);
      return hipGetLastError();
    }
  }
};
template <int N> struct InvZ {
  static hipError_t run(const float2* g1, const float2* g2, const float2* g3, float* out,
                        const float2* tw, float kf, int nbox, hipStream_t s, int v) {
    auto go = [&](auto ty) -> hipError_t {
      constexpr int TY = decltype(ty)::value;
      dim3 grid(N / TY, N, nbox);
      hipLaunchKernelGGL((inv_z_kernel<N, TY>), grid, dim3(kInvZNT), 0, s, g1, g2, g3, out, tw, kf,
                         nbox);
      return hipGetLastError();
    };
    return with_tile<PMNU_TILES(IZ)>(go, v);
  }
};
template <int N> struct CopyModes {
  static hipError_t run(const float2* ck, float2* out, int box, hipStream_t s) {
    hipLaunchKernelGGL(copy_modes_kernel<N>, dim3(1024), dim3(256), 0, s, ck, out, box);
    return hipGetLastError();
  }
};
template <int N> struct Partials {
  static hipError_t run(int* out, int v) {
    return with_tile<PMNU_TILES(FX)>([&](auto tx) {
      *out = (N / decltype(tx)::value) * Shape<N>::NK;
      return hipSuccess;
    }, v);
  }
};
template <int N> struct TileOf {
  static hipError_t run(int* out, int pass, int v) {
    const int i = (v == 1 || v == 2) ? v : 0;
    switch (pass) {
      case 0: *out = Tiles<N>::FZ[i]; break;
      case 1: *out = Tiles<N>::FY[i]; break;
      case 2: *out = Tiles<N>::FX[i]; break;
      case 3: *out = Tiles<N>::IX[i]; break;
      case 4: *out = Tiles<N>::IY[i]; break;
      case 5: *out = Tiles<N>::IZ[i]; break;
      default: return hipErrorInvalidValue;
    }
    return hipSuccess;
  }
};

}  // namespace

hipError_t launch_fwd_z(int n, const unsigned long long* rho, const float* delta, int* reset,
                        int* clear, int n_clear, float2* out, const float2* tw, double scale,
                        int nbox, hipStream_t s, int v) {
  return dispatch_n<FwdZ>(n, rho, delta, reset, clear, n_clear, out, tw, scale, nbox, s, v);
}
hipError_t launch_fwd_y(int n, const float2* in, float2* out, const float2* tw, int nbox,
                        hipStream_t s, int v, int* reset, int* clear, int n_clear) {
  return dispatch_n<FwdY>(n, in, out, tw, nbox, s, v, reset, clear, n_clear);
}
hipError_t launch_fwd_zy(int n, const unsigned long long* rho, const float* delta, int* reset,
                         int* clear, int n_clear, float2* out, const float2* tw, double scale,
                         int nbox, hipStream_t s) {
  return dispatch_n<FwdZY>(n, rho, delta, reset, clear, n_clear, out, tw, scale, nbox, s);
}
template <int N> struct PatchFwdZ {
  static hipError_t run(const unsigned long long* patches, int pcap, const int* reg_count,
                        const int4* reg_list, unsigned long long* rho_fb, const int* n_fb,
                        float2* out, const float2* tw, double scale, int nbox, hipStream_t s,
                        float* delta_out) {
    if constexpr (N < 32) {
      return hipErrorInvalidValue;                 // the fused pass needs N / 16 >= 2 cells
    } else {
      const dim3 grid(static_cast<unsigned>(N / 16 * N), nbox);
      hipLaunchKernelGGL(patch_fwd_z_kernel<N>, grid, dim3(kPatchFwdNT), 0, s, patches, pcap,
                         reg_count, reg_list, rho_fb, n_fb, out, tw, scale, delta_out);
      return hipGetLastError();
    }
  }
};
hipError_t launch_patch_fwd_z(int n, const unsigned long long* patches, const int* reg_count,
                              const int4* reg_list, unsigned long long* rho_fb, const int* n_fb,
                              float2* out, const float2* tw, double scale, int nbox,
                              hipStream_t s, float* delta_out) {
  return dispatch_n<PatchFwdZ>(n, patches, kPatchCap, reg_count, reg_list, rho_fb, n_fb, out, tw,
                               scale, nbox, s, delta_out);
}
hipError_t launch_fwd_x_bin(int n, float2* data, const float2* tw, const uint16_t* bin_of_n2,
                            double* partial, int nbins, int nbox, hipStream_t s, int v) {
  return dispatch_n<FwdX>(n, data, tw, bin_of_n2, partial, nbins, nbox, s, v);
}
int fwd_x_partials(int n, int v) {
  int out = 0;
  if (dispatch_n<Partials>(n, &out, v) != hipSuccess) return 0;
  return out;
}
int fft_tile(int n, int pass, int v) {
  int out = 0;
  if (dispatch_n<TileOf>(n, &out, pass, v) != hipSuccess) return 0;
  return out;
}
hipError_t launch_inv_x(int n, const float2* dk, float2* f1, float2* f2, const float2* tw,
                        const uint32_t* ridx, const int* next, const double* ratio,
                        const RespBox* boxes, int nbins, const float* inv_w2, float cfac,
                        float kf, int nbox, hipStream_t s, int v) {
  return dispatch_n<InvX>(n, dk, f1, f2, tw, ridx, next, ratio, boxes, nbins, inv_w2, cfac, kf,
                          nbox, s, v);
}
hipError_t launch_inv_y(int n, const float2* f1, const float2* f2, float2* g1, float2* g2,
                        float2* g3, const float2* tw, float kf, int nbox, hipStream_t s, int v) {
  return dispatch_n<InvY>(n, f1, f2, g1, g2, g3, tw, kf, nbox, s, v);
}
hipError_t launch_inv_xy(int n, const float2* dk, float2* g1, float2* g2, float2* g3,
                         const float2* tw, const uint32_t* ridx, const int* next,
                         const double* ratio, const RespBox* boxes, int nbins, const float* iw,
                         float cgreen, float kf, int nbox, hipStream_t s) {
  return dispatch_n<InvXY>(n, dk, g1, g2, g3, tw, ridx, next, ratio, boxes, nbins, iw, cgreen,
                           kf, nbox, s);
}
hipError_t launch_inv_yz(int n, const float2* f1, const float2* f2, float* out, const float2* tw,
                         float kf, int nbox, hipStream_t s) {
  return dispatch_n<InvYZ>(n, f1, f2, out, tw, kf, nbox, s);
}
hipError_t launch_inv_z(int n, const float2* g1, const float2* g2, const float2* g3, float* out,
                        const float2* tw, float kf, int nbox, hipStream_t s, int v) {
  return dispatch_n<InvZ>(n, g1, g2, g3, out, tw, kf, nbox, s, v);
}
hipError_t launch_copy_modes(int n, const float2* ck, float2* out, int box, hipStream_t s) {
  return dispatch_n<CopyModes>(n, ck, out, box, s);
}

}  // namespace pmnu
