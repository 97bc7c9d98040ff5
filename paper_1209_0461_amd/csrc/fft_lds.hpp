// Radix-2/4/8/16 Stockham FFT passes over lines held in LDS (gfx950, wave64, FP32).
//
// A workgroup keeps NL lines of length N (power of two, 8..512) in LDS, interleaved:
// element e of line l sits at lds[e * ES + l] with ES = NL + 1. Consecutive threads take
// consecutive lines, so every pass reads and writes LDS with unit stride across a wave;
// the odd element stride keeps the one strided transpose at load/store time (rows that
// are contiguous in HBM) from piling onto one bank.
//
// One pass of radix R at sub-transform size Ns (Stockham autosort, natural order in and
// out): butterfly j in [0, N/R) reads elements j + r N/R, multiplies element r by
// w^(r k), k = j mod Ns, w = exp(DIR 2 pi i / (Ns R)), does a length-R DFT in registers
// and writes element r to (j / Ns) Ns R + k + r Ns. Passes run for Ns = 1, R1, R1 R2, ...
// until Ns = N. DIR = -1 is the forward transform, +1 the (unnormalised) inverse.
#pragma once
#include <hip/hip_runtime.h>

namespace pmnu {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by DIR * i  (DIR = -1: by -i)
template <int DIR>
__device__ __forceinline__ float2 mul_dir_i(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// --------------------------------------------------------------- register DFTs ----
template <int R, int DIR> struct Dft;

template <int DIR> struct Dft<2, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int DIR> struct Dft<4, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = mul_dir_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

// exp(DIR 2 pi i m / 8) and exp(DIR 2 pi i m / 16) for the internal twiddles
__device__ __forceinline__ float2 w8(int m, int dir) {
  constexpr float h = 0.70710678118654752440f;
  float c, s;
  switch (m & 7) {
    case 0: c = 1.f; s = 0.f; break;
    case 1: c = h; s = h; break;
    case 2: c = 0.f; s = 1.f; break;
    case 3: c = -h; s = h; break;
    case 4: c = -1.f; s = 0.f; break;
    case 5: c = -h; s = -h; break;
    case 6: c = 0.f; s = -1.f; break;
    default: c = h; s = -h; break;
  }
  return make_float2(c, dir * s);
}

__device__ __forceinline__ float2 w16(int m, int dir) {
  // cos and sin of 2 pi m / 16 for m = 0..15
  constexpr float c1 = 0.92387953251128675613f;   // cos(pi/8)
  constexpr float s1 = 0.38268343236508977173f;   // sin(pi/8)
  constexpr float h = 0.70710678118654752440f;
  const float cs[16] = {1.f, c1, h, s1, 0.f, -s1, -h, -c1, -1.f, -c1, -h, -s1, 0.f, s1, h, c1};
  const float sn[16] = {0.f, s1, h, c1, 1.f, c1, h, s1, 0.f, -s1, -h, -c1, -1.f, -c1, -h, -s1};
  return make_float2(cs[m & 15], dir * sn[m & 15]);
}

// 8 = 4 (inner, over m) x 2 (outer, over p): n = 2m + p, k = k1 + 4 k2
template <int DIR> struct Dft<8, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 y0[4] = {v[0], v[2], v[4], v[6]};
    float2 y1[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, DIR>::run(y0);
    Dft<4, DIR>::run(y1);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 b = k1 ? cmul(y1[k1], w8(k1, DIR)) : y1[k1];
      v[k1] = cadd(y0[k1], b);
      v[k1 + 4] = csub(y0[k1], b);
    }
  }
};

// 16 = 4 x 4: n = 4m + p, k = k1 + 4 k2
template <int DIR> struct Dft<16, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 y[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
#pragma unroll
      for (int m = 0; m < 4; ++m) y[p][m] = v[4 * m + p];
      Dft<4, DIR>::run(y[p]);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 z[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) z[p] = (p && k1) ? cmul(y[p][k1], w16(p * k1, DIR)) : y[p][k1];
      Dft<4, DIR>::run(z);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = z[k2];
    }
  }
};

// ------------------------------------------------------------------ radix plans ----
// Radix of pass P for a length-N transform; 0 ends the plan.
__host__ __device__ constexpr int plan_radix(int n, int pass) {
  return n == 8 ? (pass == 0 ? 8 : 0)
       : n == 16 ? (pass == 0 ? 16 : 0)
       : n == 32 ? (pass == 0 ? 8 : pass == 1 ? 4 : 0)
       : n == 64 ? (pass < 2 ? 8 : 0)
       : n == 128 ? (pass == 0 ? 16 : pass == 1 ? 8 : 0)
       : n == 256 ? (pass < 2 ? 16 : 0)
       : n == 512 ? (pass < 3 ? 8 : 0)
       : 0;
}

__host__ __device__ constexpr int plan_ns(int n, int pass) {
  return pass == 0 ? 1 : plan_ns(n, pass - 1) * plan_radix(n, pass - 1);
}

// One Stockham pass over all NL lines; NT threads cooperate. tw[m] = exp(-2 pi i m / N).
template <int N, int NL, int NT, int R, int NS, int DIR, int ES>
__device__ __forceinline__ void stockham_pass(float2* lds, const float2* tw) {
  constexpr int NB = N / R;                 // butterflies per line
  constexpr int TOTAL = NL * NB;
  constexpr int CNT = (TOTAL + NT - 1) / NT;
  float2 v[CNT][R];
  const int tid = threadIdx.x;
#pragma unroll
  for (int c = 0; c < CNT; ++c) {
    const int i = tid + c * NT;
    if (TOTAL % NT == 0 || i < TOTAL) {
      const int l = i % NL, j = i / NL;
#pragma unroll
      for (int r = 0; r < R; ++r) v[c][r] = lds[(j + r * NB) * ES + l];
      if (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[(r * k * (N / (NS * R))) & (N - 1)];
          if (DIR > 0) w.y = -w.y;
          v[c][r] = cmul(v[c][r], w);
        }
      }
      Dft<R, DIR>::run(v[c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CNT; ++c) {
    const int i = tid + c * NT;
    if (TOTAL % NT == 0 || i < TOTAL) {
      const int l = i % NL, j = i / NL;
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[(base + r * NS) * ES + l] = v[c][r];
    }
  }
  __syncthreads();
}

template <int N, int NL, int NT, int DIR, int PASS, int ES>
__device__ __forceinline__ void fft_passes(float2* lds, const float2* tw) {
  if constexpr (plan_radix(N, PASS) != 0) {
    stockham_pass<N, NL, NT, plan_radix(N, PASS), plan_ns(N, PASS), DIR, ES>(lds, tw);
    fft_passes<N, NL, NT, DIR, PASS + 1, ES>(lds, tw);
  }
}

// Transform lines 0..NL-1 in place (element stride ES, NL + 1 unless the lines are the
// first NL of a wider layout). Caller must __syncthreads() before (data written) and may
// read the result after return (the last pass ends with a barrier).
template <int N, int NL, int NT, int DIR, int ES = NL + 1>
__device__ __forceinline__ void fft_lines(float2* lds, const float2* tw) {
  fft_passes<N, NL, NT, DIR, 0, ES>(lds, tw);
}

// Load the N-entry twiddle table exp(-2 pi i m / N) into LDS.
template <int N, int NT>
__device__ __forceinline__ void load_twiddles(float2* tw_lds, const float2* tw_global) {
  for (int m = threadIdx.x; m < N; m += NT) tw_lds[m] = tw_global[m];
}

}  // namespace pmnu
