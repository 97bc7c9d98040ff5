// Surrogate network for the neutrino history integral (gfx950): an MLP
// 16 -> 128 -> 128 -> 128 -> 1 with GELU hidden activations. Weights are rounded to
// bfloat16 (round to nearest even); every layer's input is carried as two bfloat16 parts,
// hi = bf16(v) and lo = bf16(v - hi) (a 16-bit significand), and multiplied by the weights as
// two bf16 products with FP32 accumulation; biases, pre-activations, GELU, the loss and all
// gradients are FP32. (A layer input rounded to one bfloat16 alone limits the network to
// about 2e-3 in ln R; the second part removes that floor.)
//
// Training runs on the matrix cores: mlp_train_kernel takes 32 samples per workgroup
// through the forward pass (bf16 MFMA tiles, 16x16x32 where K is a multiple of 32 and
// 16x16x16 for the 16 inputs, activations kept in LDS) and the backward pass (weight
// gradients H^T dZ and input gradients dZ W^T, also on MFMA, with dZ rounded to bfloat16
// as MFMA operand), and adds its share of the gradient to an FP32 buffer with global
// atomics. adam_kernel applies one Adam step to the FP32 masters.
//
// Inside the step one bin is one row, so a matrix-core tile would be 1/16 full:
// surrogate_response_kernel, one workgroup per (bin, box) like the exact response, forms
// P_cdm and the bin's inputs and takes the row through the network as FP32 dot products
// with the bfloat16 weights (packed once per weight change) held in registers, fetched at
// the start so that their latency hides behind the P_cdm reduction; it runs the exact
// integral (response_device.hpp) for a bin whose inputs fall outside the training range
// (or for every bin when checking). Its activations are FP32 where training carries them
// as hi + lo bfloat16 pairs (16-bit significand): the two agree to about 1e-5 in ln R.
#include "response_device.hpp"
#include "surrogate_layout.hpp"

namespace pmnu {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;
constexpr int TB = 32;   // samples per training workgroup

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<unsigned short>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<unsigned short>(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(static_cast<unsigned>(h) << 16); }
__device__ __forceinline__ float bfr(float f) { return bf2f(f2bf(f)); }
// v as hi + lo, both bfloat16
__device__ __forceinline__ void split_bf(float v, unsigned short& hi, unsigned short& lo) {
  hi = f2bf(v);
  lo = f2bf(v - bf2f(hi));
}

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// acc += A(16 x K) * B(K x 16) for one 16x16 tile, K a multiple of 16, operands bf16 in
// LDS with element (m, k) of A at A[m*sam + k*sak] and (k, n) of B at B[k*sbk + n*sbn].
// With K a multiple of 32 it takes gfx950's 16x16x32 steps (lane l supplies row l%16 of A /
// column l%16 of B for k = 8*(l/16) .. +7 of every 32-wide step), otherwise 16x16x16 steps
// (k = 4*(l/16) .. +3 of every 16-wide step); either way lane l receives rows
// 4*(l/16) .. +3 of column l%16 of the result.
__device__ __forceinline__ f32x4 mma16(const unsigned short* A, int sam, int sak,
                                       const unsigned short* B, int sbk, int sbn, int K,
                                       f32x4 acc) {
  const int l = threadIdx.x & 63, r = l & 15;
  if (K % 32 == 0) {
    const int kb = (l >> 4) << 3;
    for (int k0 = 0; k0 < K; k0 += 32) {
      s16x8 a, b;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a[q] = static_cast<short>(A[r * sam + (k0 + kb + q) * sak]);
        b[q] = static_cast<short>(B[(k0 + kb + q) * sbk + r * sbn]);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                     __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
    }
    return acc;
  }
  const int kb = (l >> 4) << 2;
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = static_cast<short>(A[r * sam + (k0 + kb + q) * sak]);
      b[q] = static_cast<short>(B[(k0 + kb + q) * sbk + r * sbn]);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

struct Smem {
  unsigned short x[2][TB * 16];       // standardised inputs, K padded to 16 (bf16 hi, lo)
  unsigned short h[3][2][TB * 128];   // inputs of layers 2, 3, 4: H1, H2, H3 (bf16 hi, lo)
  float z[3][TB * 128];               // pre-activations Z1..Z3, later dZ (FP32)
  alignas(16) unsigned short w[128 * 128];   // one staged weight matrix as [out][in] (bf16)
  unsigned short d[TB * 128];         // dZ of the current layer (bf16)
  float y[TB];
  float dy[TB];
};

// W[in][out] (FP32 master, row-major) -> S.w[out*kin + in] (bf16); rows in >= nin are 0.
// Loads go out in batches of 16 per thread before their LDS stores.
__device__ __forceinline__ void stage_weights(Smem& S, const float* W, int nin, int kin) {
  constexpr int BATCH = 16;
  const int total = kin * 128;
  for (int t0 = 0; t0 < total; t0 += BATCH * NT) {
    float v[BATCH];
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int t = t0 + threadIdx.x + q * NT, i = t / 128, o = t % 128;
      v[q] = (t < total && i < nin) ? W[i * 128 + o] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int t = t0 + threadIdx.x + q * NT, i = t / 128, o = t % 128;
      if (t < total) S.w[o * kin + i] = f2bf(v[q]);
    }
  }
}

// Z = H W + b for the 32 x 128 tile (H as its hi and lo parts); writes Z (FP32) and
// GELU(Z) as hi and lo parts
__device__ __forceinline__ void dense_gelu(Smem& S, const unsigned short* Hhi,
                                           const unsigned short* Hlo, int kin,
                                           const float* bias, float* Z, unsigned short* Ohi,
                                           unsigned short* Olo) {
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int t = wv; t < 16; t += NT / 64) {
    const int mt = t >> 3, nt = t & 7;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mma16(Hhi + mt * 16 * kin, kin, 1, S.w + nt * 16 * kin, 1, kin, kin, acc);
    acc = mma16(Hlo + mt * 16 * kin, kin, 1, S.w + nt * 16 * kin, 1, kin, kin, acc);
    const int col = nt * 16 + (l & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = mt * 16 + ((l >> 4) << 2) + q;
      const float z = acc[q] + bias[col];
      Z[row * 128 + col] = z;
      split_bf(gelu(z), Ohi[row * 128 + col], Olo[row * 128 + col]);
    }
  }
}

// output layer: 8 lanes per sample, 16 products each, FP32
__device__ __forceinline__ void output_layer(Smem& S, const float* P) {
  const int tid = threadIdx.x;
  {
    const int s = tid >> 3, part = tid & 7;
    float acc = 0.f;
#pragma unroll
    for (int j = part * 16; j < part * 16 + 16; ++j)
      acc += (bf2f(S.h[2][0][s * 128 + j]) + bf2f(S.h[2][1][s * 128 + j])) * bfr(P[kOffW4 + j]);
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    if (part == 0) S.y[s] = acc + P[kOffB4];
  }
  __syncthreads();
}

// bfloat16 image of W1..W3 in the staged layout ([out][in], the first layer's K padded to
// 16), so that inference stages a layer with 16-byte copies
constexpr int kPackW1 = 0;
constexpr int kPackW2 = kPackW1 + 128 * 16;
constexpr int kPackW3 = kPackW2 + 128 * 128;
constexpr int kPackSize = kPackW3 + 128 * 128;

// Layers 1-3 of the forward pass on S.x (already standardised, bf16); weights staged from
// the FP32 masters P.
__device__ __forceinline__ void hidden_layers(Smem& S, const float* P) {
  stage_weights(S, P + kOffW1, kSurIn, 16);
  __syncthreads();
  dense_gelu(S, S.x[0], S.x[1], 16, P + kOffB1, S.z[0], S.h[0][0], S.h[0][1]);
  __syncthreads();
  stage_weights(S, P + kOffW2, 128, 128);
  __syncthreads();
  dense_gelu(S, S.h[0][0], S.h[0][1], 128, P + kOffB2, S.z[1], S.h[1][0], S.h[1][1]);
  __syncthreads();
  stage_weights(S, P + kOffW3, 128, 128);
  __syncthreads();
  dense_gelu(S, S.h[1][0], S.h[1][1], 128, P + kOffB3, S.z[2], S.h[2][0], S.h[2][1]);
  __syncthreads();
  output_layer(S, P);
}

// Forward pass of up to TB rows starting at row0 (through perm if given). Leaves y (the
// standardised output) in S.y.
__device__ __forceinline__ void forward_tile(Smem& S, const float* P, const float* x, const int* perm,
                             int64_t row0, int count) {
  const int tid = threadIdx.x;
  for (int t = tid; t < TB * 16; t += NT) {
    const int s = t >> 4, i = t & 15;
    float v = 0.f;
    if (i < kSurIn && s < count) {
      const int64_t r = perm ? perm[row0 + s] : row0 + s;
      v = (x[r * kSurIn + i] - P[kOffMu + i]) / P[kOffSigma + i];
    }
    split_bf(v, S.x[0][t], S.x[1][t]);
  }
  hidden_layers(S, P);
}

// dW (kin x 128) += Hin^T dZ for the 32-row tile (rows i < nin), Hin as hi and lo parts,
// with atomics
__device__ __forceinline__ void weight_grad(Smem& S, const unsigned short* Hhi,
                                            const unsigned short* Hlo, int kin, int nin,
                                            float* gW) {
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int ntiles = (kin / 16) * 8;
  for (int t = wv; t < ntiles; t += NT / 64) {
    const int mt = t >> 3, nt = t & 7;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mma16(Hhi + mt * 16, 1, kin, S.d + nt * 16, 128, 1, TB, acc);
    acc = mma16(Hlo + mt * 16, 1, kin, S.d + nt * 16, 128, 1, TB, acc);
    const int col = nt * 16 + (l & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = mt * 16 + ((l >> 4) << 2) + q;
      if (row < nin) atomicAdd(gW + row * 128 + col, acc[q]);
    }
  }
}

// db (128) += column sums of dZ (FP32, held in Z)
__device__ __forceinline__ void bias_grad(const float* dZ, float* gb) {
  const int j = threadIdx.x;
  if (j < 128) {
    float s = 0.f;
    for (int r = 0; r < TB; ++r) s += dZ[r * 128 + j];
    atomicAdd(gb + j, s);
  }
}

// dZ_prev = (dZ W^T) * GELU'(Z_prev), W staged as [out][in] with in = 128
__device__ __forceinline__ void backprop_hidden(Smem& S, float* Zprev) {
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  f32x4 res[4];
  int tiles = 0;
  for (int t = wv; t < 16; t += NT / 64, ++tiles) {
    const int mt = t >> 3, nt = t & 7;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    // A(m = sample, k = out) = dZ[s][o]; B(k = out, n = in) = W[in][out] = S.w[out*128 + in]
    res[tiles] = mma16(S.d + mt * 16 * 128, 128, 1, S.w + nt * 16, 128, 1, 128, acc);
  }
  __syncthreads();   // every wave is done reading S.d
  tiles = 0;
  for (int t = wv; t < 16; t += NT / 64, ++tiles) {
    const int mt = t >> 3, nt = t & 7;
    const int col = nt * 16 + (l & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = mt * 16 + ((l >> 4) << 2) + q;
      const float dz = res[tiles][q] * gelu_grad(Zprev[row * 128 + col]);
      Zprev[row * 128 + col] = dz;
      S.d[row * 128 + col] = f2bf(dz);
    }
  }
  __syncthreads();
}

// Forward + backward of one 32-row tile of the minibatch rows [row0, row0 + count).
__global__ __launch_bounds__(NT) void mlp_train_kernel(const float* __restrict__ P,
                                                       const float* __restrict__ x,
                                                       const float* __restrict__ y,
                                                       const int* __restrict__ perm,
                                                       int64_t row0, int64_t count,
                                                       float inv_batch, float* __restrict__ grad,
                                                       float* __restrict__ loss_sum) {
  __shared__ Smem S;
  const int tid = threadIdx.x;
  const int64_t base = row0 + static_cast<int64_t>(blockIdx.x) * TB;
  const int cnt = static_cast<int>(min(static_cast<int64_t>(TB), row0 + count - base));
  forward_tile(S, P, x, perm, base, cnt);

  // loss and dL/dy on the standardised target
  if (tid < 64) {
    float l2 = 0.f, dy = 0.f;
    if (tid < TB && tid < cnt) {
      const int64_t r = perm ? perm[base + tid] : base + tid;
      const float t = (y[r] - P[kOffYMu]) / P[kOffYSigma];
      if (isfinite(t)) {
        const float res = S.y[tid] - t;
        l2 = res * res;
        dy = 2.0f * res * inv_batch;
      }
    }
    if (tid < TB) S.dy[tid] = dy;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) l2 += __shfl_xor(l2, off, 64);
    if (tid == 0) atomicAdd(loss_sum, l2);
  }
  __syncthreads();
  // output layer
  if (tid < 128) {
    float g = 0.f;
    for (int s = 0; s < TB; ++s)
      g += (bf2f(S.h[2][0][s * 128 + tid]) + bf2f(S.h[2][1][s * 128 + tid])) * S.dy[s];
    atomicAdd(grad + kOffW4 + tid, g);
  } else if (tid == 128) {
    float g = 0.f;
    for (int s = 0; s < TB; ++s) g += S.dy[s];
    atomicAdd(grad + kOffB4, g);
  }
  for (int t = tid; t < TB * 128; t += NT) {
    const int s = t >> 7, j = t & 127;
    const float dz = S.dy[s] * bfr(P[kOffW4 + j]) * gelu_grad(S.z[2][t]);
    S.z[2][t] = dz;
    S.d[t] = f2bf(dz);
  }
  __syncthreads();
  // layer 3: W3 (H2 -> Z3)
  bias_grad(S.z[2], grad + kOffB3);
  weight_grad(S, S.h[1][0], S.h[1][1], 128, 128, grad + kOffW3);
  stage_weights(S, P + kOffW3, 128, 128);
  __syncthreads();
  backprop_hidden(S, S.z[1]);
  // layer 2: W2 (H1 -> Z2)
  bias_grad(S.z[1], grad + kOffB2);
  weight_grad(S, S.h[0][0], S.h[0][1], 128, 128, grad + kOffW2);
  stage_weights(S, P + kOffW2, 128, 128);
  __syncthreads();
  backprop_hidden(S, S.z[0]);
  // layer 1: W1 (X -> Z1)
  bias_grad(S.z[0], grad + kOffB1);
  weight_grad(S, S.x[0], S.x[1], 16, kSurIn, grad + kOffW1);
}

__global__ __launch_bounds__(NT) void mlp_predict_kernel(const float* __restrict__ P,
                                                         const float* __restrict__ x,
                                                         float* __restrict__ y, int64_t n) {
  __shared__ Smem S;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * TB;
  const int cnt = static_cast<int>(min(static_cast<int64_t>(TB), n - base));
  forward_tile(S, P, x, nullptr, base, cnt);
  if (threadIdx.x < cnt) y[base + threadIdx.x] = S.y[threadIdx.x] * P[kOffYSigma] + P[kOffYMu];
}

__global__ void adam_kernel(float* __restrict__ P, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- in the step ----
// Inputs of (box, bin) as surrogate_layout.hpp defines them, from the stored history
// (hpm, hpn: this box's rows), the lag brackets the host put in the box's constants and
// box constants the host precomputed. Every value read from memory is one entry of a
// staging array, so that a workgroup can fetch them with one load per lane, all in flight
// together, before the P_cdm reduction (gather_value), and the inputs are formed once
// P_cdm^{1/2} is known (finish_features).
enum : int {
  kGLo = 0,                    // A at node sur_j[m]
  kGHi = kSurLags,             // A at node sur_j[m] + 1 (node sur_j[m] itself when sur_t = 0)
  kGT = 2 * kSurLags,          // sur_t[m]
  kGPn = 3 * kSurLags,         // P_nu^{1/2} at the last stored node
  kGLnA, kGM, kGGap, kGLnA0, kGLnX0,
  kGCount
};

__device__ __forceinline__ bool features_defined(const RespBox& bx) {
  return bx.sur_ok && bx.sur_hist && bx.kfs > 0.0;
}

__device__ __forceinline__ double gather_value(const RespBox* __restrict__ bxp,
                                               const double* hpm, const double* hpn, int nbins,
                                               int b, int i) {
  if (i < kGHi) return hpm[static_cast<size_t>(bxp->sur_j[i]) * nbins + b];
  if (i < kGT) {
    const int m = i - kGHi;
    return hpm[static_cast<size_t>(bxp->sur_j[m] + (bxp->sur_t[m] > 0.0 ? 1 : 0)) * nbins + b];
  }
  if (i < kGPn) return bxp->sur_t[i - kGT];
  switch (i) {
    case kGPn: return hpn[static_cast<size_t>(bxp->n_cur - 1) * nbins + b];
    case kGLnA: return bxp->sur_lna;
    case kGM: return bxp->m_total;
    case kGGap: return bxp->sur_gap;
    case kGLnA0: return bxp->sur_lna0;
    default: return bxp->sur_lnx0;
  }
}

// Input i (FP64, before the rounding to FP32), one input per call so that the lanes of a
// wave can form the inputs of a row together
__device__ __forceinline__ double feature_value(int i, double k, double pcdm_half,
                                                const double* g) {
  switch (i) {
    case 0: return log(k);
    case 1: return g[kGLnA];
    case 2: return g[kGM];
    case 3: return g[kGGap];
    case 4: return g[kGPn] / pcdm_half;
    case 5: return g[kGLnA0];
    case 6: return log(k) + g[kGLnX0];
    default: {
      const int m = i - 7;
      const double t = g[kGT + m];
      return ((1.0 - t) * g[kGLo + m] + t * g[kGHi + m]) / pcdm_half;
    }
  }
}

// whether input i's value keeps the row in the network's domain (input 6, the
// free-streaming argument across the last interval, at most kSurXLastMax)
__device__ __forceinline__ bool feature_in_domain(int i, double v) {
  return i != 6 || v <= kSurXLastMax;
}

__device__ __forceinline__ bool finish_features(double k, double pcdm_half, const double* g,
                                                float* f) {
  if (!(pcdm_half > 0.0)) return false;
  bool in = true;
  for (int i = 0; i < kSurIn; ++i) {
    const double v = feature_value(i, k, pcdm_half, g);
    in = in && feature_in_domain(i, v);
    f[i] = static_cast<float>(v);
  }
  return in;
}

// The inputs of one (box, bin) in one thread (training rows)
__device__ __forceinline__ bool make_features(const RespBox* __restrict__ bxp, double k,
                                              double pcdm_half, const double* hpm,
                                              const double* hpn, int nbins, int b, float* f) {
  if (!features_defined(*bxp)) return false;
  double g[kGCount];
#pragma unroll
  for (int i = 0; i < kGCount; ++i) g[i] = gather_value(bxp, hpm, hpn, nbins, b, i);
  return finish_features(k, pcdm_half, g, f);
}

__device__ __forceinline__ double approx_factor(double k, double kfs) {
  const double t = 1.0 + k / kfs;
  return 1.0 / (t * t);
}

__global__ void pack_weights_kernel(const float* __restrict__ P, unsigned short* __restrict__ Q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kPackW2) {
    const int o = i / 16, in = i % 16;
    Q[i] = in < kSurIn ? f2bf(P[kOffW1 + in * 128 + o]) : static_cast<unsigned short>(0);
  } else if (i < kPackW3) {
    const int j = i - kPackW2, o = j / 128, in = j % 128;
    Q[i] = f2bf(P[kOffW2 + in * 128 + o]);
  } else if (i < kPackSize) {
    const int j = i - kPackW3, o = j / 128, in = j % 128;
    Q[i] = f2bf(P[kOffW3 + in * 128 + o]);
  }
}

// ---- one row through the network inside a workgroup of RT = 256 threads ----
// The weights come from the packed bfloat16 image Q ([out][in] rows) in 16-byte chunks of 8
// inputs. Layer 1 (128 x 16, 256 chunks): thread t holds chunk t, output t / 2, inputs
// 8 (t % 2) .. +7. Layers 2 and 3 (128 x 128, 2048 chunks): thread t holds chunks
// t + 256 u, u = 0..7, i.e. inputs 8 (t % 16) .. +7 of outputs t / 16 + 16 u; each load
// instruction of a wave covers 1 KB of contiguous weights. Activations stay FP32.
// The biases a thread adds are those of the output it finishes: t / 2 in layer 1 and
// hidden_out(t) in layers 2 and 3; thread t holds W4[t % 128] (threads t < 128 use it).
// Every load here is unconditional and its value first used after the P_cdm reduction, so
// that no wait for one of them stands between the loads and the reduction's own.
__device__ __forceinline__ int hidden_out(int t) {
  return (t >> 4) + 16 * (4 * ((t >> 3) & 1) + 2 * ((t >> 2) & 1) + ((t >> 1) & 1));
}

struct NetRegs {
  uint4 w1;
  uint4 w2[8], w3[8];
  float b1, b2, b3, w4;
  float b4, ymu, ysg;   // output bias, target mean and scale
};

__device__ __forceinline__ void load_net_weights(const float* __restrict__ P,
                                                 const unsigned short* __restrict__ Q, int t,
                                                 NetRegs& r) {
  const uint4* q = reinterpret_cast<const uint4*>(Q);
  r.w1 = q[kPackW1 / 8 + t];
#pragma unroll
  for (int u = 0; u < 8; ++u) r.w2[u] = q[kPackW2 / 8 + t + 256 * u];
#pragma unroll
  for (int u = 0; u < 8; ++u) r.w3[u] = q[kPackW3 / 8 + t + 256 * u];
  const int o = hidden_out(t);
  r.b1 = P[kOffB1 + (t >> 1)];
  r.b2 = P[kOffB2 + o];
  r.b3 = P[kOffB3 + o];
  r.w4 = P[kOffW4 + (t & 127)];   // used (bf16-rounded) by threads t < 128
  r.b4 = P[kOffB4];
  r.ymu = P[kOffYMu];
  r.ysg = P[kOffYSigma];
}

// sum_j a[j] w[j] over one chunk (w: 8 bfloat16 in a uint4)
__device__ __forceinline__ float chunk_dot(const float* a, const uint4& w) {
  const unsigned v[4] = {w.x, w.y, w.z, w.w};
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    s += a[2 * i] * __uint_as_float(v[i] << 16);
    s += a[2 * i + 1] * __uint_as_float(v[i] & 0xffff0000u);
  }
  return s;
}

// One 128 x 128 layer: h_out = GELU(W h_in + b). Each thread has the partial sums of 8
// outputs over its 8 inputs; the 16 threads sharing those outputs (16 consecutive lanes)
// add them in a butterfly that halves the outputs each lane carries at every step, after
// which lane pair (2v, 2v+1) of the group holds output (t / 16) + 16 u with
// u = 4 b3 + 2 b2 + b1 from the lane's bits.
__device__ __forceinline__ void hidden_128(const float* __restrict__ hin, const uint4* w,
                                           float bias, float* hout) {
  const int t = threadIdx.x, c = t & 15;
  float a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = hin[8 * c + j];
  float v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = chunk_dot(a, w[u]);
  const bool b3 = (t >> 3) & 1, b2 = (t >> 2) & 1, b1 = (t >> 1) & 1;
  float x4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float keep = b3 ? v[4 + i] : v[i], send = b3 ? v[i] : v[4 + i];
    x4[i] = keep + __shfl_xor(send, 8, 64);
  }
  float x2[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float keep = b2 ? x4[2 + i] : x4[i], send = b2 ? x4[i] : x4[2 + i];
    x2[i] = keep + __shfl_xor(send, 4, 64);
  }
  const float keep = b1 ? x2[1] : x2[0], send = b1 ? x2[0] : x2[1];
  float z = keep + __shfl_xor(send, 2, 64);
  z += __shfl_xor(z, 1, 64);
  if (!(t & 1)) hout[hidden_out(t)] = gelu(z + bias);
}

// The row's output y (standardised target) without the output bias, in every thread.
// x: the 16 standardised inputs in LDS; h0, h1: two 128-float LDS rows; red: RT / 64 floats.
__device__ __forceinline__ float net_forward(const NetRegs& r, const float* x, float* h0,
                                             float* h1, float* red) {
  const int t = threadIdx.x;
  {
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = x[8 * (t & 1) + j];
    float z = chunk_dot(a, r.w1);
    z += __shfl_xor(z, 1, 64);
    if (!(t & 1)) h0[t >> 1] = gelu(z + r.b1);
  }
  __syncthreads();
  hidden_128(h0, r.w2, r.b2, h1);
  __syncthreads();
  hidden_128(h1, r.w3, r.b3, h0);
  __syncthreads();
  float s = t < 128 ? h0[t] * bfr(r.w4) : 0.f;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  if ((t & 63) == 0) red[t >> 6] = s;
  __syncthreads();
  float y = 0.f;
#pragma unroll
  for (int w = 0; w < RT / 64; ++w) y += red[w];
  return y;
}

// The surrogate's response, one workgroup per (bin b, box), as response_kernel but with the
// network in place of the history integral where it can answer: P_cdm from the deposit's
// partial sums, the bin's inputs (their memory reads and the network's weights are issued
// before the partial sums, so that the latencies overlap), the
// network's R, and the exact integral (response_device.hpp) for a bin whose inputs are not
// defined or fall outside the training range. Mode 1 keeps the network's R; mode 2 (check)
// keeps the exact result and records the network's beside it.
__global__ __launch_bounds__(RT) void surrogate_response_kernel(
    const float* __restrict__ P, const unsigned short* __restrict__ Q, int mode,
    const RespBox* __restrict__ boxes, const double* __restrict__ partial, int n_partial,
    const double* __restrict__ counts, const double* __restrict__ kmean,
    double* __restrict__ hist_pm, double* __restrict__ hist_pnu,
    const double* __restrict__ ic_pnu, const double* __restrict__ ic_theta,
    const double* __restrict__ tg_ds, const double* __restrict__ tg_l2,
    const double* __restrict__ tg_w, int nbins, int jcap, int qcap, int q_sub, int iterations,
    double norm, double* __restrict__ pcdm_out, double* __restrict__ pnu_out,
    double* __restrict__ ratio_out, double* __restrict__ sur_r, double* __restrict__ chk_exact,
    double* __restrict__ chk_sur) {
  __shared__ double red[2 * RT / 64];
  __shared__ float xs[kSurIn];
  __shared__ float h0[128], h1[128];
  __shared__ float redf[RT / 64];
  __shared__ float scal[4 * kSurIn];   // the inputs' mean, scale, minimum, maximum
  __shared__ double gsh[kGCount];      // the staged values of the inputs
  __shared__ int s_ok;
  const int tid = threadIdx.x;
  const int b = blockIdx.x, box = blockIdx.y;
  const size_t ob = static_cast<size_t>(box) * nbins + b;
  const RespBox* bxp = boxes + box;
  const RespBox bx = *bxp;
  double* hpm = hist_pm + static_cast<size_t>(box) * jcap * nbins;
  double* hpn = hist_pnu + static_cast<size_t>(box) * jcap * nbins;
  const size_t row = static_cast<size_t>(bx.n_cur) * nbins + b;
  const double cb = counts[b];
  const bool defined = cb > 0.0 && features_defined(bx);   // uniform over the workgroup
  const double kb = kmean[b];
  // fetched before the reduction: one staged value per lane and the scalers
  double gv = 0.0;
  float sc = 0.f;
  if (defined) {
    if (tid < kGCount) gv = gather_value(bxp, hpm, hpn, nbins, b, tid);
    if (tid < 4 * kSurIn) sc = P[kOffMu + tid];   // kOffMu .. kOffMax + kSurIn are contiguous
  }
  // the weights too: the reduction then waits for them as well (a wave consumes its loads
  // in issue order), which costs less than their latency after it (14.5 against 15.3 us)
  NetRegs w;
  if (defined) load_net_weights(P, Q, tid, w);
  const double msum = bin_mode_sum(partial, n_partial, nbins, box, b, red);   // has barriers
  const double pcdm = cb > 0.0 ? norm * msum / cb : 0.0;
  const double ph = sqrt(pcdm);
  if (defined) {
    if (tid < 4 * kSurIn) scal[tid] = sc;
    if (tid < kGCount) gsh[tid] = gv;
    __syncthreads();
  }
  if (tid < 64) {
    // lane i < kSurIn forms input i; the row is used when every input is in the network's
    // domain and within the training range (5% margin)
    bool in = true;
    float fv = 0.f;
    if (defined && ph > 0.0 && tid < kSurIn) {
      const double v = feature_value(tid, kb, ph, gsh);
      fv = static_cast<float>(v);
      const float lo = scal[2 * kSurIn + tid], hi = scal[3 * kSurIn + tid];
      const float mg = 0.05f * (hi - lo);
      in = feature_in_domain(tid, v) && fv >= lo - mg && fv <= hi + mg;
    }
    const bool ok = defined && ph > 0.0 && __all(in);
    if (ok && tid < kSurIn) xs[tid] = (fv - scal[tid]) / scal[kSurIn + tid];
    if (tid == 0) s_ok = ok ? 1 : 0;
  }
  if (tid == 0) {
    const bool ok = s_ok != 0;
    pcdm_out[ob] = pcdm;
    if (!(cb > 0.0)) {
      sur_r[ob] = __builtin_nan("");
      pnu_out[ob] = ratio_out[ob] = 0.0;
      hpm[row] = hpn[row] = 0.0;
      if (chk_exact) chk_exact[ob] = chk_sur[ob] = 0.0;
    } else if (!ok) {
      sur_r[ob] = __builtin_nan("");
    }
  }
  __syncthreads();
  const bool ok = s_ok != 0;
  if (ok) {
    const float y = net_forward(w, xs, h0, h1, redf) + w.b4;
    if (tid == 0) {
      const double r_net = exp(static_cast<double>(y * w.ysg + w.ymu)) *
                           approx_factor(kb, bx.kfs);
      sur_r[ob] = r_net;
      if (mode == 1) {
        const double pnu = r_net * ph;
        pnu_out[ob] = pnu;
        ratio_out[ob] = r_net;
        hpm[row] = (1.0 - bx.f_nu) * ph + bx.f_nu * pnu;
        hpn[row] = pnu;
      } else if (chk_sur) {
        chk_sur[ob] = r_net;
      }
    }
  }
  if (cb > 0.0 && (!ok || mode == 2)) {
    const double pnu = exact_pnu(bx, kb, ph, (bx.n_cur > 0 ? hpn[row - nbins] : 0.0),
                                 ic_pnu + static_cast<size_t>(box) * kMaxSpecies * nbins,
                                 ic_theta[ob], hpm, nbins, b,
                                 tg_ds + static_cast<size_t>(box) * qcap,
                                 tg_l2 + static_cast<size_t>(box) * qcap,
                                 tg_w + static_cast<size_t>(box) * qcap, q_sub, iterations, red);
    if (tid == 0) {
      const double r = ph > 0.0 ? pnu / ph : 0.0;   // no CDM power in the bin: R = 0
      pnu_out[ob] = pnu;
      ratio_out[ob] = r;
      hpm[row] = (1.0 - bx.f_nu) * ph + bx.f_nu * pnu;
      hpn[row] = pnu;
      if (chk_exact) {
        chk_exact[ob] = r;
        if (!ok) chk_sur[ob] = r;             // the network did not answer for this bin
      }
    }
  }
}

// Training rows from the step's state after an exact response: one thread per (box, bin).
__global__ void dataset_kernel(const RespBox* __restrict__ boxes, const double* __restrict__ pcdm,
                               const double* __restrict__ ratio, const double* __restrict__ kmean,
                               const double* __restrict__ hist_pm,
                               const double* __restrict__ hist_pnu, int nbins, int jcap,
                               int nbox, float* __restrict__ x, float* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbox * nbins) return;
  const int box = i / nbins, b = i % nbins;
  const RespBox bx = boxes[box];
  const double ph = sqrt(pcdm[i]);
  const double r = ratio[i];
  float f[kSurIn];
  const size_t hoff = static_cast<size_t>(box) * jcap * nbins;
  bool ok = make_features(boxes + box, kmean[b], ph, hist_pm + hoff, hist_pnu + hoff, nbins, b,
                          f) &&
            r > 0.0;
  for (int c = 0; c < kSurIn; ++c) x[static_cast<size_t>(i) * kSurIn + c] = ok ? f[c] : 0.f;
  y[i] = ok ? static_cast<float>(log(r / approx_factor(kmean[b], bx.kfs)))
            : __builtin_nanf("");
}

}  // namespace

hipError_t launch_mlp_train(const float* P, const float* x, const float* y, const int* perm,
                            int64_t row0, int64_t count, float inv_batch, float* grad,
                            float* loss_sum, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((count + TB - 1) / TB);
  hipLaunchKernelGGL(mlp_train_kernel, dim3(blocks), dim3(NT), 0, s, P, x, y, perm, row0, count,
                     inv_batch, grad, loss_sum);
  return hipGetLastError();
}

hipError_t launch_mlp_predict(const float* P, const float* x, float* y, int64_t n, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((n + TB - 1) / TB);
  hipLaunchKernelGGL(mlp_predict_kernel, dim3(blocks), dim3(NT), 0, s, P, x, y, n);
  return hipGetLastError();
}

hipError_t launch_adam(float* P, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, P, g, m, v, n, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const float* P, unsigned short* Q, hipStream_t s) {
  hipLaunchKernelGGL(pack_weights_kernel, dim3((kPackSize + 255) / 256), dim3(256), 0, s, P, Q);
  return hipGetLastError();
}

int64_t packed_weight_count() { return kPackSize; }

hipError_t launch_surrogate_response(const float* P, const unsigned short* Q, int mode,
                                     const RespBox* boxes, const double* partial, int n_partial,
                                     const double* counts, const double* kmean, double* hist_pm,
                                     double* hist_pnu, const double* ic_pnu,
                                     const double* ic_theta, const double* tg_ds,
                                     const double* tg_l2, const double* tg_w, int nbins, int jcap,
                                     int qcap, int q_sub, int iterations, double norm, int nbox,
                                     double* pcdm, double* pnu, double* ratio, double* sur_r,
                                     double* chk_exact, double* chk_sur, hipStream_t s) {
  hipLaunchKernelGGL(surrogate_response_kernel, dim3(nbins, nbox), dim3(RT), 0, s, P, Q, mode,
                     boxes, partial, n_partial, counts, kmean, hist_pm, hist_pnu, ic_pnu,
                     ic_theta, tg_ds, tg_l2, tg_w, nbins, jcap, qcap, q_sub, iterations, norm, pcdm,
                     pnu, ratio, sur_r, chk_exact, chk_sur);
  return hipGetLastError();
}

hipError_t launch_surrogate_dataset(const RespBox* boxes, const double* pcdm, const double* ratio,
                                    const double* kmean, const double* hist_pm,
                                    const double* hist_pnu, int nbins, int jcap, int nbox,
                                    float* x, float* y, hipStream_t s) {
  const int n = nbox * nbins;
  hipLaunchKernelGGL(dataset_kernel, dim3((n + 255) / 256), dim3(256), 0, s, boxes, pcdm, ratio,
                     kmean, hist_pm, hist_pnu, nbins, jcap, nbox, x, y);
  return hipGetLastError();
}

}  // namespace pmnu
