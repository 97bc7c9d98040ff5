// Surrogate network for the neutrino history integral (gfx950): an MLP
// 11 -> 128 -> 128 -> 128 -> 1 with GELU hidden activations. Weights and every layer's
// input are rounded to bfloat16 (round to nearest even) and multiplied with FP32
// accumulation; biases, pre-activations, GELU, the loss and all gradients are FP32.
//
// Training runs on the matrix cores: mlp_train_kernel takes 32 samples per workgroup
// through the forward pass (16x16x16 bf16 MFMA tiles, activations kept in LDS) and the
// backward pass (weight gradients H^T dZ and input gradients dZ W^T, also on MFMA, with
// dZ rounded to bfloat16 as MFMA operand), and adds its share of the gradient to an FP32
// buffer with global atomics. adam_kernel applies one Adam step to the FP32 masters.
//
// Inside the step the network sees one row per k-bin: surrogate_response_kernel, one
// workgroup per (bin, box), forms P_cdm, takes the bin's row through the same MFMA forward
// pass with the weights staged at once from a bfloat16 image packed once per weight
// change, and falls back to the exact integral (response_device.hpp) in the same
// workgroup when the inputs are outside the training range (or when checking).
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

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// acc += A(16 x K) * B(K x 16) for one 16x16 tile, K a multiple of 16, operands bf16 in
// LDS with element (m, k) of A at A[m*sam + k*sak] and (k, n) of B at B[k*sbk + n*sbn].
// Lane l supplies row l%16 of A / column l%16 of B for k = 4*(l/16) .. +3 of every
// 16-wide K step and receives rows 4*(l/16) .. +3 of column l%16 of the result.
__device__ __forceinline__ f32x4 mma16(const unsigned short* A, int sam, int sak,
                                       const unsigned short* B, int sbk, int sbn, int K,
                                       f32x4 acc) {
  const int l = threadIdx.x & 63, r = l & 15, kb = (l >> 4) << 2;
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
  unsigned short x[TB * 16];          // standardised inputs, K padded to 16 (bf16)
  unsigned short h[3][TB * 128];      // inputs of layers 2, 3, 4: H1, H2, H3 (bf16)
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

// Z = H W + b for the 32 x 128 tile; writes Z (FP32) and GELU(Z) (bf16)
__device__ __forceinline__ void dense_gelu(Smem& S, const unsigned short* Hin, int kin,
                                           const float* bias, float* Z, unsigned short* Hout) {
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int t = wv; t < 16; t += NT / 64) {
    const int mt = t >> 3, nt = t & 7;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mma16(Hin + mt * 16 * kin, kin, 1, S.w + nt * 16 * kin, 1, kin, kin, acc);
    const int col = nt * 16 + (l & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = mt * 16 + ((l >> 4) << 2) + q;
      const float z = acc[q] + bias[col];
      Z[row * 128 + col] = z;
      Hout[row * 128 + col] = f2bf(gelu(z));
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
      acc += bf2f(S.h[2][s * 128 + j]) * bfr(P[kOffW4 + j]);
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
  dense_gelu(S, S.x, 16, P + kOffB1, S.z[0], S.h[0]);
  __syncthreads();
  stage_weights(S, P + kOffW2, 128, 128);
  __syncthreads();
  dense_gelu(S, S.h[0], 128, P + kOffB2, S.z[1], S.h[1]);
  __syncthreads();
  stage_weights(S, P + kOffW3, 128, 128);
  __syncthreads();
  dense_gelu(S, S.h[1], 128, P + kOffB3, S.z[2], S.h[2]);
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
    S.x[t] = f2bf(v);
  }
  hidden_layers(S, P);
}

// dW (kin x 128) += Hin^T dZ for the 32-row tile (rows i < nin), with atomics
__device__ __forceinline__ void weight_grad(Smem& S, const unsigned short* Hin, int kin, int nin,
                                            float* gW) {
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int ntiles = (kin / 16) * 8;
  for (int t = wv; t < ntiles; t += NT / 64) {
    const int mt = t >> 3, nt = t & 7;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mma16(Hin + mt * 16, 1, kin, S.d + nt * 16, 128, 1, TB, acc);
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
    for (int s = 0; s < TB; ++s) g += bf2f(S.h[2][s * 128 + tid]) * S.dy[s];
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
  weight_grad(S, S.h[1], 128, 128, grad + kOffW3);
  stage_weights(S, P + kOffW3, 128, 128);
  __syncthreads();
  backprop_hidden(S, S.z[1]);
  // layer 2: W2 (H1 -> Z2)
  bias_grad(S.z[1], grad + kOffB2);
  weight_grad(S, S.h[0], 128, 128, grad + kOffW2);
  stage_weights(S, P + kOffW2, 128, 128);
  __syncthreads();
  backprop_hidden(S, S.z[0]);
  // layer 1: W1 (X -> Z1)
  bias_grad(S.z[0], grad + kOffB1);
  weight_grad(S, S.x, 16, kSurIn, grad + kOffW1);
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
// Features of (box, bin): ln k, ln a, M_nu, stored P_M^{1/2}(a_{n-m}) / P_cdm^{1/2}, m=1..8.
__device__ __forceinline__ bool make_features(const RespBox& bx, double k, double pcdm_half,
                                              const double* hpm, int nbins, int b, float* f) {
  if (!bx.sur_ok || bx.n_cur < kSurHistory + 1 || !(pcdm_half > 0.0) || !(bx.kfs > 0.0))
    return false;
  f[0] = static_cast<float>(log(k));
  f[1] = static_cast<float>(log(bx.a_now));
  f[2] = static_cast<float>(bx.m_total);
  for (int mm = 1; mm <= kSurHistory; ++mm)
    f[2 + mm] = static_cast<float>(hpm[static_cast<size_t>(bx.n_cur - mm) * nbins + b] / pcdm_half);
  return true;
}

__device__ __forceinline__ double approx_factor(double k, double kfs) {
  const double t = 1.0 + k / kfs;
  return 1.0 / (t * t);
}

__device__ __forceinline__ bool in_range(const float* P, const float* f) {
  for (int i = 0; i < kSurIn; ++i) {
    const float lo = P[kOffMin + i], hi = P[kOffMax + i], mg = 0.05f * (hi - lo);
    if (!(f[i] >= lo - mg && f[i] <= hi + mg)) return false;
  }
  return true;
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

// Inference-only shared memory for one bin: all three packed weight matrices at once, the
// biases and the tail of the blob, activations of one 16-row tile ping-ponged.
struct SmemInfer {
  unsigned short x[16 * 16];
  unsigned short h[2][16 * 128];
  alignas(16) unsigned short w[kPackSize];   // W1 | W2 | W3 as packed ([out][in])
  float b[3][128];                           // b1, b2, b3
  float tail[kSurBlob - kOffW4];             // the FP32 blob from W4 on (W4, b4, scalers)
  float y;
};

// acc += A(16 x K) * B(K x 16) with A = act[row][k] and B(k, n) = W[n][k], both bf16 rows of
// length K in LDS: each lane's four consecutive k of a row are one 8-byte read. Same
// operands, in the same order, as mma16 with (sam, sak) = (K, 1) and (sbk, sbn) = (1, K).
template <int K>
__device__ __forceinline__ f32x4 mma16_rows(const unsigned short* A, const unsigned short* W,
                                            f32x4 acc) {
  const int l = threadIdx.x & 63, r = l & 15, kb = (l >> 4) << 2;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x4 a = *reinterpret_cast<const bf16x4*>(A + r * K + k0 + kb);
    const bf16x4 b = *reinterpret_cast<const bf16x4*>(W + r * K + k0 + kb);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// GELU(H W + b) (bf16) for one 16 x 128 tile of rows, as dense_gelu without keeping Z
template <int K>
__device__ __forceinline__ void dense_gelu_rows(const unsigned short* Hin,
                                                const unsigned short* W, const float* bias,
                                                unsigned short* Hout) {
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int nt = wv; nt < 8; nt += RT / 64) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mma16_rows<K>(Hin, W + nt * 16 * K, acc);
    const int col = nt * 16 + (l & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = ((l >> 4) << 2) + q;
      Hout[row * 128 + col] = f2bf(gelu(acc[q] + bias[col]));
    }
  }
}

// The surrogate's response, one workgroup per (bin, box): P_cdm from the deposit's partial
// sums, the network's R for the bin (features from P_cdm and the stored history, forward
// pass on the matrix cores; the arithmetic of the training kernels' forward pass), and the
// exact integral (response_device.hpp) when the network cannot answer (inputs outside the
// training range) or when checking (mode 2, which keeps the exact result and records
// both). The whole packed weight image is staged first (one unrolled copy: the compiler
// issues the loads ahead of the LDS stores).
__global__ __launch_bounds__(RT) void surrogate_response_kernel(
    const float* __restrict__ P, const unsigned short* __restrict__ Q, int mode,
    const RespBox* __restrict__ boxes, const double* __restrict__ partial, int n_partial,
    const double* __restrict__ counts, const double* __restrict__ kmean,
    double* __restrict__ hist_pm, double* __restrict__ hist_pnu,
    const double* __restrict__ ic_pnu, const double* __restrict__ ic_theta,
    const double* __restrict__ tg_ds, const double* __restrict__ tg_w, int nbins, int jcap,
    int qcap, int q_sub, int iterations, double norm, double* __restrict__ pcdm_out,
    double* __restrict__ pnu_out, double* __restrict__ ratio_out, double* __restrict__ sur_r,
    int* __restrict__ sur_use, double* __restrict__ chk_exact, double* __restrict__ chk_sur) {
  __shared__ SmemInfer S;
  __shared__ double red[2 * RT / 64];
  __shared__ int s_ok;
  const int tid = threadIdx.x;
  const int b = blockIdx.x, box = blockIdx.y;
  const size_t ob = static_cast<size_t>(box) * nbins + b;
  constexpr int WV = kPackSize / 8, WIT = (WV + RT - 1) / RT;   // 16-byte pieces
  constexpr int TV = kSurBlob - kOffW4;
  static_assert(3 * 128 + TV <= 3 * RT, "three values per thread");
  {
    static_assert(WV % RT == 0, "whole rounds");
    const uint4* src = reinterpret_cast<const uint4*>(Q);
    uint4* dst = reinterpret_cast<uint4*>(S.w);
#pragma unroll
    for (int i = 0; i < WIT; ++i) dst[tid + i * RT] = src[tid + i * RT];
    // slot t of 3 * 128 + TV: the biases, then the tail of the blob
    auto src_of = [&](int t) {
      return t < 128 ? kOffB1 + t : t < 256 ? kOffB2 + t - 128
                                            : t < 384 ? kOffB3 + t - 256 : kOffW4 + t - 384;
    };
    float pr[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int t = tid + i * RT;
      if (t < 384 + TV) pr[i] = P[src_of(t)];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int t = tid + i * RT;
      if (t < 384) S.b[t / 128][t % 128] = pr[i];
      else if (t < 384 + TV) S.tail[t - 384] = pr[i];
    }
  }
  const float* Ps = S.tail - kOffW4;         // blob offsets from W4 on, in LDS
  const RespBox bx = boxes[box];
  double* hpm = hist_pm + static_cast<size_t>(box) * jcap * nbins;
  double* hpn = hist_pnu + static_cast<size_t>(box) * jcap * nbins;
  const size_t row = static_cast<size_t>(bx.n_cur) * nbins + b;
  const double cb = counts[b];
  const double msum = bin_mode_sum(partial, n_partial, nbins, box, b, red);   // has barriers
  const double pcdm = cb > 0.0 ? norm * msum / cb : 0.0;
  if (!(cb > 0.0)) {
    if (tid == 0) {
      pcdm_out[ob] = 0.0;
      sur_r[ob] = __builtin_nan("");
      sur_use[ob] = 0;
      pnu_out[ob] = ratio_out[ob] = 0.0;
      hpm[row] = hpn[row] = 0.0;
      if (chk_exact) chk_exact[ob] = chk_sur[ob] = 0.0;
    }
    return;
  }
  const double ph = sqrt(pcdm);
  if (tid == 0) {
    float f[kSurIn];
    const bool ok = make_features(bx, kmean[b], ph, hpm, nbins, b, f) && in_range(Ps, f);
    s_ok = ok ? 1 : 0;
    for (int i = 0; i < 16; ++i)
      S.x[i] = f2bf(ok && i < kSurIn ? (f[i] - Ps[kOffMu + i]) / Ps[kOffSigma + i] : 0.f);
  } else if (tid >= 16 && tid < 16 * 16) {
    S.x[tid] = 0;                            // rows 1..15 of the tile (row 0: thread 0)
  }
  __syncthreads();
  const bool ok = s_ok != 0;
  double r_net = __builtin_nan("");
  if (ok) {
    dense_gelu_rows<16>(S.x, S.w + kPackW1, S.b[0], S.h[0]);
    __syncthreads();
    dense_gelu_rows<128>(S.h[0], S.w + kPackW2, S.b[1], S.h[1]);
    __syncthreads();
    dense_gelu_rows<128>(S.h[1], S.w + kPackW3, S.b[2], S.h[0]);
    __syncthreads();
    if (tid < 8) {
      // output layer: 8 lanes, 16 products each, FP32 (as output_layer)
      float acc = 0.f;
#pragma unroll
      for (int j = tid * 16; j < tid * 16 + 16; ++j)
        acc += bf2f(S.h[0][j]) * bfr(Ps[kOffW4 + j]);
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      acc += __shfl_xor(acc, 4, 64);
      if (tid == 0) S.y = acc + Ps[kOffB4];
    }
    __syncthreads();
    r_net = exp(static_cast<double>(S.y * Ps[kOffYSigma] + Ps[kOffYMu])) *
            approx_factor(kmean[b], bx.kfs);
  }
  if (tid == 0) {
    pcdm_out[ob] = pcdm;
    sur_r[ob] = r_net;
    sur_use[ob] = ok ? 1 : 0;
  }
  if (ok && mode == 1) {                     // answered by the network
    if (tid == 0) {
      const double pnu = r_net * ph;
      pnu_out[ob] = pnu;
      ratio_out[ob] = r_net;
      hpm[row] = (1.0 - bx.f_nu) * ph + bx.f_nu * pnu;
      hpn[row] = pnu;
    }
    return;
  }
  const double pnu = exact_pnu(bx, kmean[b], ph, (bx.n_cur > 0 ? hpn[row - nbins] : 0.0),
                               ic_pnu + static_cast<size_t>(box) * kMaxSpecies * nbins,
                               ic_theta[ob], hpm, nbins, b,
                               tg_ds + static_cast<size_t>(box) * qcap,
                               tg_w + static_cast<size_t>(box) * qcap, q_sub, iterations, red);
  if (tid == 0) {
    const double r = ph > 0.0 ? pnu / ph : 0.0;   // no CDM power in the bin: R = 0
    pnu_out[ob] = pnu;
    ratio_out[ob] = r;
    hpm[row] = (1.0 - bx.f_nu) * ph + bx.f_nu * pnu;
    hpn[row] = pnu;
    if (chk_exact) {
      chk_exact[ob] = r;
      chk_sur[ob] = ok ? r_net : r;
    }
  }
}

// Training rows from the step's state after an exact response: one thread per (box, bin).
__global__ void dataset_kernel(const RespBox* __restrict__ boxes, const double* __restrict__ pcdm,
                               const double* __restrict__ ratio, const double* __restrict__ kmean,
                               const double* __restrict__ hist_pm, int nbins, int jcap,
                               int nbox, float* __restrict__ x, float* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbox * nbins) return;
  const int box = i / nbins, b = i % nbins;
  const RespBox bx = boxes[box];
  const double ph = sqrt(pcdm[i]);
  const double r = ratio[i];
  float f[kSurIn];
  bool ok = make_features(bx, kmean[b], ph, hist_pm + static_cast<size_t>(box) * jcap * nbins,
                          nbins, b, f) && r > 0.0;
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
                                     const double* tg_w, int nbins, int jcap, int qcap,
                                     int q_sub, int iterations, double norm, int nbox,
                                     double* pcdm, double* pnu, double* ratio, double* sur_r,
                                     int* sur_use, double* chk_exact, double* chk_sur,
                                     hipStream_t s) {
  hipLaunchKernelGGL(surrogate_response_kernel, dim3(nbins, nbox), dim3(RT), 0, s, P, Q, mode,
                     boxes, partial, n_partial, counts, kmean, hist_pm, hist_pnu, ic_pnu,
                     ic_theta, tg_ds, tg_w, nbins, jcap, qcap, q_sub, iterations, norm, pcdm,
                     pnu, ratio, sur_r, sur_use, chk_exact, chk_sur);
  return hipGetLastError();
}

hipError_t launch_surrogate_dataset(const RespBox* boxes, const double* pcdm, const double* ratio,
                                    const double* kmean, const double* hist_pm, int nbins,
                                    int jcap, int nbox, float* x, float* y, hipStream_t s) {
  const int n = nbox * nbins;
  hipLaunchKernelGGL(dataset_kernel, dim3((n + 255) / 256), dim3(256), 0, s, boxes, pcdm, ratio,
                     kmean, hist_pm, nbins, jcap, nbox, x, y);
  return hipGetLastError();
}

}  // namespace pmnu
