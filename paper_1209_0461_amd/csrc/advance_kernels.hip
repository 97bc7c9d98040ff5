// Leapfrog updates of the particles in the superconformal time s (gfx950). Later kicks and
// drifts are applied by the interpolation itself; this kernel serves the first one.
//
// kick_drift_kernel: u += K_b acc, then (if drift) x += D_b u wrapped into [0, L), on the
// flat [box][particle][3] arrays; K_b, D_b per box. Every float is independent, so each
// thread takes four consecutive floats with 16-byte loads and stores (the arrays are
// torch allocations, 256-byte aligned; a tail of fewer than four floats goes one by one).
// Streaming, HBM-bound: 20 bytes per float with the drift (x, u, acc in; x, u out), 12
// without.
#include "pm_nu_internal.hpp"

namespace pmnu {
namespace {

template <bool DRIFT>
__global__ __launch_bounds__(256) void kick_drift_kernel(float* __restrict__ pos,
                                                         float* __restrict__ vel,
                                                         const float* __restrict__ acc,
                                                         const double2* __restrict__ kd,
                                                         int64_t per_box, int64_t total,
                                                         float L) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t j0 = 4 * t;
  if (j0 >= total) return;
  const int64_t b0 = j0 / per_box;
  const int64_t edge = (b0 + 1) * per_box;   // first float of the next box
  if (j0 + 4 <= total) {
    float4 v = reinterpret_cast<const float4*>(vel)[t];
    const float4 a = reinterpret_cast<const float4*>(acc)[t];
    float4 x;
    if (DRIFT) x = reinterpret_cast<const float4*>(pos)[t];
    float kk[4], dd[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double2 f = kd[j0 + e < edge ? b0 : b0 + 1];
      kk[e] = static_cast<float>(f.x);
      dd[e] = static_cast<float>(f.y);
    }
    v.x += kk[0] * a.x;
    v.y += kk[1] * a.y;
    v.z += kk[2] * a.z;
    v.w += kk[3] * a.w;
    reinterpret_cast<float4*>(vel)[t] = v;
    if (DRIFT) {
      x.x = wrap_box(x.x + dd[0] * v.x, L);
      x.y = wrap_box(x.y + dd[1] * v.y, L);
      x.z = wrap_box(x.z + dd[2] * v.z, L);
      x.w = wrap_box(x.w + dd[3] * v.w, L);
      reinterpret_cast<float4*>(pos)[t] = x;
    }
  } else {
    for (int64_t j = j0; j < total; ++j) {
      const double2 f = kd[j < edge ? b0 : b0 + 1];
      const float v = vel[j] + static_cast<float>(f.x) * acc[j];
      vel[j] = v;
      if (DRIFT) pos[j] = wrap_box(pos[j] + static_cast<float>(f.y) * v, L);
    }
  }
}

}  // namespace

hipError_t launch_kick_drift(float* pos, float* vel, const float* acc, const double* kd,
                             int64_t n_particles, int nbox, float box, bool drift,
                             hipStream_t s) {
  const int64_t per_box = 3 * n_particles;
  const int64_t total = per_box * nbox;
  const int64_t threads = (total + 3) / 4;
  const int64_t blocks = (threads + 255) / 256;
  const double2* f = reinterpret_cast<const double2*>(kd);
  if (drift)
    hipLaunchKernelGGL(kick_drift_kernel<true>, dim3(static_cast<unsigned>(blocks)), dim3(256),
                       0, s, pos, vel, acc, f, per_box, total, box);
  else
    hipLaunchKernelGGL(kick_drift_kernel<false>, dim3(static_cast<unsigned>(blocks)),
                       dim3(256), 0, s, pos, vel, acc, f, per_box, total, box);
  return hipGetLastError();
}

}  // namespace pmnu
