// Host side of the surrogate network: weight/statistics storage on the device, the
// training loop (per-epoch shuffles, minibatch gradient + Adam launches, half-cosine
// learning-rate decay), prediction, gradients for checking, the training-set builder and
// the response launch used by response modes 1 and 2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "pm_nu_internal.hpp"
#include "surrogate_layout.hpp"

namespace pmnu {

struct Surrogate {
  float* P = nullptr;          // [kSurBlob] FP32 masters + statistics
  float* g = nullptr;          // [kSurParams] gradient
  float* m = nullptr;          // [kSurParams] Adam first moment
  float* v = nullptr;          // [kSurParams] Adam second moment
  float* loss = nullptr;       // [1]
  int* perm = nullptr;         // [perm_cap]
  int64_t perm_cap = 0;
  double* chk_exact = nullptr; // [nbox][B]
  double* chk_sur = nullptr;   // [nbox][B]
  unsigned short* packed = nullptr;  // bf16 image of W1..W3 for inference
  double* sur_r = nullptr;     // [nbox][B] the network's R of the last response
  bool packed_valid = false;   // cleared whenever the FP32 masters change
  bool loaded = false;
  int64_t step = 0;
};

void surrogate_free(Ctx& c) {
  Surrogate* s = c.sur;
  if (!s) return;
  void* bufs[] = {s->P, s->g, s->m, s->v, s->loss, s->perm, s->chk_exact, s->chk_sur,
                  s->packed, s->sur_r};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  delete s;
  c.sur = nullptr;
}

namespace {

int ensure(Ctx& c) {
  if (c.sur) return PM_NU_OK;
  Surrogate* s = new Surrogate();
  c.sur = s;
  const size_t nb = static_cast<size_t>(c.nbox) * c.B;
  hipError_t e = hipMalloc(&s->P, kSurBlob * sizeof(float));
  if (!e) e = hipMalloc(&s->g, kSurParams * sizeof(float));
  if (!e) e = hipMalloc(&s->m, kSurParams * sizeof(float));
  if (!e) e = hipMalloc(&s->v, kSurParams * sizeof(float));
  if (!e) e = hipMalloc(&s->loss, sizeof(float));
  if (!e) e = hipMalloc(&s->chk_exact, nb * sizeof(double));
  if (!e) e = hipMalloc(&s->chk_sur, nb * sizeof(double));
  if (!e) e = hipMalloc(&s->packed, packed_weight_count() * sizeof(unsigned short));
  if (!e) e = hipMalloc(&s->sur_r, nb * sizeof(double));
  if (!e) e = hipMemset(s->P, 0, kSurBlob * sizeof(float));
  if (!e) e = hipMemset(s->chk_exact, 0, nb * sizeof(double));
  if (!e) e = hipMemset(s->chk_sur, 0, nb * sizeof(double));
  if (e) {
    surrogate_free(c);
    return set_error(PM_NU_ENOMEM, "surrogate allocation failed: %s", hipGetErrorString(e));
  }
  return PM_NU_OK;
}

int reset_optimizer(Ctx& c) {
  Surrogate* s = c.sur;
  PMNU_HIP(hipMemset(s->m, 0, kSurParams * sizeof(float)));
  PMNU_HIP(hipMemset(s->v, 0, kSurParams * sizeof(float)));
  s->step = 0;
  s->packed_valid = false;
  return PM_NU_OK;
}

int need_loaded(Ctx* c) {
  if (!c) return set_error(PM_NU_EINVAL, "ctx is NULL");
  if (!c->sur || !c->sur->loaded)
    return set_error(PM_NU_ESURROGATE, "no surrogate weights (load or init first)");
  return PM_NU_OK;
}

#define SUR_LAUNCH(call)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return set_error(PM_NU_EHIP, "surrogate launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

}  // namespace

int surrogate_launch(Ctx& c, int mode, double norm) {
  int rc = need_loaded(&c);
  if (rc) return rc;
  Surrogate* s = c.sur;
  if (!s->packed_valid) {
    hipError_t e = launch_pack_weights(s->P, s->packed, c.stream);
    if (e != hipSuccess) return set_error(PM_NU_EHIP, "weight packing: %s", hipGetErrorString(e));
    s->packed_valid = true;
  }
  timer_begin(c, ST_SURROGATE);
  hipError_t e = launch_surrogate_response(
      s->P, s->packed, mode, c.d_resp, c.bin_partial, c.n_partial, c.d_counts, c.d_kmean,
      c.hist_pm, c.hist_pnu, c.ic_pnu, c.ic_theta, c.tg_ds, c.tg_l2, c.tg_w, c.B, c.Jcap, c.qcap,
      c.Q,
      c.cfg.iterations, norm, c.nbox, c.pcdm, c.pnu, c.ratio, s->sur_r, s->chk_exact,
      s->chk_sur, c.stream);
  timer_end(c);
  if (e != hipSuccess) return set_error(PM_NU_EHIP, "surrogate response: %s", hipGetErrorString(e));
  return PM_NU_OK;
}

}  // namespace pmnu

using namespace pmnu;

extern "C" {

int64_t pm_nu_surrogate_blob_floats(void) { return kSurBlob; }

int pm_nu_surrogate_load(pm_nu_ctx* ctx, const float* blob, int64_t n_floats) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  if (!c || !blob) return set_error(PM_NU_EINVAL, "ctx/blob is NULL");
  drop_graph(*c);   // new weights
  if (n_floats != kSurBlob)
    return set_error(PM_NU_EINVAL, "blob must hold %d floats (got %lld)", kSurBlob,
                     static_cast<long long>(n_floats));
  for (int i = 0; i < kSurIn; ++i)
    if (!(blob[kOffSigma + i] > 0.f)) return set_error(PM_NU_EINVAL, "feature scale must be > 0");
  if (!(blob[kOffYSigma] > 0.f)) return set_error(PM_NU_EINVAL, "target scale must be > 0");
  int rc = ensure(*c);
  if (rc) return rc;
  PMNU_HIP(hipStreamSynchronize(c->stream));
  PMNU_HIP(hipMemcpy(c->sur->P, blob, kSurBlob * sizeof(float), hipMemcpyHostToDevice));
  rc = reset_optimizer(*c);
  if (rc) return rc;
  c->sur->loaded = true;
  return PM_NU_OK;
}

int pm_nu_surrogate_save(pm_nu_ctx* ctx, float* blob, int64_t n_floats) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  int rc = need_loaded(c);
  if (rc) return rc;
  if (!blob || n_floats < kSurBlob) return set_error(PM_NU_EINVAL, "blob too small");
  PMNU_HIP(hipStreamSynchronize(c->stream));
  PMNU_HIP(hipMemcpy(blob, c->sur->P, kSurBlob * sizeof(float), hipMemcpyDeviceToHost));
  return PM_NU_OK;
}

int pm_nu_surrogate_init(pm_nu_ctx* ctx, const float* x, const float* y, int64_t n,
                         uint64_t seed) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  if (!c || !x || !y || n < 2) return set_error(PM_NU_EINVAL, "bad arguments");
  drop_graph(*c);   // new weights
  int rc = ensure(*c);
  if (rc) return rc;
  PMNU_HIP(hipStreamSynchronize(c->stream));
  std::vector<float> hx(static_cast<size_t>(n) * kSurIn), hy(static_cast<size_t>(n));
  PMNU_HIP(hipMemcpy(hx.data(), x, hx.size() * sizeof(float), hipMemcpyDeviceToHost));
  PMNU_HIP(hipMemcpy(hy.data(), y, hy.size() * sizeof(float), hipMemcpyDeviceToHost));
  std::vector<float> blob(kSurBlob, 0.f);
  // statistics over the rows with a finite target
  std::vector<double> sum(kSurIn, 0.0), sum2(kSurIn, 0.0), mn(kSurIn, 1e300), mx(kSurIn, -1e300);
  double ys = 0.0, ys2 = 0.0;
  int64_t cnt = 0;
  for (int64_t r = 0; r < n; ++r) {
    if (!std::isfinite(hy[r])) continue;
    ++cnt;
    ys += hy[r];
    ys2 += static_cast<double>(hy[r]) * hy[r];
    for (int i = 0; i < kSurIn; ++i) {
      const double v = hx[r * kSurIn + i];
      sum[i] += v;
      sum2[i] += v * v;
      mn[i] = std::min(mn[i], v);
      mx[i] = std::max(mx[i], v);
    }
  }
  if (cnt < 2) return set_error(PM_NU_EINVAL, "fewer than 2 rows with a finite target");
  for (int i = 0; i < kSurIn; ++i) {
    const double mu = sum[i] / cnt;
    const double var = std::max(sum2[i] / cnt - mu * mu, 0.0);
    blob[kOffMu + i] = static_cast<float>(mu);
    blob[kOffSigma + i] = static_cast<float>(var > 1e-24 ? std::sqrt(var) : 1.0);
    blob[kOffMin + i] = static_cast<float>(mn[i]);
    blob[kOffMax + i] = static_cast<float>(mx[i]);
  }
  const double ymu = ys / cnt, yvar = std::max(ys2 / cnt - ymu * ymu, 0.0);
  blob[kOffYMu] = static_cast<float>(ymu);
  blob[kOffYSigma] = static_cast<float>(yvar > 1e-24 ? std::sqrt(yvar) : 1.0);
  // Glorot-uniform weights, zero biases
  std::mt19937_64 rng(seed);
  auto fill = [&](int off, int fan_in, int fan_out) {
    const double a = std::sqrt(6.0 / (fan_in + fan_out));
    std::uniform_real_distribution<double> u(-a, a);
    for (int i = 0; i < fan_in * fan_out; ++i) blob[off + i] = static_cast<float>(u(rng));
  };
  fill(kOffW1, kSurIn, 128);
  fill(kOffW2, 128, 128);
  fill(kOffW3, 128, 128);
  fill(kOffW4, 128, 1);
  PMNU_HIP(hipMemcpy(c->sur->P, blob.data(), kSurBlob * sizeof(float), hipMemcpyHostToDevice));
  rc = reset_optimizer(*c);
  if (rc) return rc;
  c->sur->loaded = true;
  return PM_NU_OK;
}

int pm_nu_surrogate_train_part(pm_nu_ctx* ctx, const float* x, const float* y, int64_t n,
                               int first_epoch, int epochs, int total_epochs, int batch,
                               float lr, uint64_t seed, float* loss_out) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  int rc = need_loaded(c);
  if (rc) return rc;
  drop_graph(*c);   // new weights
  if (!x || !y || n < 1 || epochs < 1 || batch < 32 || batch % 32 || !(lr > 0.f) ||
      first_epoch < 0 || total_epochs < first_epoch + epochs)
    return set_error(PM_NU_EINVAL, "bad training arguments");
  if (n > (1ll << 31) - 1) return set_error(PM_NU_EINVAL, "too many rows");
  Surrogate* s = c->sur;
  if (s->perm_cap < n) {
    if (s->perm) (void)hipFree(s->perm);
    s->perm = nullptr;
    s->perm_cap = 0;
    PMNU_HIP(hipMalloc(&s->perm, n * sizeof(int)));
    s->perm_cap = n;
  }
  std::vector<int> perm(n);
  const int64_t nb = (n + batch - 1) / batch;
  const int64_t total = nb * total_epochs;
  int64_t t = nb * first_epoch;
  float last = 0.f;
  for (int ep = first_epoch; ep < first_epoch + epochs; ++ep) {
    for (int64_t i = 0; i < n; ++i) perm[i] = static_cast<int>(i);
    std::mt19937_64 rng(seed + 0x9E3779B97F4A7C15ull * (ep + 1));
    for (int64_t i = n - 1; i > 0; --i) {
      std::uniform_int_distribution<int64_t> d(0, i);
      std::swap(perm[i], perm[d(rng)]);
    }
    PMNU_HIP(hipStreamSynchronize(c->stream));
    PMNU_HIP(hipMemcpy(s->perm, perm.data(), n * sizeof(int), hipMemcpyHostToDevice));
    SUR_LAUNCH(launch_fill_zero(s->loss, sizeof(float), c->stream));
    for (int64_t b = 0; b < nb; ++b, ++t) {
      const int64_t r0 = b * batch, cnt = std::min<int64_t>(batch, n - r0);
      SUR_LAUNCH(launch_fill_zero(s->g, kSurParams * sizeof(float), c->stream));
      SUR_LAUNCH(launch_mlp_train(s->P, x, y, s->perm, r0, cnt, 1.0f / cnt, s->g, s->loss,
                                  c->stream));
      ++s->step;
      const double frac = static_cast<double>(t) / std::max<int64_t>(1, total - 1);
      const float lr_t =
          static_cast<float>(lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(kPi * frac))));
      const float c1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(s->step)));
      const float c2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(s->step)));
      s->packed_valid = false;
      SUR_LAUNCH(launch_adam(s->P, s->g, s->m, s->v, kSurParams, lr_t, 0.9f, 0.999f, 1e-8f, c1, c2,
                             c->stream));
    }
    float lsum = 0.f;
    PMNU_HIP(hipStreamSynchronize(c->stream));
    PMNU_HIP(hipMemcpy(&lsum, s->loss, sizeof(float), hipMemcpyDeviceToHost));
    last = lsum / static_cast<float>(n);
  }
  if (loss_out) *loss_out = last;
  return PM_NU_OK;
}

int pm_nu_surrogate_train(pm_nu_ctx* ctx, const float* x, const float* y, int64_t n,
                          int epochs, int batch, float lr, uint64_t seed, float* loss_out) {
  return pm_nu_surrogate_train_part(ctx, x, y, n, 0, epochs, epochs, batch, lr, seed, loss_out);
}

int pm_nu_surrogate_predict(pm_nu_ctx* ctx, const float* x, float* y, int64_t n) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  int rc = need_loaded(c);
  if (rc) return rc;
  if (!x || !y || n < 1) return set_error(PM_NU_EINVAL, "bad arguments");
  SUR_LAUNCH(launch_mlp_predict(c->sur->P, x, y, n, c->stream));
  return PM_NU_OK;
}

int pm_nu_surrogate_grad(pm_nu_ctx* ctx, const float* x, const float* y, int64_t n, float* grad,
                         float* loss_out) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  int rc = need_loaded(c);
  if (rc) return rc;
  if (!x || !y || !grad || n < 1) return set_error(PM_NU_EINVAL, "bad arguments");
  Surrogate* s = c->sur;
  SUR_LAUNCH(launch_fill_zero(s->g, kSurParams * sizeof(float), c->stream));
  SUR_LAUNCH(launch_fill_zero(s->loss, sizeof(float), c->stream));
  SUR_LAUNCH(launch_mlp_train(s->P, x, y, nullptr, 0, n, 1.0f / n, s->g, s->loss, c->stream));
  PMNU_HIP(hipMemcpyAsync(grad, s->g, kSurParams * sizeof(float), hipMemcpyDeviceToDevice,
                          c->stream));
  float lsum = 0.f;
  PMNU_HIP(hipStreamSynchronize(c->stream));
  PMNU_HIP(hipMemcpy(&lsum, s->loss, sizeof(float), hipMemcpyDeviceToHost));
  if (loss_out) *loss_out = lsum / static_cast<float>(n);
  return PM_NU_OK;
}

int pm_nu_surrogate_dataset(pm_nu_ctx* ctx, double a_now, float* x, float* y) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  if (!c || !x || !y) return set_error(PM_NU_EINVAL, "bad arguments");
  int rc = do_response_mode(*c, a_now, 0);
  if (rc) return rc;
  SUR_LAUNCH(launch_surrogate_dataset(c->d_resp, c->pcdm, c->ratio, c->d_kmean, c->hist_pm,
                                      c->hist_pnu, c->B, c->Jcap, c->nbox, x, y, c->stream));
  return PM_NU_OK;
}

int pm_nu_get_surrogate_check(pm_nu_ctx* ctx, int box, double* ratio_exact,
                              double* ratio_surrogate) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  int rc = need_loaded(c);
  if (rc) return rc;
  if (box < 0 || box >= c->nbox) return set_error(PM_NU_EINVAL, "box out of range");
  PMNU_HIP(hipStreamSynchronize(c->stream));
  const size_t B = c->B;
  if (ratio_exact)
    PMNU_HIP(hipMemcpy(ratio_exact, c->sur->chk_exact + box * B, B * sizeof(double),
                       hipMemcpyDeviceToHost));
  if (ratio_surrogate)
    PMNU_HIP(hipMemcpy(ratio_surrogate, c->sur->chk_sur + box * B, B * sizeof(double),
                       hipMemcpyDeviceToHost));
  return PM_NU_OK;
}

}  // extern "C"
