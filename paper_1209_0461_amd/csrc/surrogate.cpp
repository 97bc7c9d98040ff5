// Surrogate network for the history integral: placeholder entry points until the
// training and inference kernels are in place.
#include <hip/hip_runtime.h>

#include "pm_nu_internal.hpp"

namespace pmnu {
struct Surrogate {};
void surrogate_free(Ctx& c) {
  delete c.sur;
  c.sur = nullptr;
}
int surrogate_response(Ctx& c, double) {
  (void)c;
  return set_error(PM_NU_ESURROGATE, "no surrogate network loaded");
}
}  // namespace pmnu

using namespace pmnu;

extern "C" {
int64_t pm_nu_surrogate_blob_floats(void) { return 34689 + 2 * PM_NU_SUR_IN + 2; }
int pm_nu_surrogate_load(pm_nu_ctx*, const float*, int64_t) {
  return set_error(PM_NU_ESURROGATE, "surrogate not available");
}
int pm_nu_surrogate_save(pm_nu_ctx*, float*, int64_t) {
  return set_error(PM_NU_ESURROGATE, "surrogate not available");
}
int pm_nu_surrogate_init(pm_nu_ctx*, const float*, const float*, int64_t, uint64_t) {
  return set_error(PM_NU_ESURROGATE, "surrogate not available");
}
int pm_nu_surrogate_train(pm_nu_ctx*, const float*, const float*, int64_t, int, int, float,
                          uint64_t, float*) {
  return set_error(PM_NU_ESURROGATE, "surrogate not available");
}
int pm_nu_surrogate_predict(pm_nu_ctx*, const float*, float*, int64_t) {
  return set_error(PM_NU_ESURROGATE, "surrogate not available");
}
int pm_nu_surrogate_grad(pm_nu_ctx*, const float*, const float*, int64_t, float*, float*) {
  return set_error(PM_NU_ESURROGATE, "surrogate not available");
}
int pm_nu_surrogate_features(pm_nu_ctx*, double, float*) {
  return set_error(PM_NU_ESURROGATE, "surrogate not available");
}
int pm_nu_get_surrogate_check(pm_nu_ctx*, int, double*, double*) {
  return set_error(PM_NU_ESURROGATE, "surrogate not available");
}
}
