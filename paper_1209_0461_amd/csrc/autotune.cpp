// Launch-shape autotuner: times the candidate block sizes of the particle kernels with
// HIP events on the context's own buffers and keeps the fastest; the choice can be
// cached as JSON keyed by (device name, N, n_boxes).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "pm_nu_internal.hpp"

using namespace pmnu;

namespace {

std::string cache_key(const Ctx& c) {
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, c.device) == hipSuccess) dev = prop.gcnArchName;
  std::ostringstream o;
  o << dev << "/N" << c.N << "/boxes" << c.nbox;
  return o.str();
}

std::string tuning_json(const Ctx& c) {
  std::ostringstream o;
  o << "{\"deposit_block\": " << c.tune.deposit_block << ", \"interp_block\": "
    << c.tune.interp_block << "}";
  return o.str();
}

// Minimal reader for the cache file: lines "key deposit_block interp_block".
bool read_cache(const char* path, const std::string& key, Tuning& t) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    // format: {"key": "...", "deposit_block": D, "interp_block": I}
    if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
    int d = 0, i = 0;
    const size_t pd = line.find("\"deposit_block\": ");
    const size_t pi = line.find("\"interp_block\": ");
    if (pd == std::string::npos || pi == std::string::npos) continue;
    d = std::atoi(line.c_str() + pd + 17);
    i = std::atoi(line.c_str() + pi + 16);
    if (d >= 64 && d <= 1024 && i >= 64 && i <= 1024) {
      t.deposit_block = d;
      t.interp_block = i;
      return true;
    }
  }
  return false;
}

void write_cache(const char* path, const std::string& key, const Tuning& t) {
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line))
      if (!line.empty() && line.find("\"key\": \"" + key + "\"") == std::string::npos)
        keep.push_back(line);
  }
  std::ofstream f(path, std::ios::trunc);
  for (const std::string& l : keep) f << l << "\n";
  f << "{\"key\": \"" << key << "\", \"deposit_block\": " << t.deposit_block
    << ", \"interp_block\": " << t.interp_block << "}\n";
}

}  // namespace

extern "C" {

int pm_nu_autotune(pm_nu_ctx* ctx, const float* pos, float* acc, double a_now,
                   const char* cache_path) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  if (!c) return set_error(PM_NU_EINVAL, "ctx is NULL");
  if (!pos || !acc) return set_error(PM_NU_EINVAL, "pos/acc is NULL");
  const std::string key = cache_key(*c);
  if (cache_path && read_cache(cache_path, key, c->tune)) return PM_NU_OK;
  const bool was_timing = c->timer.enabled;
  c->timer.enabled = false;
  const int blocks[] = {128, 256, 512, 1024};
  hipEvent_t e0, e1;
  PMNU_HIP(hipEventCreate(&e0));
  PMNU_HIP(hipEventCreate(&e1));
  int rc = pm_nu_step(ctx, pos, acc, a_now);   // warm everything up once
  if (rc) return rc;
  const double inv_cell = c->N / c->cfg.box_size;
  float best_d = 1e30f, best_i = 1e30f;
  Tuning best = c->tune;
  for (int bsz : blocks) {
    float tot_d = 0.f, tot_i = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      PMNU_HIP(launch_fill_zero(c->rho, c->M * c->nbox * 8, c->stream));
      PMNU_HIP(hipEventRecord(e0, c->stream));
      PMNU_HIP(launch_deposit(pos, c->rho, c->Np, c->nbox, c->N, inv_cell, c->d_flags, bsz, 1,
                              c->stream));
      PMNU_HIP(hipEventRecord(e1, c->stream));
      PMNU_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      PMNU_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep) tot_d += ms;
      PMNU_HIP(hipEventRecord(e0, c->stream));
      PMNU_HIP(launch_interp(pos, c->force, acc, c->Np, c->nbox, c->N, inv_cell, bsz, 1,
                             c->stream));
      PMNU_HIP(hipEventRecord(e1, c->stream));
      PMNU_HIP(hipEventSynchronize(e1));
      PMNU_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep) tot_i += ms;
    }
    if (tot_d < best_d) {
      best_d = tot_d;
      best.deposit_block = bsz;
    }
    if (tot_i < best_i) {
      best_i = tot_i;
      best.interp_block = bsz;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->tune = best;
  c->timer.enabled = was_timing;
  // leave the context in a consistent state: recompute one full step with the choice
  rc = pm_nu_step(ctx, pos, acc, a_now);
  if (rc) return rc;
  if (cache_path) write_cache(cache_path, key, c->tune);
  return PM_NU_OK;
}

int pm_nu_tuning(pm_nu_ctx* ctx, char* out, size_t cap) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  if (!c || !out || cap == 0) return set_error(PM_NU_EINVAL, "bad arguments");
  const std::string s = tuning_json(*c);
  std::snprintf(out, cap, "%s", s.c_str());
  return PM_NU_OK;
}

}  // extern "C"
