// Launch-shape autotuner: times the candidate launch shapes of the particle kernels (the
// deposit's chunking mode / block size, the interpolation's block size) with HIP events
// on the context's own buffers and keeps the fastest; the choice can be cached as JSON
// lines keyed by (device name, N, n_boxes, particles per box).
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
  o << dev << "/N" << c.N << "/boxes" << c.nbox << "/np" << c.Np;
  return o.str();
}

std::string tuning_json(const Ctx& c) {
  std::ostringstream o;
  o << "{\"deposit_mode\": " << c.tune.deposit_mode << ", \"deposit_block\": "
    << c.tune.deposit_block << ", \"interp_mode\": " << c.tune.interp_mode
    << ", \"interp_block\": " << c.tune.interp_block << "}";
  return o.str();
}

int json_int(const std::string& line, const char* field, int fallback) {
  const std::string f = std::string("\"") + field + "\": ";
  const size_t p = line.find(f);
  return p == std::string::npos ? fallback : std::atoi(line.c_str() + p + f.size());
}

// Cache file: one JSON object per line,
// {"key": "...", "deposit_mode": M, "deposit_block": D, "interp_block": I}
bool read_cache(const char* path, const std::string& key, Tuning& t) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
    const int m = json_int(line, "deposit_mode", -1);
    const int d = json_int(line, "deposit_block", -1);
    const int im = json_int(line, "interp_mode", -1);
    const int i = json_int(line, "interp_block", -1);
    if (m >= 0 && m <= 7 && d >= 64 && d <= 1024 && im >= 0 && im <= 3 && i >= 64 && i <= 1024) {
      t.deposit_mode = m;
      t.deposit_block = d;
      t.interp_mode = im;
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
  f << "{\"key\": \"" << key << "\", \"deposit_mode\": " << t.deposit_mode
    << ", \"deposit_block\": " << t.deposit_block << ", \"interp_mode\": " << t.interp_mode
    << ", \"interp_block\": " << t.interp_block << "}\n";
}

}  // namespace

extern "C" {

int pm_nu_autotune(pm_nu_ctx* ctx, const float* pos, float* acc, double a_now,
                   const char* cache_path) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  if (!c) return set_error(PM_NU_EINVAL, "ctx is NULL");
  if (!pos || !acc) return set_error(PM_NU_EINVAL, "pos/acc is NULL");
  drop_graph(*c);   // the launch shapes may change
  const std::string key = cache_key(*c);
  if (cache_path && read_cache(cache_path, key, c->tune)) return PM_NU_OK;
  const bool was_timing = c->timer.enabled;
  c->timer.enabled = false;
  struct DepCand { int mode, block; };
  const DepCand dep[] = {{0, 256}, {1, 256}, {2, 256}, {3, 256}, {4, 256}, {5, 256}, {6, 256},
                         {7, 256}};
  const DepCand itp[] = {{0, 256}, {0, 512}, {0, 1024}, {1, 256}, {2, 256}, {3, 256}};
  hipEvent_t e0, e1;
  PMNU_HIP(hipEventCreate(&e0));
  PMNU_HIP(hipEventCreate(&e1));
  int rc = pm_nu_step(ctx, pos, acc, a_now);   // warm everything up once
  if (rc) return rc;
  const double inv_cell = c->N / c->cfg.box_size;
  auto time_ms = [&](auto&& launch) -> float {
    float tot = 0.f;
    for (int rep = 0; rep < 4; ++rep) {
      if (launch(true) != hipSuccess) return 1e30f;
      if (hipEventRecord(e0, c->stream) != hipSuccess) return 1e30f;
      if (launch(false) != hipSuccess) return 1e30f;
      if (hipEventRecord(e1, c->stream) != hipSuccess) return 1e30f;
      if (hipEventSynchronize(e1) != hipSuccess) return 1e30f;
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (rep) tot += ms;
    }
    return tot;
  };
  Tuning best = c->tune;
  float best_d = 1e30f, best_i = 1e30f;
  // the deposit candidates are timed as whole deposits (including the forward transform)
  // since the patch mode replaces the zero pass and changes what the first FFT pass reads
  for (const DepCand& d : dep) {
    c->tune.deposit_mode = d.mode;
    c->tune.deposit_block = d.block;
    float ms = 0.f;
    for (int rep = 0; rep < 4 && ms < 1e29f; ++rep) {
      if (hipEventRecord(e0, c->stream) != hipSuccess || pm_nu_deposit(ctx, pos) != PM_NU_OK ||
          hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        ms = 1e30f;
        break;
      }
      float v = 0.f;
      hipEventElapsedTime(&v, e0, e1);
      if (rep) ms += v;
    }
    if (ms < best_d) {
      best_d = ms;
      best.deposit_mode = d.mode;
      best.deposit_block = d.block;
    }
  }
  for (const DepCand& d : itp) {
    const float ms = time_ms([&](bool prep) -> hipError_t {
      if (prep) return hipSuccess;
      return launch_interp(pos, c->force, acc, c->Np, c->nbox, c->N, inv_cell, d.mode, d.block,
                           c->stream);
    });
    if (ms < best_i) {
      best_i = ms;
      best.interp_mode = d.mode;
      best.interp_block = d.block;
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

int pm_nu_set_launch(pm_nu_ctx* ctx, int deposit_mode, int deposit_block, int interp_mode,
                     int interp_block) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  if (!c) return set_error(PM_NU_EINVAL, "ctx is NULL");
  drop_graph(*c);   // a captured step keeps its launch shapes
  auto block_ok = [](int b) { return b >= 64 && b <= 1024 && b % 64 == 0; };
  if (deposit_mode < 0 || deposit_mode > 7 || interp_mode < 0 || interp_mode > 3 ||
      !block_ok(deposit_block) || !block_ok(interp_block))
    return set_error(PM_NU_EINVAL, "bad launch shape");
  c->tune.deposit_mode = deposit_mode;
  c->tune.deposit_block = deposit_block;
  c->tune.interp_mode = interp_mode;
  c->tune.interp_block = interp_block;
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
