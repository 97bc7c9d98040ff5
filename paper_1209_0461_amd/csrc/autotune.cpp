// Launch-shape autotuner: times the candidate launch shapes of the particle kernels (the
// deposit's chunking mode / block size, the interpolation's mode / block size) and the tile
// candidates of the six FFT passes with HIP events on the context's own buffers and keeps
// the fastest of each; the choice can be cached as JSON lines keyed by (device
// architecture, N, n_boxes, particles per box).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
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

const char* const kFftPass[6] = {"fwd_z", "fwd_y", "fwd_x", "inv_x", "inv_y", "inv_z"};

std::string tuning_json(const Ctx& c) {
  std::ostringstream o;
  o << "{\"deposit_mode\": " << c.tune.deposit_mode << ", \"deposit_block\": "
    << c.tune.deposit_block << ", \"interp_mode\": " << c.tune.interp_mode
    << ", \"interp_block\": " << c.tune.interp_block << ", \"fft\": [";
  for (int p = 0; p < 6; ++p) o << (p ? ", " : "") << c.tune.fft[p];
  o << "], \"fft_tiles\": {";
  for (int p = 0; p < 6; ++p)
    o << (p ? ", " : "") << "\"" << kFftPass[p] << "\": " << fft_tile(c.N, p, c.tune.fft[p]);
  o << "}, \"response_threads\": " << response_threads(c.B, c.nbox) << "}";
  return o.str();
}

// The FFT candidates of a cache line: "fft": [a, b, c, d, e, f], each 0..2.
bool json_fft(const std::string& line, int* fft) {
  const std::string f = "\"fft\": [";
  const size_t p = line.find(f);
  if (p == std::string::npos) return false;
  const char* q = line.c_str() + p + f.size();
  for (int i = 0; i < 6; ++i) {
    char* end = nullptr;
    const long v = std::strtol(q, &end, 10);
    if (end == q || v < 0 || v > 2) return false;
    fft[i] = static_cast<int>(v);
    q = end;
    while (*q == ',' || *q == ' ') ++q;
  }
  return true;
}

int json_int(const std::string& line, const char* field, int fallback) {
  const std::string f = std::string("\"") + field + "\": ";
  const size_t p = line.find(f);
  return p == std::string::npos ? fallback : std::atoi(line.c_str() + p + f.size());
}

// Cache file: one JSON object per line,
// {"key": "...", "deposit_mode": M, "deposit_block": D, "interp_block": I}; a line is taken
// only if every field is a shape that pm_nu_set_launch would accept for a mesh of n
bool read_cache(const char* path, const std::string& key, int n, Tuning& t) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
    const int m = json_int(line, "deposit_mode", -1);
    const int d = json_int(line, "deposit_block", -1);
    const int im = json_int(line, "interp_mode", -1);
    const int i = json_int(line, "interp_block", -1);
    int fft[6];
    if (m >= 0 && m <= 9 && (m < 8 || n >= 32) && d >= 64 && d <= 1024 && im >= 0 && im <= 3 &&
        i >= 64 && i <= 1024 && json_fft(line, fft)) {
      t.deposit_mode = m;
      t.deposit_block = d;
      t.interp_mode = im;
      t.interp_block = i;
      for (int p = 0; p < 6; ++p) t.fft[p] = fft[p];
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
    << ", \"interp_block\": " << t.interp_block << ", \"fft\": [";
  for (int p = 0; p < 6; ++p) f << (p ? ", " : "") << t.fft[p];
  f << "]}\n";
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
  if (cache_path && read_cache(cache_path, key, c->N, c->tune)) return PM_NU_OK;
  const bool was_timing = c->timer.enabled;
  c->timer.enabled = false;
  struct DepCand { int mode, block; };
  const DepCand dep[] = {{0, 256}, {0, 512}, {0, 1024}, {1, 256}, {2, 256}, {3, 256}, {4, 256},
                         {5, 256}, {6, 256}, {7, 256}, {8, 256}, {9, 256}};
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
  // the FFT passes, one at a time on the buffers of the step just run, each into an output
  // other than its input (the data are whatever the step left there; the closing step below
  // recomputes everything)
  c->tune = best;
  rc = pm_nu_step(ctx, pos, acc, a_now);
  if (rc) return rc;
  const float kf = static_cast<float>(2.0 * kPi / c->cfg.box_size);
  const float cgreen =
      static_cast<float>(1.5 * c->cfg.omega_m * kH0 * kH0 / a_now / static_cast<double>(c->M));
  const double scale = static_cast<double>(c->M) / static_cast<double>(c->Np) / kFixScale;
  for (int p = 0; p < 6; ++p) {
    float best_ms = 1e30f;
    for (int v = 0; v < 3; ++v) {
      if (v > 0 && fft_tile(c->N, p, v) == fft_tile(c->N, p, 0)) continue;   // same tile
      const float ms = time_ms([&](bool prep) -> hipError_t {
        if (prep) return hipSuccess;
        switch (p) {
          case 0:   // the density as the step's deposit left it (delta or the fixed-point sum)
            return c->density_is_delta
                       ? launch_fwd_z(c->N, nullptr, c->delta, nullptr, nullptr, 0, c->ck[2],
                                      c->tw, scale, c->nbox, c->stream, v)
                       : launch_fwd_z(c->N, c->rho, nullptr, nullptr, nullptr, 0, c->ck[2],
                                      c->tw, scale, c->nbox, c->stream, v);
          case 1: return launch_fwd_y(c->N, c->ck[1], c->ck[2], c->tw, c->nbox, c->stream, v);
          case 2:
            return launch_fwd_x_bin(c->N, c->ck[0], c->tw, c->bin_of_n2, c->bin_partial, c->B,
                                    c->nbox, c->stream, v);
          case 3:
            return launch_inv_x(c->N, c->ck[0], c->ck[1], c->ck[2], c->tw, c->ridx, c->d_next,
                                c->ratio, c->d_resp, c->B, c->inv_w2, cgreen, kf, c->nbox,
                                c->stream, v);
          case 4:
            return launch_inv_y(c->N, c->ck[1], c->ck[2], c->ck[0], c->ck[3], c->ck[4], c->tw, kf,
                                c->nbox, c->stream, v);
          default:
            return launch_inv_z(c->N, c->ck[0], c->ck[3], c->ck[4], c->force, c->tw, kf,
                                c->nbox, c->stream, v);
        }
      });
      if (ms < best_ms) {
        best_ms = ms;
        best.fft[p] = v;
      }
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
  if (deposit_mode < 0 || deposit_mode > 9 || interp_mode < 0 || interp_mode > 3 ||
      (deposit_mode >= 8 && c->N < 32) ||
      !block_ok(deposit_block) || !block_ok(interp_block))
    return set_error(PM_NU_EINVAL, "bad launch shape");
  c->tune.deposit_mode = deposit_mode;
  c->tune.deposit_block = deposit_block;
  c->tune.interp_mode = interp_mode;
  c->tune.interp_block = interp_block;
  return PM_NU_OK;
}

int pm_nu_set_fft_tiles(pm_nu_ctx* ctx, const int32_t* candidates) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  if (!c) return set_error(PM_NU_EINVAL, "ctx is NULL");
  if (!candidates) return set_error(PM_NU_EINVAL, "candidates is NULL");
  for (int p = 0; p < 6; ++p)
    if (candidates[p] < 0 || candidates[p] > 2)
      return set_error(PM_NU_EINVAL, "FFT tile candidate %d of pass %d: must be 0, 1 or 2",
                       candidates[p], p);
  drop_graph(*c);   // a captured step keeps its launch shapes
  for (int p = 0; p < 6; ++p) c->tune.fft[p] = candidates[p];
  c->stage = 0;     // the next step starts with a deposit (its bin partials follow the tile)
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
