// Host runtime of the pm_nu library: configuration, bin geometry, the FP64 time grid of
// the history integral, buffer ownership, stage ordering, timing and graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "background.hpp"
#include "host_math.hpp"
#include "pm_nu_internal.hpp"

namespace pmnu {

const char* const kStageNames[ST_COUNT] = {
    "zero_mesh", "cic_deposit", "fft_fwd_z", "fft_fwd_y", "fft_fwd_x_bin", "nu_response",
    "inv_x_green", "fft_inv_y", "fft_inv_z", "cic_interp", "surrogate",
    "patch_reduce", "kick_drift", "patch_fwd_z", "inv_xy_green", "fft_fwd_zy", "inv_yz"};

namespace {
thread_local std::string g_err = "no error";
}

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void timer_begin(Ctx& c, int stage) {
  Timer& t = c.timer;
  t.open = false;
  if (!t.enabled || c.capturing || !((t.mask >> stage) & 1u)) return;
  if (2 * (t.used + 1) > t.pool.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      t.pool.push_back(e);
    }
  }
  if (t.stage_of.size() <= t.used) t.stage_of.resize(t.used + 1);
  t.stage_of[t.used] = stage;
  (void)hipEventRecord(t.pool[2 * t.used], c.stream);
  t.open = true;
}

void timer_end(Ctx& c) {
  Timer& t = c.timer;
  if (!t.open) return;
  t.open = false;
  if (2 * t.used + 1 >= t.pool.size()) return;
  (void)hipEventRecord(t.pool[2 * t.used + 1], c.stream);
  ++t.used;
}

void drop_graph(Ctx& c) {
  if (c.graph_exec) hipGraphExecDestroy(c.graph_exec);
  if (c.graph) hipGraphDestroy(c.graph);
  c.graph_exec = nullptr;
  c.graph = nullptr;
}

namespace {

// k_fs(a) = sqrt(3/2 Omega_M(a) <v^-2>) a H, <v^-2> = 2 ln2/(3 zeta(3)) (m a / T_nu0)^2
double k_free_streaming(double a, double m_single, double om) {
  if (!(m_single > 0.0)) return 0.0;
  const double e2 = om / (a * a * a) + 1.0 - om;
  const double om_a = om / (a * a * a * e2);
  const double v2 = (2.0 * std::log(2.0) / (3.0 * 1.2020569031595942)) *
                    std::pow(m_single * a / kTnu0, 2);
  return std::sqrt(1.5 * om_a * v2) * a * kH0 * std::sqrt(e2);
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int validate(const pm_nu_config* c) {
  if (!c) return set_error(PM_NU_EINVAL, "config is NULL");
  if (!is_pow2(c->n_mesh) || c->n_mesh < 8 || c->n_mesh > 512)
    return set_error(PM_NU_EINVAL, "n_mesh must be a power of two in [8, 512] (got %d)",
                     c->n_mesh);
  if (c->n_boxes < 1 || c->n_boxes > 65535)
    return set_error(PM_NU_EINVAL, "n_boxes must be in [1, 65535]");
  if (c->n_particles < 1) return set_error(PM_NU_EINVAL, "n_particles must be >= 1");
  if (!(c->box_size > 0.0) || !std::isfinite(c->box_size))
    return set_error(PM_NU_EINVAL, "box_size must be positive");
  if (!(c->omega_m > 0.0 && c->omega_m <= 1.0))
    return set_error(PM_NU_EINVAL, "omega_m must be in (0, 1]");
  if (!(c->hubble > 0.0)) return set_error(PM_NU_EINVAL, "hubble must be positive");
  if (c->n_kbins < 1 || c->n_kbins > kMaxBins)
    return set_error(PM_NU_EINVAL, "n_kbins must be in [1, %d]", kMaxBins);
  if (c->max_history < 2) return set_error(PM_NU_EINVAL, "max_history must be >= 2");
  if (c->substeps < 1 || c->substeps > 1024)
    return set_error(PM_NU_EINVAL, "substeps must be in [1, 1024]");
  if (c->iterations < 1 || c->iterations > 16)
    return set_error(PM_NU_EINVAL, "iterations must be in [1, 16]");
  if (c->response_mode < 0 || c->response_mode > 2)
    return set_error(PM_NU_EINVAL, "response_mode must be 0, 1 or 2");
  if (c->n_species < 1) return set_error(PM_NU_EINVAL, "n_species must be >= 1");
  const double qcap = (static_cast<double>(c->max_history) - 1.0) * c->substeps + 1.0;
  if (qcap > 1e8) return set_error(PM_NU_EINVAL, "max_history * substeps too large");
  return PM_NU_OK;
}

template <typename T>
int dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess)
    return set_error(PM_NU_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                     hipGetErrorString(e));
  return PM_NU_OK;
}

void free_ctx(Ctx* c);

// Bin geometry (host_math.cpp) and its table of bins per integer |n|^2 on the device.
void build_bins(Ctx& c) {
  BinGeometry g = make_bin_geometry(c.N, c.cfg.box_size, c.B);
  c.edges = g.edges;
  c.counts = g.counts;
  c.kmean = g.kmean;
  c.nonempty = g.nonempty;
  hipMemcpy(c.bin_of_n2, g.bin_of_n2.data(), g.bin_of_n2.size() * sizeof(uint16_t),
            hipMemcpyHostToDevice);
}

// Node list of one box for a response at a_now: the stored nodes strictly before a_now
// (a stored node equal to a_now is recomputed) plus a_now itself.
int nodes_for(const Ctx& c, int box, double a_now, std::vector<double>& nodes, int& n_cur) {
  const std::vector<double>& ha = c.hist_a[box];
  if (ha.empty()) return set_error(PM_NU_EHISTORY, "box %d has no stored history", box);
  size_t m = ha.size();
  if (std::fabs(ha.back() - a_now) <= 1e-12 * a_now) --m;
  else if (a_now < ha.back())
    return set_error(PM_NU_EHISTORY, "a_now=%g precedes the last stored node %g of box %d",
                     a_now, ha.back(), box);
  // m = 0: a_now is the first stored node, where eq. (P-final) reduces to the initial
  // amplitude (no interval to integrate over)
  if (static_cast<int>(m) >= c.Jcap)
    return set_error(PM_NU_EHISTORY, "box %d: history full (%d nodes)", box, c.Jcap);
  nodes.assign(ha.begin(), ha.begin() + m);
  nodes.push_back(a_now);
  n_cur = static_cast<int>(m);
  return PM_NU_OK;
}

// Time grid of eq. (P-final) for every box at a_now (host FP64). The sub-intervals between
// stored nodes are kept per box and only the newest interval, to a_now, is integrated
// afresh; the arrays go to the device by stream-ordered copies from pinned staging.
int prepare_time_grid(Ctx& c, double a_now) {
  std::vector<std::vector<double>> all_nodes(c.nbox);
  std::vector<int> ncur(c.nbox);
  for (int b = 0; b < c.nbox; ++b) {
    int rc = nodes_for(c, b, a_now, all_nodes[b], ncur[b]);
    if (rc) return rc;
  }
  bool same = (c.tg_a_now == a_now) && (c.tg_version == c.hist_version) && ncur == c.n_cur;
  if (same) return PM_NU_OK;
  const double om = c.cfg.omega_m;
  const double pref = 1.5 * om * kH0 * kH0;   // the source keeps all matter, Omega_M
  const int Q = c.Q;
  const size_t qcap = static_cast<size_t>(c.qcap);
  PMNU_HIP(hipEventSynchronize(c.ev_tg));     // the staging's previous upload has run
  double* ds_all = c.h_tg;
  double* w_all = c.h_tg + c.nbox * qcap;
  double* l2_all = c.h_tg + 2 * c.nbox * qcap;
  std::vector<double> a_last(Q), seg_last(Q), hinv_last(Q);
  for (int b = 0; b < c.nbox; ++b) {
    const std::vector<double>& nd = all_nodes[b];
    const int n = ncur[b];
    const int nq = n * Q + 1;
    const Background bg = make_background(c.relativistic, om, c.cfg.hubble, c.species[b],
                                          c.nu_mult[b], c.nu_massless[b]);
    TgCache& cc = c.tgc[b];
    if (cc.bg_version != c.bg_version) {
      cc = TgCache();
      cc.bg_version = c.bg_version;
    }
    size_t keep = 0;   // leading stored nodes the cache was built from
    while (keep < cc.nodes.size() && keep < static_cast<size_t>(n) && cc.nodes[keep] == nd[keep])
      ++keep;
    const int kept = keep > 0 ? static_cast<int>(keep) - 1 : 0;   // intervals still valid
    cc.a.resize(static_cast<size_t>(kept) * Q);
    cc.seg.resize(cc.a.size());
    cc.hinv.resize(cc.a.size());
    for (int jj = kept; jj + 1 < n; ++jj) {                       // stored intervals to add
      const size_t o = cc.a.size();
      cc.a.resize(o + Q);
      cc.seg.resize(o + Q);
      cc.hinv.resize(o + Q);
      interval_nodes(bg, nd[jj], nd[jj + 1], Q, &cc.a[o], &cc.seg[o], &cc.hinv[o]);
    }
    cc.nodes.assign(nd.begin(), nd.begin() + n);
    if (n > 0)
      interval_nodes(bg, nd[n - 1], nd[n], Q, a_last.data(), seg_last.data(), hinv_last.data());
    double* dsb = ds_all + b * qcap;
    double* wb = w_all + b * qcap;
    assemble_time_grid(bg, nd.data(), n, Q, pref, cc.seg.data(), cc.hinv.data(),
                       seg_last.data(), hinv_last.data(), dsb, wb);
    // log2 of each s difference, for the fit's fractional power (0 where ds = 0: the
    // fit's x^4.1811 term is then 0 whatever this value)
    double* l2b = l2_all + b * qcap;
    for (int q = 0; q < nq; ++q) l2b[q] = dsb[q] > 0.0 ? std::log2(dsb[q]) : 0.0;
    RespBox& rb = c.h_resp[b];
    rb = RespBox();
    rb.f_nu = c.f_nu[b];
    const std::vector<double>& sp = c.species[b];
    rb.n_sp = static_cast<int>(sp.size());
    const double msum = std::accumulate(sp.begin(), sp.end(), 0.0);
    for (int s = 0; s < kMaxSpecies; ++s) {
      const bool on = s < rb.n_sp;
      rb.w_sp[s] = on ? (rb.n_sp == 1 ? 1.0 : sp[s] / msum) : 0.0;
      rb.tm_sp[s] = on ? kTnu0 / sp[s] : 0.0;
    }
    rb.t_over_m = rb.n_sp > 0 ? rb.tm_sp[0] : 0.0;
    // the network was trained on matter + Lambda with the fit for I(x)
    rb.sur_ok = c.sur_setting[b] && !c.relativistic && !c.series;
    rb.series = c.series ? 1 : 0;
    rb.ds_ic = dsb[0];
    rb.a_i = nd[0];
    rb.kfs = k_free_streaming(a_now, c.m_nu[b] / c.cfg.n_species, om);
    rb.m_total = c.m_nu[b];
    rb.a_now = a_now;
    rb.nq = nq;
    rb.n_cur = n;
    // the surrogate's history samples at fixed lags in ln a below the last stored node
    rb.sur_hist = 0;
    rb.sur_gap = n > 0 ? std::log(a_now) - std::log(nd[n - 1]) : 0.0;
    rb.sur_ds_last = n > 0 ? dsb[(n - 1) * Q] : 0.0;
    rb.sur_lna = std::log(a_now);
    rb.sur_lna0 = std::log(a_now / nd[0]);
    rb.sur_lnx0 = rb.sur_ds_last > 0.0 && rb.t_over_m > 0.0
                      ? std::log(rb.sur_ds_last * rb.t_over_m)
                      : -std::numeric_limits<double>::infinity();
    if (n >= 2 && std::log(nd[n - 1]) - kSurLag[kSurLags - 1] >= std::log(nd[0])) {
      rb.sur_hist = 1;
      const double u_last = std::log(nd[n - 1]);
      int j = n - 1;
      for (int m = 0; m < kSurLags; ++m) {
        const double u = u_last - kSurLag[m];
        while (j > 0 && std::log(nd[j]) > u) --j;
        if (j >= n - 1) {
          rb.sur_j[m] = n - 1;
          rb.sur_t[m] = 0.0;
        } else {
          const double u0 = std::log(nd[j]), u1 = std::log(nd[j + 1]);
          rb.sur_j[m] = j;
          rb.sur_t[m] = (u - u0) / (u1 - u0);
        }
      }
    }
  }
  const size_t bytes = c.nbox * qcap * sizeof(double);
  PMNU_HIP(hipMemcpyAsync(c.tg_ds, ds_all, bytes, hipMemcpyHostToDevice, c.stream));
  PMNU_HIP(hipMemcpyAsync(c.tg_w, w_all, bytes, hipMemcpyHostToDevice, c.stream));
  PMNU_HIP(hipMemcpyAsync(c.tg_l2, l2_all, bytes, hipMemcpyHostToDevice, c.stream));
  PMNU_HIP(hipMemcpyAsync(c.d_resp, c.h_resp, c.nbox * sizeof(RespBox), hipMemcpyHostToDevice,
                          c.stream));
  PMNU_HIP(hipEventRecord(c.ev_tg, c.stream));
  c.tg_a_now = a_now;
  c.tg_version = c.hist_version;
  c.n_cur = ncur;
  return PM_NU_OK;
}

}  // namespace

#define TIMED(ctx, stage, launch)                                                      \
  do {                                                                                 \
    timer_begin(ctx, stage);                                                           \
    hipError_t e_ = (launch);                                                          \
    timer_end(ctx);                                                                    \
    if (e_ != hipSuccess)                                                              \
      return set_error(PM_NU_EHIP, "kernel launch (%s) failed: %s", kStageNames[stage], \
                       hipGetErrorString(e_));                                         \
  } while (0)

namespace {

int do_deposit(Ctx& c, const float* pos) {
  if (!pos) return set_error(PM_NU_EINVAL, "pos is NULL");
  const int64_t cells = c.M * c.nbox;
  const double inv_cell = c.N / c.cfg.box_size;
  const double scale = static_cast<double>(c.M) / static_cast<double>(c.Np) / kFixScale;
  const bool fused = c.tune.deposit_mode >= 8;
  const int n_cells = static_cast<int>(c.nbox * patch_coarse_cells(c.N));
  // N <= 128: the x-plane fits the LDS and the z and y passes are one kernel, writing the
  // y-transformed modes straight to ck[0]
  const bool zy = c.N <= 128 && c.tune.fwd_zy && !fused;
  if (c.tune.deposit_mode >= 6) {
    const bool big = c.tune.deposit_mode == 7 || c.tune.deposit_mode == 9;
    TIMED(c, ST_DEPOSIT,
          launch_deposit_patch(pos, c.patches, c.reg_count, c.reg_list, c.rho_fb, c.n_fb,
                               c.Np, c.nbox, c.N, inv_cell, c.d_flags, big, c.stream));
    if (fused) {
      // the patch sums and the z pass in one kernel; fwd_y resets the registry
      TIMED(c, ST_PATCH_FWD_Z,
            launch_patch_fwd_z(c.N, c.patches, c.reg_count, c.reg_list, c.rho_fb, c.n_fb,
                               c.ck[1], c.tw, scale, c.nbox, c.stream,
                               c.keep_density ? c.delta : nullptr));
    } else {
      TIMED(c, ST_PATCH_REDUCE,
            launch_patch_reduce(c.patches, c.reg_count, c.reg_list, c.rho_fb, c.n_fb, c.delta,
                                c.nbox, c.N, scale, c.stream));
      if (zy)
        TIMED(c, ST_FWD_ZY, launch_fwd_zy(c.N, nullptr, c.delta, c.n_fb, c.reg_count, n_cells,
                                          c.ck[0], c.tw, scale, c.nbox, c.stream));
      else
        TIMED(c, ST_FFT_Z, launch_fwd_z(c.N, nullptr, c.delta, c.n_fb, c.reg_count, n_cells,
                                        c.ck[1], c.tw, scale, c.nbox, c.stream, c.tune.fft[0]));
    }
    c.density_is_delta = true;
    c.density_kept = !fused || c.keep_density;
  } else {
    TIMED(c, ST_ZERO, launch_fill_zero(c.rho, cells * 8, c.stream));
    TIMED(c, ST_DEPOSIT, launch_deposit(pos, c.rho, c.Np, c.nbox, c.N, inv_cell, c.d_flags,
                                        c.tune.deposit_mode, c.tune.deposit_block, c.stream));
    if (zy)
      TIMED(c, ST_FWD_ZY, launch_fwd_zy(c.N, c.rho, nullptr, nullptr, nullptr, 0, c.ck[0], c.tw,
                                        scale, c.nbox, c.stream));
    else
      TIMED(c, ST_FFT_Z, launch_fwd_z(c.N, c.rho, nullptr, nullptr, nullptr, 0, c.ck[1], c.tw,
                                      scale, c.nbox, c.stream, c.tune.fft[0]));
    c.density_is_delta = false;
    c.density_kept = true;
  }
  if (!zy)
    TIMED(c, ST_FFT_Y, launch_fwd_y(c.N, c.ck[1], c.ck[0], c.tw, c.nbox, c.stream,
                                    c.tune.fft[1], fused ? c.n_fb : nullptr,
                                    fused ? c.reg_count : nullptr, fused ? n_cells : 0));
  // the number of partial bin sums follows the tile of this pass
  c.n_partial = fwd_x_partials(c.N, c.tune.fft[2]);
  TIMED(c, ST_FFT_X_BIN, launch_fwd_x_bin(c.N, c.ck[0], c.tw, c.bin_of_n2, c.bin_partial,
                                          c.B, c.nbox, c.stream, c.tune.fft[2]));
  c.stage = 1;
  c.modes_valid = true;
  c.pos_dep = pos;
  return PM_NU_OK;
}

}  // namespace

int do_response_mode(Ctx& c, double a_now, int mode) {
  if (c.stage < 1) return set_error(PM_NU_ESTATE, "pm_nu_response needs pm_nu_deposit first");
  if (!(a_now > 0.0) || !std::isfinite(a_now)) return set_error(PM_NU_EINVAL, "bad a_now");
  if (!c.capturing) {
    // an eager step at another a moves the history past what a captured graph recomputes
    if (c.graph_exec && a_now != c.graph_a) drop_graph(c);
    int rc = prepare_time_grid(c, a_now);
    if (rc) return rc;
  } else if (c.tg_a_now != a_now) {
    return set_error(PM_NU_ESTATE, "time grid not prepared before capture");
  }
  const double norm = std::pow(c.cfg.box_size, 3) / (static_cast<double>(c.M) * c.M);
  if (mode == 0) {
    TIMED(c, ST_RESPONSE,
          launch_response(c.d_resp, c.bin_partial, c.n_partial, c.d_counts, c.d_kmean,
                          c.hist_pm, c.hist_pnu, c.ic_pnu, c.ic_theta, c.tg_ds, c.tg_l2, c.tg_w, c.B,
                          c.Jcap, c.qcap, c.Q, c.cfg.iterations, norm, c.nbox, c.pcdm, c.pnu,
                          c.ratio, c.stream, response_threads(c.B, c.nbox), c.series,
                          std::any_of(c.h_resp, c.h_resp + c.nbox,
                                      [](const RespBox& r) { return r.n_sp > 1; })));
  } else {
    int rc = surrogate_launch(c, mode, norm);
    if (rc) return rc;
  }
  // commit the node on the host side (the kernel wrote row n_cur)
  for (int b = 0; b < c.nbox; ++b) {
    std::vector<double>& ha = c.hist_a[b];
    if (static_cast<int>(ha.size()) == c.n_cur[b]) {
      ha.push_back(a_now);
    } else {
      ha.resize(c.n_cur[b] + 1);
      ha.back() = a_now;
    }
  }
  c.stage = 2;
  c.a_resp = a_now;
  return PM_NU_OK;
}

namespace {

int do_force(Ctx& c, const float* pos, float* acc, double a_now, const Leap* lp = nullptr) {
  if (c.stage != 2) return set_error(PM_NU_ESTATE, "pm_nu_force needs pm_nu_response first");
  if (!c.modes_valid)
    return set_error(PM_NU_ESTATE, "pm_nu_force needs the modes of a deposit (the power was set)");
  if (a_now != c.a_resp)
    return set_error(PM_NU_ESTATE, "pm_nu_force a_now differs from the response's");
  if (!pos || !acc) return set_error(PM_NU_EINVAL, "pos/acc is NULL");
  const float kf = static_cast<float>(2.0 * kPi / c.cfg.box_size);
  const double cgreen = 1.5 * c.cfg.omega_m * kH0 * kH0 / a_now / static_cast<double>(c.M);
  // N <= 64: an x-plane's F1 and F2 fit the LDS and the last two inverse passes are one
  // kernel; else the k_z slab fits the LDS and the first two are one kernel, whose G1 goes to
  // ck[1] (ck[0] still holds the modes it reads)
  const bool inv_yz = c.N <= 64 && c.tune.inv_yz;
  const bool inv_xy = c.N <= 64 && c.tune.inv_xy && !inv_yz;
  float2* g1 = inv_xy ? c.ck[1] : c.ck[0];
  if (inv_yz) {
    TIMED(c, ST_INV_X_GREEN,
          launch_inv_x(c.N, c.ck[0], c.ck[1], c.ck[2], c.tw, c.ridx, c.d_next, c.ratio,
                       c.d_resp, c.B, c.inv_w2, static_cast<float>(cgreen), kf, c.nbox, c.stream,
                       c.tune.fft[3]));
    TIMED(c, ST_INV_YZ, launch_inv_yz(c.N, c.ck[1], c.ck[2], c.force, c.tw, kf, c.nbox,
                                      c.stream));
  } else if (inv_xy) {
    TIMED(c, ST_INV_XY,
          launch_inv_xy(c.N, c.ck[0], g1, c.ck[3], c.ck[4], c.tw, c.ridx, c.d_next, c.ratio,
                        c.d_resp, c.B, c.inv_w2, static_cast<float>(cgreen), kf, c.nbox,
                        c.stream));
  } else {
    TIMED(c, ST_INV_X_GREEN,
          launch_inv_x(c.N, c.ck[0], c.ck[1], c.ck[2], c.tw, c.ridx, c.d_next, c.ratio,
                       c.d_resp, c.B, c.inv_w2, static_cast<float>(cgreen), kf, c.nbox, c.stream,
                       c.tune.fft[3]));
    TIMED(c, ST_INV_Y, launch_inv_y(c.N, c.ck[1], c.ck[2], g1, c.ck[3], c.ck[4], c.tw, kf,
                                    c.nbox, c.stream, c.tune.fft[4]));
  }
  if (!inv_yz)
    TIMED(c, ST_INV_Z, launch_inv_z(c.N, g1, c.ck[3], c.ck[4], c.force, c.tw, kf, c.nbox,
                                    c.stream, c.tune.fft[5]));
  TIMED(c, ST_INTERP, launch_interp(pos, c.force, acc, c.Np, c.nbox, c.N,
                                    c.N / c.cfg.box_size, c.tune.interp_mode,
                                    c.tune.interp_block, c.stream, lp));
  c.stage = 0;
  return PM_NU_OK;
}

void free_ctx(Ctx* c) {
  if (!c) return;
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  if (c->graph) hipGraphDestroy(c->graph);
  for (hipEvent_t e : c->timer.pool) hipEventDestroy(e);
  void* bufs[] = {c->rho, c->ck[0], c->ck[1], c->ck[2], c->ck[3], c->ck[4], c->force,
                  c->bin_partial,
                  c->bin_of_n2, c->d_counts, c->d_kmean, c->d_lnk, c->d_nonempty, c->pcdm, c->pnu,
                  c->ratio, c->hist_pm, c->hist_pnu, c->ic_pnu, c->ic_theta, c->tg_ds,
                  c->tg_l2, c->tg_w, c->d_resp, c->ridx, c->d_next, c->tw, c->inv_w2,
                  c->d_flags, c->patches, c->reg_count, c->reg_list, c->rho_fb, c->n_fb,
                  c->delta, c->d_kd};
  for (void* p : bufs)
    if (p) hipFree(p);
  for (void* p : {static_cast<void*>(c->h_tg), static_cast<void*>(c->h_resp),
                  static_cast<void*>(c->h_kd)})
    if (p) hipHostFree(p);
  if (c->ev_tg) hipEventDestroy(c->ev_tg);
  if (c->ev_kd) hipEventDestroy(c->ev_kd);
  delete c;
}

}  // namespace

}  // namespace pmnu

using namespace pmnu;

extern "C" {

void pm_nu_default_config(pm_nu_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->n_mesh = 32;
  cfg->n_boxes = 1;
  cfg->n_particles = 32768;
  cfg->box_size = 128.0;
  cfg->omega_m = 0.3;
  cfg->hubble = 0.7;
  cfg->n_kbins = 32;
  cfg->max_history = 256;
  cfg->substeps = 8;
  cfg->iterations = 1;
  cfg->deconvolve = 1;
  cfg->response_mode = 0;
  cfg->n_species = 3;
  cfg->stream = nullptr;
}

const char* pm_nu_last_error(void) { return g_err.c_str(); }

int pm_nu_init(const pm_nu_config* cfg, const double* m_nu_total, pm_nu_ctx** out) {
  if (!out) return set_error(PM_NU_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  if (!m_nu_total) return set_error(PM_NU_EINVAL, "m_nu_total is NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return set_error(PM_NU_ENODEV, "no HIP device");
  Ctx* c = new (std::nothrow) Ctx();
  if (!c) return set_error(PM_NU_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  hipGetDevice(&c->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess &&
      std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    delete c;
    return set_error(PM_NU_ENODEV, "device %d is %s, this library is built for gfx950",
                     c->device, prop.gcnArchName);
  }
  c->N = cfg->n_mesh;
  c->NK = c->N / 2 + 1;
  c->nbox = cfg->n_boxes;
  c->B = cfg->n_kbins;
  c->Jcap = cfg->max_history;
  c->Q = cfg->substeps;
  c->Np = cfg->n_particles;
  c->M = static_cast<int64_t>(c->N) * c->N * c->N;
  c->MH = static_cast<int64_t>(c->NK) * c->N * c->N;
  c->n2max = 3 * c->N * c->N / 4;
  c->qcap = (c->Jcap - 1) * c->Q + 1;
  c->n_partial = fwd_x_partials(c->N, 0);
  // room for the partial sums of every tile candidate of the binning pass
  int max_partial = c->n_partial;
  for (int v = 1; v < 3; ++v) max_partial = std::max(max_partial, fwd_x_partials(c->N, v));
  c->n_partial_cap = max_partial;
  // the patch deposit is the faster one once the mesh holds many coarse cells
  c->tune.deposit_mode = c->N >= 64 ? 6 : 4;
  c->stream = static_cast<hipStream_t>(cfg->stream);
  c->m_nu.assign(m_nu_total, m_nu_total + c->nbox);
  for (int b = 0; b < c->nbox; ++b) {
    const double m = c->m_nu[b];
    if (!(m >= 0.0) || !std::isfinite(m)) {
      delete c;
      return set_error(PM_NU_EINVAL, "m_nu_total[%d] must be >= 0", b);
    }
    c->f_nu.push_back(m / (93.14 * cfg->omega_m * cfg->hubble * cfg->hubble));
    const double m1 = m / cfg->n_species;
    c->t_over_m.push_back(m1 > 0 ? kTnu0 / m1 : 0.0);
    // n_species equal masses: one kernel with weight 1
    c->species.push_back(m1 > 0 ? std::vector<double>{m1} : std::vector<double>{});
    c->nu_mult.push_back(cfg->n_species);
    c->nu_massless.push_back(m1 > 0 ? 0 : cfg->n_species);
    c->sur_setting.push_back(cfg->n_species == 3 ? 1 : 0);
  }
  c->ic_base.assign(c->nbox, std::vector<double>(c->B, 0.0));
  const size_t nb = c->nbox, B = c->B;
#define ALLOC(ptr, count)                 \
  do {                                    \
    int rc_ = dalloc(&(ptr), (count));    \
    if (rc_) {                            \
      free_ctx(c);                        \
      return rc_;                         \
    }                                     \
  } while (0)
  ALLOC(c->rho, nb * c->M);
  for (int i = 0; i < 5; ++i) ALLOC(c->ck[i], nb * c->MH);
  ALLOC(c->force, 3 * nb * c->M);
  ALLOC(c->bin_partial, nb * c->n_partial_cap * B);
  ALLOC(c->bin_of_n2, static_cast<size_t>(c->n2max) + 1);
  ALLOC(c->d_counts, B);
  ALLOC(c->d_kmean, B);
  ALLOC(c->d_lnk, B);
  ALLOC(c->d_nonempty, B);
  ALLOC(c->pcdm, nb * B);
  ALLOC(c->pnu, nb * B);
  ALLOC(c->ratio, nb * B);
  ALLOC(c->hist_pm, nb * c->Jcap * B);
  ALLOC(c->hist_pnu, nb * c->Jcap * B);
  ALLOC(c->ic_pnu, nb * kMaxSpecies * B);
  ALLOC(c->ic_theta, nb * B);
  ALLOC(c->tg_ds, nb * c->qcap);
  ALLOC(c->tg_l2, nb * c->qcap);
  ALLOC(c->tg_w, nb * c->qcap);
  ALLOC(c->d_resp, nb);
  ALLOC(c->ridx, static_cast<size_t>(c->n2max) + 1);
  ALLOC(c->d_next, B);
  ALLOC(c->tw, static_cast<size_t>(c->N));
  ALLOC(c->inv_w2, static_cast<size_t>(c->N));
  ALLOC(c->d_flags, 1);
  {
    const size_t chunks = nb * static_cast<size_t>(patch_chunks(c->Np));
    const size_t coarse = nb * static_cast<size_t>(patch_coarse_cells(c->N));
    ALLOC(c->patches, chunks * kPatchCap);
    ALLOC(c->reg_count, coarse);
    ALLOC(c->reg_list, coarse * 32);
    ALLOC(c->rho_fb, nb * c->M);
    ALLOC(c->n_fb, 2);
    ALLOC(c->delta, nb * c->M);
  }
  ALLOC(c->d_kd, 2 * nb);
#undef ALLOC
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_tg), 3 * nb * c->qcap * sizeof(double)) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_resp), nb * sizeof(RespBox)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_kd), 2 * nb * sizeof(double)) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_tg, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_kd, hipEventDisableTiming) != hipSuccess) {
    free_ctx(c);
    return set_error(PM_NU_ENOMEM, "pinned staging or events could not be created");
  }
  std::memset(c->h_tg, 0, 3 * nb * c->qcap * sizeof(double));
  c->tgc.resize(c->nbox);
  build_bins(*c);
  if (c->nonempty.empty()) {
    free_ctx(c);
    return set_error(PM_NU_EINVAL, "all k-bins are empty");
  }
  std::vector<float2> tw(c->N);
  std::vector<float> iw(c->N);
  for (int m = 0; m < c->N; ++m) {
    const double ph = -2.0 * kPi * m / c->N;
    tw[m] = make_float2(static_cast<float>(std::cos(ph)), static_cast<float>(std::sin(ph)));
    const int nm = m < c->N / 2 ? m : m - c->N;
    const double t = kPi * nm / c->N;
    const double sinc = (nm == 0) ? 1.0 : std::sin(t) / t;
    iw[m] = cfg->deconvolve ? static_cast<float>(1.0 / std::pow(sinc, 4)) : 1.0f;
  }
  std::vector<int> ne(c->nonempty);
  ne.resize(B, 0);
  std::vector<int> next(B);                       // next non-empty bin (the last: itself)
  for (size_t b = 0; b < B; ++b) next[b] = static_cast<int>(b);
  for (size_t i = 0; i + 1 < c->nonempty.size(); ++i) next[c->nonempty[i]] = c->nonempty[i + 1];
  hipError_t e = hipSuccess;
  e = e ? e : hipMemcpy(c->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(c->inv_w2, iw.data(), iw.size() * sizeof(float), hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(c->d_counts, c->counts.data(), B * sizeof(double), hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(c->d_kmean, c->kmean.data(), B * sizeof(double), hipMemcpyHostToDevice);
  std::vector<double> lnk(B, 0.0);
  for (size_t b = 0; b < B; ++b) lnk[b] = c->kmean[b] > 0 ? std::log(c->kmean[b]) : 0.0;
  e = e ? e : hipMemcpy(c->d_lnk, lnk.data(), B * sizeof(double), hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(c->d_nonempty, ne.data(), B * sizeof(int), hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(c->d_next, next.data(), B * sizeof(int), hipMemcpyHostToDevice);
  e = e ? e : launch_ratio_index(c->d_lnk, c->d_nonempty, static_cast<int>(c->nonempty.size()),
                                 c->n2max, 2.0 * kPi / cfg->box_size, c->ridx, nullptr);
  e = e ? e : hipMemset(c->d_flags, 0, sizeof(int));
  e = e ? e : hipMemset(c->hist_pm, 0, nb * c->Jcap * B * sizeof(double));
  e = e ? e : hipMemset(c->hist_pnu, 0, nb * c->Jcap * B * sizeof(double));
  e = e ? e : hipMemset(c->ic_pnu, 0, nb * kMaxSpecies * B * sizeof(double));
  e = e ? e : hipMemset(c->ic_theta, 0, nb * B * sizeof(double));
  e = e ? e : hipMemset(c->pcdm, 0, nb * B * sizeof(double));
  e = e ? e : hipMemset(c->pnu, 0, nb * B * sizeof(double));
  e = e ? e : hipMemset(c->ratio, 0, nb * B * sizeof(double));
  // the patch deposit keeps these at zero between deposits
  e = e ? e : hipMemset(c->reg_count, 0, nb * patch_coarse_cells(c->N) * sizeof(int));
  e = e ? e : hipMemset(c->rho_fb, 0, nb * c->M * sizeof(unsigned long long));
  e = e ? e : hipMemset(c->n_fb, 0, 2 * sizeof(int));
  e = e ? e : hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_ctx(c);
    return set_error(PM_NU_EHIP, "init upload failed: %s", hipGetErrorString(e));
  }
  c->hist_a.assign(c->nbox, {});
  c->has_ic.assign(c->nbox, 0);
  c->n_cur.assign(c->nbox, -1);
  *out = reinterpret_cast<pm_nu_ctx*>(c);
  return PM_NU_OK;
}

void pm_nu_destroy(pm_nu_ctx* ctx) {
  Ctx* c = reinterpret_cast<Ctx*>(ctx);
  if (!c) return;
  hipDeviceSynchronize();
  surrogate_free(*c);
  free_ctx(c);
}

#define GET_CTX(ctx)                                                    \
  Ctx* c = reinterpret_cast<Ctx*>(ctx);                                 \
  if (!c) return set_error(PM_NU_EINVAL, "ctx is NULL")

int pm_nu_get_bins(pm_nu_ctx* ctx, int64_t* edge_n2, double* mode_count, double* k_mean) {
  GET_CTX(ctx);
  if (edge_n2) std::copy(c->edges.begin(), c->edges.end(), edge_n2);
  if (mode_count) std::copy(c->counts.begin(), c->counts.end(), mode_count);
  if (k_mean) std::copy(c->kmean.begin(), c->kmean.end(), k_mean);
  return PM_NU_OK;
}

int pm_nu_set_history(pm_nu_ctx* ctx, int box, int n_nodes, const double* a,
                      const double* pm_half, const double* pnu_half,
                      const double* pnu_half_init, const double* theta_over_delta_init) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step would not see the change
  if (box < 0 || box >= c->nbox) return set_error(PM_NU_EINVAL, "box %d out of range", box);
  if (n_nodes < 1 || n_nodes >= c->Jcap)
    return set_error(PM_NU_EHISTORY, "n_nodes must be in [1, max_history-1] (got %d)", n_nodes);
  if (!a || !pm_half || !pnu_half || !pnu_half_init || !theta_over_delta_init)
    return set_error(PM_NU_EINVAL, "history array is NULL");
  for (int j = 0; j < n_nodes; ++j) {
    if (!(a[j] > 0.0) || !std::isfinite(a[j]) || (j > 0 && !(a[j] > a[j - 1])))
      return set_error(PM_NU_EHISTORY, "history scale factors must be positive and increasing");
  }
  const size_t B = c->B;
  PMNU_HIP(hipStreamSynchronize(c->stream));
  const size_t off = static_cast<size_t>(box) * c->Jcap * B;
  PMNU_HIP(hipMemcpy(c->hist_pm + off, pm_half, n_nodes * B * sizeof(double),
                     hipMemcpyHostToDevice));
  PMNU_HIP(hipMemcpy(c->hist_pnu + off, pnu_half, n_nodes * B * sizeof(double),
                     hipMemcpyHostToDevice));
  // every species starts from this amplitude (pm_nu_set_species may give their own)
  for (int sp = 0; sp < kMaxSpecies; ++sp)
    PMNU_HIP(hipMemcpy(c->ic_pnu + (static_cast<size_t>(box) * kMaxSpecies + sp) * B,
                       pnu_half_init, B * sizeof(double), hipMemcpyHostToDevice));
  c->ic_base[box].assign(pnu_half_init, pnu_half_init + B);
  PMNU_HIP(hipMemcpy(c->ic_theta + box * B, theta_over_delta_init, B * sizeof(double),
                     hipMemcpyHostToDevice));
  c->hist_a[box].assign(a, a + n_nodes);
  c->has_ic[box] = 1;
  ++c->hist_version;
  return PM_NU_OK;
}

int pm_nu_get_history(pm_nu_ctx* ctx, int box, int* n_nodes, double* a, double* pm_half,
                      double* pnu_half) {
  GET_CTX(ctx);
  if (box < 0 || box >= c->nbox) return set_error(PM_NU_EINVAL, "box %d out of range", box);
  const int n = static_cast<int>(c->hist_a[box].size());
  if (n_nodes) *n_nodes = n;
  if (a) std::copy(c->hist_a[box].begin(), c->hist_a[box].end(), a);
  PMNU_HIP(hipStreamSynchronize(c->stream));
  const size_t B = c->B, off = static_cast<size_t>(box) * c->Jcap * B;
  if (pm_half && n)
    PMNU_HIP(hipMemcpy(pm_half, c->hist_pm + off, n * B * sizeof(double), hipMemcpyDeviceToHost));
  if (pnu_half && n)
    PMNU_HIP(hipMemcpy(pnu_half, c->hist_pnu + off, n * B * sizeof(double),
                       hipMemcpyDeviceToHost));
  return PM_NU_OK;
}

int pm_nu_deposit(pm_nu_ctx* ctx, const float* pos) {
  GET_CTX(ctx);
  return do_deposit(*c, pos);
}

int pm_nu_response(pm_nu_ctx* ctx, double a_now) {
  GET_CTX(ctx);
  return do_response_mode(*c, a_now, c->cfg.response_mode);
}

int pm_nu_set_response_mode(pm_nu_ctx* ctx, int mode) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step would not see the change
  if (mode < 0 || mode > 2) return set_error(PM_NU_EINVAL, "response_mode must be 0, 1 or 2");
  c->cfg.response_mode = mode;
  return PM_NU_OK;
}

int pm_nu_set_mass(pm_nu_ctx* ctx, int box, double m_nu_total) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step would not see the change
  ++c->bg_version;   // H(a) may change
  if (box < 0 || box >= c->nbox) return set_error(PM_NU_EINVAL, "box %d out of range", box);
  if (!(m_nu_total >= 0.0) || !std::isfinite(m_nu_total))
    return set_error(PM_NU_EINVAL, "m_nu_total must be >= 0");
  const double h = c->cfg.hubble;
  c->m_nu[box] = m_nu_total;
  c->f_nu[box] = m_nu_total / (93.14 * c->cfg.omega_m * h * h);
  const double m1 = m_nu_total / c->cfg.n_species;
  c->t_over_m[box] = m1 > 0 ? kTnu0 / m1 : 0.0;
  c->species[box] = m1 > 0 ? std::vector<double>{m1} : std::vector<double>{};
  c->nu_mult[box] = c->cfg.n_species;
  c->nu_massless[box] = m1 > 0 ? 0 : c->cfg.n_species;
  c->sur_setting[box] = c->cfg.n_species == 3 ? 1 : 0;
  c->tg_a_now = -1.0;   // the per-box constants of the response are rebuilt
  return PM_NU_OK;
}

int pm_nu_set_species(pm_nu_ctx* ctx, int box, int n_species, const double* m_species,
                      const double* pnu_half_init) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step would not see the change
  ++c->bg_version;   // H(a) may change
  if (box < 0 || box >= c->nbox) return set_error(PM_NU_EINVAL, "box %d out of range", box);
  if (n_species < 1 || n_species > kMaxSpecies || !m_species)
    return set_error(PM_NU_EINVAL, "n_species must be in [1, %d] with masses given",
                     kMaxSpecies);
  std::vector<double> massive;
  std::vector<int> src;
  double total = 0.0;
  for (int i = 0; i < n_species; ++i) {
    if (!(m_species[i] >= 0.0) || !std::isfinite(m_species[i]))
      return set_error(PM_NU_EINVAL, "species masses must be finite and >= 0");
    total += m_species[i];
    if (m_species[i] > 0.0) {
      massive.push_back(m_species[i]);
      src.push_back(i);
    }
  }
  const size_t B = c->B;
  if (pnu_half_init)
    for (size_t i = 0; i < static_cast<size_t>(n_species) * B; ++i)
      if (!std::isfinite(pnu_half_init[i]))
        return set_error(PM_NU_EINVAL, "species initial amplitudes must be finite");
  PMNU_HIP(hipStreamSynchronize(c->stream));
  // initial amplitudes of the massive species, compacted into slots 0..n-1
  for (size_t s = 0; s < massive.size(); ++s) {
    const double* from = pnu_half_init ? pnu_half_init + src[s] * B : c->ic_base[box].data();
    PMNU_HIP(hipMemcpy(c->ic_pnu + (static_cast<size_t>(box) * kMaxSpecies + s) * B, from,
                       B * sizeof(double), hipMemcpyHostToDevice));
  }
  const double h = c->cfg.hubble;
  c->m_nu[box] = total;
  c->f_nu[box] = total / (93.14 * c->cfg.omega_m * h * h);
  c->t_over_m[box] = massive.empty() ? 0.0 : kTnu0 / massive[0];
  c->species[box] = massive;
  c->nu_mult[box] = 1;
  c->nu_massless[box] = n_species - static_cast<int>(massive.size());
  bool equal3 = n_species == 3 && massive.size() == 3 && !pnu_half_init;
  for (size_t s = 1; equal3 && s < massive.size(); ++s) equal3 = massive[s] == massive[0];
  c->sur_setting[box] = equal3 ? 1 : 0;
  c->tg_a_now = -1.0;   // the per-box constants of the response are rebuilt
  return PM_NU_OK;
}

int pm_nu_set_background(pm_nu_ctx* ctx, int relativistic) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step would not see the change
  ++c->bg_version;   // H(a) may change
  if (relativistic != 0 && relativistic != 1)
    return set_error(PM_NU_EINVAL, "relativistic must be 0 or 1 (got %d)", relativistic);
  c->relativistic = relativistic == 1;
  c->tg_a_now = -1.0;   // the time grid is rebuilt on the next response
  return PM_NU_OK;
}

int pm_nu_set_kernel(pm_nu_ctx* ctx, int series) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step would not see the change
  if (series != 0 && series != 1)
    return set_error(PM_NU_EINVAL, "series must be 0 or 1 (got %d)", series);
  c->series = series == 1;
  c->tg_a_now = -1.0;   // the per-box constants of the response are rebuilt
  return PM_NU_OK;
}

int pm_nu_set_iterations(pm_nu_ctx* ctx, int iterations) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step would not see the change
  if (iterations < 1 || iterations > 16)
    return set_error(PM_NU_EINVAL, "iterations must be in [1, 16] (got %d)", iterations);
  c->cfg.iterations = iterations;
  return PM_NU_OK;
}

int pm_nu_kernel_values(const double* x, int64_t n, int series, double* out, void* stream) {
  if (n < 0 || (n > 0 && (!x || !out)))
    return set_error(PM_NU_EINVAL, "x and out must be device arrays of n >= 0 doubles");
  if (series != 0 && series != 1)
    return set_error(PM_NU_EINVAL, "series must be 0 or 1 (got %d)", series);
  hipError_t e = launch_kernel_values(x, n, series, out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return set_error(PM_NU_EHIP, "kernel_values: %s", hipGetErrorString(e));
  return PM_NU_OK;
}

int pm_nu_set_power(pm_nu_ctx* ctx, int box, const double* p_cdm) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step would not see the change
  if (box < 0 || box >= c->nbox || !p_cdm) return set_error(PM_NU_EINVAL, "bad box/p_cdm");
  // The response sums the per-workgroup partial mode sums of each bin ([bin][workgroup]):
  // put the whole sum w |delta_k|^2 = P C_b N^6 / L^3 in the first partial, zero the rest.
  const double norm = std::pow(c->cfg.box_size, 3) / (static_cast<double>(c->M) * c->M);
  std::vector<double> part(static_cast<size_t>(c->n_partial) * c->B, 0.0);
  for (int b = 0; b < c->B; ++b) {
    if (!std::isfinite(p_cdm[b]) || p_cdm[b] < 0.0)
      return set_error(PM_NU_EINVAL, "p_cdm[%d] must be finite and >= 0", b);
    if (c->counts[b] > 0) part[static_cast<size_t>(b) * c->n_partial] = p_cdm[b] * c->counts[b] / norm;
  }
  PMNU_HIP(hipStreamSynchronize(c->stream));
  PMNU_HIP(hipMemcpy(c->bin_partial + static_cast<size_t>(box) * c->n_partial * c->B, part.data(),
                     part.size() * sizeof(double), hipMemcpyHostToDevice));
  c->stage = 1;
  c->modes_valid = false;
  return PM_NU_OK;
}

int pm_nu_force(pm_nu_ctx* ctx, const float* pos, float* acc, double a_now) {
  GET_CTX(ctx);
  if (pos != c->pos_dep) return set_error(PM_NU_EINVAL, "pos differs from the deposit's array");
  return do_force(*c, pos, acc, a_now);
}

int pm_nu_step(pm_nu_ctx* ctx, const float* pos, float* acc, double a_now) {
  int rc = pm_nu_deposit(ctx, pos);
  if (rc) return rc;
  rc = pm_nu_response(ctx, a_now);
  if (rc) return rc;
  return pm_nu_force(ctx, pos, acc, a_now);
}

namespace {

// Kick and drift factors of every box, copied in stream order ahead of the next kick_drift
// launch.
int upload_kd(Ctx& c, const std::vector<double>& kd) {
  PMNU_HIP(hipEventSynchronize(c.ev_kd));     // the staging's previous upload has run
  std::copy(kd.begin(), kd.end(), c.h_kd);
  PMNU_HIP(hipMemcpyAsync(c.d_kd, c.h_kd, kd.size() * sizeof(double), hipMemcpyHostToDevice,
                          c.stream));
  PMNU_HIP(hipEventRecord(c.ev_kd, c.stream));
  return PM_NU_OK;
}

}  // namespace

int pm_nu_advance(pm_nu_ctx* ctx, float* pos, float* vel, float* acc, const double* a_steps,
                  int n_steps) {
  GET_CTX(ctx);
  if (!pos || !vel || !acc || !a_steps || n_steps < 1)
    return set_error(PM_NU_EINVAL, "pos, vel, acc and a_steps are needed, n_steps >= 1");
  for (const void* p : {static_cast<const void*>(pos), static_cast<const void*>(vel),
                        static_cast<const void*>(acc)})
    if (reinterpret_cast<uintptr_t>(p) % 16)
      return set_error(PM_NU_EINVAL, "pos, vel and acc must be 16-byte aligned");
  for (int j = 0; j <= n_steps; ++j)
    if (!(a_steps[j] > 0.0) || !std::isfinite(a_steps[j]) || (j && !(a_steps[j] > a_steps[j - 1])))
      return set_error(PM_NU_EINVAL, "a_steps must be finite, positive and increasing");
  for (int b = 0; b < c->nbox; ++b) {
    const std::vector<double>& ha = c->hist_a[b];
    if (ha.empty()) return set_error(PM_NU_EHISTORY, "box %d has no stored history", b);
    if (a_steps[1] <= ha.back() * (1.0 + 1e-12))
      return set_error(PM_NU_EHISTORY, "box %d: a_steps[1]=%g does not follow the last stored "
                       "node %g", b, a_steps[1], ha.back());
    if (static_cast<int>(ha.size()) + n_steps > c->Jcap)
      return set_error(PM_NU_EHISTORY, "box %d: %d more nodes do not fit the history (%d of %d "
                       "used)", b, n_steps, static_cast<int>(ha.size()), c->Jcap);
  }
  std::vector<Background> bg(c->nbox);
  for (int b = 0; b < c->nbox; ++b)
    bg[b] = make_background(c->relativistic, c->cfg.omega_m, c->cfg.hubble, c->species[b],
                            c->nu_mult[b], c->nu_massless[b]);
  const float L = static_cast<float>(c->cfg.box_size);
  std::vector<double> kd(2 * static_cast<size_t>(c->nbox));
  auto a_mid = [&](int j) { return std::sqrt(a_steps[j] * a_steps[j + 1]); };
  // opening half kick with the given force, and the first drift
  for (int b = 0; b < c->nbox; ++b) {
    kd[2 * b] = a_steps[0] * kick_of(bg[b], a_steps[0], a_mid(0));
    kd[2 * b + 1] = ds_of(bg[b], a_steps[0], a_steps[1]);
  }
  int rc = upload_kd(*c, kd);
  if (rc) return rc;
  TIMED(*c, ST_KICK_DRIFT, launch_kick_drift(pos, vel, acc, c->d_kd, c->Np, c->nbox, L, true,
                                             c->stream));
  for (int j = 0; j < n_steps; ++j) {
    const double a1 = a_steps[j + 1];
    rc = do_deposit(*c, pos);
    if (rc) return rc;
    rc = do_response_mode(*c, a1, c->cfg.response_mode);
    if (rc) return rc;
    // the interpolation applies the force at a1 at once: the closing half kick of this step
    // with the opening one of the next and the next drift, or (last step) the closing half
    // kick alone, storing the force
    const bool last = j + 1 == n_steps;
    for (int b = 0; b < c->nbox; ++b) {
      kd[2 * b] = a1 * kick_of(bg[b], a_mid(j), last ? a1 : a_mid(j + 1));
      kd[2 * b + 1] = last ? 0.0 : ds_of(bg[b], a1, a_steps[j + 2]);
    }
    rc = upload_kd(*c, kd);
    if (rc) return rc;
    Leap lp;
    lp.vel = vel;
    lp.pos = last ? nullptr : pos;
    lp.kd = c->d_kd;
    lp.box = L;
    lp.store_acc = last ? 1 : 0;
    rc = do_force(*c, pos, acc, a1, &lp);
    if (rc) return rc;
  }
  return PM_NU_OK;
}

int pm_nu_get_spectrum(pm_nu_ctx* ctx, int box, double* p_cdm, double* pnu_half,
                       double* ratio) {
  GET_CTX(ctx);
  if (box < 0 || box >= c->nbox) return set_error(PM_NU_EINVAL, "box %d out of range", box);
  if (c->stage == 1) {
    // deposited (or power set) but no response yet: reduce the bin partials now
    const double norm = std::pow(c->cfg.box_size, 3) / (static_cast<double>(c->M) * c->M);
    hipError_t e = launch_bin_power(c->bin_partial, c->n_partial, c->d_counts, c->B, norm,
                                    c->nbox, c->pcdm, c->stream);
    if (e != hipSuccess) return set_error(PM_NU_EHIP, "bin power: %s", hipGetErrorString(e));
  }
  PMNU_HIP(hipStreamSynchronize(c->stream));
  const size_t B = c->B;
  if (p_cdm) PMNU_HIP(hipMemcpy(p_cdm, c->pcdm + box * B, B * sizeof(double), hipMemcpyDeviceToHost));
  if (pnu_half)
    PMNU_HIP(hipMemcpy(pnu_half, c->pnu + box * B, B * sizeof(double), hipMemcpyDeviceToHost));
  if (ratio) PMNU_HIP(hipMemcpy(ratio, c->ratio + box * B, B * sizeof(double), hipMemcpyDeviceToHost));
  int flags = 0;
  PMNU_HIP(hipMemcpy(&flags, c->d_flags, sizeof(int), hipMemcpyDeviceToHost));
  if (flags & 1) {
    PMNU_HIP(hipMemset(c->d_flags, 0, sizeof(int)));
    return set_error(PM_NU_ENONFINITE, "a non-finite particle position was skipped");
  }
  return PM_NU_OK;
}

int pm_nu_side_grid_uses(pm_nu_ctx* ctx, int64_t* uses) {
  GET_CTX(ctx);
  if (!uses) return set_error(PM_NU_EINVAL, "uses is NULL");
  *uses = 0;
  if (!c->n_fb) return PM_NU_OK;            // no patch deposit buffers (N < 64 by default)
  PMNU_HIP(hipStreamSynchronize(c->stream));
  unsigned total = 0;
  PMNU_HIP(hipMemcpy(&total, c->n_fb + 1, sizeof(unsigned), hipMemcpyDeviceToHost));
  *uses = static_cast<int64_t>(total - c->fb_seen);   // modulo 2^32, like the device count
  c->fb_seen = total;
  return PM_NU_OK;
}

int pm_nu_copy_density(pm_nu_ctx* ctx, int box, float* out) {
  GET_CTX(ctx);
  if (box < 0 || box >= c->nbox || !out) return set_error(PM_NU_EINVAL, "bad box/out");
  if (c->tune.deposit_mode >= 8 && !c->density_kept)
    return set_error(PM_NU_ESTATE, "deposit modes 8 and 9 store the density only after "
                                   "pm_nu_set_keep_density(ctx, 1)");
  hipError_t e =
      c->density_is_delta
          ? launch_delta_to_density(c->delta + box * c->M, out, c->M,
                                    static_cast<float>(static_cast<double>(c->Np) / c->M),
                                    c->stream)
          : launch_fixed_to_float(c->rho + box * c->M, out, c->M, c->stream);
  if (e != hipSuccess) return set_error(PM_NU_EHIP, "copy_density: %s", hipGetErrorString(e));
  return PM_NU_OK;
}

int pm_nu_set_inverse_xy(pm_nu_ctx* ctx, int fused) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step keeps its kernels
  c->tune.inv_xy = fused != 0 ? 1 : 0;
  return PM_NU_OK;
}

int pm_nu_set_inverse_yz(pm_nu_ctx* ctx, int fused) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step keeps its kernels
  c->tune.inv_yz = fused != 0 ? 1 : 0;
  return PM_NU_OK;
}

int pm_nu_set_forward_zy(pm_nu_ctx* ctx, int fused) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step keeps its kernels
  c->tune.fwd_zy = fused != 0 ? 1 : 0;
  return PM_NU_OK;
}

int pm_nu_set_keep_density(pm_nu_ctx* ctx, int on) {
  GET_CTX(ctx);
  drop_graph(*c);   // a captured step keeps its kernel arguments
  c->keep_density = on != 0;
  return PM_NU_OK;
}

int pm_nu_copy_modes(pm_nu_ctx* ctx, int box, float* out) {
  GET_CTX(ctx);
  if (box < 0 || box >= c->nbox || !out) return set_error(PM_NU_EINVAL, "bad box/out");
  if (c->stage < 1) return set_error(PM_NU_ESTATE, "modes are valid after pm_nu_deposit");
  // the step keeps the field before its x transform (the inverse pass redoes it): transform
  // a copy along x here and read the modes from it
  const size_t bytes = static_cast<size_t>(c->nbox) * c->MH * sizeof(float2);
  PMNU_HIP(hipMemcpyAsync(c->ck[2], c->ck[0], bytes, hipMemcpyDeviceToDevice, c->stream));
  hipError_t e = launch_fwd_x_bin(c->N, c->ck[2], c->tw, c->bin_of_n2, nullptr, c->B, c->nbox,
                                  c->stream);
  if (e == hipSuccess)
    e = launch_copy_modes(c->N, c->ck[2], reinterpret_cast<float2*>(out), box, c->stream);
  if (e != hipSuccess) return set_error(PM_NU_EHIP, "copy_modes: %s", hipGetErrorString(e));
  return PM_NU_OK;
}

int pm_nu_copy_force_grid(pm_nu_ctx* ctx, int box, int axis, float* out) {
  GET_CTX(ctx);
  if (box < 0 || box >= c->nbox || axis < 0 || axis > 2 || !out)
    return set_error(PM_NU_EINVAL, "bad box/axis/out");
  hipError_t e = launch_extract_component(c->force + static_cast<size_t>(box) * c->M * 3, out,
                                          c->M, axis, c->stream);
  if (e != hipSuccess) return set_error(PM_NU_EHIP, "copy_force_grid: %s", hipGetErrorString(e));
  return PM_NU_OK;
}

int pm_nu_set_timing(pm_nu_ctx* ctx, int enable) {
  GET_CTX(ctx);
  c->timer.enabled = enable != 0;
  c->timer.mask = ~0u;
  return PM_NU_OK;
}

int pm_nu_set_timing_mask(pm_nu_ctx* ctx, uint32_t stage_mask) {
  GET_CTX(ctx);
  c->timer.enabled = stage_mask != 0;
  c->timer.mask = stage_mask;
  return PM_NU_OK;
}

int pm_nu_read_timing(pm_nu_ctx* ctx, int* n_stages, const char** names, double* total_ms,
                      int64_t* launches) {
  GET_CTX(ctx);
  if (!n_stages) return set_error(PM_NU_EINVAL, "n_stages is NULL");
  Timer& t = c->timer;
  std::vector<double> ms(ST_COUNT, 0.0);
  std::vector<int64_t> cnt(ST_COUNT, 0);
  if (t.used > 0) {
    PMNU_HIP(hipEventSynchronize(t.pool[2 * t.used - 1]));
    for (size_t i = 0; i < t.used; ++i) {
      float v = 0.f;
      PMNU_HIP(hipEventElapsedTime(&v, t.pool[2 * i], t.pool[2 * i + 1]));
      ms[t.stage_of[i]] += v;
      cnt[t.stage_of[i]] += 1;
    }
  }
  t.used = 0;
  const int cap = *n_stages;
  const int n = std::min<int>(cap, ST_COUNT);
  for (int i = 0; i < n; ++i) {
    if (names) names[i] = kStageNames[i];
    if (total_ms) total_ms[i] = ms[i];
    if (launches) launches[i] = cnt[i];
  }
  *n_stages = n;
  return PM_NU_OK;
}

int pm_nu_graph_capture(pm_nu_ctx* ctx, const float* pos, float* acc, double a_now) {
  GET_CTX(ctx);
  if (!c->stream) return set_error(PM_NU_EINVAL, "graph capture needs a non-null stream");
  if (c->cfg.response_mode == 2)
    return set_error(PM_NU_EINVAL, "the surrogate check mode cannot be captured");
  int rc = prepare_time_grid(*c, a_now);
  if (rc) return rc;
  // run one step eagerly so that the node a_now exists and later replays recompute it
  rc = pm_nu_step(ctx, pos, acc, a_now);
  if (rc) return rc;
  rc = prepare_time_grid(*c, a_now);
  if (rc) return rc;
  PMNU_HIP(hipStreamSynchronize(c->stream));
  if (c->graph_exec) {
    hipGraphExecDestroy(c->graph_exec);
    c->graph_exec = nullptr;
  }
  if (c->graph) {
    hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
  PMNU_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  rc = pm_nu_step(ctx, pos, acc, a_now);
  c->capturing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (rc) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return set_error(PM_NU_EHIP, "end capture: %s", hipGetErrorString(e));
  c->graph = g;
  PMNU_HIP(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
  c->graph_a = a_now;
  return PM_NU_OK;
}

int pm_nu_graph_launch(pm_nu_ctx* ctx) {
  GET_CTX(ctx);
  if (!c->graph_exec)
    return set_error(PM_NU_ESTATE,
                     "no captured graph (none captured, or a setting changed since capture)");
  PMNU_HIP(hipGraphLaunch(c->graph_exec, c->stream));
  return PM_NU_OK;
}

}  // extern "C"
