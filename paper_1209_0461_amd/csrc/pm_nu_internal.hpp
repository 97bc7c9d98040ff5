// Internal interfaces of the pm_nu library: the context and the host-side launchers of
// every kernel. Only the C ABI in include/pm_nu.h is exported.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pm_nu.h"
#include "host_consts.hpp"
#include "surrogate_layout.hpp"

namespace pmnu {

// Per-box constants of the response kernel (device copy, one per box).

struct RespBox {
  double f_nu;       // Omega_nu / Omega_M
  double t_over_m;   // T_nu0 / m of the first massive species (0 without neutrinos)
  double w_sp[kMaxSpecies];    // m_s / M_nu of each massive species (equal masses: one, w = 1)
  double tm_sp[kMaxSpecies];   // T_nu0 / m_s
  int n_sp;          // massive species with distinct masses (0 without neutrinos)
  int sur_ok;        // three equal masses: the setting the surrogate network was trained on
  double ds_ic;      // s(a_now) - s(a_i)
  double a_i;        // scale factor of node 0
  double kfs;        // free-streaming wavenumber k_fs(a_now) [h/Mpc] (0 without neutrinos)
  double m_total;    // total neutrino mass [eV]
  double a_now;      // scale factor of the current step
  int nq;            // sub-nodes of the quadrature (current step included)
  int n_cur;         // history row of the current step
  int series;        // 1: exact series for I(x), 0: the fit eq. (fit)
  // the surrogate's history samples (surrogate_layout.hpp): lag m reads the stored nodes
  // sur_j[m] and sur_j[m] + 1 with weights 1 - sur_t[m] and sur_t[m] (sur_t = 0: node
  // sur_j alone); sur_hist = 0 when the history does not reach back far enough
  int sur_hist;
  int sur_j[kSurLags];
  double sur_t[kSurLags];
  double sur_gap;    // ln a_now - ln a_{n-1}
  double sur_ds_last;  // s(a_now) - s(a_{n-1})
  double sur_lna;      // ln a_now
  double sur_lna0;     // ln(a_now / a_0)
  double sur_lnx0;     // ln((s(a_now) - s(a_{n-1})) T_nu0 / m): input 6 is ln k + sur_lnx0
};

// A coordinate moved back into [0, L) (exact: fmodf; x + L may round up to L, which wraps to 0).
__device__ __forceinline__ float wrap_box(float x, float L) {
  if (x >= 0.f && x < L) return x;
  x = fmodf(x, L);
  if (x < 0.f) x += L;
  return x < L ? x : 0.f;
}

// What the interpolation does with each particle's acceleration: store it (a step), or also
// apply the leapfrog of pm_nu_advance on the spot, u += K_b acc and, between steps,
// x += D_b u wrapped into [0, L) (positions updated in place).
struct Leap {
  float* vel = nullptr;          // null: store the acceleration only
  float* pos = nullptr;          // null: no drift
  const double* kd = nullptr;    // [nbox][2] K_b, D_b
  float box = 0.f;
  int store_acc = 1;
};

// Launch shapes chosen by the autotuner (defaults are safe for every N).
struct Tuning {
  int deposit_mode = 4;      // see launch_deposit
  int deposit_block = 256;   // block size of mode 0
  int interp_mode = 1;       // see launch_interp
  int interp_block = 256;    // block size of mode 0
  // tile candidate (0 default, 1, 2) of each FFT pass: fwd_z, fwd_y, fwd_x, inv_x, inv_y,
  // inv_z (fft_tile gives the tile); the same result for every candidate
  int fft[6] = {0, 0, 0, 0, 0, 0};
  // N <= 64: the last two inverse passes as one kernel (inv_yz, after inv_x), else the first
  // two (inv_xy, before inv_z) when inv_xy is set; 0 and 0: three passes
  int inv_yz = 1;
  int inv_xy = 1;
  // N <= 128: the first two forward passes as one kernel (fwd_zy); 0: as two
  int fwd_zy = 1;
};

struct Timer {
  bool enabled = false;
  unsigned mask = ~0u;            // stages that get an event pair (bit = Stage)
  bool open = false;              // an event pair was begun and not yet ended
  std::vector<hipEvent_t> pool;   // events recorded since the last read
  std::vector<int> stage_of;      // stage of each event pair
  size_t used = 0;                // pairs in use
};

enum Stage {
  ST_ZERO = 0, ST_DEPOSIT, ST_FFT_Z, ST_FFT_Y, ST_FFT_X_BIN, ST_RESPONSE, ST_INV_X_GREEN, ST_INV_Y, ST_INV_Z, ST_INTERP, ST_SURROGATE, ST_PATCH_REDUCE, ST_KICK_DRIFT,
  ST_PATCH_FWD_Z, ST_INV_XY, ST_FWD_ZY, ST_INV_YZ, ST_COUNT
};
extern const char* const kStageNames[ST_COUNT];

struct Surrogate;  // defined in surrogate.cpp

// Where |n|^2 falls among the non-empty bins, packed in 32 bits: bits 0..9 the bin lo of
// the lower bracketing mean, bits 10..31 the weight t of the next non-empty bin in units of
// 2^-22, so that R(|k|) = R[lo] + t (R[next(lo)] - R[lo]) (t = 0 below the first and above
// the last bin mean, and at n^2 = 0). Fixed by the geometry; the first inverse pass forms
// the step's T(n^2) from it.
constexpr int kRatioBinBits = 10;                 // kMaxBins = 2^10
constexpr double kRatioUnit = 1.0 / 4194304.0;    // 2^-22

// Per box: the quadrature sub-nodes of the intervals between stored history nodes (they do
// not change as the history grows, only the interval to the current step does).
struct TgCache {
  std::vector<double> nodes;            // the stored nodes they were built from
  std::vector<double> a, seg, hinv;     // per sub-node: a, s to the next sub-node, 1/(a H)
  int64_t bg_version = -1;              // Ctx::bg_version they were built with
};

struct Ctx {
  pm_nu_config cfg{};
  int N = 0, NK = 0, nbox = 0, B = 0, Jcap = 0, Q = 0;
  int64_t Np = 0, M = 0, MH = 0;   // particles per box, N^3, (N/2+1) N^2
  int n2max = 0;                   // 3 N^2 / 4
  int qcap = 0;                    // sub-node capacity per box
  int n_partial = 0;               // per-box partial bin sums (of the binning pass's tile)
  int n_partial_cap = 0;           // the most any tile candidate writes (buffer size)
  hipStream_t stream = nullptr;
  int device = 0;

  std::vector<double> m_nu, f_nu, t_over_m;
  std::vector<std::vector<double>> species;   // per box: masses of the massive species [eV]
                                              // (the default equal masses: one entry)
  std::vector<int> nu_mult;        // per box: how many species share each entry of species
  std::vector<int> nu_massless;    // per box: massless species (radiation in the background)
  bool relativistic = false;       // background with radiation and eq. (relativistic)
  bool series = false;             // exact I(x) series instead of the fit
  std::vector<int> sur_setting;    // per box: n_species = 3 equal masses (the network's)
  std::vector<std::vector<double>> ic_base;   // per box: the initial amplitude of set_history
  std::vector<int64_t> edges;      // [B+1]
  std::vector<double> counts, kmean;
  std::vector<int> nonempty;       // bins with counts > 0

  // device buffers
  unsigned long long* rho = nullptr;   // [nbox][M] deposit, fixed point (unit 2^-40)
  // complex fields, (N/2+1) N^2 each per box: ck[0] holds the field transformed along z
  // and y, [kz][x][ky], from the forward passes to the first inverse pass (which applies
  // the x transform itself); the others hold intermediates
  float2* ck[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  float* force = nullptr;          // [nbox][M][3] accelerations, components interleaved
  double* bin_partial = nullptr;   // [nbox][n_partial][B]
  uint16_t* bin_of_n2 = nullptr;   // [n2max+1]
  double* d_counts = nullptr;      // [B]
  double* d_kmean = nullptr;       // [B]
  double* d_lnk = nullptr;         // [B] ln of the bin means (0 for empty bins)
  int* d_nonempty = nullptr;       // [B]
  double* pcdm = nullptr;          // [nbox][B]
  double* pnu = nullptr;           // [nbox][B]
  double* ratio = nullptr;         // [nbox][B]
  double* hist_pm = nullptr;       // [nbox][Jcap][B]
  double* hist_pnu = nullptr;      // [nbox][Jcap][B]
  double* ic_pnu = nullptr;        // [nbox][kMaxSpecies][B] per massive species
  double* ic_theta = nullptr;      // [nbox][B]
  double* tg_ds = nullptr;         // [nbox][qcap]
  double* tg_l2 = nullptr;         // [nbox][qcap] log2 of tg_ds (the fit's x^0.1811)
  double* tg_w = nullptr;          // [nbox][qcap]
  RespBox* d_resp = nullptr;       // [nbox]
  uint32_t* ridx = nullptr;        // [n2max+1] packed bin and weight of |n|^2
  int* d_next = nullptr;           // [B] next non-empty bin after each non-empty bin (or itself)
  float2* tw = nullptr;            // [N] exp(-2 pi i m/N)
  float* inv_w2 = nullptr;         // [N] 1/sinc^4(pi n/N) per axis index (or 1)
  int* d_flags = nullptr;          // [1] bit 0: non-finite position seen
  // patch deposit (deposit modes 6 and 7)
  unsigned long long* patches = nullptr;   // [chunks][kPatchCap] per-chunk tiles
  int* reg_count = nullptr;        // [nbox][coarse cells] patches registered
  int4* reg_list = nullptr;        // [nbox][coarse cells][32] (chunk, origin, extents, 0)
  unsigned long long* rho_fb = nullptr;    // [nbox][M] side grid, kept at zero
  int* n_fb = nullptr;             // [2] chunks that used the side grid this deposit; running
                                   // total of earlier deposits (added by the first FFT pass)
  unsigned fb_seen = 0;            // running total at the last pm_nu_side_grid_uses
  float* delta = nullptr;          // [nbox][M] delta in FP32 (modes 6, 7)
  double* d_kd = nullptr;          // [nbox][2] kick and drift factors of the leapfrog
  // pinned staging of the host-built arrays (copied in stream order) and the last copies
  double* h_tg = nullptr;          // ds [nbox][qcap], then w, then log2 ds
  RespBox* h_resp = nullptr;       // [nbox]
  double* h_kd = nullptr;          // [nbox][2]
  hipEvent_t ev_tg = nullptr, ev_kd = nullptr;
  bool density_is_delta = false;   // the last deposit wrote delta (modes 6..9), not rho
  bool keep_density = false;       // modes 8, 9: also store delta (pm_nu_set_keep_density)
  bool density_kept = false;       // the last deposit left a readable density

  // host state
  std::vector<std::vector<double>> hist_a;   // committed node scale factors per box
  std::vector<int> has_ic;
  int stage = 0;                   // 0: idle, 1: deposited, 2: responded
  bool modes_valid = false;        // the modes come from a deposit (not pm_nu_set_power)
  double a_resp = 0.0;
  const float* pos_dep = nullptr;
  // time-grid cache: valid for (a_now, history version)
  double tg_a_now = -1.0;
  std::vector<TgCache> tgc;        // per box
  int64_t bg_version = 0;          // bumped whenever H(a) of a box may change
  int64_t hist_version = 0, tg_version = -1;
  std::vector<int> n_cur;          // row of the current step per box (valid after prepare)

  Tuning tune;
  Timer timer;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  double graph_a = -1.0;           // a_now of the captured step
  bool capturing = false;

  Surrogate* sur = nullptr;
};

// ---- error helpers (host.cpp) -------------------------------------------------------
int set_error(int code, const char* fmt, ...);
#define PMNU_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::pmnu::set_error(PM_NU_EHIP, "%s failed: %s (%s:%d)", #call,              \
                               hipGetErrorString(e_), __FILE__, __LINE__);              \
  } while (0)

// Event-bracketed launch helpers (host.cpp)
void timer_begin(Ctx& c, int stage);
void timer_end(Ctx& c);
// Discard a captured step graph (after any change that the captured launches would miss).
void drop_graph(Ctx& c);
// Response at a_now with the exact integral (mode 0) or the surrogate (modes 1, 2).
int do_response_mode(Ctx& c, double a_now, int mode);
// surrogate.cpp: the kernel launch of the surrogate response (modes 1, 2)
int surrogate_launch(Ctx& c, int mode, double norm);
void surrogate_free(Ctx& c);

// ---- kernel launchers (each returns hipGetLastError() of its launch) -----------------
// grid_kernels.hip
constexpr double kFixScale = 1099511627776.0;   // 2^40: fixed-point unit of the deposit
constexpr int kMaxBins = 1024;                   // largest n_kbins
static_assert(kMaxBins <= (1 << kRatioBinBits), "bin index of the packed ratio index");
// patch deposit (deposit mode 6): chunk of particles, LDS tile / patch capacity in nodes,
// threads per workgroup
// patch deposit: chunks of kPatchCH particles on kPatchNT threads; the LDS tile holds
// kPatchTile nodes (mode 6, three workgroups per CU) or kPatchCap (mode 7, room for larger
// boxes); a stored patch has room for kPatchCap nodes
constexpr int kPatchCH = 4096, kPatchCap = 9216, kPatchTile = 6144, kPatchNT = 512;
hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s);
hipError_t launch_fixed_to_float(const unsigned long long* src, float* dst, int64_t n,
                                 hipStream_t s);
hipError_t launch_extract_component(const float* src, float* dst, int64_t n, int comp,
                                   hipStream_t s);
// mode 0: one thread per particle, 8 global atomics each; modes 1-3: LDS-privatised
// chunks of 1024 / 2048 / 4096 particles (global atomics for chunks that do not fit)
// modes 0-5 (modes 6 and 7 are the patch deposit, launched by launch_deposit_patch)
hipError_t launch_deposit(const float* pos, unsigned long long* rho, int64_t np, int nbox, int N,
                          double inv_cell, int* flags, int mode, int block, hipStream_t s);
// mode 0: one thread per particle gathering from HBM; modes 1-3: chunks of 1024 / 2048 /
// 4096 particles with their bounding-box tile of the acceleration grid staged in LDS; lp
// (may be NULL) applies the leapfrog of pm_nu_advance with each acceleration
hipError_t launch_interp(const float* pos, const float* force, float* acc, int64_t np,
                         int nbox, int N, double inv_cell, int mode, int block, hipStream_t s,
                         const Leap* lp = nullptr);
// fft_kernels.hip
// input: the fixed-point density rho, or (if delta is not NULL) delta in FP32; reset[0] (may
// be NULL) is added to reset[1] and cleared by the kernel when reading delta, and the n_clear
// ints at clear are cleared
// (NULL: none); a clear larger than the launch's thread count is rejected
hipError_t launch_fwd_z(int N, const unsigned long long* rho, const float* delta, int* reset,
                        int* clear, int n_clear, float2* out, const float2* tw, double scale,
                        int nbox, hipStream_t s, int v = 0);
// reset, clear, n_clear: the patch registry's end-of-step work after launch_patch_fwd_z
hipError_t launch_fwd_y(int N, const float2* in, float2* out, const float2* tw, int nbox,
                        hipStream_t s, int v = 0, int* reset = nullptr, int* clear = nullptr,
                        int n_clear = 0);
// N <= 128: fwd_z and fwd_y in one kernel (rho or delta in as for launch_fwd_z; out: the
// y-transformed modes fwd_y would write)
hipError_t launch_fwd_zy(int N, const unsigned long long* rho, const float* delta, int* reset,
                         int* clear, int n_clear, float2* out, const float2* tw, double scale,
                         int nbox, hipStream_t s);
// the patch sums and the first (z) forward pass in one kernel (N >= 32); delta_out, when
// given, also receives delta
hipError_t launch_patch_fwd_z(int n, const unsigned long long* patches, const int* reg_count,
                              const int4* reg_list, unsigned long long* rho_fb, const int* n_fb,
                              float2* out, const float2* tw, double scale, int nbox,
                              hipStream_t s, float* delta_out);
// partial != NULL: FFT along x and the mode sums per bin, data left unchanged (the step);
// partial == NULL: FFT along x stored in place, no sums (reading the modes out)
hipError_t launch_fwd_x_bin(int N, float2* data, const float2* tw, const uint16_t* bin_of_n2,
                            double* partial, int B, int nbox, hipStream_t s, int v = 0);
// partial bin sums per box written by launch_fwd_x_bin with tile candidate v
int fwd_x_partials(int N, int v = 0);
// tile of FFT pass `pass` (0 fwd_z rows, 1 fwd_y lines, 2 fwd_x columns, 3 inv_x columns,
// 4 inv_y lines, 5 inv_z rows) for candidate v (0 default, 1, 2); 0 for a bad N or pass
int fft_tile(int N, int pass, int v);
// T(n^2) = (1 - f_nu) + f_nu R from ridx and next, the per-bin R ([nbox][nbins]) and the
// boxes' f_nu
hipError_t launch_inv_x(int N, const float2* dk, float2* f1, float2* f2, const float2* tw,
                        const uint32_t* ridx, const int* next, const double* ratio,
                        const RespBox* boxes, int nbins, const float* inv_w2, float cfac,
                        float kf, int nbox, hipStream_t s, int v = 0);
hipError_t launch_inv_y(int N, const float2* f1, const float2* f2, float2* g1, float2* g2,
                        float2* g3, const float2* tw, float kf, int nbox, hipStream_t s,
                        int v = 0);
// N <= 64: inv_x and inv_y in one kernel (g1 must not be dk: the layouts differ)
hipError_t launch_inv_xy(int N, const float2* dk, float2* g1, float2* g2, float2* g3,
                         const float2* tw, const uint32_t* ridx, const int* next,
                         const double* ratio, const RespBox* boxes, int nbins,
                         const float* inv_w2, float cgreen, float kf, int nbox, hipStream_t s);
// N <= 64: inv_y and inv_z in one kernel (f1, f2 as inv_x writes them)
hipError_t launch_inv_yz(int N, const float2* f1, const float2* f2, float* out, const float2* tw,
                         float kf, int nbox, hipStream_t s);
hipError_t launch_inv_z(int N, const float2* g1, const float2* g2, const float2* g3,
                        float* out, const float2* tw, float kf, int nbox, hipStream_t s,
                        int v = 0);
hipError_t launch_copy_modes(int N, const float2* ck, float2* out, int box, hipStream_t s);
// response_kernels.hip
hipError_t launch_response(const RespBox* boxes, const double* partial, int n_partial,
                           const double* counts, const double* kmean, const double* hist_pm,
                           const double* hist_pnu, const double* ic_pnu,
                           const double* ic_theta, const double* tg_ds, const double* tg_l2,
                           const double* tg_w, int B, int Jcap, int qcap, int Q, int iterations,
                           double norm,
                           int nbox, double* pcdm, double* pnu, double* ratio,
                           hipStream_t s, int threads, bool series, bool hierarchy);
// threads per workgroup of the exact response for this many (bin, box) pairs: 64 or 256
int response_threads(int nbins, int nbox);
// mlp_kernels.hip
hipError_t launch_mlp_train(const float* P, const float* x, const float* y, const int* perm,
                            int64_t row0, int64_t count, float inv_batch, float* grad,
                            float* loss_sum, hipStream_t s);
hipError_t launch_mlp_predict(const float* P, const float* x, float* y, int64_t n, hipStream_t s);
hipError_t launch_adam(float* P, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_pack_weights(const float* P, unsigned short* Q, hipStream_t s);
int64_t packed_weight_count();
hipError_t launch_surrogate_response(const float* P, const unsigned short* Q, int mode,
                                     const RespBox* boxes, const double* partial, int n_partial,
                                     const double* counts, const double* kmean, double* hist_pm,
                                     double* hist_pnu, const double* ic_pnu,
                                     const double* ic_theta, const double* tg_ds,
                                     const double* tg_l2, const double* tg_w, int nbins, int jcap,
                                     int qcap, int q_sub, int iterations, double norm, int nbox,
                                     double* pcdm, double* pnu, double* ratio, double* sur_r,
                                     double* chk_exact, double* chk_sur, hipStream_t s);
hipError_t launch_surrogate_dataset(const RespBox* boxes, const double* pcdm, const double* ratio,
                                    const double* kmean, const double* hist_pm,
                                    const double* hist_pnu, int nbins, int jcap, int nbox,
                                    float* x, float* y, hipStream_t s);
int patch_cb_log2(int n);
int64_t patch_coarse_cells(int n);
int64_t patch_chunks(int64_t np);
// big_tile: the kPatchCap-node LDS tile (mode 7) instead of kPatchTile (mode 6); reg_list
// entries are (chunk, packed box origin, packed extents, 0), n <= 1024
hipError_t launch_deposit_patch(const float* pos, unsigned long long* patches, int* reg_count,
                                int4* reg_list, unsigned long long* rho_fb, int* n_fb,
                                int64_t np, int nbox, int n, double inv_cell, int* flags,
                                bool big_tile, hipStream_t s);
hipError_t launch_patch_reduce(const unsigned long long* patches, const int* reg_count,
                               const int4* reg_list, unsigned long long* rho_fb,
                               const int* n_fb, float* delta, int nbox, int n, double scale,
                               hipStream_t s);
hipError_t launch_delta_to_density(const float* delta, float* out, int64_t n, float rho_bar,
                                   hipStream_t s);
hipError_t launch_kick_drift(float* pos, float* vel, const float* acc, const double* kd,
                             int64_t n_particles, int nbox, float box, bool drift,
                             hipStream_t s);
hipError_t launch_kernel_values(const double* x, int64_t n, int series, double* out,
                                hipStream_t s);
hipError_t launch_bin_power(const double* partial, int n_partial, const double* counts,
                            int nbins, double norm, int nbox, double* pcdm, hipStream_t s);
hipError_t launch_ratio_index(const double* lnk, const int* nonempty, int n_nonempty,
                              int n2max, double kf, uint32_t* out, hipStream_t s);

}  // namespace pmnu
