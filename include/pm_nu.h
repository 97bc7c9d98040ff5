/* pm_nu.h -- C ABI of the MI355X (gfx950) particle-mesh gravity step with the massive-
 * neutrino density added by linear response (Ali-Haimoud & Bird, arXiv:1209.0461).
 *
 * The step follows the loop of the paper's Sec. 4.3 (ii)-(iv):
 *   pm_nu_deposit   CDM density by cloud-in-cell, forward FFT, binned P_cdm(k)     (ii)
 *   pm_nu_response  P_nu^{1/2}(k, a) from the history integral eq. (P-final),
 *                   the ratio R(k) = (P_nu/P_cdm)^{1/2} (eq. (phases)) and the new
 *                   total-matter amplitude appended to the history                 (iii)
 *   pm_nu_force     delta_M = [(1 - f_nu) + f_nu R(|k|)] delta_cdm (Sec. 4.3 (iv)),
 *                   Poisson's equation eq. (Poisson), spectral gradient, inverse FFT
 *                   and cloud-in-cell interpolation of the acceleration             (iv)
 *
 * Conventions
 *   Units: c = 1, lengths in Mpc/h, wavenumbers in h/Mpc, H0 = 1/2997.92458 h/Mpc.
 *   Positions: FP32 array [n_boxes][n_particles][3]; component 0 is mesh axis 0 (the
 *     slowest index of a C-order N^3 grid). Values outside [0, L) are wrapped.
 *   Accelerations: FP32 [n_boxes][n_particles][3], acc = -grad(phi) with
 *     k^2 phi = -(3/2) H0^2 Omega_M delta_M / a  (units h/Mpc with c = 1).
 *   Pointers marked (dev) are device pointers owned by the caller; pointers marked
 *     (host) are host memory owned by the caller. The library owns all other memory.
 *   Work is enqueued on cfg.stream and runs asynchronously unless marked (sync).
 *   Every int-returning call returns PM_NU_OK (0) or a negative PM_NU_E* code; the
 *     message of the last failure on the calling thread is pm_nu_last_error().
 *   Per step the calls must come in the order deposit -> response -> force
 *     (pm_nu_step does all three); any other order returns PM_NU_ESTATE.
 *   Mesh sizes: powers of two from 8 to 512.
 */
#ifndef PM_NU_H
#define PM_NU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PM_NU_OK = 0,
  PM_NU_EINVAL = -1,      /* bad argument or configuration                          */
  PM_NU_ENOMEM = -2,      /* device or host allocation failed                        */
  PM_NU_EHIP = -3,        /* a HIP runtime call failed                               */
  PM_NU_ESTATE = -4,      /* call order violated (e.g. force before response)        */
  PM_NU_EHISTORY = -5,    /* history missing, not increasing in a, or full           */
  PM_NU_ENODEV = -6,      /* no usable gfx950 device                                 */
  PM_NU_ESURROGATE = -7,  /* surrogate requested but not loaded / input out of range */
  PM_NU_ENONFINITE = -8   /* a non-finite particle position was seen by the deposit  */
};

typedef struct pm_nu_ctx pm_nu_ctx;

typedef struct {
  int32_t n_mesh;          /* N: mesh points per side, power of two in [8, 512]         */
  int32_t n_boxes;         /* independent boxes sharing N, L, bins (>= 1)                */
  int64_t n_particles;     /* CDM particles per box (>= 1)                               */
  double box_size;         /* L [Mpc/h]                                                  */
  double omega_m;          /* Omega_M today, neutrinos included                          */
  double hubble;           /* h                                                          */
  int32_t n_kbins;         /* B: log-spaced bins over [2 pi/L, sqrt(3) pi N/L], 1..1024  */
  int32_t max_history;     /* history capacity in nodes per box, current step included   */
  int32_t substeps;        /* Q: quadrature steps per history interval (>= 1)            */
  int32_t iterations;      /* iterations of the implicit equation (Sec. 4.3 (iii)), >= 1 */
  int32_t deconvolve;      /* 1: divide the Green's function by the CIC window squared  */
  int32_t response_mode;   /* 0: exact integral; 1: surrogate network; 2: surrogate with
                              the exact integral run beside it as a check                */
  int32_t n_species;       /* degenerate neutrino species sharing the total mass (3)    */
  void* stream;            /* hipStream_t for all work; NULL = the null stream           */
} pm_nu_config;

/* Fill *cfg with defaults: N = 32, one box, 32768 particles, L = 128, Omega_M = 0.3,
 * h = 0.7, 32 bins, 256 history nodes, Q = 8, 1 iteration, deconvolution on, exact
 * response, 3 species, null stream. */
void pm_nu_default_config(pm_nu_config* cfg);

/* Create a context on the current HIP device. m_nu_total (host) [n_boxes]: total
 * neutrino mass per box in eV (0 allowed: plain CDM). Allocates every buffer the step
 * needs; later calls allocate nothing on the device (sync). */
int pm_nu_init(const pm_nu_config* cfg, const double* m_nu_total, pm_nu_ctx** out);

/* Release everything owned by ctx (sync). NULL is ignored. */
void pm_nu_destroy(pm_nu_ctx* ctx);

/* Thread-local text of the last error (never NULL). */
const char* pm_nu_last_error(void);

/* Bin geometry (host, sync): integer |n|^2 edges [B+1] (mode n is in bin b when
 * edge[b] <= |n|^2 < edge[b+1], the top bin also takes |n|^2 = 3N^2/4), mode counts
 * [B] (full-sphere counts) and mean |k| [B] in h/Mpc. Any pointer may be NULL. */
int pm_nu_get_bins(pm_nu_ctx* ctx, int64_t* edge_n2, double* mode_count, double* k_mean);

/* Load the stored history of one box (sync). Nodes j = 0..n_nodes-1 at strictly
 * increasing scale factors a (host) [n]; node 0 is the initial time a_i.
 *   pm_half  (host) [n][B]: P_M^{1/2}(k_b, a_j), the stored total-matter amplitudes
 *   pnu_half (host) [n][B]: P_nu^{1/2}(k_b, a_j) (the last row seeds the first iteration)
 *   pnu_half_init (host) [B]: P_nu^{1/2}(k_b, a_i) of the initial-condition term
 *   theta_over_delta_init (host) [B]: [theta_nu/delta_nu]_i(k_b) in h/Mpc
 * (eq. (P-final), eq. (deltaI-nu)). Replaces any previous history of the box. */
int pm_nu_set_history(pm_nu_ctx* ctx, int box, int n_nodes, const double* a,
                      const double* pm_half, const double* pnu_half,
                      const double* pnu_half_init, const double* theta_over_delta_init);

/* Read the history of one box (sync): *n_nodes, a [n], pm_half [n][B], pnu_half [n][B]
 * (caller sizes the arrays with max_history; any array pointer may be NULL). */
int pm_nu_get_history(pm_nu_ctx* ctx, int box, int* n_nodes, double* a, double* pm_half,
                      double* pnu_half);

/* Stage (ii): CIC mass of every particle (unit mass), delta = rho/rho_bar - 1, forward
 * real FFT and the binned power P_cdm(k_b) = (L^3/N^6) sum_b w |delta_k|^2 / C_b with
 * FP64 sums. pos (dev) [n_boxes][n_particles][3]. */
int pm_nu_deposit(pm_nu_ctx* ctx, const float* pos);

/* Stage (iii) at scale factor a_now, which must not precede the last stored node.
 * Evaluates eq. (P-final) in FP64 by the trapezoid rule in ln a (Q steps per history
 * interval, P_M^{1/2} linear in ln a between nodes, dtau = dln a/(a H), H(a) of
 * pm_nu_set_background), using P_nu(a_now) ~ P_nu(previous node) inside the integral for
 * the first iteration (Sec. 4.3 (iii), Appendix B). Writes P_nu^{1/2}, R_b and appends the
 * node a_now with P_M^{1/2} = (1-f_nu) P_cdm^{1/2} + f_nu P_nu^{1/2}; if a_now equals
 * the last stored node that node is recomputed from the ones before it instead (when it is
 * the only node, a_now = a_i and P_nu^{1/2} is the initial amplitude: the start of a run). A box
 * with m_nu_total = 0 has f_nu = 0: its P_nu^{1/2} and R read 0 and the step is plain CDM.
 * Needs pm_nu_deposit first. */
int pm_nu_response(pm_nu_ctx* ctx, double a_now);

/* Stage (iv): rescale the modes by (1 - f_nu) + f_nu R(|k|) (R linear in ln k between
 * non-empty bin means, held outside), phi = -(3/2) H0^2 Omega_M delta_M /(a k^2 W^2)
 * (W = prod sinc^2(pi n_a/N) when deconvolve), g_a = -i k_a phi (zero on the Nyquist
 * index of axis a), inverse FFT, CIC interpolation into acc (dev)
 * [n_boxes][n_particles][3]. pos must be the array given to the deposit. a_now must
 * equal the one given to pm_nu_response. */
int pm_nu_force(pm_nu_ctx* ctx, const float* pos, float* acc, double a_now);

/* deposit + response + force. */
int pm_nu_step(pm_nu_ctx* ctx, const float* pos, float* acc, double a_now);

/* Per-box spectra of the last step (host, sync), each [B], any may be NULL:
 * P_cdm(k_b) [(Mpc/h)^3], P_nu^{1/2}(k_b), R_b = P_nu^{1/2}/P_cdm^{1/2}. Empty bins
 * read 0; R_b reads 0 in a bin whose P_cdm is 0 (no CDM mode to carry the neutrino
 * phase, eq. (phases)). Returns PM_NU_ENONFINITE if the last deposit saw a non-finite position. */
int pm_nu_get_spectrum(pm_nu_ctx* ctx, int box, double* p_cdm, double* pnu_half,
                       double* ratio);

/* ---- stage (ii) without allocation ------------------------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the binned power of one box, as pm_nu_deposit
 * followed by pm_nu_get_spectrum's p_cdm, with no context. The CIC mass of every particle
 * (unit mass), delta = rho/rho_bar - 1, the forward real FFT and
 * P_cdm(k_b) = (L^3/N^6) sum_b w |delta_k|^2 / C_b (FP64 sums) over the bins of
 * pm_nu_get_bins for this N, L and B.
 *   pos (dev) [n_particles][3] FP32 positions (wrapped into [0, L)); p_cdm (dev) [n_kbins]
 *   FP64 output; stream: hipStream_t (NULL: the null stream). Asynchronous on the stream.
 * Every intermediate lives in one static device array of 5 MiB per device, held until the
 * process ends, which limits n_mesh to powers of two from 8 to 64 and n_kbins to 1..256.
 * It allocates nothing, on the device or the host. Calls on one device share that array:
 * calls that overlap on one device (several streams or threads) race. A non-finite
 * position is skipped, not reported. Errors: PM_NU_EINVAL for sizes beyond those limits or
 * bad arguments, PM_NU_EHIP if a launch fails. */
int pm_nu_binned_power_noalloc(const float* pos, int64_t n_particles, int n_mesh,
                               double box_size, int n_kbins, double* p_cdm, void* stream);

/* ---- diagnostics (copies of internal state, enqueued on the stream) ---------------- */
/* (sync) How many chunk parts the patch deposit (deposit modes 6..9) has sent through its
 * atomic side grid since the last call (a chunk whose bounding box exceeds the LDS tile,
 * or its part in a coarse cell whose patch list was full); 0 when every chunk went
 * through its patch, and always 0 for the other deposit modes. */
int pm_nu_side_grid_uses(pm_nu_ctx* ctx, int64_t* uses);
/* Deposited mass rho (unit mass per particle) of one box into out (dev) [N][N][N].
 * Deposit modes 8 and 9 never write the density to HBM unless asked to by
 * pm_nu_set_keep_density before the deposit; otherwise PM_NU_ESTATE. */
int pm_nu_copy_density(pm_nu_ctx* ctx, int box, float* out);
/* For N <= 64 the first two inverse FFT passes (Green's function, x and y) can run as one
 * kernel per k_z slab, whose modes fit the LDS (fused != 0, the default), when the last two
 * are not fused (pm_nu_set_inverse_yz, which takes precedence); 0 runs them as the two passes
 * that larger meshes use. Every choice gives the same forces bit for bit. */
int pm_nu_set_inverse_xy(pm_nu_ctx* ctx, int fused);
/* For N <= 64 the last two inverse FFT passes (y, then z into the acceleration grid) run as
 * one kernel per x-plane, whose modes fit the LDS, after the x pass (fused != 0, the
 * default); 0 leaves the choice to pm_nu_set_inverse_xy. The same forces bit for bit. */
int pm_nu_set_inverse_yz(pm_nu_ctx* ctx, int fused);
/* For N <= 128 the first two forward FFT passes (z, then y) run as one kernel per x-plane,
 * which fits the LDS (fused != 0, the default; not with deposit modes 8 and 9, whose patch
 * pass already does the z pass); 0 runs them as the two passes that larger meshes use. Both
 * give the same modes bit for bit. */
int pm_nu_set_forward_zy(pm_nu_ctx* ctx, int fused);
/* With deposit modes 8 and 9, also store delta at every deposit (67 MB more writes per
 * 256^3 box) so that pm_nu_copy_density can read it (on != 0); the default is off. The
 * other deposit modes always keep it. */
int pm_nu_set_keep_density(pm_nu_ctx* ctx, int on);
/* delta_k of one box (after pm_nu_deposit) into out (dev) as complex64 pairs in the
 * layout of numpy.fft.rfftn: [N][N][N/2+1][2]. */
int pm_nu_copy_modes(pm_nu_ctx* ctx, int box, float* out);
/* Acceleration grid of one axis (after pm_nu_force) into out (dev) [N][N][N]. */
int pm_nu_copy_force_grid(pm_nu_ctx* ctx, int box, int axis, float* out);

/* ---- per-kernel timing with HIP events on the library's stream ---------------------- */
/* enable != 0 starts recording an event pair around every kernel launch. */
int pm_nu_set_timing(pm_nu_ctx* ctx, int enable);
/* Record event pairs only around the stages whose bit is set (bit i = the i-th stage as
 * listed by pm_nu_read_timing); 0 stops recording. Fewer events, less overhead. */
int pm_nu_set_timing_mask(pm_nu_ctx* ctx, uint32_t stage_mask);
/* (sync) Sums of kernel times [ms] and launch counts per stage since the last read,
 * then resets them. names[i] are static strings. Arrays hold *n_stages entries on
 * input (capacity) and output (count). */
int pm_nu_read_timing(pm_nu_ctx* ctx, int* n_stages, const char** names, double* total_ms,
                      int64_t* launches);

/* ---- HIP graph of a whole step (for batched small boxes and launch-bound loops) ------ */
/* Capture deposit + response + force at a_now for the given pointers into a graph
 * (sync). The time grid for a_now is prepared before capture. Replays recompute the
 * node a_now each time. Any later call that changes what a step computes (set_history,
 * set_mass, set_species, set_background, set_kernel, set_iterations, set_response_mode,
 * set_power, set_launch, autotune, surrogate load/init/train) discards the graph; launch
 * then fails with PM_NU_ESTATE until the step is captured again. */
int pm_nu_graph_capture(pm_nu_ctx* ctx, const float* pos, float* acc, double a_now);
/* Launch the captured graph on the stream. An eager response at another a_now (which moves
 * the history on) also discards the graph. */
int pm_nu_graph_launch(pm_nu_ctx* ctx);

/* ---- time stepping: the loop of Sec. 4.3 (ii)-(iv) ------------------------------------ */
/* Advance the particles from a_steps[0] to a_steps[n_steps] by n_steps kick-drift-kick
 * leapfrog steps in the superconformal time s (ds = dt/a^2, Sec. 3.2), in which comoving
 * positions obey d^2x/ds^2 = a^2 acc, acc being the force of pm_nu_step (so a acc is what
 * stays constant in the linear matter era). One step a0 -> a1, a_m = sqrt(a0 a1):
 *   u += a0 acc(a0) int_{a0}^{a_m} da/(a^2 H);   x += u int_{a0}^{a1} da/(a^3 H), wrapped;
 *   acc(a1) from deposit -> response -> force at a1 (the response stores the node a1);
 *   u += a1 acc(a1) int_{a_m}^{a1} da/(a^2 H).
 * The two half kicks that meet between steps are applied as one. H(a) is the background of
 * pm_nu_set_background.
 *   pos (dev) [n_boxes][N_p][3] in [0, L); vel (dev) same layout, u = dx/ds = a^2 dx/dt
 *   [dimensionless with c = 1]; acc (dev): on entry the force at a_steps[0] for these
 *   positions (pm_nu_step at a_steps[0]), on exit the force at a_steps[n_steps]. All three
 *   16-byte aligned; updated in place.
 *   a_steps (host) [n_steps + 1], increasing, a_steps[1] after the last stored node.
 * Velocities leave synchronised with positions at a_steps[n_steps]. Sync per step (the time
 * grid of each new a is built on the host). Errors: PM_NU_EINVAL for bad arguments,
 * PM_NU_EHISTORY if the history lacks room for n_steps nodes, then those of the step. */
int pm_nu_advance(pm_nu_ctx* ctx, float* pos, float* vel, float* acc, const double* a_steps,
                  int n_steps);

/* ---- launch-shape autotuning ----------------------------------------------------------- */
/* Time the candidate launch shapes of the tunable kernels on this context's buffers with
 * HIP events (pos/acc (dev) as for pm_nu_step, a_now as for pm_nu_response; the history
 * must be set): the deposit mode and block, the interpolation mode and block, and the three
 * tile candidates of each FFT pass (pm_nu_set_fft_tiles); keep the fastest of each, and if
 * cache_path is not NULL read/write the choice as JSON keyed by (device architecture, N,
 * n_boxes, particles per box) (sync). Ends with one full step at a_now. */
int pm_nu_autotune(pm_nu_ctx* ctx, const float* pos, float* acc, double a_now,
                   const char* cache_path);
/* Set the launch shapes directly: deposit_mode 0 (one thread per particle, global atomics;
 * deposit_block = threads per workgroup), 1..5 (LDS-privatised chunks of 1024/2048/4096
 * particles on 256 threads, 4096 on 512 threads, 8192 on 1024 threads, flushed with global
 * atomics), 6 (chunks of 4096 written to per-chunk patches and summed per 16^3 coarse
 * cell without atomics; a chunk whose box exceeds 6144 nodes, or its part in a coarse cell
 * already listing 32 patches, goes through atomics on a side grid),
 * 7 (as 6 with room for boxes of 9216 nodes, at lower occupancy), 8 and 9 (as 6 and 7 with
 * the coarse-cell sums and the first forward FFT pass in one kernel, so that delta never
 * goes to HBM; N >= 32), interp_mode
 * 0 (direct gather; interp_block = particles per workgroup, rounded down to 256, 512 or
 * 1024) or 1/2/3 (LDS-staged chunks). Blocks: multiples of 64 in 64..1024. Until this or
 * pm_nu_autotune is called: deposit_mode 6 for N >= 64 (4 below, where one coarse cell
 * covers the mesh), interp_mode 1. */
int pm_nu_set_launch(pm_nu_ctx* ctx, int deposit_mode, int deposit_block, int interp_mode,
                     int interp_block);
/* Tile candidates of the six FFT passes, candidates[6] (host) in the order fwd_z (real rows
 * per workgroup), fwd_y (lines), fwd_x + binning (k_y columns), inv_x (k_y columns), inv_y
 * (lines), inv_z (rows); each 0 (the default), 1 or 2, the tile sizes pm_nu_tuning reports
 * (below N = 64 all three are the default). Every candidate computes the same transform;
 * only the speed differs. pm_nu_autotune times them and keeps the fastest of each pass.
 * The next step must start with pm_nu_deposit. Errors: PM_NU_EINVAL for a value outside
 * 0..2. */
int pm_nu_set_fft_tiles(pm_nu_ctx* ctx, const int32_t* candidates);
/* Current launch-shape choice as a short JSON text (host buffer of cap bytes, sync):
 * deposit and interpolation modes and blocks, the FFT tile candidates ("fft") and their
 * tiles ("fft_tiles"), and the threads per (bin, box) of the exact response
 * ("response_threads": 64 when there are at least 1024 pairs, 256 otherwise). */
int pm_nu_tuning(pm_nu_ctx* ctx, char* out, size_t cap);

/* Switch the response between the exact integral (0), the surrogate (1) and the surrogate
 * checked against the exact integral (2) between steps. */
int pm_nu_set_response_mode(pm_nu_ctx* ctx, int mode);

/* Change the total neutrino mass of one box (eV, >= 0) between steps (sync); the box gets
 * cfg.n_species equal masses again. */
int pm_nu_set_mass(pm_nu_ctx* ctx, int box, double m_nu_total);

/* Neutrino mass hierarchy (the paper's Sec. 6.2): give one box n_species (1..4) species
 * with their own masses m_species[n_species] (eV, >= 0, host). Each massive species
 * free-streams with its own kernel I(k (s - s') T_nu0 / m_s) and the neutrino contrast is
 * the mean over species weighted by m_s / M_nu, M_nu = sum of the masses (f_nu follows M_nu);
 * a massless species adds nothing. pnu_half_init (host, [n_species][B], or NULL) gives each
 * species its initial amplitude; NULL uses the one of pm_nu_set_history for all (a later
 * pm_nu_set_history resets all species to its amplitude). The surrogate answers only for
 * three equal masses (the setting it was trained on); otherwise the exact integral runs.
 * Sync. Errors: PM_NU_EINVAL for a bad box, count, mass or amplitude. */
int pm_nu_set_species(pm_nu_ctx* ctx, int box, int n_species, const double* m_species,
                      const double* pnu_half_init);

/* ---- background expansion -------------------------------------------------------------- */
/* Choose the flat background whose H(a) enters the time grid of eq. (P-final): the
 * superconformal time s = int da/(a^3 H) and the measure dtau = d ln a/(a H).
 *   relativistic = 0 (default): matter + Lambda, the neutrinos counted as matter.
 *   relativistic = 1: the background of Sec. 4.4. Each massive species carries the energy
 *     density of eq. (relativistic), a^-3 int sqrt(m^2 + q^2/a^2) f_0(q) 4 pi q^2 dq
 *     (Fermi-Dirac f_0 at T_nu0 = 1.95 K), normalised so that a non-relativistic species
 *     has Omega_nu h^2 = m/93.14 eV; photons (T_gamma = (11/4)^{1/3} T_nu0) and massless
 *     species are radiation; cold matter is Omega_M minus the neutrino rest mass; Lambda
 *     closes the budget today (H(1) = H0).
 * Applies to every box from the next response. f_nu and the source of eq. (P-final) and of
 * the Poisson equation keep Omega_M. The surrogate was trained on the default background
 * and steps aside under the relativistic one (the exact integral runs). Sync. Errors:
 * PM_NU_EINVAL unless relativistic is 0 or 1. */
int pm_nu_set_background(pm_nu_ctx* ctx, int relativistic);

/* ---- free-streaming kernel I(x) ------------------------------------------------------- */
/* Choose I(x) in eq. (P-final) for every box from the next response:
 *   series = 0 (default): the rational fit eq. (fit) of Appendix C;
 *   series = 1: the exact function of Appendix C, 4/(3 zeta(3)) sum_{n>=1} (-1)^{n+1}
 *     n/(n^2+x^2)^2, summed with the alternating-series acceleration of Cohen, Rodriguez
 *     Villegas and Zagier (32 terms; relative error at rounding level for x <= 1e3 and
 *     below 1e-12 for x <= 1e4).
 * The surrogate was trained with the fit and steps aside under the series. Sync.
 * Errors: PM_NU_EINVAL unless series is 0 or 1. */
int pm_nu_set_kernel(pm_nu_ctx* ctx, int series);

/* I(x) at n points (series as above): x and out are device arrays of n doubles, launched
 * on `stream` (NULL: the default stream) and not waited for. A diagnostic of the device
 * kernels; needs no context. Errors: PM_NU_EINVAL for n < 0, a NULL array with n > 0 or a
 * bad flag; PM_NU_EHIP if the launch fails. */
int pm_nu_kernel_values(const double* x, int64_t n, int series, double* out, void* stream);

/* Iterations of the implicit equation for the current node (Sec. 4.3 (iii), Appendix B),
 * as pm_nu_config.iterations, from the next response. The quadrature is gathered once as
 * a stored-node part plus a coefficient of the current node, so each further iteration is a
 * scalar update. Sync. Errors: PM_NU_EINVAL outside [1, 16]. */
int pm_nu_set_iterations(pm_nu_ctx* ctx, int iterations);

/* ---- binned power from elsewhere ------------------------------------------------------- */
/* Set P_cdm(k_b) of one box (host) [B] in place of a deposit, for a response computed
 * from a spectrum measured elsewhere (or for building the surrogate's training set). The
 * response may follow; the force may not (it needs the modes of a deposit). Empty bins
 * are ignored (sync). */
int pm_nu_set_power(pm_nu_ctx* ctx, int box, const double* p_cdm);

/* ---- learned surrogate for the history integral (not in the paper) -------------------- */
/* A fully connected network 16 -> 128 -> 128 -> 128 -> 1, GELU after each hidden layer,
 * weights and layer inputs rounded to bfloat16 with FP32 accumulation (matrix cores in
 * training and in the step), FP32 master weights and Adam moments. Inputs per (box, bin),
 * with a_0 < ... < a_{n-1} the stored nodes before a_now and A(u) the stored
 * P_M^{1/2}(k_b) linear in u = ln a between them (as the history integral reads it):
 *   ln k_b, ln a_now, M_nu [eV], ln a_now - ln a_{n-1},
 *   P_nu^{1/2}(k_b, a_{n-1}) / P_cdm^{1/2}(k_b, a_now) (what the first iteration puts into
 *   the current node), ln(a_now / a_0), ln(k_b (s(a_now) - s(a_{n-1})) T_nu0 / m) (the
 *   free-streaming kernel's argument across the last interval, m = M_nu / n_species), and
 *   A(ln a_{n-1} - L_m) / P_cdm^{1/2}(k_b, a_now) for the nine lags
 *   L_m = 0, 0.05, 0.1, 0.2, 0.35, 0.55, 0.8, 1.2, 2.1 in ln a
 * (lags in ln a, so the inputs mean the same for any spacing of the stored nodes; they
 * exist once the history reaches 2.1 in ln a below its last node), standardised with the
 * stored mean/scale. Output (after un-standardising):
 *   y = ln(R (1 + k_b/k_fs(a_now))^2),
 * i.e. R relative to the Appendix A approximation 1/(1 + k/k_fs)^2 with k_fs of
 * eq. (kfs-formal) for one species of mass M_nu/n_species. In the step (response_mode 1)
 * a bin whose inputs do not exist or fall outside the training range (5% margin) uses the
 * exact integral instead; response_mode 2 runs both and keeps the exact result. Blob layout
 * (FP32): W1[16][128], b1[128], W2[128][128], b2, W3[128][128], b3, W4[128], b4, then
 * feature mean[16], scale[16], min[16], max[16], target mean, scale. */
enum { PM_NU_SUR_IN = 16, PM_NU_SUR_HIDDEN = 128, PM_NU_SUR_PARAMS = 35329 };
/* Number of FP32 values in a weight blob (35329 + 4*16 + 2). */
int64_t pm_nu_surrogate_blob_floats(void);
/* Load weights and statistics (host) (sync). */
int pm_nu_surrogate_load(pm_nu_ctx* ctx, const float* blob, int64_t n_floats);
/* Copy the current weights and statistics out (host) (sync). */
int pm_nu_surrogate_save(pm_nu_ctx* ctx, float* blob, int64_t n_floats);
/* Training rows for the step's current state: runs the exact response at a_now (after
 * pm_nu_deposit or pm_nu_set_power for every box, history set) and writes the inputs
 * x (dev) [n_boxes*B][16] and targets y (dev) [n_boxes*B] in row box*B + b; rows that
 * cannot be used (empty bin, inputs that do not exist, no neutrinos) get y = NaN. */
int pm_nu_surrogate_dataset(pm_nu_ctx* ctx, double a_now, float* x, float* y);
/* Initialise weights (seeded, uniform +-sqrt(6/(fan_in+fan_out))) and the feature and
 * target statistics from the n rows of x (dev) [n][16], y (dev) [n] (sync). */
int pm_nu_surrogate_init(pm_nu_ctx* ctx, const float* x, const float* y, int64_t n,
                         uint64_t seed);
/* Adam (lr, betas 0.9/0.999, eps 1e-8) on the mean squared error of the standardised
 * target over x (dev) [n][16], y (dev) [n]: `epochs` passes in minibatches of `batch`
 * rows (a multiple of 32), reshuffled every epoch from `seed`; the learning rate decays
 * by half-cosine to lr/100 over the call. *loss_out (host) = mean loss of the last epoch
 * (sync). */
int pm_nu_surrogate_train(pm_nu_ctx* ctx, const float* x, const float* y, int64_t n,
                          int epochs, int batch, float lr, uint64_t seed, float* loss_out);
/* The same training split over several calls: epochs first_epoch .. first_epoch+epochs-1 of
 * a run of total_epochs, the learning rate following the half-cosine of the whole run (the
 * shuffles and Adam moments continue from the previous call). pm_nu_surrogate_train is the
 * call with first_epoch = 0 and total_epochs = epochs. */
int pm_nu_surrogate_train_part(pm_nu_ctx* ctx, const float* x, const float* y, int64_t n,
                               int first_epoch, int epochs, int total_epochs, int batch,
                               float lr, uint64_t seed, float* loss_out);
/* Network output y (dev) [n] (un-standardised) for raw inputs x (dev) [n][16]. */
int pm_nu_surrogate_predict(pm_nu_ctx* ctx, const float* x, float* y, int64_t n);
/* Mean squared error of the standardised target over x (dev) [n][16], y (dev) [n] and its
 * FP32 gradient (dev) [35329] in blob order, with the current weights (sync). */
int pm_nu_surrogate_grad(pm_nu_ctx* ctx, const float* x, const float* y, int64_t n,
                         float* grad, float* loss_out);
/* After a response in mode 2: exact and surrogate R of one box (host) [B] (sync);
 * bins that used the exact fallback report the same value twice. */
int pm_nu_get_surrogate_check(pm_nu_ctx* ctx, int box, double* ratio_exact,
                              double* ratio_surrogate);

#ifdef __cplusplus
}
#endif
#endif /* PM_NU_H */
