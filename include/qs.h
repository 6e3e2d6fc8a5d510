/*
 * qs.h -- C ABI of the MI355X quasistatic beam-plasma instability solver.
 *
 * The model (San Miguel Claveria et al., "Quasistatic modeling of ultrarelativistic
 * beam-plasma instabilities", Sec. II):  a dilute, cold beam of one or more species
 * (charge q_s, mass m_s, unperturbed density n_bs, common Lorentz factor gamma_b) crosses
 * a cold plasma of immobile ions.  In the co-moving coordinates xi = t - x (distance
 * behind the beam front) and tau = t, with every quantity normalized as in Sec. II, the
 * linear perturbations of one transverse Fourier mode exp(i k.r_perp) obey
 *
 *   (d_xi^2 + 1) n_p = rho                         plasma response, Eq. plasma_oscillations_QSA
 *   (1 + k^2) Psi  = n_p                           pseudo-potential, Eq. poisson_QSA
 *   d_tau rho      = d_xi j_par - i k j_perp       beam charge continuity, Eq. beam_continuity
 *   d_tau j_par    = -gamma^-3 Omega d_xi Psi      beam current response, Eq. beam_momentum
 *   d_tau j_perp   = +gamma^-1 Omega i k Psi
 *
 * with rho = sum_s q_s n_s the perturbed beam charge density, j_par, j_perp the perturbed
 * beam current densities sum_s q_s n0_s v_s, and Omega(xi) = sum_s q_s^2 n0_s(xi)/m_s
 * (for a xi-dependent profile the continuity equation is in flux form, Sec. III.D).  The
 * solver marches the plasma response causally in xi from the front (n_p = d_xi n_p = 0
 * ahead of the beam), with no slowly-varying-envelope approximation, alternating with a
 * fourth-order Runge-Kutta push of (rho, j_par, j_perp) in tau.  Eliminating the currents
 * gives the master equation, Eq. full_master_eq (Eq. full_master_eq_v2 for a profile).
 *
 * Fields written by the solver (ln of magnitudes, at cell centres):
 *   E_par = -d_xi Psi,  E_perp = -i k (rho - n_p)/(1+k^2),  B_perp = -i k rho/(1+k^2),
 *   |E| = sqrt(|E_par|^2 + |E_perp|^2),  A = sqrt(|E|^2 + |B_perp|^2).
 *
 * Discretization: cells j = 0..n_xi-1 of width h = length/n_xi; rho and j_perp at cell
 * centres, j_par on the interior faces (j+1)h (the two outer faces carry no current); the
 * oscillator is advanced through each cell with its exact solution for a cell-constant
 * source.  Each mode is renormalized after every step by an exact power of two; every
 * output already includes that scale.
 *
 * Conventions for every entry point:
 *   - Return value: QS_OK or a negative qs_status.  No entry point aborts, throws or exits.
 *     The message of the last failure on the calling thread is returned by qs_last_error().
 *   - Argument errors (QS_ERR_ARG) are detected before any device work and leave every
 *     buffer and the context unchanged.
 *   - Pointers documented as "device" must point to device memory of the device that was
 *     current at qs_init; "host" pointers to host memory.  The caller owns every buffer it
 *     passes; the library keeps no pointer to them after the call returns, except the
 *     workspace given to qs_init, which must stay alive until qs_free.
 *   - Device work is queued on the stream given to qs_init, in call order.  Calls returning
 *     host data synchronize that stream.  A context may be used by one thread at a time;
 *     distinct contexts are independent.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QS_ABI_VERSION 1

typedef enum {
    QS_OK = 0,
    QS_ERR_ARG = -1,         /* invalid argument (nothing was changed) */
    QS_ERR_ALLOC = -2,       /* device or host allocation failed, or workspace too small */
    QS_ERR_HIP = -3,         /* a HIP runtime call failed; the message names it */
    QS_ERR_NUMERIC = -4,     /* a non-finite value was found when renormalizing */
    QS_ERR_UNSUPPORTED = -5, /* valid request that the library does not implement */
    QS_ERR_STATE = -6        /* the context is in a state that does not allow the call */
} qs_status;

enum { QS_FP64 = 0, QS_FP32 = 1 };           /* FP32: FP32 state, FP64 oscillator carry */
enum { QS_PROFILE_FLATTOP = 0, QS_PROFILE_GAUSSIAN = 1, QS_PROFILE_TABLE = 2 };
enum { QS_GEOM_SPECTRAL = 0, QS_GEOM_TRANSVERSE_GRID = 1 };
enum {
    QS_SEED_NOISE = 0,         /* rho = amp f(xi_j) exp(i theta), theta uniform from rng_seed */
    QS_SEED_UNIFORM = 1,       /* rho = amp f(xi_j): the extended disturbance of Appendix C */
    QS_SEED_FRONT_IMPULSE = 2, /* d_tau rho = amp/h in cell 0 at tau = 0+ (Appendix B impulse) */
    QS_SEED_CENTROID = 3,      /* transverse-grid runs only: displaced beam plus noise */
    QS_SEED_NONE = 4           /* state is zero until qs_set_state */
};
enum {
    QS_FLAG_DROP_LONGITUDINAL = 1, /* drop the gamma^-2 d_xi^2 term: Eq. CFI_st_master */
    QS_FLAG_NO_RESTORING = 2,      /* plasma operator d_xi^2 only: Eq. CFI_st_master_front */
    QS_FLAG_STEADY_INFLOW = 4,     /* plasma ahead of the front equals cell 0 (uniform test) */
    QS_FLAG_FPERP_SNAPSHOTS = 8,   /* output option: snapshots' ln_e holds ln|F_perp| (below) */
    QS_FLAG_STATIONARY_FRONT = 16  /* plasma ahead of the front held at its tau = 0 value (below) */
};

/*
 * One problem instance, in the paper's normalized units (Sec. II).
 *   n_species, q, m, nb_over_np : beam species (charge/e, mass/m_e, peak n_bs/n_p), host
 *                                 arrays of n_species entries.  Only sum q^2 nb/m enters.
 *   gamma_b                     : common Lorentz factor (> 1).
 *   length                      : beam length L; the grid covers 0 <= xi <= L.
 *   profile                     : longitudinal shape f(xi) <= 1 of n_b0 (Sec. III.D):
 *                                 FLATTOP f = 1; GAUSSIAN exp(-(xi-xi_center)^2/2 sigma_xi^2);
 *                                 TABLE profile_table[n_xi] (host) at the cell centres.
 *   geometry                    : QS_GEOM_SPECTRAL (list of k_perp), or
 *                                 QS_GEOM_TRANSVERSE_GRID (finite-width beam, Sec. IV.B: the
 *                                 perturbations on a periodic nx x ny grid per xi cell; one
 *                                 instance per context, QS_FP32 only, flags DROP_LONGITUDINAL
 *                                 and NO_RESTORING only; see "Finite-width contexts" below).
 *   n_modes, kx, ky             : transverse wavevectors, host arrays; ky may be NULL (slab).
 *                                 Only |k| enters the dynamics.  Ignored for TRANSVERSE_GRID.
 *   nx, ny, lx, ly, sigma_r     : transverse grid (TRANSVERSE_GRID only; ignored otherwise):
 *                                 nx, ny powers of two in [2, 256], n_xi <= 65535, periodic
 *                                 box lx x ly,
 *                                 points x_i = (i - nx/2) lx/nx (likewise y); the beam's
 *                                 transverse profile g = exp(-(x^2+y^2)/(2 sigma_r^2)), or
 *                                 g = 1 for sigma_r = 0, so n_b0 = nb f(xi) g(x, y).
 *   n_xi                        : number of xi cells (>= 1).
 *   d_tau                       : tau step of the Runge-Kutta push (> 0).
 *   precision                   : QS_FP64, or QS_FP32 (FP32 state, FP64 oscillator carry).
 *   seed_kind, seed_amp,        : initial perturbation (see the enum); for NOISE the phase of
 *   rng_seed                      (instance i, mode m, cell j) is 2 pi u, u the top 53 bits of
 *                                 output number (i*n_modes + m)*n_xi + j of SplitMix64 started
 *                                 at rng_seed, over 2^53.
 *   centroid_offset             : TRANSVERSE_GRID only: the CENTROID seed is
 *                                 rho = (centroid_offset x / sigma_r^2 + seed_amp (2u - 1)) f g,
 *                                 the first-order density change of a beam displaced by
 *                                 centroid_offset in x plus uniform noise (u as for NOISE with
 *                                 index (j ny + iy) nx + ix); NOISE is seed_amp (2u - 1) f g,
 *                                 UNIFORM seed_amp f g.
 *   flags                       : QS_FLAG_* model test hooks (0 for the physical model) and
 *                                 the output option QS_FLAG_FPERP_SNAPSHOTS (spectral
 *                                 geometry only): snapshot ln_e then receives
 *                                 ln|F_perp| = ln(k kappa |n_p|) (+ the log-scale), the
 *                                 transverse force E_perp - B_perp = i k Psi on a beam particle
 *                                 (Sec. III.D, the quantity of Figs. 3 and 4); ln_b and the
 *                                 per-step max ln A are unchanged.
 *                                 QS_FLAG_STATIONARY_FRONT (spectral geometry only; not with
 *                                 QS_FLAG_STEADY_INFLOW): the plasma ahead of the beam is held
 *                                 at its tau = 0 state for every step, the boundary value that
 *                                 Sec. III.D's numerical solution keeps (F_perp(xi = 0, tau) =
 *                                 F_perp(xi = 0, 0)) and that Appendix C's extended
 *                                 disturbance has (Eq. extended_BC): per mode n_p = F and
 *                                 d_xi n_p = 0 at the front, F the charge density of cell 0 in
 *                                 the state qs_init seeds (the plasma in equilibrium with the
 *                                 beam's first cell at tau = 0).  F belongs to the context, not
 *                                 to the state: qs_set_state and checkpoints leave it as
 *                                 seeded (0 for QS_SEED_NONE and the front impulse).
 */
typedef struct qs_params {
    int32_t n_species;
    const double *q;
    const double *m;
    const double *nb_over_np;
    double gamma_b;
    double length;
    int32_t profile;
    double sigma_xi;
    double xi_center;
    const double *profile_table;
    int32_t geometry;
    int64_t n_modes;
    const double *kx;
    const double *ky;
    int32_t nx, ny;
    double lx, ly;
    double sigma_r;
    int32_t n_xi;
    double d_tau;
    int32_t precision;
    int32_t seed_kind;
    double seed_amp;
    uint64_t rng_seed;
    double centroid_offset;
    int32_t flags;
} qs_params;

typedef struct qs_ctx qs_ctx;

/*
 * Execution plan of the march kernel (library design choice, not physics):
 *   columns_per_lane : real columns per SIMD lane, 1 (the two parts of a mode in adjacent
 *                      lanes) or 2 (one mode per lane); 0 = default (1, or the value of the
 *                      environment variable QS_COLUMNS_PER_LANE).
 *   segment_cells    : target cells per xi-segment.  Each 64-lane block of modes is split
 *                      into ceil(n_xi/segment_cells) segments (at most 16 for FP32 with one
 *                      column per lane, else 8), one
 *                      wavefront each, pipelined over tau-steps with the oscillator carries
 *                      passed between segments in LDS.  0 = automatic (fill one round of
 *                      workgroups); >= n_xi = no segmentation.
 *   max_segments     : (output of qs_get_plan) largest segment count of any instance.
 */
typedef struct qs_plan {
    int32_t columns_per_lane;
    int32_t segment_cells;
    int32_t max_segments;
    int32_t reserved;
} qs_plan;

/* ABI version of the loaded library (QS_ABI_VERSION at build time). */
int32_t qs_abi_version(void);

/* Thread-local text of the last failure on this thread ("" if none).  Never NULL. */
const char *qs_last_error(void);

/*
 * Bytes of device workspace qs_init needs for these instances (0 on invalid arguments).
 * params: host array of n_instances problem descriptions.
 */
size_t qs_workspace_size(const qs_params *params, int32_t n_instances);

/* As qs_workspace_size, for an explicit execution plan (NULL = automatic). */
size_t qs_workspace_size_ex(const qs_params *params, int32_t n_instances, const qs_plan *plan);

/*
 * Create a solver context for n_instances >= 1 instances (Sec. II problem statement per
 * instance), build the per-instance tables (Omega(xi) at centres and faces, per-mode
 * constants) and write the seed state.  All instances must share one precision; their
 * n_xi, d_tau, species and modes may differ (a batched sweep).
 *   hip_stream      : hipStream_t to queue device work on (NULL = the null stream).
 *   workspace       : device buffer of workspace_bytes >= qs_workspace_size(...), owned by
 *                     the caller and kept alive until qs_free; or NULL, in which case the
 *                     library allocates (and frees) its own.
 *   out             : receives the context (host).  Unchanged on failure.
 * Errors: QS_ERR_ARG (invalid parameter: the message names it), QS_ERR_UNSUPPORTED,
 *         QS_ERR_ALLOC, QS_ERR_HIP.
 */
qs_status qs_init(const qs_params *params, int32_t n_instances, void *hip_stream,
                  void *workspace, size_t workspace_bytes, qs_ctx **out);

/* As qs_init, with an explicit execution plan (NULL = automatic).  QS_ERR_ARG for an invalid
 * plan.  The plan changes only the schedule and the association of the arithmetic: in FP64
 * the results of different plans agree to rounding (~1e-15 relative); in FP32 the stored
 * state is rounded after a different number of operations per segment, so plans differ by
 * FP32 rounding, a few 1e-7 relative per step (at most 2e-6 in ln A over the tests' runs).
 * For one plan the results are bitwise reproducible. */
qs_status qs_init_ex(const qs_params *params, int32_t n_instances, const qs_plan *plan,
                     void *hip_stream, void *workspace, size_t workspace_bytes, qs_ctx **out);

/* The plan in use (host): columns per lane, segment cells, largest segment count; and the
 * workgroup count and wave slots per workgroup of one march launch.  Any output may be NULL. */
qs_status qs_get_plan(const qs_ctx *ctx, qs_plan *plan, int32_t *n_workgroups,
                      int32_t *waves_per_workgroup);

/*
 * Advance every instance by n_steps >= 0 tau-steps of its own d_tau (the hot path: one
 * fused causal march over xi per step carrying all four Runge-Kutta stages; each snapshot
 * interval runs as one persistent launch, which writes the interval's snapshot during its
 * first sweep when the plan has one column per lane; snapshots at every step run as one
 * launch whose sweeps, with one column per lane, still take two steps and write both).
 * Outputs (device pointers, each may be NULL; element type double for QS_FP64, float for
 * QS_FP32), for the modes of all instances concatenated in instance order (mode index
 * M = sum of n_modes of the earlier instances + m):
 *   out_ln_e, out_ln_b : field snapshots of the state at the start of every step s of this
 *                        call with s % out_every == 0; snapshot t of instance i starts at
 *                        element t * S + off_i with S = sum_i n_xi_i * n_modes_i and
 *                        off_i = sum_{i'<i} n_xi_i' * n_modes_i', then [n_xi_i][n_modes_i]
 *                        (rows padded instead after qs_set_snapshot_align).
 *                        With n_steps == 0 one snapshot of the current state is written and
 *                        the state does not change.
 *   out_max_ln_a       : [n_steps][total modes] max over xi of ln A at the start of each step.
 *   out_every >= 1 (ignored when both snapshot pointers are NULL).
 * Errors: QS_ERR_ARG, QS_ERR_HIP.  Does not synchronize.
 */
qs_status qs_step_tau(qs_ctx *ctx, int32_t n_steps, int32_t out_every, void *out_ln_e,
                      void *out_ln_b, void *out_max_ln_a);

/*
 * Synchronize the context's stream and report any failure of the launches since the last
 * call:
 *   QS_ERR_NUMERIC : a renormalization met a non-finite value; the message names the first
 *                    one found: the instance, its mode index (as given in qs_params) and the
 *                    tau-step after which the state was non-finite;
 *   QS_ERR_HIP     : a xi-segment hand-off wait of the march kernel gave up (a device that
 *                    stalled a workgroup beyond the wait budget); that launch's results are
 *                    invalid.
 * After either failure, if the rollback copy is enabled (qs_set_rollback) and holds a state,
 * the state, scales and step count are restored to it -- the state at the start of the last
 * qs_step_tau call (or graph replay) that began with no failure pending, i.e. the last good
 * tau -- and the message names that step; the context is usable again.  Otherwise the
 * context is marked invalid: qs_step_tau and qs_graph_launch return QS_ERR_STATE until
 * qs_set_state, qs_grid_set_state or qs_load_checkpoint replaces the state (qs_get_state
 * still reads it).  The failure is reported once.
 */
qs_status qs_sync_check(qs_ctx *ctx);

/*
 * Rollback copy (spectral contexts): with enable != 0 the library allocates a device copy
 * of the state and its scales (the size of a checkpoint, qs_checkpoint_size) and every
 * stepping call first refreshes it, on the context's stream, unless a failure is pending; a
 * failure reported by qs_sync_check then restores it (above).  The copy costs one device
 * read and write of the state per qs_step_tau call.  enable == 0 frees it.
 * Errors: QS_ERR_ARG, QS_ERR_UNSUPPORTED (transverse-grid context), QS_ERR_ALLOC.
 */
qs_status qs_set_rollback(qs_ctx *ctx, int32_t enable);

/*
 * Snapshot row alignment (spectral contexts; library design choice, not physics).  With
 * align > 1 the snapshots that later qs_step_tau and qs_graph_create calls write pad each
 * instance's rows to a multiple of `align` modes: instance i holds [n_xi_i][ld_i] elements of
 * each snapshot, ld_i = n_modes_i rounded up to a multiple of align, the row of cell j holding
 * mode m at j * ld_i + m, from off_i = sum_{i'<i} n_xi_i' ld_i'; a snapshot holds
 * S = sum_i n_xi_i ld_i elements (*snapshot_elems, may be NULL) and the padding is not
 * written.  The march writes the modes of one wavefront (32 with one column per lane) as one
 * piece of each row, so with rows aligned to that piece (align 32, and a buffer aligned to
 * 128 bytes) each piece fills whole cache lines: partly written lines otherwise cost the
 * memory a read before the write.  align = 1 restores the dense layout (the default).  The
 * state, checkpoints and every other output are unaffected.  Synchronous.
 * Errors: QS_ERR_ARG (align not a power of two in [1, 1024]), QS_ERR_UNSUPPORTED
 * (transverse-grid context), QS_ERR_STATE (the context has graphs: free them first, they
 * keep the layout they were made with), QS_ERR_HIP.
 */
qs_status qs_set_snapshot_align(qs_ctx *ctx, int32_t align, int64_t *snapshot_elems);

/*
 * Number of tau-steps taken since qs_init (host).  Returns -1 for a NULL context.
 */
int64_t qs_steps_done(const qs_ctx *ctx);

/*
 * Copy the state out (synchronizes).  Host arrays of 2 * sum_i n_modes_i * n_xi_i doubles
 * each, complex interleaved, instance-major then mode then cell:
 *   rho    : beam charge density at the cell centres,
 *   j_par  : longitudinal beam current density at the rear face of each cell (the last
 *            cell's entry, the outer face, is 0),
 *   j_perp : transverse beam current density along k at the cell centres,
 *   log2_scale : [total modes] the state of mode M is (rho, j_par, j_perp) * 2^log2_scale[M].
 * Any array may be NULL.  Errors: QS_ERR_ARG, QS_ERR_HIP.
 */
qs_status qs_get_state(qs_ctx *ctx, double *rho, double *j_par, double *j_perp,
                       double *log2_scale);

/*
 * Replace the state (same layout as qs_get_state; all four arrays required, host).
 * log2_scale must hold integers.  Values are rounded to the context's precision.
 * Errors: QS_ERR_ARG, QS_ERR_HIP.
 */
qs_status qs_set_state(qs_ctx *ctx, const double *rho, const double *j_par,
                       const double *j_perp, const double *log2_scale);

/*
 * Checkpoint: an opaque, bitwise-exact image of the context's state (stored values, per-mode
 * scale exponents, steps done) in the library's own layout, for resuming the same problem.
 * qs_checkpoint_size returns its size in bytes (0 for a NULL context).
 * qs_save_checkpoint writes it to host memory `dst` of `bytes` >= that size (synchronizes).
 * qs_load_checkpoint restores it from host memory; it must come from a context created with
 * identical parameters (checked through the stored shape header: QS_ERR_ARG otherwise).
 * Continuing after a load is bitwise identical to continuing the saved context.
 * (qs_get_state / qs_set_state instead use the documented canonical layout; a round trip
 * through them is exact up to one rounding of the stored scaled currents.)
 */
size_t qs_checkpoint_size(const qs_ctx *ctx);
qs_status qs_save_checkpoint(qs_ctx *ctx, void *dst, size_t bytes);
qs_status qs_load_checkpoint(qs_ctx *ctx, const void *src, size_t bytes);

/*
 * Autotuner (library design choice, not physics): time candidate execution plans for these
 * instances on the current device and return the fastest for calls of steps_per_call tau-
 * steps that output the per-step maxima.  Candidates: columns_per_lane 1 and 2, each with
 * 1, 2, 3, 4, 6, 8, 12 or 16 xi-segments (as many as the workgroup holds) and the automatic
 * plan.  Each is initialized on a scratch workspace that qs_tune allocates (hipMalloc) and
 * frees before returning, and timed: directly for steps_per_call <= 96, else as calls of 16
 * and 96 steps fitted to a + b n (a segmented plan pays a pipeline fill once per call) and
 * evaluated at n = steps_per_call.  With QS_TUNE_VERBOSE set, each candidate's time is
 * printed to stderr.  If
 * the environment variable QS_TUNE_CACHE names a file, a result for the same parameters
 * (seed excluded), steps_per_call and device is taken from it instead of timing, and new
 * results are appended to it.
 *   best        : receives columns_per_lane and segment_cells (pass it to qs_init_ex).
 *   ms_per_step : optional; the projected time per tau-step of the chosen plan.
 * Synchronizes the device.  Errors: QS_ERR_ARG (as qs_init), QS_ERR_ALLOC, QS_ERR_HIP.
 */
qs_status qs_tune(const qs_params *params, int32_t n_instances, int32_t steps_per_call,
                  qs_plan *best, double *ms_per_step);

/*
 * Captured step sequences: qs_graph_create records the kernel launches of one
 * qs_step_tau(ctx, n_steps, out_every, out_ln_e, out_ln_b, out_max_ln_a) call (same
 * arguments and meaning) into a HIP graph without running them; qs_graph_launch replays it
 * on the context's stream, advancing the state by n_steps each time and writing the same
 * output buffers.  The graph holds only kernel nodes (no memset or copy nodes).  The output
 * pointers must stay valid while the graph exists; the graph must be freed before its
 * context.  Errors: QS_ERR_ARG (as qs_step_tau; n_steps >= 1), QS_ERR_HIP.
 */
typedef struct qs_graph qs_graph;
qs_status qs_graph_create(qs_ctx *ctx, int32_t n_steps, int32_t out_every, void *out_ln_e,
                          void *out_ln_b, void *out_max_ln_a, qs_graph **out);
qs_status qs_graph_launch(qs_graph *graph);
void qs_graph_free(qs_graph *graph);

/*
 * Finite-width contexts (geometry QS_GEOM_TRANSVERSE_GRID).  qs_step_tau advances them like
 * spectral ones; its outputs are float32 with snapshots laid out [snap][n_xi][ny][nx] and
 * out_max_ln_a [step] holding ln of the largest (|E|^2 + |B|^2)^(1/2) over the whole grid at
 * the start of each step.  The state (host, float64, [n_xi][ny][nx] each): rho at cell
 * centres, j_par on the rear face of each cell (the last face carries none), j_x and j_y at
 * centres.  qs_grid_get_state / qs_grid_set_state read and replace it (set: all four
 * arrays required; get: any may be NULL).  The spectral state calls, checkpoints and
 * qs_tune return QS_ERR_UNSUPPORTED for these contexts, and the grid calls for spectral
 * ones.  Errors: QS_ERR_ARG, QS_ERR_UNSUPPORTED, QS_ERR_HIP.
 */
qs_status qs_grid_get_state(qs_ctx *ctx, double *rho, double *j_par, double *j_x, double *j_y);
qs_status qs_grid_set_state(qs_ctx *ctx, const double *rho, const double *j_par, const double *j_x,
                            const double *j_y);

/* Release the context and anything the library allocated for it.  NULL is ignored. */
void qs_free(qs_ctx *ctx);

/*
 * Test hook: the wall-clock budget of each xi-segment hand-off wait of this context's march
 * launches, in seconds (-1: the default, 2 s plus 20 us per segment cell).  A small budget
 * makes the waits give up -- every wave of the launch still exits -- so that the stall path
 * of qs_sync_check can be exercised.  Errors: QS_ERR_ARG.
 */
qs_status qs_debug_set_wait_budget(qs_ctx *ctx, double seconds);

/*
 * Diagnostics: output number i (0-based) of the SplitMix64 stream started at `seed`, as the
 * device seed kernel evaluates it (Steele, Lea and Flood, OOPSLA 2014), computed on the host.
 */
uint64_t qs_debug_splitmix64(uint64_t seed, uint64_t i);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
