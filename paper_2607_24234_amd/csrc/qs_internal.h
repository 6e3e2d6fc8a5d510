// Internal declarations shared by the HIP sources of libqs (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qs.h"

struct qs_mlp;

namespace qs {

constexpr int kWave = 64;  // lanes per wavefront on CDNA
constexpr int32_t kFlatProfile = 1 << 16;  // InstDev.flags bit: Omega is constant over the beam

// Per-instance constants, read by every workgroup of that instance (wave-uniform).
struct InstDev {
    int32_t n_xi;        // cells
    int32_t n_modes;     // active modes
    int32_t n_blocks;    // 64-lane blocks of this instance
    int32_t block0;      // first global block index
    int32_t pmode0;      // first padded global mode index
    int32_t mode0;       // first global (unpadded) mode index
    int32_t flags;       // QS_FLAG_*
    int32_t snap_first;  // first cell written to snapshots (rows j - snap_first); 0 unless narrowed
    int64_t state_off;   // element offset of block 0 in the state array
    int64_t omega_off;   // element offset of this instance's Omega tables (centres, then faces)
    int64_t snap_off;    // element offset of this instance inside one snapshot
    int64_t scale_off;   // offset of (segment 0, mode 0) in the per-(mode, segment) scale arrays
    int32_t n_seg;       // xi-segments (waves per block) of this instance
    int32_t seg_len;     // cells per segment (the last one may be shorter)
    int32_t snap_ld;     // elements between the snapshot rows of consecutive cells (>= n_modes)
    int32_t pad_;
    double h, ih;        // cell width, 1/h (0 when the longitudinal term is dropped)
    double dtau;
    double ginv, g3inv;  // gamma^-1, gamma^-3 (g3inv is 0 when the longitudinal term is dropped)
    double c1, s1;       // cos h, sin h
    double c2, s2;       // cos h/2, sin h/2
};

// Arguments of one tau-step launch.
struct StepArgs {
    void *state;              // TS elements, layout [block][cell][var 3][col NC][lane 64]
    const int32_t *blk_inst;  // global block -> instance
    const InstDev *inst;
    const void *omega;        // TC elements: per instance [n_xi] centres then [n_xi] faces
    const double *kmode;      // |k| per padded mode
    const double *coef;       // per padded mode (cT, cP): d_tau T' = cT Omega n_p and
                              // d_tau P' = cP Omega d_xi n_p (k^2 kappa/gamma, -kappa/(gamma^3 h))
    int32_t *log2s;           // per (segment, padded mode): applied power of two (L)
    int32_t *epend;           // per (segment, padded mode): pending exponent (next step)
    void *ln_e, *ln_b;        // snapshot outputs (TS) or null
    void *max_ln_a;           // [step][total modes] (TS) or null
    int64_t snap_base;        // element offset of the launch's first snapshot (ln_e/ln_b)
    int64_t snap_stride;      // elements between the snapshots of consecutive steps of one
                              // launch (snapshot launches that take several steps)
    int64_t max_base;         // element offset of the launch's first row in max_ln_a
    int32_t total_modes;      // unpadded total modes (row length of max_ln_a)
    int32_t update;           // 1: advance the state; 0: fields only
    int32_t n_steps;          // tau-steps of this launch
    int32_t keyed;            // 1: max_ln_a holds order-preserving keys (combined by atomic max)
    uint64_t wait_ticks;      // wall-clock ticks a segment hand-off wait allows before giving up
    const int2 *wave_table;   // per (workgroup, wave slot): (global block, segment) or (-1, -1)
    const double *front0;     // [global block][column][lane]: rho of cell 0 at tau = 0 (the
                              // stationary front's n_p, unscaled)
    uint32_t *err;            // [0]: 1 + padded mode after a non-finite renormalization;
                              // [1]: 1 if a segment hand-off wait gave up;
                              // [2..3]: uint64 ~(step << 32 | padded mode) of the first
                              //         non-finite value (largest complement = first step);
                              // [4..5]: int64 tau-steps done (the device's step counter)
};

// Device copy of the state and scales, taken at the start of a stepping call when no error
// is pending (the rollback guard); meta[0] receives the step count of the copy.
struct GuardArgs {
    const uint4 *src[3];
    uint4 *dst[3];
    int64_t n16[3];           // 16-byte words per region
    const uint32_t *err;
    int64_t *meta;
};

struct SeedArgs {
    void *state;
    const int32_t *blk_inst;
    const InstDev *inst;
    const double *shape;      // per instance at omega_off: f(xi_j) (double)
    const double *kmode;
    int32_t *log2s, *epend;
    int32_t kind;
    double amp;
    uint64_t rng_seed;
    const int32_t *inst_index; // instance index per instance (for the RNG counter)
    int32_t block_base;        // global block index of blockIdx.x == 0
};

// Replace the per-mode push coefficients (cT, cP above; host arrays of the context's modes in
// qs_params order) of a spectral context: lets modes of one instance stand for beams of other
// densities, Lorentz factors and steps (qs_growth.hip).  Synchronous.
qs_status set_mode_coefficients(qs_ctx *c, const double *cT, const double *cP);

// Narrow the snapshots of a spectral context to the cells j >= first[i] of each instance i
// (host array of n_instances, 0 <= first[i] < n_xi): instance i then holds
// [n_xi - first[i]][snap_ld] elements of each snapshot, row j - first[i] for cell j, at the
// running offset over the instances (qs_growth.hip reads only the rear cells).  *snap_elems
// receives the elements of one snapshot.  Synchronous; QS_ERR_ARG for an invalid cell.
qs_status set_snapshot_cells(qs_ctx *c, const int32_t *first, int64_t *snap_elems);

// The tables of a flat-top instance: Omega = q2nm at every centre and at every inner face (the
// outer face 0), profile 1, at element offset `off` of the tables ([n] centres, [n] faces).
struct FlatTable {
    int64_t off;
    int32_t n;
    int32_t pad;
    double q2nm;   // sum over species of q^2 n_b / m
};

// launchers (qs_spectral.hip)
// flat-top instances' tables: shape (double) and omega (TC of the precision), one block each
hipError_t launch_flat_tables(int precision, const FlatTable *ft, int n, double *shape, void *omega, hipStream_t s);
// front0[(gb * nc + c) * 64 + lane] = rho of cell 0 of that column of the stored state (the
// state at tau = 0 when called after seeding)
hipError_t launch_front_capture(int precision, int nc, const void *state, const int32_t *blk_inst,
                                const InstDev *inst, int n_blocks, double *front0, hipStream_t s);
constexpr int kMaxSegments = 16;  // most waves per workgroup of the march kernel
// Tau-steps the one-column stepping kernels advance per sweep over the state (1 or 2).
// With 2 the second step follows the first through every cell: its stage inputs at cell j
// need the first step's results at cells <= j only, which are in registers by then, so the
// state is read and written once per two steps.
#ifndef QS_STEPS_PER_SWEEP
#define QS_STEPS_PER_SWEEP 2
#endif
// waves per workgroup of the march kernel: for FP32 with one column per lane 16 (12 when a
// sweep takes two steps, whose carries need up to 170 registers), else 8 (the register
// budget of the larger column counts and of FP64 allows half the waves; a two-step FP64
// sweep needs up to 228)
inline int march_wg_waves(int precision, int nc) {
    return precision == QS_FP32 && nc == 1 ? (QS_STEPS_PER_SWEEP == 2 ? 12 : 16) : 8;
}
// snap_first_only: with snapshot outputs, write them for the launch's first step only, from
// the stepping kernel (a launch of several steps keeps its two-step sweeps); otherwise every
// step of the launch is written, one step per sweep.
hipError_t launch_march(int precision, int nc, bool restoring, bool fields, bool flat, int n_wg,
                        int wg_waves, bool segmented, bool snap_first_only, const StepArgs &a, hipStream_t s);
size_t march_lds_bytes(int precision, int nc, int wg_waves, bool segmented);
// resident workgroups per CU of the march kernel for this shape (-1 if the runtime cannot
// tell, e.g. without a device)
int march_wgs_per_cu(int precision, int nc, bool restoring, bool flat, int wg_waves, bool segmented);
hipError_t allow_march_lds(int precision, int nc, size_t bytes);
hipError_t launch_key_fill(int precision, void *p, int64_t n, hipStream_t s);
hipError_t launch_advance_steps(uint32_t *err, int32_t n, hipStream_t s);
hipError_t launch_guard_copy(const GuardArgs &g, hipStream_t s);
hipError_t launch_key_decode(int precision, void *p, int64_t n, hipStream_t s);
hipError_t launch_seed(int precision, int nc, int n_blocks, int max_n_xi, const SeedArgs &a,
                       hipStream_t s);

// finite-width (transverse-grid) contexts (qs_grid.hip)
struct GridCtx;
size_t grid_workspace_size(const qs_params &p);
qs_status grid_create(const qs_params &p, void *workspace, size_t ws_bytes, hipStream_t s, GridCtx **out,
                      std::string *err);
void grid_free(GridCtx *c, hipStream_t s);
qs_status grid_step(GridCtx *c, int32_t n_steps, int32_t out_every, void *ln_e, void *ln_b, void *max_ln_a,
                    hipStream_t s, std::string *err);
qs_status grid_sync_check(GridCtx *c, hipStream_t s, std::string *err);
qs_status grid_get_state(GridCtx *c, double *rho, double *jpar, double *jx, double *jy, hipStream_t s,
                         std::string *err);
qs_status grid_set_state(GridCtx *c, const double *rho, const double *jpar, const double *jx, const double *jy,
                         hipStream_t s, std::string *err);

// text returned by qs_last_error on this thread
void set_last_error(const std::string &msg);

// stream and device a surrogate network was created with (qs_mlp.hip)
hipStream_t mlp_stream(const qs_mlp *net);
int mlp_device(const qs_mlp *net);

// host helper mirroring the device SplitMix64 (exported for the generator tests)
uint64_t splitmix64_host(uint64_t seed, uint64_t i);

}  // namespace qs
