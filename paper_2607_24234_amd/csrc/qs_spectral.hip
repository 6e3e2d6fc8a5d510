// Spectral hot path for gfx950: one wavefront per block of 64 lanes, each lane owning NC
// real columns (the real and imaginary parts of a mode evolve independently because every
// coefficient below is real), marching causally in xi.
//
// Per mode the model of Sec. II (Eqs. plasma_oscillations_QSA, poisson_QSA,
// beam_continuity, beam_momentum, flux form of Sec. III.D) is written in the
// charge/current variables
//     rho,  P = j_par (on the rear face of each cell),  T = -i j_perp,
// for which, with kappa = 1/(1+k^2) and Omega(xi) = sum_s q_s^2 n0_s(xi)/m_s,
//     d_tau rho = (P_{j+1/2} - P_{j-1/2})/h + k T
//     d_tau T   = (k kappa/gamma) Omega_j n_p(centre j)
//     d_tau P   = -(kappa/gamma^3) Omega_{j+1/2} d_xi n_p(face j+1/2)
// and n_p is the response of the plasma oscillator (d_xi^2 + 1) n_p = rho, marched from
// n_p = d_xi n_p = 0 at the front with the exact propagator of a cell-constant source.
//
// All four Runge-Kutta stages of one tau-step advance together in a single sweep: the
// stage-m input at cell j needs only stage m-1 rates at cell j, which need stage m-2's
// march up to the rear face of cell j (causality in xi).  Each lane therefore carries four
// oscillator states (n_p, d_xi n_p) per column in FP64 and reads and writes the state of
// each cell once per sweep; the one-column stepping kernels take two tau-steps per sweep
// (QS_STEPS_PER_SWEEP).
#include <type_traits>

#include "qs_internal.h"

// Cells of state loads the march keeps in flight ahead of the one it computes.
#ifndef QS_PREFETCH
#define QS_PREFETCH 3
#endif

namespace qs {
namespace {

// ----------------------------------------------------------------------------- RNG
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number i of the stream whose
// state starts at `seed`.
__host__ __device__ inline uint64_t sm64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Stored values of a mode stay within [2^-R, 2^R] of 1 (largest |rho|).
template <typename TS> struct RenormRange;
template <> struct RenormRange<float> { static constexpr int R = 24; };
template <> struct RenormRange<double> { static constexpr int R = 100; };

// ----------------------------------------------------------------------------- buffer I/O
// State traffic goes through raw buffer instructions: one 128-bit descriptor per 64-lane
// block (base = the block's region, hardware bounds check against its size), a wave-
// uniform byte offset in an SGPR and one per-lane VGPR offset.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // gfx9-family raw-buffer format word

__device__ __forceinline__ rsrc_t make_rsrc(void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, kRsrcWord3);
}
template <typename T> __device__ __forceinline__ T bload(rsrc_t r, int voff, int soff);
template <> __device__ __forceinline__ float bload<float>(rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ double bload<double>(rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void bstore(float x, rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(double x, rsrc_t r, int voff, int soff) {
    using u2 = __attribute__((ext_vector_type(2))) uint32_t;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, voff, soff, 0);
}

// ----------------------------------------------------------------------------- seed
template <int NC> struct Cols;

template <typename TS, int NC>
__global__ void __launch_bounds__(256) seed_kernel(SeedArgs a, int max_n_xi) {
    const int gb = a.block_base + (int)blockIdx.x;
    const int ii = a.blk_inst[gb];
    const InstDev I = a.inst[ii];
    const int b = gb - I.block0;
    const int N = I.n_xi;
    const int lane = threadIdx.x & (kWave - 1);
    const int j = blockIdx.y * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (j >= N) return;
    const double f = a.shape[I.omega_off + j];
    TS *cell = static_cast<TS *>(a.state) + I.state_off + ((int64_t)b * N + j) * 3 * NC * kWave;
    const uint64_t inst_idx = (uint64_t)a.inst_index[ii];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int m = Cols<NC>::mode(b, lane, NC >= 2 ? c / 2 : 0);
        const int part = NC >= 2 ? (c & 1) : (lane & 1);
        double re = 0.0, im = 0.0, tre = 0.0;
        if (m < I.n_modes) {
            if (a.kind == QS_SEED_NOISE) {
                uint64_t q = (inst_idx * (uint64_t)I.n_modes + (uint64_t)m) * (uint64_t)N + (uint64_t)j;
                double u = (double)(sm64(a.rng_seed, q) >> 11) * (1.0 / 9007199254740992.0);
                double sn, cs;
                sincos(6.283185307179586476925286766559 * u, &sn, &cs);
                re = a.amp * f * cs;
                im = a.amp * f * sn;
            } else if (a.kind == QS_SEED_UNIFORM) {
                re = a.amp * f;
            } else if (a.kind == QS_SEED_FRONT_IMPULSE) {
                // d_tau rho_0 = T' = amp/h (T' = k T)
                if (j == 0) tre = a.amp / I.h;
            }
        }
        // rows: var 0 = rho, 1 = P' = j_par/h, 2 = T' = -i k j_perp
        cell[(0 * NC + c) * kWave + lane] = (TS)(part ? im : re);
        cell[(1 * NC + c) * kWave + lane] = (TS)0;
        cell[(2 * NC + c) * kWave + lane] = (TS)(part ? 0.0 : tre);
        if (j == 0 && (NC >= 2 ? part == 0 : (lane & 1) == 0)) {
            // start inside the renormalization range: rescale by the exponent of |amp|
            // when it lies outside
            int e = 0;
            const double am = fabs(a.amp);
            constexpr int R = RenormRange<TS>::R;
            if (am > 0.0 && (am > ldexp(1.0, R) || am < ldexp(1.0, -R))) (void)frexp(am, &e);
            for (int sg = 0; sg < I.n_seg; ++sg) {
                const int64_t si = I.scale_off + (int64_t)sg * I.n_blocks * Cols<NC>::MODES_PER_BLOCK + m;
                a.log2s[si] = 0;
                a.epend[si] = e;
            }
        }
    }
}

// ----------------------------------------------------------------------------- step
// Stored state (per column): rho, P' = j_par/h on the rear face of each cell, and
// T' = k T = -i k j_perp, so that
//     d_tau rho = (P'_{j+1/2} - P'_{j-1/2}) + T'
//     d_tau T'  = (k^2 kappa/gamma) Omega_j n_p(centre j)
//     d_tau P'  = -(kappa/(gamma^3 h)) Omega_{j+1/2} d_xi n_p(face j+1/2).
// The tau-step is classic RK4.  For this linear, tau-independent system its update is
// the degree-4 Taylor polynomial of exp(dtau A), evaluated here in nested form:
//     W1 = U,  W_{m+1} = U + c_m A W_m (c = dtau/4, dtau/3, dtau/2),  U' = U + dtau A W4,
// so no stage sums are kept.  The stored values of a mode are a power of two away from the
// true ones (log2s); when the largest |rho| of a mode leaves [2^-R, 2^R] the next step
// rescales it exactly (epend).
//
// TS: storage type, TC: arithmetic type of everything except the oscillator carries
// (always double).  RESTORING selects the plasma operator (d_xi^2 + 1) or d_xi^2.
// Column layout: a block is 64 lanes x NC real columns; column q = lane*NC + c of block b
// is part (q & 1) (0 = real, 1 = imaginary) of local mode b*32*NC + q/2.  With NC = 1 the
// two parts of a mode sit in adjacent lanes and are combined with a lane swap when the
// fields and the renormalization need the mode's modulus.
template <int NC> struct Cols {
    static constexpr int MPL = NC >= 2 ? NC / 2 : 1;   // modes per lane
    static constexpr int MODES_PER_BLOCK = 32 * NC;
    __device__ static int mode(int b, int lane, int t) {
        return NC >= 2 ? b * MODES_PER_BLOCK + lane * (NC / 2) + t : b * MODES_PER_BLOCK + (lane >> 1);
    }
    __device__ static int col(int t, int part) { return NC >= 2 ? 2 * t + part : 0; }
};

// value of the neighbouring lane (lane ^ 1) through a DPP quad permutation [1, 0, 3, 2]
__device__ __forceinline__ float lane_swap(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_swap(double x) {
    const int2 v = __builtin_bit_cast(int2, x);
    int2 r;
    r.x = __builtin_amdgcn_update_dpp(0, v.x, 0xB1, 0xF, 0xF, false);
    r.y = __builtin_amdgcn_update_dpp(0, v.y, 0xB1, 0xF, 0xF, false);
    return __builtin_bit_cast(double, r);
}
template <typename TC> __device__ __forceinline__ TC pair_sum(TC x) { return x + lane_swap(x); }
template <typename TC> __device__ __forceinline__ TC pair_max(TC x) {
    const TC y = lane_swap(x);
    return (y > x || !(y <= y)) ? y : x;
}

// ------------------------------------------------------------- max over segments
// Order-preserving integer keys of floating-point values: max of keys = key of the max, so
// segments of one mode combine their maxima with integer atomics in any order.
__device__ __forceinline__ uint32_t fkey(float x) {
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float funkey(uint32_t k) {
    return __builtin_bit_cast(float, (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}
__device__ __forceinline__ uint64_t fkey(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double funkey(uint64_t k) {
    return __builtin_bit_cast(double, (k & 0x8000000000000000ull) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k);
}
__device__ __forceinline__ void atomic_max_key(float *dst, float v) {
    atomicMax(reinterpret_cast<unsigned int *>(dst), fkey(v));
}
__device__ __forceinline__ void atomic_max_key(double *dst, double v) {
    atomicMax(reinterpret_cast<unsigned long long *>(dst), (unsigned long long)fkey(v));
}

// ----------------------------------------------------------------------------- march
// One workgroup per 64-lane block of modes, one wave per xi-segment of that block.  Wave s
// owns cells [s*seg_len, min(N, (s+1)*seg_len)) and runs every tau-step of the launch on
// them; at a segment boundary it hands the four stage carries (n_p, d_xi n_p) and the stage
// inputs of P' at the boundary face to wave s+1 through LDS.  Wave s+1 can start step n as
// soon as wave s has finished step n on its cells, so the segments of one block pipeline
// over tau-steps (tau-skew).  Each (mode, segment) keeps its own power-of-two scale: carries
// crossing a boundary are rescaled exactly by the difference of the two exponents.
//
// LDS layout (dynamic): int ready[16], taken[16], abort, 3 pad; then per boundary w (0..S-2)
// the payload: per step of a sweep (slot s) double Y[4][NC][64], V[4][NC][64], TC PP[4][NC][64];
// then int32 LL[MPL][64].  The flags count sweeps.
constexpr int kMaxSeg = 16;
constexpr int kFlagInts = 2 * kMaxSeg + 4;
constexpr int kSweepSlots = QS_STEPS_PER_SWEEP;

template <typename TC, int NC>
struct Payload {
    static constexpr int MPL = NC >= 2 ? NC / 2 : 1;
    static constexpr int SLOT = kWave * (8 * NC * 8 + 4 * NC * (int)sizeof(TC));
    static constexpr int BYTES = kSweepSlots * SLOT + kWave * MPL * 4;
    __device__ static double *Y(char *p, int s) { return reinterpret_cast<double *>(p + s * SLOT); }
    __device__ static double *V(char *p, int s) { return reinterpret_cast<double *>(p + s * SLOT) + 4 * NC * kWave; }
    __device__ static TC *PP(char *p, int s) { return reinterpret_cast<TC *>(p + s * SLOT + 8 * NC * kWave * 8); }
    __device__ static int32_t *LL(char *p) { return reinterpret_cast<int32_t *>(p + kSweepSlots * SLOT); }
};

// Wait until *flag >= target (LDS, same workgroup).  Gives up (false) when another wave of
// the workgroup gave up (*abort set) or after `ticks` of the constant-rate wall clock, and
// then sets *abort so that every other waiting wave of the workgroup stops too.
__device__ __forceinline__ bool wait_flag(int *flag, int target, int *abort, uint64_t ticks) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return false;
        if (wall_clock64() - t0 > ticks) {
            __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Snapshot forms of the march: none; every step of the launch (with one column per lane the
// sweeps keep two steps and write the fields of both; one step per sweep otherwise); the
// launch's first step only, inside the stepping kernel (its sweeps keep their step count).
constexpr int kSnapNone = 0, kSnapEvery = 1, kSnapFirst = 2;

template <typename TS, typename TC, int NC, bool RESTORING, bool FIELDS, int SNAP, bool FLAT>
__global__ void __launch_bounds__(sizeof(TS) == 4 && NC == 1 ? (kSweepSlots == 2 ? 768 : 1024) : 512)
__attribute__((amdgpu_waves_per_eu(NC == 1 ? (sizeof(TS) == 8 ? (kSweepSlots == 2 ? 2 : 4) : (kSweepSlots == 2 ? 3 : 5)) : 1)))
march_kernel(StepArgs a) {
    using CL = Cols<NC>;
    using PL = Payload<TC, NC>;
    constexpr int MPL = CL::MPL;
    constexpr int ROW = 3 * NC;        // rows of 64 values per cell
    extern __shared__ __align__(16) char lds[];
    int *ready = reinterpret_cast<int *>(lds);
    int *taken = ready + kMaxSeg;
    int *abort = ready + 2 * kMaxSeg;
    char *payload = lds + kFlagInts * sizeof(int);

    // wave slot -> (block, segment) from the packing table; slots of one block's segments
    // are consecutive, so the hand-off of slot w goes to slot w+1
    const int slot = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);  // wave-uniform
    const int lane = (int)threadIdx.x % kWave;
    if (threadIdx.x < kFlagInts) ready[threadIdx.x] = 0;  // also clears taken[] and abort
    __syncthreads();
    const int2 ent = a.wave_table[(int64_t)blockIdx.x * (blockDim.x / kWave) + slot];
    if (ent.x < 0) return;  // idle slot
    const int gb = ent.x, wave = ent.y;  // global block, segment index
    const int ii = a.blk_inst[gb];
    const InstDev I = a.inst[ii];
    const int b = gb - I.block0;

    const int N = I.n_xi;
    const int c0 = wave * I.seg_len;
    const int c1 = min(N, c0 + I.seg_len);
    const bool has_next = wave + 1 < I.n_seg;
    const bool steady = (I.flags & QS_FLAG_STEADY_INFLOW) != 0;
    const bool stationary = (I.flags & QS_FLAG_STATIONARY_FRONT) != 0;
    const bool writer = NC >= 2 || (lane & 1) == 0;   // lane that writes per-mode results

    TC cT[MPL], cP[MPL], kap2[MPL], k2kap2[MPL];
    int32_t L[MPL], ep[MPL];
    int mloc[MPL];
    int64_t sidx[MPL];  // index of this (mode, segment) in the scale arrays
#pragma unroll
    for (int t = 0; t < MPL; ++t) {
        mloc[t] = CL::mode(b, lane, t);
        const double k = a.kmode[I.pmode0 + mloc[t]];
        const double kp = 1.0 / (1.0 + k * k);
        kap2[t] = (TC)(kp * kp);
        k2kap2[t] = (TC)(k * k * kp * kp);
        cT[t] = (TC)a.coef[2 * (I.pmode0 + mloc[t])];
        cP[t] = (TC)a.coef[2 * (I.pmode0 + mloc[t]) + 1];
        sidx[t] = I.scale_off + (int64_t)wave * I.n_blocks * CL::MODES_PER_BLOCK + mloc[t];
        L[t] = a.log2s[sidx[t]];
        ep[t] = a.epend[sidx[t]];
    }
    const TC c1s = (TC)(0.25 * I.dtau), c2s = (TC)(I.dtau / 3.0), c3s = (TC)(0.5 * I.dtau);
    const TC dt = (TC)I.dtau;
    const double C1 = I.c1, S1 = I.s1, C2 = I.c2, S2 = I.s2, h = I.h;

    // Omega at centres then faces; a flat profile has one value (the last face carries 0)
    const TC *omc = static_cast<const TC *>(a.omega) + I.omega_off;
    const rsrc_t ro = make_rsrc(const_cast<TC *>(omc), (uint32_t)(2 * N * sizeof(TC)));
    const TC om0 = omc[0];

    // this block's region of the state: [cell][row][lane] of TS
    TS *blk = static_cast<TS *>(a.state) + I.state_off + (int64_t)b * N * ROW * kWave;
    const rsrc_t rs = make_rsrc(blk, (uint32_t)((int64_t)N * ROW * kWave * sizeof(TS)));
    const int voff = lane * (int)sizeof(TS);
    constexpr int RB = kWave * (int)sizeof(TS);  // bytes per row
    constexpr int XW = ROW + (FLAT ? 0 : 2);
    auto ldx = [&](int j, TS (&x)[XW]) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < ROW; ++r) x[r] = bload<TS>(rs, voff, (j * ROW + r) * RB);
        if (!FLAT) {
            x[ROW] = (TS)bload<TC>(ro, 0, j * (int)sizeof(TC));
            x[ROW + 1] = (TS)bload<TC>(ro, 0, (N + j) * (int)sizeof(TC));
        }
    };

    // steps one sweep can take: two for the stepping kernels with one column per lane, where
    // the second step's carries still fit the register budget; one otherwise
    constexpr int NS = NC == 1 ? kSweepSlots : 1;
    double y[NS][4][NC], v[NS][4][NC];  // per step of the sweep and stage: n_p and d_xi n_p at the front face
    TC pp[NS][4][NC];                   // stage inputs of P' at the front face of the current cell
    TC scale[MPL], rmax[MPL], a2max[NS][MPL];
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;

    int64_t snap_row = a.snap_base;  // snapshot of the sweep's first step (kSnapEvery: the next at + snap_stride)
    bool snap_now = SNAP == kSnapEvery;  // kSnapFirst: the first sweep's first step

    // One segment pass of a sweep of K tau-steps: per cell, all four stages of each step, the
    // fields of the state at the step's start (stage-1 values) and the update.
    // init_front: the pass starts at the beam front with a steady or stationary front
    // condition: n_p ahead of the beam is cell 0's current stage value (steady) or held at
    // cell 0's charge density at tau = 0, in this sweep's units (stationary); d_xi n_p = 0
    auto pass = [&](const bool init_front, auto steps) __attribute__((always_inline)) {
        constexpr int K = decltype(steps)::value;
        // step `slot` of the sweep at cell j from its stage-1 values u (TC, pending power of
        // two applied) and Omega at the centre and the rear face: fields, and the updated
        // values un rounded to the storage type
        auto step_cell = [&](const int j, const TC (&u)[3][NC], const TC Oc, const TC Of, TS (&un)[3][NC],
                             auto first, auto slot) __attribute__((always_inline)) {
            constexpr bool FIRST = decltype(first)::value;
            constexpr int sl = decltype(slot)::value;
            const TC(&r0)[NC] = u[0];
            const TC(&P0)[NC] = u[1];
            const TC(&T0)[NC] = u[2];
            TC cTO[NC], cPO[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int t = NC >= 2 ? c / 2 : 0;
                cTO[c] = cT[t] * Oc;
                cPO[c] = cP[t] * Of;
            }
            TC dr[NC], dT[NC], dP[NC];   // A W_m at this cell
            TC ncf0[NC], vcf0[NC];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const TC cm = (m == 1) ? c1s : (m == 2 ? c2s : c3s);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const TC rm = (m == 0) ? r0[c] : r0[c] + cm * dr[c];
                    const TC Pm = (m == 0) ? P0[c] : P0[c] + cm * dP[c];
                    const TC Tm = (m == 0) ? T0[c] : T0[c] + cm * dT[c];
                    const double rd = (double)rm;
                    double &ym = y[sl][m][c], &vm = v[sl][m][c];
                    if (FIRST && init_front) {
                        ym = steady ? rd
                                    : a.front0[((int64_t)gb * NC + c) * kWave + lane] * ldexp(1.0, -L[NC >= 2 ? c / 2 : 0]);
                        vm = 0.0;
                    }
                    double nc, yn, vn, vc;
                    if (RESTORING) {
                        const double uu = ym - rd;
                        nc = rd + C2 * uu + S2 * vm;
                        yn = rd + C1 * uu + S1 * vm;
                        vn = C1 * vm - S1 * uu;
                        if (FIELDS && m == 0) vc = C2 * vm - S2 * uu;
                    } else {
                        nc = ym + 0.5 * h * vm + 0.125 * h * h * rd;
                        yn = ym + h * vm + 0.5 * h * h * rd;
                        vn = vm + h * rd;
                        if (FIELDS && m == 0) vc = vm + 0.5 * h * rd;
                    }
                    ym = yn;
                    vm = vn;
                    if (FIELDS && m == 0) { ncf0[c] = (TC)nc; vcf0[c] = (TC)vc; }
                    dr[c] = (Pm - pp[sl][m][c]) + Tm;
                    pp[sl][m][c] = Pm;
                    dT[c] = cTO[c] * (TC)nc;
                    dP[c] = cPO[c] * (TC)vn;
                }
            }
            if (FIELDS) {
#pragma unroll
                for (int t = 0; t < MPL; ++t) {
                    // |E_par|^2 = kappa^2 |n_p'|^2, |E_perp|^2 = k^2 kappa^2 |rho - n_p|^2,
                    // |B_perp|^2 = k^2 kappa^2 |rho|^2, summed over the two parts of the mode
                    const bool snap_here = SNAP == kSnapEvery || (SNAP == kSnapFirst && sl == 0 && snap_now);
                    TC e2 = (TC)0, b2 = (TC)0, a2;
                    if (NC >= 2) {
                        const int ca = 2 * t, cb = 2 * t + 1;
                        const TC en = vcf0[ca] * vcf0[ca] + vcf0[cb] * vcf0[cb];
                        const TC d0 = r0[ca] - ncf0[ca], d1 = r0[cb] - ncf0[cb];
                        e2 = kap2[t] * en + k2kap2[t] * (d0 * d0 + d1 * d1);
                        b2 = k2kap2[t] * (r0[ca] * r0[ca] + r0[cb] * r0[cb]);
                        a2 = e2 + b2;
                    } else {
                        const TC d0 = r0[0] - ncf0[0];
                        if (snap_here) {
                            e2 = pair_sum(kap2[0] * vcf0[0] * vcf0[0] + k2kap2[0] * d0 * d0);
                            b2 = pair_sum(k2kap2[0] * r0[0] * r0[0]);
                            a2 = e2 + b2;
                        } else {
                            // A^2 alone: one sum over the mode's two lanes
                            a2 = pair_sum(kap2[0] * vcf0[0] * vcf0[0] + k2kap2[0] * (d0 * d0 + r0[0] * r0[0]));
                        }
                    }
                    a2max[sl][t] = a2 > a2max[sl][t] ? a2 : a2max[sl][t];
                    if (snap_here) {
                        // snapshot option: |F_perp|^2 = k^2 kappa^2 |n_p|^2 in place of |E|^2
                        TC s2 = e2;
                        if (I.flags & QS_FLAG_FPERP_SNAPSHOTS) {
                            if (NC >= 2) s2 = k2kap2[t] * (ncf0[2 * t] * ncf0[2 * t] + ncf0[2 * t + 1] * ncf0[2 * t + 1]);
                            else s2 = pair_sum(k2kap2[0] * ncf0[0] * ncf0[0]);
                        }
                        if (mloc[t] < I.n_modes && j >= I.snap_first) {
                            const double sh = (double)L[t] * 0.69314718055994530942;
                            const int64_t o = snap_row + (SNAP == kSnapEvery ? sl * a.snap_stride : 0) + I.snap_off +
                                              (int64_t)(j - I.snap_first) * I.snap_ld + mloc[t];
                            if (NC >= 2) {
                                static_cast<TS *>(a.ln_e)[o] = (TS)(0.5 * (double)log(s2) + sh);
                                static_cast<TS *>(a.ln_b)[o] = (TS)(0.5 * (double)log(b2) + sh);
                            } else {
                                // the mode's two lanes hold the same sums: the even lane writes
                                // ln|E|, the odd one ln|B|, in one store
                                const bool odd = (lane & 1) != 0;
                                TS *dst = static_cast<TS *>(odd ? a.ln_b : a.ln_e);
                                dst[o] = (TS)(0.5 * (double)log(odd ? b2 : s2) + sh);
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                un[0][c] = (TS)(r0[c] + dt * dr[c]);
                un[1][c] = (TS)(P0[c] + dt * dP[c]);
                un[2][c] = (TS)(T0[c] + dt * dT[c]);
            }
        };
        auto cell = [&](const int j, const TS (&x)[XW], auto first) __attribute__((always_inline)) {
            const bool last = (j == N - 1);
            const TC Oc = FLAT ? om0 : (TC)x[ROW];
            const TC Of = last ? (TC)0 : (FLAT ? om0 : (TC)x[ROW + 1]);
            TC u[3][NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int t = NC >= 2 ? c / 2 : 0;
                // stored values times the pending exact power of two (1 when none)
#pragma unroll
                for (int r = 0; r < 3; ++r) u[r][c] = (TC)x[r * NC + c] * scale[t];
            }
            TS un[3][NC];
            step_cell(j, u, Oc, Of, un, first, I0{});
            if constexpr (K == 2) {
                // the second step of the sweep starts from the first one's stored values
                TC u2[3][NC];
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < NC; ++c) u2[r][c] = (TC)un[r][c];
                step_cell(j, u2, Oc, Of, un, first, std::integral_constant<int, NS - 1>{});
            }
            if (a.update) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const int t = NC >= 2 ? c / 2 : 0;
#pragma unroll
                    for (int r = 0; r < 3; ++r) bstore(un[r][c], rs, voff, (j * ROW + r * NC + c) * RB);
                    const TC ar = (TC)fabs((TC)un[0][c]);
                    rmax[t] = (ar > rmax[t] || !(ar <= ar)) ? ar : rmax[t];  // NaN sticks
                }
            }
        };
        // Cell c0 first (it may carry the front condition), then c0+1..c1-1 with the loads
        // of cell j+D issued before cell j is computed, into a ring of D+1 register sets
        // indexed by compile-time constants (the loop is unrolled D+1 times), so neither
        // the buffers nor the carries are copied at the loop edge and every wait covers only
        // the oldest loads.  Loads past the end of the block's region are bounds-checked by
        // the descriptor (0 returned, unused).
        using first_t = std::integral_constant<bool, true>;
        using rest_t = std::integral_constant<bool, false>;
        // a two-step sweep computes twice per cell loaded: two cells in flight suffice
        constexpr int D = (K == 2 && QS_PREFETCH > 2) ? 2 : QS_PREFETCH;
        TS xs[D + 1][XW];
#pragma unroll
        for (int d = 0; d <= D; ++d) ldx(c0 + d, xs[d]);
        cell(c0, xs[0], first_t{});
        int j = c0 + 1;
        // whole groups of D+1 cells: ring slot (k+1) mod (D+1) holds cell j+k
        for (; j + D < c1; j += D + 1) {
#pragma unroll
            for (int k = 0; k <= D; ++k) {
                ldx(j + k + D, xs[k]);
                cell(j + k, xs[(k + 1) % (D + 1)], rest_t{});
            }
        }
        // the last (at most D) cells are already loaded
#pragma unroll
        for (int k = 0; k < D; ++k)
            if (j + k < c1) cell(j + k, xs[(k + 1) % (D + 1)], rest_t{});
    };

    constexpr int R = RenormRange<TS>::R;
    int sweeps = 0;   // sweeps done; the hand-off flags count these
    for (int n = 0; n < a.n_steps; ++sweeps) {
        // steps of this sweep: two while at least two remain (stepping kernels only)
        const int k = (NS == 2 && a.update && n + 1 < a.n_steps) ? 2 : 1;
        snap_row = a.snap_base + (int64_t)n * a.snap_stride;
        if (SNAP == kSnapFirst) snap_now = n == 0;
        // apply the pending renormalization of each (mode, segment): this sweep's loads are
        // multiplied by 2^-e; a fields-only launch (no update) reads the stored values with
        // their current exponent
#pragma unroll
        for (int t = 0; t < MPL; ++t) {
            scale[t] = (TC)1;
            if (a.update) {
                L[t] += ep[t];
                scale[t] = (TC)ldexp(1.0, -ep[t]);
            }
            rmax[t] = (TC)0;
#pragma unroll
            for (int sl = 0; sl < NS; ++sl) a2max[sl][t] = (TC)0;
        }
        // carries at the segment's front face: zero at the beam front (unperturbed plasma; the
        // steady and stationary front conditions set n_p at the first cell), else from wave-1
        if (wave == 0) {
#pragma unroll
            for (int sl = 0; sl < NS; ++sl)
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int c = 0; c < NC; ++c) { y[sl][m][c] = 0.0; v[sl][m][c] = 0.0; pp[sl][m][c] = (TC)0; }
        } else {
            if (!wait_flag(&ready[slot - 1], sweeps + 1, abort, a.wait_ticks)) { a.err[1] = 1u; return; }
            char *pl = payload + (slot - 1) * PL::BYTES;
#pragma unroll
            for (int t = 0; t < MPL; ++t) {
                const int lp = PL::LL(pl)[t * kWave + lane];
                const double f = ldexp(1.0, lp - L[t]);  // predecessor units -> ours (exact)
#pragma unroll
                for (int sl = 0; sl < NS; ++sl) {
                    if (sl >= k) break;
#pragma unroll
                    for (int m = 0; m < 4; ++m)
#pragma unroll
                        for (int p = 0; p < (NC >= 2 ? 2 : 1); ++p) {
                            const int c = NC >= 2 ? 2 * t + p : 0;
                            y[sl][m][c] = PL::Y(pl, sl)[(m * NC + c) * kWave + lane] * f;
                            v[sl][m][c] = PL::V(pl, sl)[(m * NC + c) * kWave + lane] * f;
                            pp[sl][m][c] = PL::PP(pl, sl)[(m * NC + c) * kWave + lane] * (TC)f;
                        }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) __hip_atomic_store(&taken[slot - 1], sweeps + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if constexpr (NS == 2) {
            if (k == 2) pass(wave == 0 && (steady || stationary), std::integral_constant<int, 2>{});
            else pass(wave == 0 && (steady || stationary), std::integral_constant<int, 1>{});
        } else {
            pass(wave == 0 && (steady || stationary), std::integral_constant<int, 1>{});
        }

        // hand the carries at this segment's rear face to the next segment
        if (has_next) {
            if (!wait_flag(&taken[slot], sweeps, abort, a.wait_ticks)) { a.err[1] = 1u; return; }
            char *pl = payload + slot * PL::BYTES;
#pragma unroll
            for (int sl = 0; sl < NS; ++sl) {
                if (sl >= k) break;
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        PL::Y(pl, sl)[(m * NC + c) * kWave + lane] = y[sl][m][c];
                        PL::V(pl, sl)[(m * NC + c) * kWave + lane] = v[sl][m][c];
                        PL::PP(pl, sl)[(m * NC + c) * kWave + lane] = pp[sl][m][c];
                    }
            }
#pragma unroll
            for (int t = 0; t < MPL; ++t) PL::LL(pl)[t * kWave + lane] = L[t];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) __hip_atomic_store(&ready[slot], sweeps + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }

#pragma unroll
        for (int t = 0; t < MPL; ++t) {
            if (NC == 1) rmax[t] = pair_max(rmax[t]);
            if (FIELDS && a.max_ln_a && writer && mloc[t] < I.n_modes) {
                const double sh = (double)L[t] * 0.69314718055994530942;
#pragma unroll
                for (int sl = 0; sl < NS; ++sl) {
                    if (sl >= k) break;
                    const TS val = (TS)(0.5 * (double)log(a2max[sl][t]) + sh);
                    TS *dst = static_cast<TS *>(a.max_ln_a) + a.max_base + (int64_t)(n + sl) * a.total_modes + I.mode0 + mloc[t];
                    if (a.keyed) atomic_max_key(dst, val);
                    else *dst = val;
                }
            }
            int e = 0;
            if (a.update) {
                const double mx = (double)rmax[t];
                if (!isfinite(mx)) {
                    if (writer) {
                        const uint32_t pm = (uint32_t)(I.pmode0 + mloc[t]);
                        a.err[0] = 1u + pm;
                        // the step after which the stored state is non-finite; the first
                        // (lowest step, then mode) wins through a max of complements
                        const int64_t step = *reinterpret_cast<const int64_t *>(a.err + 4) + n + k;
                        atomicMax(reinterpret_cast<unsigned long long *>(a.err + 2),
                                  ~(((unsigned long long)step << 32) | pm));
                    }
                } else if (mx > 0.0 && (mx > ldexp(1.0, R) || mx < ldexp(1.0, -R))) {
                    (void)frexp(mx, &e);
                }
            }
            ep[t] = e;
        }
        n += k;
    }
    if (a.update) {
#pragma unroll
        for (int t = 0; t < MPL; ++t) {
            if (!writer) continue;
            a.log2s[sidx[t]] = L[t];
            a.epend[sidx[t]] = ep[t];
        }
    }
}

template <typename TS>
__global__ void __launch_bounds__(256) key_fill(TS *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const auto k = fkey((TS)-INFINITY);
        p[i] = __builtin_bit_cast(TS, k);
    }
}
template <typename TS>
__global__ void __launch_bounds__(256) key_decode(TS *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        using K = decltype(fkey((TS)0));
        p[i] = funkey(__builtin_bit_cast(K, p[i]));
    }
}

template <typename TS, typename TC, int NC, bool RESTORING>
hipError_t launch_march_r(bool fields, int snap, bool flat, int n_wg, int wg_waves, bool segmented,
                          const StepArgs &a, hipStream_t s) {
    dim3 grid(n_wg), block(kWave * wg_waves);
    const size_t lds = march_lds_bytes(sizeof(TS) == 8 ? QS_FP64 : QS_FP32, NC, wg_waves, segmented);
#define QS_LAUNCH(F, S, FL) hipLaunchKernelGGL((march_kernel<TS, TC, NC, RESTORING, F, S, FL>), grid, block, lds, s, a)
    // the first-step form exists where sweeps take two steps (one column per lane)
    if (NC != 1 && snap == kSnapFirst) snap = kSnapEvery;
    if (flat) {
        if (snap == kSnapEvery) QS_LAUNCH(true, kSnapEvery, true);
        else if (snap == kSnapFirst) QS_LAUNCH(true, NC == 1 ? kSnapFirst : kSnapEvery, true);
        else if (fields) QS_LAUNCH(true, kSnapNone, true);
        else QS_LAUNCH(false, kSnapNone, true);
    } else {
        if (snap == kSnapEvery) QS_LAUNCH(true, kSnapEvery, false);
        else if (snap == kSnapFirst) QS_LAUNCH(true, NC == 1 ? kSnapFirst : kSnapEvery, false);
        else if (fields) QS_LAUNCH(true, kSnapNone, false);
        else QS_LAUNCH(false, kSnapNone, false);
    }
#undef QS_LAUNCH
    return hipGetLastError();
}

template <typename TS, typename TC, int NC>
hipError_t launch_march_t(bool restoring, bool fields, int snap, bool flat, int n_wg, int wg_waves,
                          bool segmented, const StepArgs &a, hipStream_t s) {
    if (restoring) return launch_march_r<TS, TC, NC, true>(fields, snap, flat, n_wg, wg_waves, segmented, a, s);
    return launch_march_r<TS, TC, NC, false>(fields, snap, flat, n_wg, wg_waves, segmented, a, s);
}

// rho of cell 0 of every column: the front value of the stationary front condition
template <typename TS, int NC>
__global__ void __launch_bounds__(256) front_capture(const TS *__restrict__ state, const int32_t *__restrict__ blk_inst,
                                                     const InstDev *__restrict__ inst, int n_blocks,
                                                     double *__restrict__ front0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_blocks * NC * kWave) return;
    const int gb = (int)(i / (NC * kWave));
    const int c = (int)(i / kWave) % NC, lane = (int)(i % kWave);
    const InstDev I = inst[blk_inst[gb]];
    const int b = gb - I.block0;
    front0[i] = (double)state[I.state_off + (int64_t)b * I.n_xi * 3 * NC * kWave + (int64_t)c * kWave + lane];
}

template <typename TC>
__global__ void __launch_bounds__(256) flat_tables(const FlatTable *__restrict__ ft, double *__restrict__ shape,
                                                   TC *__restrict__ omega) {
    const FlatTable F = ft[blockIdx.x];
    const int64_t n2 = 2 * (int64_t)F.n;
    for (int64_t j = threadIdx.x; j < n2; j += blockDim.x) {
        shape[F.off + j] = j < F.n ? 1.0 : 0.0;
        omega[F.off + j] = (TC)(j + 1 < n2 ? F.q2nm : 0.0);   // the last face is the outer one
    }
}

template <typename TS, int NC>
hipError_t launch_seed_t(int n_blocks, int max_n_xi, const SeedArgs &a, hipStream_t s) {
    constexpr int kCellsPerWg = 4;
    dim3 grid(n_blocks, (max_n_xi + kCellsPerWg - 1) / kCellsPerWg), block(kCellsPerWg * kWave);
    hipLaunchKernelGGL((seed_kernel<TS, NC>), grid, block, 0, s, a, max_n_xi);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_flat_tables(int precision, const FlatTable *ft, int n, double *shape, void *omega, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (precision == QS_FP64)
        hipLaunchKernelGGL(flat_tables<double>, dim3(n), dim3(256), 0, s, ft, shape, static_cast<double *>(omega));
    else
        hipLaunchKernelGGL(flat_tables<float>, dim3(n), dim3(256), 0, s, ft, shape, static_cast<float *>(omega));
    return hipGetLastError();
}

hipError_t launch_front_capture(int precision, int nc, const void *state, const int32_t *blk_inst,
                                const InstDev *inst, int n_blocks, double *front0, hipStream_t s) {
    const int64_t n = (int64_t)n_blocks * nc * kWave;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (precision == QS_FP64) {
        if (nc == 1) hipLaunchKernelGGL((front_capture<double, 1>), grid, block, 0, s, static_cast<const double *>(state), blk_inst, inst, n_blocks, front0);
        else hipLaunchKernelGGL((front_capture<double, 2>), grid, block, 0, s, static_cast<const double *>(state), blk_inst, inst, n_blocks, front0);
    } else {
        if (nc == 1) hipLaunchKernelGGL((front_capture<float, 1>), grid, block, 0, s, static_cast<const float *>(state), blk_inst, inst, n_blocks, front0);
        else hipLaunchKernelGGL((front_capture<float, 2>), grid, block, 0, s, static_cast<const float *>(state), blk_inst, inst, n_blocks, front0);
    }
    return hipGetLastError();
}

size_t march_lds_bytes(int precision, int nc, int wg_waves, bool segmented) {
    if (!segmented) return kFlagInts * sizeof(int);  // no hand-offs: the flags only
    size_t pay;
    if (precision == QS_FP64) pay = nc == 1 ? Payload<double, 1>::BYTES : Payload<double, 2>::BYTES;
    else pay = nc == 1 ? Payload<float, 1>::BYTES : Payload<float, 2>::BYTES;
    return kFlagInts * sizeof(int) + (size_t)(wg_waves - 1) * pay;
}

hipError_t launch_march(int precision, int nc, bool restoring, bool fields, bool flat, int n_wg,
                        int wg_waves, bool segmented, bool snap_first_only, const StepArgs &a, hipStream_t s) {
    const int snap = a.ln_e == nullptr ? kSnapNone : (snap_first_only ? kSnapFirst : kSnapEvery);
    if (wg_waves < 1 || wg_waves > march_wg_waves(precision, nc)) return hipErrorInvalidConfiguration;
    if (precision == QS_FP64) {
        if (nc == 1) return launch_march_t<double, double, 1>(restoring, fields, snap, flat, n_wg, wg_waves, segmented, a, s);
        return launch_march_t<double, double, 2>(restoring, fields, snap, flat, n_wg, wg_waves, segmented, a, s);
    }
    if (nc == 1) return launch_march_t<float, float, 1>(restoring, fields, snap, flat, n_wg, wg_waves, segmented, a, s);
    return launch_march_t<float, float, 2>(restoring, fields, snap, flat, n_wg, wg_waves, segmented, a, s);
}

int march_wgs_per_cu(int precision, int nc, bool restoring, bool flat, int wg_waves, bool segmented) {
    // occupancy of the variant that steps with per-step maxima (fields, no snapshot)
    const size_t lds = march_lds_bytes(precision, nc, wg_waves, segmented);
    const void *f = nullptr;
#define QS_PICK(TS, TC, NCc)                                                                          \
    f = restoring ? (flat ? reinterpret_cast<const void *>(&march_kernel<TS, TC, NCc, true, true, kSnapNone, true>)   \
                          : reinterpret_cast<const void *>(&march_kernel<TS, TC, NCc, true, true, kSnapNone, false>)) \
                  : (flat ? reinterpret_cast<const void *>(&march_kernel<TS, TC, NCc, false, true, kSnapNone, true>)  \
                          : reinterpret_cast<const void *>(&march_kernel<TS, TC, NCc, false, true, kSnapNone, false>));
    if (precision == QS_FP64) {
        if (nc == 1) { QS_PICK(double, double, 1) } else { QS_PICK(double, double, 2) }
    } else {
        if (nc == 1) { QS_PICK(float, float, 1) } else { QS_PICK(float, float, 2) }
    }
#undef QS_PICK
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kWave * wg_waves, lds) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return n;
}

hipError_t allow_march_lds(int precision, int nc, size_t bytes) {
    // kernels that need more than the default dynamic LDS must opt in
#define QS_ALLOW(TS, TC, NCc, R, F, S, FL) \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&march_kernel<TS, TC, NCc, R, F, S, FL>), \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes); \
    if (e != hipSuccess) return e;
#define QS_ALLOW_R(TS, TC, NCc, R) \
    QS_ALLOW(TS, TC, NCc, R, true, kSnapEvery, true) QS_ALLOW(TS, TC, NCc, R, true, kSnapNone, true) \
    QS_ALLOW(TS, TC, NCc, R, false, kSnapNone, true) QS_ALLOW(TS, TC, NCc, R, true, kSnapEvery, false) \
    QS_ALLOW(TS, TC, NCc, R, true, kSnapNone, false) QS_ALLOW(TS, TC, NCc, R, false, kSnapNone, false)
#define QS_ALLOW_ALL(TS, TC, NCc) QS_ALLOW_R(TS, TC, NCc, true) QS_ALLOW_R(TS, TC, NCc, false)
#define QS_ALLOW_FIRST(TS, TC) \
    QS_ALLOW(TS, TC, 1, true, true, kSnapFirst, true) QS_ALLOW(TS, TC, 1, true, true, kSnapFirst, false) \
    QS_ALLOW(TS, TC, 1, false, true, kSnapFirst, true) QS_ALLOW(TS, TC, 1, false, true, kSnapFirst, false)
    hipError_t e = hipSuccess;
    if (precision == QS_FP64) {
        if (nc == 1) { QS_ALLOW_ALL(double, double, 1) QS_ALLOW_FIRST(double, double) } else { QS_ALLOW_ALL(double, double, 2) }
    } else {
        if (nc == 1) { QS_ALLOW_ALL(float, float, 1) QS_ALLOW_FIRST(float, float) } else { QS_ALLOW_ALL(float, float, 2) }
    }
#undef QS_ALLOW_FIRST
#undef QS_ALLOW_ALL
#undef QS_ALLOW_R
#undef QS_ALLOW
    return e;
}

// The device's step counter advances after each stepping launch (a kernel node, so that
// replays of a captured step sequence count their steps too).
__global__ void advance_steps(uint32_t *err, int32_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *reinterpret_cast<int64_t *>(err + 4) += n;
}

// Rollback guard: copy the state regions unless an error is pending (then the guard keeps
// the last good copy); the first thread records the step count of the copy.
__global__ void __launch_bounds__(256) guard_copy(GuardArgs g) {
    if (g.err[0] != 0u || g.err[1] != 0u) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int r = 0; r < 3; ++r)
        for (int64_t i = t0; i < g.n16[r]; i += stride) g.dst[r][i] = g.src[r][i];
    if (t0 == 0) g.meta[0] = *reinterpret_cast<const int64_t *>(g.err + 4);
}

hipError_t launch_advance_steps(uint32_t *err, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL(advance_steps, dim3(1), dim3(64), 0, s, err, n);
    return hipGetLastError();
}

hipError_t launch_guard_copy(const GuardArgs &g, hipStream_t s) {
    hipLaunchKernelGGL(guard_copy, dim3(2048), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_key_fill(int precision, void *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (precision == QS_FP64) hipLaunchKernelGGL(key_fill<double>, grid, block, 0, s, static_cast<double *>(p), n);
    else hipLaunchKernelGGL(key_fill<float>, grid, block, 0, s, static_cast<float *>(p), n);
    return hipGetLastError();
}

hipError_t launch_key_decode(int precision, void *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (precision == QS_FP64) hipLaunchKernelGGL(key_decode<double>, grid, block, 0, s, static_cast<double *>(p), n);
    else hipLaunchKernelGGL(key_decode<float>, grid, block, 0, s, static_cast<float *>(p), n);
    return hipGetLastError();
}

hipError_t launch_seed(int precision, int nc, int n_blocks, int max_n_xi, const SeedArgs &a,
                       hipStream_t s) {
    if (precision == QS_FP64) {
        if (nc == 1) return launch_seed_t<double, 1>(n_blocks, max_n_xi, a, s);
        return launch_seed_t<double, 2>(n_blocks, max_n_xi, a, s);
    }
    if (nc == 1) return launch_seed_t<float, 1>(n_blocks, max_n_xi, a, s);
    return launch_seed_t<float, 2>(n_blocks, max_n_xi, a, s);
}

uint64_t splitmix64_host(uint64_t seed, uint64_t i) { return sm64(seed, i); }

}  // namespace qs
