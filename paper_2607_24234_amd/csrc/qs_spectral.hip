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
// each cell exactly once per tau-step.
#include <type_traits>

#include "qs_internal.h"

// Tuning knobs of the step kernel (compile time): cells per register tile and the
// occupancy the register allocator targets (waves per SIMD).
#ifndef QS_STEP_TJ
#define QS_STEP_TJ 2
#endif
// waves per SIMD the register allocator targets, by storage type and columns per lane
#ifndef QS_WAVES_PER_EU
#define QS_WAVES_PER_EU(TS, NC) (NC == 1 ? (sizeof(TS) == 8 ? 4 : 5) : (sizeof(TS) == 8 ? 2 : 4))
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
            a.log2s[I.pmode0 + m] = 0;
            a.epend[I.pmode0 + m] = e;
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

template <typename TS, typename TC, int NC, bool RESTORING, bool FIELDS, bool SNAP, int TJ, bool SCALE, bool FLAT>
__device__ __forceinline__ void step_body(const StepArgs &a, const InstDev &I, const int b) {
    using CL = Cols<NC>;
    constexpr int MPL = CL::MPL;
    constexpr int ROW = 3 * NC;        // rows of 64 values per cell
    const int N = I.n_xi;
    const int lane = threadIdx.x;
    const bool steady = (I.flags & QS_FLAG_STEADY_INFLOW) != 0;
    const bool writer = NC >= 2 || (lane & 1) == 0;   // lane that writes per-mode results

    TC cT[MPL], cP[MPL], kap2[MPL], k2kap2[MPL], scale[MPL];
    int32_t L[MPL];
    int pm[MPL], mloc[MPL];
#pragma unroll
    for (int t = 0; t < MPL; ++t) {
        mloc[t] = CL::mode(b, lane, t);
        pm[t] = I.pmode0 + mloc[t];
        const double k = a.kmode[pm[t]];
        const double kp = 1.0 / (1.0 + k * k);
        kap2[t] = (TC)(kp * kp);
        k2kap2[t] = (TC)(k * k * kp * kp);
        const int e = a.epend[pm[t]];
        L[t] = a.log2s[pm[t]] + e;
        scale[t] = (TC)ldexp(1.0, -e);
        cT[t] = (TC)(k * k * kp * I.ginv);
        cP[t] = (TC)(-kp * I.g3inv * I.ih);
    }
    const TC c1 = (TC)(0.25 * I.dtau), c2 = (TC)(I.dtau / 3.0), c3 = (TC)(0.5 * I.dtau);
    const TC dt = (TC)I.dtau;
    const double C1 = I.c1, S1 = I.s1, C2 = I.c2, S2 = I.s2, h = I.h;

    // Omega at centres then faces; a flat profile has one value (the last face carries 0)
    const TC *omc = static_cast<const TC *>(a.omega) + I.omega_off;
    const rsrc_t ro = make_rsrc(const_cast<TC *>(omc), (uint32_t)(2 * N * sizeof(TC)));
    const TC om0 = omc[0];

    double y[4][NC], v[4][NC];  // oscillator carries per stage: n_p and d_xi n_p at the front face
    TC pp[4][NC];               // stage inputs of P' at the front face of the current cell
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < NC; ++c) { y[m][c] = 0.0; v[m][c] = 0.0; pp[m][c] = (TC)0; }

    TC rmax[MPL], a2max[MPL];
#pragma unroll
    for (int t = 0; t < MPL; ++t) { rmax[t] = (TC)0; a2max[t] = (TC)0; }

    // this block's region of the state: [cell][row][lane] of TS
    TS *blk = static_cast<TS *>(a.state) + I.state_off + (int64_t)b * N * ROW * kWave;
    const rsrc_t rs = make_rsrc(blk, (uint32_t)((int64_t)N * ROW * kWave * sizeof(TS)));
    const int voff = lane * (int)sizeof(TS);
    constexpr int RB = kWave * (int)sizeof(TS);  // bytes per row
    auto ld = [&](int j, int r) __attribute__((always_inline)) { return bload<TS>(rs, voff, (j * ROW + r) * RB); };

    // a cell's inputs: its state rows and (non-flat profiles) Omega at its centre and rear face
    constexpr int XW = ROW + (FLAT ? 0 : 2);
    auto ldx = [&](int j, TS (&x)[XW]) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < ROW; ++r) x[r] = ld(j, r);
        if (!FLAT) {
            x[ROW] = (TS)bload<TC>(ro, 0, j * (int)sizeof(TC));
            x[ROW + 1] = (TS)bload<TC>(ro, 0, (N + j) * (int)sizeof(TC));
        }
    };

    // one cell: four stages, fields of the state at tau_n (stage-1 values), the update.
    // FIRST (cell 0 only) applies the steady-inflow front condition of the test hook.
    auto cell = [&](const int j, const TS (&x)[XW], auto first) __attribute__((always_inline)) {
        constexpr bool FIRST = decltype(first)::value;
        const bool last = (j == N - 1);
        const TC Oc = FLAT ? om0 : (TC)x[ROW];
        const TC Of = last ? (TC)0 : (FLAT ? om0 : (TC)x[ROW + 1]);
        TC r0[NC], P0[NC], T0[NC], cTO[NC], cPO[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int t = NC >= 2 ? c / 2 : 0;
            r0[c] = SCALE ? (TC)x[0 * NC + c] * scale[t] : (TC)x[0 * NC + c];
            P0[c] = SCALE ? (TC)x[1 * NC + c] * scale[t] : (TC)x[1 * NC + c];
            T0[c] = SCALE ? (TC)x[2 * NC + c] * scale[t] : (TC)x[2 * NC + c];
            cTO[c] = cT[t] * Oc;
            cPO[c] = cP[t] * Of;
        }
        TC dr[NC], dT[NC], dP[NC];   // A W_m at this cell
        TC ncf0[NC], vcf0[NC];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const TC cm = (m == 1) ? c1 : (m == 2 ? c2 : c3);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const TC rm = (m == 0) ? r0[c] : r0[c] + cm * dr[c];
                const TC Pm = (m == 0) ? P0[c] : P0[c] + cm * dP[c];
                const TC Tm = (m == 0) ? T0[c] : T0[c] + cm * dT[c];
                const double rd = (double)rm;
                if (FIRST && steady) { y[m][c] = rd; v[m][c] = 0.0; }
                double nc, yn, vn, vc;
                if (RESTORING) {
                    const double u = y[m][c] - rd;
                    nc = rd + C2 * u + S2 * v[m][c];
                    yn = rd + C1 * u + S1 * v[m][c];
                    vn = C1 * v[m][c] - S1 * u;
                    if (FIELDS && m == 0) vc = C2 * v[m][c] - S2 * u;
                } else {
                    nc = y[m][c] + 0.5 * h * v[m][c] + 0.125 * h * h * rd;
                    yn = y[m][c] + h * v[m][c] + 0.5 * h * h * rd;
                    vn = v[m][c] + h * rd;
                    if (FIELDS && m == 0) vc = v[m][c] + 0.5 * h * rd;
                }
                y[m][c] = yn;
                v[m][c] = vn;
                if (FIELDS && m == 0) { ncf0[c] = (TC)nc; vcf0[c] = (TC)vc; }
                dr[c] = (Pm - pp[m][c]) + Tm;
                pp[m][c] = Pm;
                dT[c] = cTO[c] * (TC)nc;
                dP[c] = cPO[c] * (TC)vn;
            }
        }
        if (FIELDS) {
#pragma unroll
            for (int t = 0; t < MPL; ++t) {
                // |E_par|^2 = kappa^2 |n_p'|^2, |E_perp|^2 = k^2 kappa^2 |rho - n_p|^2,
                // |B_perp|^2 = k^2 kappa^2 |rho|^2, summed over the two parts of the mode
                TC e2, b2;
                if (NC >= 2) {
                    const int c0 = 2 * t, c1i = 2 * t + 1;
                    const TC en = vcf0[c0] * vcf0[c0] + vcf0[c1i] * vcf0[c1i];
                    const TC d0 = r0[c0] - ncf0[c0], d1 = r0[c1i] - ncf0[c1i];
                    e2 = kap2[t] * en + k2kap2[t] * (d0 * d0 + d1 * d1);
                    b2 = k2kap2[t] * (r0[c0] * r0[c0] + r0[c1i] * r0[c1i]);
                } else {
                    const TC d0 = r0[0] - ncf0[0];
                    e2 = pair_sum(kap2[0] * vcf0[0] * vcf0[0] + k2kap2[0] * d0 * d0);
                    b2 = pair_sum(k2kap2[0] * r0[0] * r0[0]);
                }
                const TC a2 = e2 + b2;
                a2max[t] = a2 > a2max[t] ? a2 : a2max[t];
                if (SNAP && writer && mloc[t] < I.n_modes) {
                    const double sh = (double)L[t] * 0.69314718055994530942;
                    const int64_t o = a.snap_base + I.snap_off + (int64_t)j * I.n_modes + mloc[t];
                    static_cast<TS *>(a.ln_e)[o] = (TS)(0.5 * (double)log(e2) + sh);
                    static_cast<TS *>(a.ln_b)[o] = (TS)(0.5 * (double)log(b2) + sh);
                }
            }
        }
        if (a.update) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int t = NC >= 2 ? c / 2 : 0;
                const TS rn = (TS)(r0[c] + dt * dr[c]);
                bstore(rn, rs, voff, (j * ROW + 0 * NC + c) * RB);
                bstore((TS)(P0[c] + dt * dP[c]), rs, voff, (j * ROW + 1 * NC + c) * RB);
                bstore((TS)(T0[c] + dt * dT[c]), rs, voff, (j * ROW + 2 * NC + c) * RB);
                const TC ar = (TC)fabs((TC)rn);
                rmax[t] = (ar > rmax[t] || !(ar <= ar)) ? ar : rmax[t];  // NaN sticks
            }
        }
    };

    // Cell 0 first (front condition), then cells 1..N-1 with a one-cell-ahead prefetch
    // ping-ponged between two register sets, unrolled by two so that neither the buffers
    // nor the oscillator carries need copies at the loop edge.  Loads past the end of the
    // block's region are bounds-checked by the buffer descriptor (they return 0, unused).
    using first_t = std::integral_constant<bool, true>;
    using rest_t = std::integral_constant<bool, false>;
    TS xa[XW], xb[XW];
    ldx(0, xa);
    ldx(1, xb);
    cell(0, xa, first_t{});
    int j = 1;
    while (j < N) {
        ldx(j + 1, xa);
        cell(j, xb, rest_t{});
        ++j;
        if (j >= N) break;
        ldx(j + 1, xb);
        cell(j, xa, rest_t{});
        ++j;
    }

    constexpr int R = RenormRange<TS>::R;
#pragma unroll
    for (int t = 0; t < MPL; ++t) {
        if (NC == 1) rmax[t] = pair_max(rmax[t]);
        if (!writer || mloc[t] >= I.n_modes) continue;
        if (FIELDS && a.max_ln_a) {
            const double sh = (double)L[t] * 0.69314718055994530942;
            static_cast<TS *>(a.max_ln_a)[a.max_base + I.mode0 + mloc[t]] =
                (TS)(0.5 * (double)log(a2max[t]) + sh);
        }
        if (a.update) {
            int e = 0;
            const double mx = (double)rmax[t];
            if (!isfinite(mx)) {
                a.err[0] = 1u + (uint32_t)pm[t];
            } else if (mx > 0.0 && (mx > ldexp(1.0, R) || mx < ldexp(1.0, -R))) {
                (void)frexp(mx, &e);
            }
            a.log2s[pm[t]] = L[t];
            a.epend[pm[t]] = e;
        }
    }
}

// FIELDS: compute the fields (max ln A per mode); SNAP: also write ln|E|, ln|B| per cell
template <typename TS, typename TC, int NC, bool RESTORING, bool FIELDS, bool SNAP, int TJ>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(QS_WAVES_PER_EU(TS, NC) - (SNAP ? 1 : 0))))
step_kernel(StepArgs a) {
    const int gb = blockIdx.x;
    const int ii = a.blk_inst[gb];
    const InstDev I = a.inst[ii];
    const int b = gb - I.block0;
    // the rescaling path runs only when a mode of this wave left the renormalization range
    bool need = false;
#pragma unroll
    for (int t = 0; t < Cols<NC>::MPL; ++t)
        need |= a.epend[I.pmode0 + Cols<NC>::mode(b, (int)threadIdx.x, t)] != 0;
    const bool flat = (I.flags & kFlatProfile) != 0;
    if (flat) {
        if (__any(need)) step_body<TS, TC, NC, RESTORING, FIELDS, SNAP, TJ, true, true>(a, I, b);
        else step_body<TS, TC, NC, RESTORING, FIELDS, SNAP, TJ, false, true>(a, I, b);
    } else {
        if (__any(need)) step_body<TS, TC, NC, RESTORING, FIELDS, SNAP, TJ, true, false>(a, I, b);
        else step_body<TS, TC, NC, RESTORING, FIELDS, SNAP, TJ, false, false>(a, I, b);
    }
}

template <typename TS, typename TC, int NC, bool RESTORING>
hipError_t launch_step_r(bool fields, bool snap, int n_blocks, const StepArgs &a, hipStream_t s) {
    constexpr int TJ = QS_STEP_TJ;
    dim3 grid(n_blocks), block(kWave);
    if (snap) hipLaunchKernelGGL((step_kernel<TS, TC, NC, RESTORING, true, true, TJ>), grid, block, 0, s, a);
    else if (fields) hipLaunchKernelGGL((step_kernel<TS, TC, NC, RESTORING, true, false, TJ>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((step_kernel<TS, TC, NC, RESTORING, false, false, TJ>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <typename TS, typename TC, int NC>
hipError_t launch_step_t(bool restoring, bool fields, bool snap, int n_blocks, const StepArgs &a, hipStream_t s) {
    if (restoring) return launch_step_r<TS, TC, NC, true>(fields, snap, n_blocks, a, s);
    return launch_step_r<TS, TC, NC, false>(fields, snap, n_blocks, a, s);
}

template <typename TS, int NC>
hipError_t launch_seed_t(int n_blocks, int max_n_xi, const SeedArgs &a, hipStream_t s) {
    constexpr int kCellsPerWg = 4;
    dim3 grid(n_blocks, (max_n_xi + kCellsPerWg - 1) / kCellsPerWg), block(kCellsPerWg * kWave);
    hipLaunchKernelGGL((seed_kernel<TS, NC>), grid, block, 0, s, a, max_n_xi);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int precision, int nc, bool restoring, bool fields, int n_blocks,
                       const StepArgs &a, hipStream_t s) {
    const bool snap = a.ln_e != nullptr;
    if (precision == QS_FP64) {
        if (nc == 1) return launch_step_t<double, double, 1>(restoring, fields, snap, n_blocks, a, s);
        return launch_step_t<double, double, 2>(restoring, fields, snap, n_blocks, a, s);
    }
    if (nc == 1) return launch_step_t<float, float, 1>(restoring, fields, snap, n_blocks, a, s);
    return launch_step_t<float, float, 2>(restoring, fields, snap, n_blocks, a, s);
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
