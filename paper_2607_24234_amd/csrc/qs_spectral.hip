// Spectral hot path for gfx950: one wavefront per block of 64 lanes, each lane owning
// MPL transverse modes (2*MPL real columns: the real and imaginary parts of a mode evolve
// independently because every coefficient below is real), marching causally in xi.
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
#include "qs_internal.h"

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

// ----------------------------------------------------------------------------- seed
template <typename TS, int MPL>
__global__ void __launch_bounds__(256) seed_kernel(SeedArgs a, int max_n_xi) {
    constexpr int NC = 2 * MPL;
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
    for (int t = 0; t < MPL; ++t) {
        const int m = (b * kWave + lane) * MPL + t;
        const bool valid = m < I.n_modes;
        double re = 0.0, im = 0.0, tre = 0.0;
        if (valid) {
            if (a.kind == QS_SEED_NOISE) {
                uint64_t c = (inst_idx * (uint64_t)I.n_modes + (uint64_t)m) * (uint64_t)N + (uint64_t)j;
                double u = (double)(sm64(a.rng_seed, c) >> 11) * (1.0 / 9007199254740992.0);
                double sn, cs;
                sincos(6.283185307179586476925286766559 * u, &sn, &cs);
                re = a.amp * f * cs;
                im = a.amp * f * sn;
            } else if (a.kind == QS_SEED_UNIFORM) {
                re = a.amp * f;
            } else if (a.kind == QS_SEED_FRONT_IMPULSE) {
                const double k = a.kmode[I.pmode0 + m];
                if (j == 0 && k != 0.0) tre = a.amp / (I.h * k);  // d_tau rho_0 = k T = amp/h
            }
        }
        // rows: var 0 = rho, 1 = P, 2 = T; column c = 2t + part
        cell[(0 * NC + 2 * t + 0) * kWave + lane] = (TS)re;
        cell[(0 * NC + 2 * t + 1) * kWave + lane] = (TS)im;
        cell[(1 * NC + 2 * t + 0) * kWave + lane] = (TS)0;
        cell[(1 * NC + 2 * t + 1) * kWave + lane] = (TS)0;
        cell[(2 * NC + 2 * t + 0) * kWave + lane] = (TS)tre;
        cell[(2 * NC + 2 * t + 1) * kWave + lane] = (TS)0;
        if (j == 0) {
            a.log2s[I.pmode0 + m] = 0;
            a.epend[I.pmode0 + m] = 0;
        }
    }
}

// ----------------------------------------------------------------------------- step
// TS: storage type, TC: arithmetic type of everything except the oscillator carries
// (always double).  RESTORING selects the plasma operator (d_xi^2 + 1) or d_xi^2.
template <typename TS, typename TC, int MPL, bool RESTORING, bool FIELDS>
__global__ void __launch_bounds__(64) step_kernel(StepArgs a) {
    constexpr int NC = 2 * MPL;        // real columns per lane
    constexpr int ROW = 3 * NC;        // rows of 64 values per cell
    constexpr int TJ = 4;              // cells per register tile
    const int gb = blockIdx.x;
    const int ii = a.blk_inst[gb];
    const InstDev I = a.inst[ii];
    const int b = gb - I.block0;
    const int N = I.n_xi;
    const int lane = threadIdx.x;
    const bool steady = (I.flags & QS_FLAG_STEADY_INFLOW) != 0;

    // per-column constants
    TC kk[NC], cT[NC], cP[NC], kap[MPL], kv[MPL];
    TC scale[MPL];
    int32_t L[MPL];
    int pm[MPL], mloc[MPL];
#pragma unroll
    for (int t = 0; t < MPL; ++t) {
        mloc[t] = (b * kWave + lane) * MPL + t;
        pm[t] = I.pmode0 + mloc[t];
        const double k = a.kmode[pm[t]];
        const double kp = 1.0 / (1.0 + k * k);
        kv[t] = (TC)k;
        kap[t] = (TC)kp;
        const int e = a.epend[pm[t]];
        L[t] = a.log2s[pm[t]] + e;
        scale[t] = (TC)ldexp(1.0, -e);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            kk[2 * t + p] = (TC)k;
            cT[2 * t + p] = (TC)(k * kp * I.ginv);
            cP[2 * t + p] = (TC)(kp * I.g3inv);
        }
    }
    const TC ih = (TC)I.ih;
    const TC dt = (TC)I.dtau, half = (TC)(0.5 * I.dtau);
    const TC w1 = (TC)(I.dtau / 6.0), w2 = (TC)(I.dtau / 3.0);
    const double C1 = I.c1, S1 = I.s1, C2 = I.c2, S2 = I.s2, h = I.h;

    const TC *omc = static_cast<const TC *>(a.omega) + I.omega_off;
    const TC *omf = omc + N;

    double y[4][NC], v[4][NC];  // oscillator carries per stage: n_p and d_xi n_p at the front face
    TC pp[4][NC];               // stage inputs of P at the front face of the current cell
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < NC; ++c) { y[m][c] = 0.0; v[m][c] = 0.0; pp[m][c] = (TC)0; }

    TC rmax[MPL], a2max[MPL];
#pragma unroll
    for (int t = 0; t < MPL; ++t) { rmax[t] = (TC)0; a2max[t] = (TC)0; }

    TS *base = static_cast<TS *>(a.state) + I.state_off + (int64_t)b * N * ROW * kWave + lane;

    TS cur[TJ][ROW], nxt[TJ][ROW];
#pragma unroll
    for (int jj = 0; jj < TJ; ++jj)
#pragma unroll
        for (int r = 0; r < ROW; ++r)
            cur[jj][r] = (jj < N) ? base[((int64_t)jj * ROW + r) * kWave] : (TS)0;

    for (int j0 = 0; j0 < N; j0 += TJ) {
        if (j0 + TJ < N) {
#pragma unroll
            for (int jj = 0; jj < TJ; ++jj)
#pragma unroll
                for (int r = 0; r < ROW; ++r)
                    nxt[jj][r] = (j0 + TJ + jj < N) ? base[((int64_t)(j0 + TJ + jj) * ROW + r) * kWave] : (TS)0;
        }
#pragma unroll
        for (int jj = 0; jj < TJ; ++jj) {
            const int j = j0 + jj;
            if (j < N) {
                const bool last = (j == N - 1);
                const TC Oc = omc[j], Of = omf[j];
                TC r0[NC], P0[NC], T0[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const TC sc = scale[c / 2];
                    r0[c] = (TC)cur[jj][0 * NC + c] * sc;
                    P0[c] = last ? (TC)0 : (TC)cur[jj][1 * NC + c] * sc;
                    T0[c] = (TC)cur[jj][2 * NC + c] * sc;
                }
                TC dr[4][NC], dT[4][NC], dP[4][NC];
                TC ncf0[NC], vcf0[NC];  // stage-0 plasma response at the centre (fields)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const TC am = (m == 0) ? (TC)0 : (m == 3 ? dt : half);
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const TC rm = (m == 0) ? r0[c] : r0[c] + am * dr[m - 1][c];
                        const TC Pm = (m == 0) ? P0[c] : (last ? (TC)0 : P0[c] + am * dP[m - 1][c]);
                        const TC Tm = (m == 0) ? T0[c] : T0[c] + am * dT[m - 1][c];
                        const double rd = (double)rm;
                        if (j == 0 && steady) { y[m][c] = rd; v[m][c] = 0.0; }
                        double nc, yn, vn, vc;
                        if (RESTORING) {
                            const double u = y[m][c] - rd;
                            nc = rd + C2 * u + S2 * v[m][c];
                            yn = rd + C1 * u + S1 * v[m][c];
                            vn = C1 * v[m][c] - S1 * u;
                            vc = C2 * v[m][c] - S2 * u;
                        } else {
                            nc = y[m][c] + 0.5 * h * v[m][c] + 0.125 * h * h * rd;
                            yn = y[m][c] + h * v[m][c] + 0.5 * h * h * rd;
                            vn = v[m][c] + h * rd;
                            vc = v[m][c] + 0.5 * h * rd;
                        }
                        y[m][c] = yn;
                        v[m][c] = vn;
                        if (FIELDS && m == 0) { ncf0[c] = (TC)nc; vcf0[c] = (TC)vc; }
                        dr[m][c] = (Pm - pp[m][c]) * ih + kk[c] * Tm;
                        pp[m][c] = Pm;
                        dT[m][c] = cT[c] * Oc * (TC)nc;
                        dP[m][c] = last ? (TC)0 : -cP[c] * Of * (TC)vn;
                    }
                }
                if (FIELDS) {
#pragma unroll
                    for (int t = 0; t < MPL; ++t) {
                        const TC k2 = kv[t] * kv[t] * kap[t] * kap[t];
                        const TC ep = kap[t] * kap[t] * (vcf0[2 * t] * vcf0[2 * t] + vcf0[2 * t + 1] * vcf0[2 * t + 1]);
                        const TC d0 = r0[2 * t] - ncf0[2 * t], d1 = r0[2 * t + 1] - ncf0[2 * t + 1];
                        const TC e2 = ep + k2 * (d0 * d0 + d1 * d1);
                        const TC b2 = k2 * (r0[2 * t] * r0[2 * t] + r0[2 * t + 1] * r0[2 * t + 1]);
                        const TC a2 = e2 + b2;
                        a2max[t] = a2 > a2max[t] ? a2 : a2max[t];
                        if (a.ln_e && mloc[t] < I.n_modes) {
                            const double sh = (double)L[t] * 0.69314718055994530942;
                            const int64_t o = a.snap_base + I.snap_off + (int64_t)j * I.n_modes + mloc[t];
                            static_cast<TS *>(a.ln_e)[o] = (TS)(0.5 * (double)log(e2) + sh);
                            static_cast<TS *>(a.ln_b)[o] = (TS)(0.5 * (double)log(b2) + sh);
                        }
                    }
                }
                if (a.update) {
                    TS *row = base + (int64_t)j * ROW * kWave;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const TC rn = r0[c] + w1 * (dr[0][c] + dr[3][c]) + w2 * (dr[1][c] + dr[2][c]);
                        const TC Pn = last ? (TC)0 : P0[c] + w1 * (dP[0][c] + dP[3][c]) + w2 * (dP[1][c] + dP[2][c]);
                        const TC Tn = T0[c] + w1 * (dT[0][c] + dT[3][c]) + w2 * (dT[1][c] + dT[2][c]);
                        row[(0 * NC + c) * kWave] = (TS)rn;
                        row[(1 * NC + c) * kWave] = (TS)Pn;
                        row[(2 * NC + c) * kWave] = (TS)Tn;
                        const TC ar = (TC)fabs((TC)(TS)rn);
                        rmax[c / 2] = ar > rmax[c / 2] ? ar : rmax[c / 2];
                        if (!(ar <= ar)) rmax[c / 2] = ar;  // keep a NaN visible
                    }
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < TJ; ++jj)
#pragma unroll
            for (int r = 0; r < ROW; ++r) cur[jj][r] = nxt[jj][r];
    }

#pragma unroll
    for (int t = 0; t < MPL; ++t) {
        if (mloc[t] >= I.n_modes) continue;
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
            } else if (mx > 0.0) {
                (void)frexp(mx, &e);
            }
            a.log2s[pm[t]] = L[t];
            a.epend[pm[t]] = e;
        }
    }
}

template <typename TS, typename TC, int MPL>
hipError_t launch_step_t(bool restoring, bool fields, int n_blocks, const StepArgs &a, hipStream_t s) {
    dim3 grid(n_blocks), block(kWave);
    if (restoring) {
        if (fields) hipLaunchKernelGGL((step_kernel<TS, TC, MPL, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((step_kernel<TS, TC, MPL, true, false>), grid, block, 0, s, a);
    } else {
        if (fields) hipLaunchKernelGGL((step_kernel<TS, TC, MPL, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((step_kernel<TS, TC, MPL, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template <typename TS, int MPL>
hipError_t launch_seed_t(int n_blocks, int max_n_xi, const SeedArgs &a, hipStream_t s) {
    constexpr int kCellsPerWg = 4;
    dim3 grid(n_blocks, (max_n_xi + kCellsPerWg - 1) / kCellsPerWg), block(kCellsPerWg * kWave);
    hipLaunchKernelGGL((seed_kernel<TS, MPL>), grid, block, 0, s, a, max_n_xi);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int precision, int mpl, bool restoring, bool fields, int n_blocks,
                       const StepArgs &a, hipStream_t s) {
    if (precision == QS_FP64) {
        if (mpl == 1) return launch_step_t<double, double, 1>(restoring, fields, n_blocks, a, s);
        return launch_step_t<double, double, 2>(restoring, fields, n_blocks, a, s);
    }
    if (mpl == 1) return launch_step_t<float, float, 1>(restoring, fields, n_blocks, a, s);
    return launch_step_t<float, float, 2>(restoring, fields, n_blocks, a, s);
}

hipError_t launch_seed(int precision, int mpl, int n_blocks, int max_n_xi, const SeedArgs &a,
                       hipStream_t s) {
    if (precision == QS_FP64) {
        if (mpl == 1) return launch_seed_t<double, 1>(n_blocks, max_n_xi, a, s);
        return launch_seed_t<double, 2>(n_blocks, max_n_xi, a, s);
    }
    if (mpl == 1) return launch_seed_t<float, 1>(n_blocks, max_n_xi, a, s);
    return launch_seed_t<float, 2>(n_blocks, max_n_xi, a, s);
}

uint64_t splitmix64_host(uint64_t seed, uint64_t i) { return sm64(seed, i); }

}  // namespace qs
