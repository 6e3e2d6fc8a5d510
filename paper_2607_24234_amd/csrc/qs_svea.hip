// Envelope-approximation (SVEA) variant of the spectral path (include/qs_svea.h, Sec. III.B):
// d_tau n = m, d_tau m = a * integral_0^xi n, one lane per transverse mode, all tau-steps of
// a call in one launch (modes are independent; each 64-mode block's cells contiguous, so a
// wave streams through one region), the four Runge-Kutta stages of two steps in one
// causal sweep down the cells with FP64 running integrals, loads kAhead cells ahead in a
// register ring, and an exact power-of-two rescale of a mode whose largest component leaves
// [2^-100, 2^100] (applied to the next sweep's loads, like the full model's sweep).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <type_traits>

#include "../../include/qs_svea.h"
#include "qs_internal.h"

namespace {

constexpr int kAhead = 3;     // cells of loads in flight per lane
// tau-steps advanced per sweep over the state (1 to 4): step q + 1 at cell j starts from step
// q's values at cell j, so the state is read and written once per sweep
#ifndef QS_SVEA_STEPS_PER_SWEEP
#define QS_SVEA_STEPS_PER_SWEEP 4
#endif
constexpr int kSweep = QS_SVEA_STEPS_PER_SWEEP;
static_assert(kSweep >= 1 && kSweep <= 4, "steps per sweep");
constexpr int kRange = 100;   // rescale when the largest component leaves [2^-kRange, 2^kRange]

struct cplx {
    double x, y;
};
__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx operator*(double s, cplx a) { return {s * a.x, s * a.y}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ double cmaxabs(cplx a) { return fmax(fabs(a.x), fabs(a.y)); }

// state element (cell j, mode k) of the blocked layout: ((k / 64) n_xi + j) 64 + k % 64
__global__ void __launch_bounds__(256) svea_seed(int64_t n_modes, int64_t total, double2 *__restrict__ n,
                                                 double2 *__restrict__ m, int32_t *__restrict__ l2s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    n[i] = make_double2(0.0, 0.0);
    m[i] = make_double2(1.0, 0.0);
    if (i < n_modes) l2s[i] = 0;
}

__global__ void __launch_bounds__(256) svea_step(int64_t n_modes, int n_xi, double h, const double2 *__restrict__ a_,
                                                 double dt, int n_steps, double2 *__restrict__ nn,
                                                 double2 *__restrict__ mm, int32_t *__restrict__ l2s) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_modes) return;
    const cplx a = {a_[k].x, a_[k].y};
    const int64_t base = (k / 64) * (int64_t)n_xi * 64 + (k % 64);   // cell j at base + 64 j
    const double hh = 0.5 * h, d2 = 0.5 * dt, d6 = dt / 6.0;
    const int last = n_xi - 1;
    double scale = 1.0;   // pending power of two, applied to this sweep's loads
    int l2 = l2s[k];
    // one RK4 step at a cell from its values (n0, m0); S holds h sum_{i<j} of each stage's n
    // for this step and advances past the cell
    auto rk4 = [&](const cplx n0, const cplx m0, cplx (&S)[4], cplx &n1, cplx &m1) __attribute__((always_inline)) {
        // stage 1
        const cplx k1n = m0, k1m = cmul(a, S[0] + hh * n0);
        S[0] = S[0] + h * n0;
        // stage 2
        const cplx n2 = n0 + d2 * k1n, m2 = m0 + d2 * k1m;
        const cplx k2n = m2, k2m = cmul(a, S[1] + hh * n2);
        S[1] = S[1] + h * n2;
        // stage 3
        const cplx n3 = n0 + d2 * k2n, m3 = m0 + d2 * k2m;
        const cplx k3n = m3, k3m = cmul(a, S[2] + hh * n3);
        S[2] = S[2] + h * n3;
        // stage 4
        const cplx n4 = n0 + dt * k3n, m4 = m0 + dt * k3m;
        const cplx k4n = m4, k4m = cmul(a, S[3] + hh * n4);
        S[3] = S[3] + h * n4;
        n1 = n0 + d6 * (k1n + 2.0 * k2n + 2.0 * k3n + k4n);
        m1 = m0 + d6 * (k1m + 2.0 * k2m + 2.0 * k3m + k4m);
    };
    // One sweep down the cells advancing K tau-steps: step 2 at cell j starts from step 1's
    // results at cell j (its inputs there need only cells <= j), so the state is read and
    // written once per sweep.
    auto sweep = [&](auto kk) __attribute__((always_inline)) {
        constexpr int K = decltype(kk)::value;
        cplx S[K][4] = {};
        double big = 0.0;
        // ring of kAhead + 1 slots: cell j sits in slot j % (kAhead + 1), loaded kAhead cells
        // early into the slot the previous cell has just freed (no copies at the loop edge)
        constexpr int R = kAhead + 1;
        double2 rn[R], rm[R];
#pragma unroll
        for (int d = 0; d < kAhead; ++d) {
            const int64_t o = base + 64 * (int64_t)min(d, last);
            rn[d] = nn[o];
            rm[d] = mm[o];
        }
        auto cell = [&](int j, double2 ln, double2 lm) __attribute__((always_inline)) {
            cplx n = {scale * ln.x, scale * ln.y}, m = {scale * lm.x, scale * lm.y};
#pragma unroll
            for (int q = 0; q < K; ++q) {
                cplx n1, m1;
                rk4(n, m, S[q], n1, m1);
                n = n1;
                m = m1;
            }
            const int64_t o = base + 64 * (int64_t)j;
            nn[o] = make_double2(n.x, n.y);
            mm[o] = make_double2(m.x, m.y);
            big = fmax(big, fmax(cmaxabs(n), cmaxabs(m)));
        };
        int jb = 0;
        for (; jb + R <= n_xi; jb += R) {
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int64_t o = base + 64 * (int64_t)min(jb + u + kAhead, last);   // the end reloads the last cell
                rn[(u + kAhead) % R] = nn[o];
                rm[(u + kAhead) % R] = mm[o];
                __builtin_amdgcn_sched_barrier(0);   // keep the loads kAhead cells ahead of their use
                cell(jb + u, rn[u], rm[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < R; ++u)
            if (jb + u < n_xi) cell(jb + u, rn[u], rm[u]);
        // power-of-two rescale of the next sweep's loads (exact), from this sweep's stored values
        scale = 1.0;
        if (big > 0.0 && (big > 0x1p100 || big < 0x1p-100)) {
            const int e = ilogb(big);
            scale = ldexp(1.0, -e);
            l2 += e;
        }
    };
    for (int s = 0; s < n_steps;) {
        const int left = n_steps - s;
        if (left >= kSweep) {
            sweep(std::integral_constant<int, kSweep>{});
            s += kSweep;
        } else {
            // the last steps of the call: one sweep of the rest
            if (kSweep > 3 && left == 3) sweep(std::integral_constant<int, (kSweep > 3 ? 3 : 1)>{});
            else if (kSweep > 2 && left == 2) sweep(std::integral_constant<int, (kSweep > 2 ? 2 : 1)>{});
            else sweep(std::integral_constant<int, 1>{});
            s += left;
        }
    }
    // a pending scale is applied in place before returning, so the stored state is exact
    if (scale != 1.0) {
        for (int j = 0; j < n_xi; ++j) {
            const int64_t o = base + 64 * (int64_t)j;
            const double2 x = nn[o], y = mm[o];
            nn[o] = make_double2(scale * x.x, scale * x.y);
            mm[o] = make_double2(scale * y.x, scale * y.y);
        }
    }
    l2s[k] = l2;
}

// ln |N| into [cell][mode] (mode fastest) from the blocked state
__global__ void __launch_bounds__(256) svea_ln(int64_t n_modes, int n_xi, const double2 *__restrict__ n,
                                               const int32_t *__restrict__ l2s, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_modes * (int64_t)n_xi) return;
    const int64_t j = i / n_modes, k = i % n_modes;
    const double2 v = n[((k / 64) * n_xi + j) * 64 + k % 64];
    const double ln2 = 0.69314718055994531;
    out[i] = log(hypot(v.x, v.y)) + (double)(l2s[k] - 1) * ln2;
}

qs_status sfail(qs_status st, const std::string &m) {
    qs::set_last_error(m);
    return st;
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

int64_t padded(int64_t n_modes) { return (n_modes + 63) / 64 * 64; }

qs_status check(int64_t n_modes, int32_t n_xi) {
    if (n_modes < 1 || n_xi < 1) return sfail(QS_ERR_ARG, "n_modes and n_xi must be >= 1");
    if ((padded(n_modes) * (int64_t)n_xi + 255) / 256 > (int64_t)0x7fffffff) return sfail(QS_ERR_ARG, "state too large");
    return QS_OK;
}

}  // namespace

extern "C" {

qs_status qs_svea_coefficients(int32_t n_species, const double *q, const double *m, const double *nb_over_np,
                               double gamma_b, int64_t n_modes, const double *k, double *a) {
    if (n_species < 1 || !q || !m || !nb_over_np || !(gamma_b >= 1.0) || n_modes < 0 || (n_modes > 0 && (!k || !a)))
        return sfail(QS_ERR_ARG, "species arrays, gamma_b >= 1, k and a are required");
    double w2 = 0.0;
    for (int s = 0; s < n_species; ++s) {
        if (!(m[s] > 0.0)) return sfail(QS_ERR_ARG, "species masses must be > 0");
        w2 += q[s] * q[s] * nb_over_np[s] / (m[s] * gamma_b);
    }
    for (int64_t i = 0; i < n_modes; ++i) {
        a[2 * i] = 0.0;
        a[2 * i + 1] = 0.5 * w2 * k[i] * k[i] / (1.0 + k[i] * k[i]);
    }
    return QS_OK;
}

qs_status qs_svea_seed_impulse(int64_t n_modes, int32_t n_xi, double *n, double *m, int32_t *log2_scale,
                               void *hip_stream) {
    qs_status st = check(n_modes, n_xi);
    if (st != QS_OK) return st;
    if (!n || !m || !log2_scale) return sfail(QS_ERR_ARG, "n, m and log2_scale are required");
    const int64_t total = padded(n_modes) * (int64_t)n_xi;
    hipLaunchKernelGGL(svea_seed, dim3(blocks_of(total)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n_modes,
                       total, reinterpret_cast<double2 *>(n), reinterpret_cast<double2 *>(m), log2_scale);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? QS_OK : sfail(QS_ERR_HIP, std::string("svea seed: ") + hipGetErrorString(e));
}

qs_status qs_svea_step(int64_t n_modes, int32_t n_xi, double h, const double *a, double d_tau, int32_t n_steps,
                       double *n, double *m, int32_t *log2_scale, void *hip_stream) {
    qs_status st = check(n_modes, n_xi);
    if (st != QS_OK) return st;
    if (!a || !n || !m || !log2_scale) return sfail(QS_ERR_ARG, "a, n, m and log2_scale are required");
    if (!(h > 0.0) || !std::isfinite(h) || !std::isfinite(d_tau) || n_steps < 0)
        return sfail(QS_ERR_ARG, "h > 0, finite d_tau and n_steps >= 0 are required");
    if (n_steps == 0) return QS_OK;
    hipLaunchKernelGGL(svea_step, dim3(blocks_of(n_modes)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n_modes,
                       (int)n_xi, h, reinterpret_cast<const double2 *>(a), d_tau, (int)n_steps,
                       reinterpret_cast<double2 *>(n), reinterpret_cast<double2 *>(m), log2_scale);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? QS_OK : sfail(QS_ERR_HIP, std::string("svea step: ") + hipGetErrorString(e));
}

qs_status qs_svea_ln_envelope(int64_t n_modes, int32_t n_xi, const double *n, const int32_t *log2_scale,
                              double *ln_abs, void *hip_stream) {
    qs_status st = check(n_modes, n_xi);
    if (st != QS_OK) return st;
    if (!n || !log2_scale || !ln_abs) return sfail(QS_ERR_ARG, "n, log2_scale and ln_abs are required");
    const int64_t total = n_modes * (int64_t)n_xi;
    hipLaunchKernelGGL(svea_ln, dim3(blocks_of(total)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), n_modes,
                       (int)n_xi, reinterpret_cast<const double2 *>(n), log2_scale, ln_abs);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? QS_OK : sfail(QS_ERR_HIP, std::string("svea envelope: ") + hipGetErrorString(e));
}

}  // extern "C"
