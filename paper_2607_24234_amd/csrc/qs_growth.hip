// Growth maps (include/qs_growth.h): windowed-growth targets from solver snapshots, training
// examples drawn from them, the surrogate's feature map, the held-out error table, and the
// query entry point with its solver fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qs_growth.h"
#include "qs_internal.h"

// Scratch of the allocation-free query entry point: the network inputs (5 floats) and the
// baseline (1 float) of at most QS_GROWTH_NOALLOC_MAX queries (6 MiB).  Each device holds its
// own copy, from the library's load until the process ends; every call on a device shares it.
static __device__ __align__(256) float scratch[(size_t)QS_GROWTH_NOALLOC_MAX * 6];

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kBinsPerFeature = 8;
constexpr double kTMax = 9.7014250014533188;  // 40/sqrt(17): Gamma_CFI tau at k = 4, tau = tau_f

qs_status gfail(qs_status st, const std::string &m) {
    qs::set_last_error(m);
    return st;
}
#define G_HIP(call, what)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return gfail(QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

// per-instance constants on the device
struct GInst {
    int64_t off;        // element offset inside one snapshot
    int64_t col0;       // first column (mode) index over all instances
    int32_t n_xi, n_modes, win;
    int32_t k0;         // first entry of this instance in the k table
    double h, d_tau, ln_s;
    float ln_nb, ln_gamma;
};

// cells of the window: two plasma wavelengths 4 pi (at least one)
int window_cells(double h) { return std::max(1, (int)std::lround(4.0 * kPi / h)); }

__host__ __device__ inline double tau_final(double nb, double g) { return 10.0 * sqrt(g / nb); }

// Box coordinates of a query (ln n_b, ln gamma, k, xi, tau): each in [-1, 1] inside the box
// n_b in [1e-3, 1e-1], gamma in [10, 1e4], k in [0.05, 4], xi in [0, 200], tau in [0, tau_f].
__device__ inline void box_coords(const float *q, float b[5]) {
    const double nb = exp((double)q[0]), g = exp((double)q[1]);
    b[0] = (float)((double)q[0] * 0.43429448190325182765 + 2.0);
    b[1] = (float)(((double)q[1] * 0.43429448190325182765 - 2.5) / 1.5);
    b[2] = (float)(((double)q[2] - 2.025) / 1.975);
    b[3] = (float)((double)q[3] / 100.0 - 1.0);
    b[4] = (float)(2.0 * (double)q[4] / tau_final(nb, g) - 1.0);
}

// For a, b >= 0: J(a, b) = ln(e^a + e^b - 1) and M(a, b) = -ln(e^-a + e^-b - e^-(a+b)), both
// 0 at a = b = 0, with J(a, 0) = a and M(a, 0) = 0, tending to max(a, b) and min(a, b) once both
// are large.  With hi = max, lo = min, d = hi - lo: e^a + e^b - 1 = e^hi (1 + e^-d - e^-hi) and
// e^-a + e^-b - e^-(a+b) = e^-lo (1 + e^-d - e^-hi), where 1 + e^-d - e^-hi >= 1.
__device__ inline double join_rest(double a, double b) { return log1p(exp(-fabs(a - b)) - exp(-fmax(a, b))); }
__device__ inline double join_up(double a, double b) { return fmax(a, b) + join_rest(a, b); }
__device__ inline double join_down(double a, double b) { return fmin(a, b) - join_rest(a, b); }

// Network inputs and baseline of a query.  Inputs: log10 n_b + 2, (log10(gamma k) - 2.1505)/
// 2.4515, 2 log10(k/0.05)/log10(80) - 1, 2 sqrt(xi/200) - 1, 2 sqrt(t/t_max) - 1 with
// t = Gamma_CFI tau = sqrt(n_b/gamma) k/sqrt(1+k^2) tau.  Baseline: the wavelength-averaged
// field of the extended disturbance at tau = 0, 1/2 ln(kappa^2 (1+3k^2)/2), plus the growth
// J(M(C, F), O): the temporal CFI growth C = ln cosh t (Appendix C) held back near the front by
// F = 2 (sqrt(1 + t xi) - 1), whose exponent tends to the spatiotemporal CFI one 2 sqrt(t xi)
// (Eq. CFI_ST), and overtaken deep in the beam by O = 3 ((1 + z)^(1/3) - 1),
// z = (3 sqrt(3)/64) t_e^2 xi, whose exponent tends to the spatiotemporal OTSI one
// (3 sqrt(3)/4) t_e^(2/3) xi^(1/3) (Eq. OTSI_ST) at t_e = t (1 + 1/(gamma k)^2)^(1/2).  F and O
// start linearly in t xi and z, so the baseline is smooth in the inputs and equals the field
// level at tau = 0.  k is floored at 1e-3 and xi, t at 0, so every query has finite inputs.
__device__ inline void net_inputs(const float *q, float x[5], float *base) {
    const double lnb = (double)q[0], lng = (double)q[1];
    const double k = fmax((double)q[2], 1e-3), xi = fmax((double)q[3], 0.0), tau = (double)q[4];
    const double kap = 1.0 / (1.0 + k * k);
    const double t = fmax(exp(0.5 * (lnb - lng)) * k * sqrt(kap) * tau, 0.0);
    const double l10 = 0.43429448190325182765;  // 1/ln 10
    x[0] = (float)(lnb * l10 + 2.0);
    x[1] = (float)(((lng + log(k)) * l10 - 2.1505) / 2.4515);
    x[2] = (float)(2.0 * log(k / 0.05) / log(80.0) - 1.0);
    x[3] = (float)(2.0 * sqrt(xi / 200.0) - 1.0);
    x[4] = (float)(2.0 * sqrt(t / kTMax) - 1.0);
    const double lcosh = t + log1p(exp(-2.0 * t)) - 0.69314718055994530942;
    // behind the front the longitudinal term adds beta^2 = Gamma_CFI^2/(gamma k)^2 to
    // Gamma_CFI^2 (the Laplace form of the transverse master equation with its gamma^-2 term)
    const double gk = exp(lng) * k;
    const double z = 0.08118988160479113 * t * t * (1.0 + 1.0 / (gk * gk)) * xi;  // 3 sqrt(3)/64
    const double otsi = 3.0 * (cbrt(1.0 + z) - 1.0);
    const double front = 2.0 * (sqrt(1.0 + t * xi) - 1.0);
    *base = (float)(0.5 * log(kap * kap * (1.0 + 3.0 * k * k) * 0.5) + join_up(join_down(lcosh, front), otsi));
}

// A^2 / S^2 of one entry from ln|E| and ln|B| (exp of -inf is 0)
__device__ inline double a2_rel(float le, float lb, double ln_s) {
    return exp(2.0 * ((double)le - ln_s)) + exp(2.0 * ((double)lb - ln_s));
}

// One thread per (snapshot, column).  Hann-weighted window of W cells ending at cell j:
// with zeta = e^(2 pi i/W) and w_i = sin^2(pi (i + 1/2)/W) = 1/2 - 1/2 Re(e^(i pi/W) zeta^i),
//   sum_i w_i a_(j-i) = S0/2 - Re(e^(i pi/W) T)/2,  S0 = sum_i a_(j-i),  T = sum_i a_(j-i) zeta^i,
// both advanced by one cell per step (T <- a_(j+1) + zeta T - a_(j+1-W), as zeta^W = 1) and
// recomputed directly every kResum cells so that no rounding accumulates; the weights present
// in a truncated window (the first W-1 cells) sum to n/2 - Re(e^(i pi/W) (1 - zeta^n)/(1 - zeta))/2.
constexpr int kResum = 64;
__global__ void __launch_bounds__(256) targets_kernel(const GInst *__restrict__ inst, int n_inst,
                                                      const float *__restrict__ le, const float *__restrict__ lb,
                                                      int64_t snap_elems, int64_t cols, int n_snap,
                                                      float *__restrict__ G) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= cols * n_snap) return;
    const int t = (int)(gid / cols);
    const int64_t c = gid % cols;
    int lo = 0, hi = n_inst - 1;  // instance of column c
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (inst[mid].col0 <= c) lo = mid; else hi = mid - 1;
    }
    const GInst I = inst[lo];
    const int m = (int)(c - I.col0);
    const int64_t base = (int64_t)t * snap_elems + I.off + m;
    const int64_t M = I.n_modes;
    const int W = I.win;
    auto a_at = [&](int j) { return a2_rel(le[base + j * M], lb[base + j * M], I.ln_s); };
    double zr = 1.0, zi = 0.0, hr = 1.0, hi2 = 0.0;  // zeta, e^(i pi/W)
    if (W > 1) {
        sincos(2.0 * kPi / W, &zi, &zr);
        sincos(kPi / W, &hi2, &hr);
    }
    double s0 = 0.0, tr = 0.0, ti = 0.0;
    for (int j = 0; j < I.n_xi; ++j) {
        const int n = min(j + 1, W);
        const double aj = a_at(j);
        if (j % kResum == 0) {  // direct sums over the window
            s0 = 0.0; tr = 0.0; ti = 0.0;
            double pr = 1.0, pi = 0.0;  // zeta^i
            for (int i = 0; i < n; ++i) {
                const double v = (i == 0) ? aj : a_at(j - i);
                s0 += v; tr += v * pr; ti += v * pi;
                const double nr = pr * zr - pi * zi;
                pi = pr * zi + pi * zr;
                pr = nr;
            }
        } else {
            const double old = (j >= W) ? a_at(j - W) : 0.0;
            s0 += aj - old;
            const double nr = aj + zr * tr - zi * ti - old;
            ti = zr * ti + zi * tr;
            tr = nr;
        }
        double num, den;
        if (W == 1) {
            num = aj;
            den = 1.0;
        } else {
            num = 0.5 * s0 - 0.5 * (hr * tr - hi2 * ti);
            // sum_{i<n} zeta^i = (1 - zeta^n)/(1 - zeta)
            double snr, cnr;
            sincos(2.0 * kPi * n / W, &snr, &cnr);
            const double ar = 1.0 - cnr, ai = -snr, br = 1.0 - zr, bi = -zi;
            const double bb = br * br + bi * bi;
            const double gr = (ar * br + ai * bi) / bb, gi = (ai * br - ar * bi) / bb;
            den = 0.5 * n - 0.5 * (hr * gr - hi2 * gi);
        }
        G[base + (int64_t)j * M] = (float)(0.5 * log(fmax(num, 0.0) / den));
    }
}

__device__ inline uint64_t sm64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Draw n examples uniformly over all (snapshot, instance, cell, mode) entries of G: the query
// (ln n_b, ln gamma, k, xi_j, tau) of the entry and its target.
__global__ void __launch_bounds__(256) sample_kernel(const GInst *__restrict__ inst, int n_inst,
                                                     const double *__restrict__ kt, const float *__restrict__ G,
                                                     int64_t snap_elems, const int32_t *__restrict__ steps, int n_snap,
                                                     uint64_t seed, int64_t n, float *__restrict__ Q,
                                                     float *__restrict__ T) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double u = (double)(sm64(seed, (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
    const uint64_t total = (uint64_t)snap_elems * (uint64_t)n_snap;
    const uint64_t e = min((uint64_t)(u * (double)total), total - 1);
    const int t = (int)(e / (uint64_t)snap_elems);
    const int64_t r = (int64_t)(e % (uint64_t)snap_elems);
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (inst[mid].off <= r) lo = mid; else hi = mid - 1;
    }
    const GInst I = inst[lo];
    const int64_t qq = r - I.off;
    const int j = (int)(qq / I.n_modes), m = (int)(qq % I.n_modes);
    Q[5 * i + 0] = I.ln_nb;
    Q[5 * i + 1] = I.ln_gamma;
    Q[5 * i + 2] = (float)kt[I.k0 + m];
    Q[5 * i + 3] = (float)((j + 0.5) * I.h);
    Q[5 * i + 4] = (float)(steps[t] * I.d_tau);
    T[i] = G[e];
}

// x [n][5] network inputs and base [n] baseline (either may be null)
__global__ void __launch_bounds__(256) features_kernel(const float *__restrict__ q, int64_t n, float *__restrict__ x,
                                                       float *__restrict__ base) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float xv[5], bv;
    net_inputs(q + 5 * i, xv, &bv);
    if (x)
        for (int d = 0; d < 5; ++d) x[5 * i + d] = xv[d];
    if (base) base[i] = bv;
}

__device__ inline int bin_of(const float *b) {
    int out = 0;
    for (int d = 0; d < 5; ++d) {
        int c = (int)floorf((b[d] + 1.0f) * (kBinsPerFeature / 2));
        c = min(kBinsPerFeature - 1, max(0, c));
        out = out * kBinsPerFeature + c;
    }
    return out;
}

__global__ void __launch_bounds__(256) fill_kernel(float *p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Held-out error histogram: bucket 0 holds |y - t| <= e0, bucket b >= 1 the range
// (e0 2^((b-1)/32), e0 2^(b/32)], the last bucket everything above e0 2^(542/32) ~ 12.5 (and
// non-finite errors): a reported percentile is at most 2^(1/32) (2.2 %) above the exact one.
constexpr int kPerOctave = 32;
constexpr int kBuckets = 544;
constexpr float kE0 = 1e-4f;
constexpr int kMinCount = 32;  // fewer held-out examples in a bin: no estimate

__host__ __device__ inline float bucket_edge(int b) {
    return b >= kBuckets - 1 ? 3.0e38f : kE0 * exp2f((float)b / kPerOctave);
}

// error of the answer y + base against the target t, binned by the query's box coordinates
__global__ void __launch_bounds__(256) hist_kernel(const float *__restrict__ q, const float *__restrict__ y,
                                                   const float *__restrict__ base, const float *__restrict__ t,
                                                   int64_t n, uint32_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float e = fabsf(y[i] + base[i] - t[i]);
    int b;
    if (!(e <= 3.0e38f)) b = kBuckets - 1;
    else if (e <= kE0) b = 0;
    else b = min(kBuckets - 1, 1 + (int)floorf((float)kPerOctave * log2f(e / kE0)));
    float bc[5];
    box_coords(q + 5 * i, bc);
    atomicAdd(cnt + (int64_t)bin_of(bc) * kBuckets + b, 1u);
}

// table[bin] = upper edge of the bucket holding the 99th percentile, -1 below kMinCount
__global__ void __launch_bounds__(256) p99_kernel(const uint32_t *__restrict__ cnt, float *__restrict__ table) {
    const int bin = blockIdx.x * blockDim.x + threadIdx.x;
    if (bin >= QS_GROWTH_BINS) return;
    const uint32_t *c = cnt + (int64_t)bin * kBuckets;
    uint32_t total = 0;
    for (int b = 0; b < kBuckets; ++b) total += c[b];
    if (total < (uint32_t)kMinCount) { table[bin] = -1.0f; return; }
    const uint32_t need = (uint32_t)ceil(0.99 * (double)total);
    uint32_t acc = 0;
    int b = 0;
    for (; b < kBuckets; ++b) {
        acc += c[b];
        if (acc >= need) break;
    }
    table[bin] = bucket_edge(min(b, kBuckets - 1));
}

// out += base (the network's residual plus the baseline); with flag != null also the routing
// flag: 1 where the solver must answer (outside the box, no held-out data in the bin, or the
// bin's held-out error above tol)
__global__ void __launch_bounds__(256) finish_kernel(const float *__restrict__ q, int64_t n,
                                                     const float *__restrict__ base, float *__restrict__ out,
                                                     const float *__restrict__ table, float tol,
                                                     uint8_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] += base[i];
    if (!flag) return;
    float b[5];
    box_coords(q + 5 * i, b);
    bool inside = true;
    for (int d = 0; d < 5; ++d) inside = inside && b[d] >= -1.0f && b[d] <= 1.0f;
    const float e = table ? table[bin_of(b)] : -1.0f;
    flag[i] = (inside && e >= 0.0f && e <= tol) ? 0 : 1;
}

__global__ void __launch_bounds__(256) scatter_kernel(const int64_t *__restrict__ idx, const float *__restrict__ val,
                                                      int64_t n, float *__restrict__ out, uint8_t *__restrict__ used) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[idx[i]] = val[i];
    if (used) used[idx[i]] = 1;
}

// The queries flagged for the solver, appended in any order (slots from a counter) with their
// positions: at most cap of them are written, the counter ends at their number.
__global__ void __launch_bounds__(256) select_kernel(const float *__restrict__ q, const uint8_t *__restrict__ flag,
                                                     int64_t n, unsigned long long *__restrict__ count,
                                                     int64_t *__restrict__ idx, float *__restrict__ rows, int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const int64_t slot = (int64_t)atomicAdd(count, 1ull);
    if (slot >= cap) return;
    idx[slot] = i;
    for (int d = 0; d < 5; ++d) rows[5 * slot + d] = q[5 * i + d];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices];  // device address of `scratch` per device (null: not yet resolved)

// Device address of this device's scratch copy, resolved once per device with that device
// current.  The host-side name `scratch` is not a device address and is never passed on.
qs_status scratch_for_device(int dev, float **out) {
    if (dev < 0 || dev >= kMaxDevices) return gfail(QS_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return gfail(QS_ERR_HIP, std::string("resolving the query scratch: ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_dev[dev];
    return QS_OK;
}

qs_status check_insts(const qs_growth_instance *inst, int32_t n_inst) {
    if (!inst || n_inst < 1) return gfail(QS_ERR_ARG, "at least one instance is required");
    for (int i = 0; i < n_inst; ++i) {
        const qs_growth_instance &g = inst[i];
        if (!(g.nb_over_np > 0) || !(g.gamma_b > 1) || !(g.length > 0) || !(g.d_tau > 0) || !(g.seed_amp > 0) ||
            g.n_xi < 1 || g.n_modes < 1 || !g.k)
            return gfail(QS_ERR_ARG, "instance " + std::to_string(i) + ": invalid description");
    }
    return QS_OK;
}

// device table of instances (+ the k table when wanted); returns snapshot elements
qs_status upload_insts(const qs_growth_instance *inst, int32_t n_inst, hipStream_t s, GInst **d_inst,
                       double **d_k, int64_t *snap_elems, int64_t *cols) {
    std::vector<GInst> gi(n_inst);
    std::vector<double> kt;
    int64_t off = 0, col = 0;
    for (int i = 0; i < n_inst; ++i) {
        const qs_growth_instance &g = inst[i];
        GInst &d = gi[i];
        d.off = off;
        d.col0 = col;
        d.n_xi = g.n_xi;
        d.n_modes = g.n_modes;
        d.h = g.length / g.n_xi;
        d.win = window_cells(d.h);
        d.k0 = (int32_t)kt.size();
        d.d_tau = g.d_tau;
        d.ln_s = std::log(g.seed_amp);
        d.ln_nb = (float)std::log(g.nb_over_np);
        d.ln_gamma = (float)std::log(g.gamma_b);
        for (int m = 0; m < g.n_modes; ++m) kt.push_back(g.k[m]);
        off += (int64_t)g.n_xi * g.n_modes;
        col += g.n_modes;
    }
    *snap_elems = off;
    *cols = col;
    G_HIP(hipMalloc(d_inst, gi.size() * sizeof(GInst)), "allocate instance table");
    G_HIP(hipMemcpyAsync(*d_inst, gi.data(), gi.size() * sizeof(GInst), hipMemcpyHostToDevice, s), "copy instance table");
    if (d_k) {
        G_HIP(hipMalloc(d_k, kt.size() * sizeof(double)), "allocate k table");
        G_HIP(hipMemcpyAsync(*d_k, kt.data(), kt.size() * sizeof(double), hipMemcpyHostToDevice, s), "copy k table");
    }
    G_HIP(hipStreamSynchronize(s), "synchronize");  // host vectors die here
    return QS_OK;
}

// The growth map's cell width: the finest of the batched sweep, 200/8192, for every beam, so
// that an answer depends on the query alone and not on the length of the beam it comes from.
constexpr double kCellWidth = 200.0 / 8192.0;

// cells of width kCellWidth that cover xi in [0, L]
int cells_for(double L) { return std::max(1, (int)std::ceil(L / kCellWidth - 1e-9)); }

// A query the solver answers: its beam (n_b, gamma), mode k, position, the step d_tau =
// tau_f/200 of its beam, the cells its answer needs, its fractional step tau/d_tau and the
// last step whose fields it reads.
struct SolverQuery {
    int64_t pos;        // position in the selection
    double nb, g, k, xi, d_tau, ts;
    int cells, last;
};

// One solver-answered query: the bilinear interpolation of the discrete windowed growth
// between the two cell centres around its xi and the two steps around its tau.
struct QueryRec {
    int64_t base;     // snapshot element of (instance, mode) at the instance's first stored cell
    int32_t stride;   // the instance's mode count (elements between cells)
    int32_t win;      // window cells
    int32_t j0, s0;   // first cell and first step
    int32_t dst;      // answer slot
    int32_t first;    // the instance's first stored cell
    double fx, ft;    // interpolation weights of cell j0 + 1 and step s0 + 1
    double ln_s;
};

// The windowed growth at cell j of one snapshot column by the direct Hann-weighted sum over
// its window (the definition, in FP64), the window's cells spread over the wavefront's lanes;
// every lane returns the result.
__device__ inline double growth_wave(const float *__restrict__ le, const float *__restrict__ lb, int64_t base,
                                     int32_t stride, int j, int first, int win, double ln_s, int lane) {
    const int cnt = min(j + 1, win);
    double num = 0.0, den = 0.0;
    for (int i = lane; i < cnt; i += qs::kWave) {
        const double s = sin(kPi * (i + 0.5) / win);
        const double w = s * s;
        const int64_t e = base + (int64_t)(j - i - first) * stride;
        num += w * a2_rel(le[e], lb[e], ln_s);
        den += w;
    }
    for (int o = qs::kWave / 2; o > 0; o >>= 1) {
        num += __shfl_xor(num, o);
        den += __shfl_xor(den, o);
    }
    return 0.5 * log(num / den);
}

// One wavefront per record of recs[0, n): the terms of its answer whose step lies in the
// window of snapshots [step_lo, step_lo + n_win) are added to acc[dst] in the order
// (step s0, cell j0), (s0, j0 + 1), (s0 + 1, j0), (s0 + 1, j0 + 1); windows pass in step order,
// so every answer is summed in that order whichever windows hold its two steps.
__global__ void __launch_bounds__(256) answer_kernel(const QueryRec *__restrict__ recs, int n,
                                                     const float *__restrict__ le, const float *__restrict__ lb,
                                                     int64_t snap_elems, int step_lo, int n_win,
                                                     double *__restrict__ acc) {
    const int r = (int)((blockIdx.x * blockDim.x + threadIdx.x) / qs::kWave);
    const int lane = (int)threadIdx.x % qs::kWave;
    if (r >= n) return;
    const QueryRec Q = recs[r];
    double sum = acc[Q.dst];
    for (int c = 0; c < 2; ++c) {
        const double wt = c == 0 ? 1.0 - Q.ft : Q.ft;
        const int t = Q.s0 + c - step_lo;
        if (wt == 0.0 || t < 0 || t >= n_win) continue;
        const int64_t row = Q.base + (int64_t)t * snap_elems;
        for (int d = 0; d < 2; ++d) {
            const double w = wt * (d == 0 ? 1.0 - Q.fx : Q.fx);
            if (w == 0.0) continue;
            sum += w * growth_wave(le, lb, row, Q.stride, Q.j0 + d, Q.first, Q.win, Q.ln_s, lane);
        }
    }
    if (lane == 0) acc[Q.dst] = sum;
}

// Budgets of one solver context: queries, and bytes of state plus snapshots.
constexpr int kChunkQueries = 32768;
constexpr size_t kChunkBytes = size_t(16) << 30;
constexpr int kGroup = 32;   // queries per instance: the modes of one 64-lane column block

// Solver answers for the queries q[a, b), every one a mode of a unit-density instance.  The
// model is linear and tau-invariant, so in units of each query's own step (tau = n d_tau)
// with T'' = d_tau T' and P'' = d_tau P' the step is 1 and the push coefficients become
// d_tau^2 cT Omega and d_tau^2 cP Omega: a beam of density n_b and Lorentz factor gamma is the
// mode with those coefficients in a unit-density instance with unit step (rho, n_p and so
// the fields are unchanged by the rescaling; the uniform seed has no current).  So 32
// queries of any beams fill a wavefront.  The chunk's queries, sorted by the cells they
// need, form instances of 32, each reaching two cells beyond its largest xi; the context
// marches without fields to the first step any query reads, then writes the fields of every
// step up to the last one read into a rolling window of snapshots, and each window's
// answers are accumulated before the next overwrites it.
qs_status solve_chunk(const std::vector<SolverQuery> &all, size_t a, size_t b, hipStream_t s,
                      std::vector<float> *vals) {
    const double S = 1e-6;
    const int nq = (int)(b - a);
    std::vector<SolverQuery> q(all.begin() + a, all.begin() + b);
    std::stable_sort(q.begin(), q.end(), [](const SolverQuery &x, const SolverQuery &y) { return x.cells < y.cells; });
    const int n_inst = (nq + kGroup - 1) / kGroup;
    std::vector<double> ks(nq), cT(nq), cP(nq);
    for (int i = 0; i < nq; ++i) {
        const SolverQuery &Q = q[i];
        const double k = Q.k, kp = 1.0 / (1.0 + k * k), d2 = Q.d_tau * Q.d_tau;
        ks[i] = k;
        cT[i] = d2 * k * k * kp * Q.nb / Q.g;                          // Omega = n_b, gamma^-1
        cP[i] = -d2 * kp * Q.nb / (Q.g * Q.g * Q.g) / kCellWidth;       // gamma^-3, 1/h
    }
    static const double qv[1] = {-1.0}, mv[1] = {1.0}, nbv[1] = {1.0};
    const int win = window_cells(kCellWidth);
    std::vector<qs_params> ps(n_inst);
    std::vector<int32_t> first(n_inst);
    std::vector<QueryRec> recs(nq);
    int64_t snap = 0;
    int s_min = 1 << 30, s_max = 0;
    for (int g = 0; g < n_inst; ++g) {
        const int i0 = g * kGroup, i1 = std::min(nq, i0 + kGroup);
        const int N = q[i1 - 1].cells;   // the group's largest
        qs_params &p = ps[g];
        std::memset(&p, 0, sizeof(p));
        p.n_species = 1;
        p.q = qv;
        p.m = mv;
        p.nb_over_np = nbv;
        p.gamma_b = 2.0;   // its push coefficients are replaced below
        p.length = N * kCellWidth;
        p.profile = QS_PROFILE_FLATTOP;
        p.geometry = QS_GEOM_SPECTRAL;
        p.n_modes = i1 - i0;
        p.kx = ks.data() + i0;
        p.n_xi = N;
        p.d_tau = 1.0;
        p.precision = QS_FP32;
        p.seed_kind = QS_SEED_UNIFORM;
        p.seed_amp = S;
        int jmin = N;
        for (int i = i0; i < i1; ++i) {
            const SolverQuery &Q = q[i];
            QueryRec &r = recs[i];
            r.stride = i1 - i0;
            r.win = win;
            // cells: centres (j + 1/2) h around xi (clamped to the first and last cell)
            const double xc = Q.xi / kCellWidth - 0.5;
            r.j0 = (int)std::floor(xc);
            r.fx = xc - r.j0;
            if (r.j0 < 0) { r.j0 = 0; r.fx = 0.0; }
            if (r.j0 >= N - 1) { r.j0 = N - 1; r.fx = 0.0; }
            r.s0 = (int)std::floor(Q.ts);
            r.ft = Q.ts - r.s0;
            r.ln_s = std::log(S);
            r.dst = i;
            jmin = std::min(jmin, r.j0);
            s_min = std::min(s_min, r.s0);
            s_max = std::max(s_max, Q.last);
        }
        // the snapshots keep the cells any window of the group reads: from its lowest cell on
        // (the group's queries lie within a few cells of each other, near its rear)
        first[g] = std::max(0, jmin - win + 1);
        for (int i = i0; i < i1; ++i) {
            recs[i].base = snap + (i - i0);
            recs[i].first = first[g];
        }
        snap += (int64_t)(N - first[g]) * (i1 - i0);
    }
    // records in step order: a window of steps [lo, hi) serves those with lo - 1 <= s0 < hi
    std::stable_sort(recs.begin(), recs.end(), [](const QueryRec &x, const QueryRec &y) { return x.s0 < y.s0; });
    std::vector<int> rs0(nq);
    for (int i = 0; i < nq; ++i) rs0[i] = recs[i].s0;

    qs_ctx *ctx = nullptr;
    qs_status st = qs_init(ps.data(), n_inst, s, nullptr, 0, &ctx);
    if (st != QS_OK) return st;
    st = qs::set_mode_coefficients(ctx, cT.data(), cP.data());
    int64_t snap_ctx = 0;
    if (st == QS_OK) st = qs::set_snapshot_cells(ctx, first.data(), &snap_ctx);
    if (st == QS_OK && snap_ctx != snap) st = gfail(QS_ERR_HIP, "growth map: snapshot layout mismatch");
    if (st != QS_OK) {
        qs_free(ctx);
        return st;
    }
    const size_t state_bytes = qs_workspace_size_ex(ps.data(), n_inst, nullptr);
    const size_t per_snap = (size_t)snap * 2 * sizeof(float);
    const size_t room = kChunkBytes > state_bytes ? kChunkBytes - state_bytes : 0;
    const int n_win = (int)std::max<size_t>(1, std::min<size_t>((size_t)(s_max - s_min + 1), room / per_snap));
    char *buf = nullptr;
    const size_t snap_bytes = ((per_snap * n_win + 255) / 256) * 256;
    const size_t rec_bytes = ((recs.size() * sizeof(QueryRec) + 255) / 256) * 256;
    if (hipMalloc(&buf, snap_bytes + rec_bytes + (size_t)nq * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        qs_free(ctx);
        return gfail(QS_ERR_ALLOC, "growth map: snapshot buffers");
    }
    float *le = reinterpret_cast<float *>(buf), *lb = le + (size_t)snap * n_win;
    QueryRec *d_recs = reinterpret_cast<QueryRec *>(buf + snap_bytes);
    double *d_acc = reinterpret_cast<double *>(buf + snap_bytes + rec_bytes);
    if (hipMemcpyAsync(d_recs, recs.data(), recs.size() * sizeof(QueryRec), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(d_acc, 0, (size_t)nq * sizeof(double), s) != hipSuccess)
        st = gfail(QS_ERR_HIP, "growth map: copy query records");
    if (st == QS_OK && s_min > 0) st = qs_step_tau(ctx, s_min, 1, nullptr, nullptr, nullptr);
    for (int lo = s_min; st == QS_OK && lo <= s_max;) {
        const int cnt = std::min(n_win, s_max + 1 - lo);   // snapshots of steps lo .. lo + cnt - 1
        // the state at the start of step lo + cnt - 1 is the last one written: a stepping call
        // writes the state before each of its steps, so the last snapshot of the run, at
        // s_max, comes from a call that only writes the current state
        const bool last = lo + cnt - 1 == s_max;
        const int n_steps = last ? cnt - 1 : cnt;
        if (n_steps > 0) st = qs_step_tau(ctx, n_steps, 1, le, lb, nullptr);
        if (st == QS_OK && last)
            st = qs_step_tau(ctx, 0, 1, le + (size_t)snap * n_steps, lb + (size_t)snap * n_steps, nullptr);
        const int ra = (int)(std::lower_bound(rs0.begin(), rs0.end(), lo - 1) - rs0.begin());
        const int rb = (int)(std::lower_bound(rs0.begin(), rs0.end(), lo + cnt) - rs0.begin());
        if (st == QS_OK && rb > ra) {
            const int64_t threads = (int64_t)(rb - ra) * qs::kWave;
            hipLaunchKernelGGL(answer_kernel, dim3(blocks_for(threads)), dim3(256), 0, s, d_recs + ra, rb - ra, le, lb,
                               snap, lo, cnt, d_acc);
            if (hipGetLastError() != hipSuccess) st = gfail(QS_ERR_HIP, "growth map: answer kernel");
        }
        lo += cnt;
    }
    std::vector<double> hv(nq);
    if (st == QS_OK && (hipMemcpyAsync(hv.data(), d_acc, hv.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
        st = gfail(QS_ERR_HIP, "growth map: copy answers");
    if (st == QS_OK) st = qs_sync_check(ctx);
    if (st == QS_OK)
        for (int i = 0; i < nq; ++i) (*vals)[q[i].pos] = (float)hv[i];
    (void)hipFree(buf);
    qs_free(ctx);
    return st;
}


// Solver answers vals[i] for the queries rows[5 i .. 5 i + 4] (host), i < sel.size(); sel[i] is
// the query's position in the caller's array (named in errors).
qs_status solve_queries(const float *rows, const std::vector<int64_t> &sel, hipStream_t s, std::vector<float> *vals) {
    // the solver needs a physical beam and a point on or behind its front at tau >= 0; the
    // step count follows tau (tau_f/200 per step), so tau beyond tau_f marches further
    for (size_t i = 0; i < sel.size(); ++i) {
        const int64_t p = sel[i];
        const float *q = rows + 5 * i;
        bool ok = true;
        for (int d = 0; d < 5; ++d) ok = ok && std::isfinite(q[d]);
        ok = ok && q[1] > 0.0f && q[2] >= 0.0f && q[3] >= 0.0f && q[4] >= 0.0f;
        if (ok) ok = (double)q[4] / (tau_final(std::exp((double)q[0]), std::exp((double)q[1])) / 200.0) < 2.0e6;
        if (!ok)
            return gfail(QS_ERR_ARG, "query " + std::to_string(p) +
                                         " cannot go to the solver: it needs finite values, gamma > 1, k >= 0, "
                                         "xi >= 0 and 0 <= tau <= 1e4 tau_f");
    }
    std::vector<SolverQuery> q(sel.size());
    for (size_t i = 0; i < sel.size(); ++i) {
        const float *x = rows + 5 * i;
        SolverQuery &Q = q[i];
        Q.pos = (int64_t)i;
        Q.nb = std::exp((double)x[0]);
        Q.g = std::exp((double)x[1]);
        Q.k = (double)x[2];
        Q.xi = (double)x[3];
        Q.d_tau = tau_final(Q.nb, Q.g) / 200.0;
        Q.ts = (double)x[4] / Q.d_tau;
        const int s0 = (int)std::floor(Q.ts);
        Q.last = s0 + (Q.ts > s0 ? 1 : 0);
        // two cells beyond xi: the cell centre behind the query is in the beam and is not the
        // last cell (the beam's rear face carries no current, which changes the last cell's
        // charge -- and only that cell's, the march being causal)
        Q.cells = cells_for(Q.xi + 2.0 * kCellWidth);
    }
    // chunks of consecutive queries in the order of the last step they read: a chunk
    // marches to its largest, so queries of similar steps share one; within the budgets of
    // queries and of state plus one snapshot per chunk
    std::sort(q.begin(), q.end(), [](const SolverQuery &x, const SolverQuery &y) {
        return x.last != y.last ? x.last < y.last : (x.cells != y.cells ? x.cells < y.cells : x.pos < y.pos);
    });
    vals->assign(sel.size(), 0.f);
    size_t a = 0;
    while (a < q.size()) {
        size_t b = a, cells = 0;
        while (b < q.size() && b - a < (size_t)kChunkQueries) {
            // state (3 rows of 64 lanes per 32 queries) and one snapshot, from the query's own
            // cells (every instance reaches its largest: bounded by the next query's cells)
            const size_t c = (size_t)q[b].cells;
            if (b > a && (cells + c) * (24 + 8) * 2 > kChunkBytes) break;
            cells += c;
            ++b;
        }
        qs_status st = solve_chunk(q, a, b, s, vals);
        if (st != QS_OK) return st;
        a = b;
    }
    return QS_OK;
}

}  // namespace

extern "C" {

qs_status qs_growth_targets(const qs_growth_instance *inst, int32_t n_inst, const float *ln_e, const float *ln_b,
                            int32_t n_snap, float *G, void *hip_stream) {
    qs_status st = check_insts(inst, n_inst);
    if (st != QS_OK) return st;
    if (!ln_e || !ln_b || !G || n_snap < 1) return gfail(QS_ERR_ARG, "ln_e, ln_b, G and n_snap >= 1 are required");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    GInst *d_inst = nullptr;
    int64_t snap = 0, cols = 0;
    st = upload_insts(inst, n_inst, s, &d_inst, nullptr, &snap, &cols);
    if (st != QS_OK) return st;
    hipLaunchKernelGGL(targets_kernel, dim3(blocks_for(cols * n_snap)), dim3(256), 0, s, d_inst, n_inst, ln_e, ln_b,
                       snap, cols, n_snap, G);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_inst);
    if (e != hipSuccess) return gfail(QS_ERR_HIP, std::string("targets kernel: ") + hipGetErrorString(e));
    return QS_OK;
}

qs_status qs_growth_sample(const qs_growth_instance *inst, int32_t n_inst, const float *G, int32_t n_snap,
                           const int32_t *snap_step, uint64_t seed, int64_t n, float *Q, float *T, void *hip_stream) {
    qs_status st = check_insts(inst, n_inst);
    if (st != QS_OK) return st;
    if (!G || !snap_step || n_snap < 1 || n < 0 || (n > 0 && (!Q || !T)))
        return gfail(QS_ERR_ARG, "G, snap_step, n_snap >= 1, n >= 0, Q and T are required");
    if (n == 0) return QS_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    GInst *d_inst = nullptr;
    double *d_k = nullptr;
    int64_t snap = 0, cols = 0;
    st = upload_insts(inst, n_inst, s, &d_inst, &d_k, &snap, &cols);
    if (st != QS_OK) return st;
    int32_t *d_steps = nullptr;
    hipError_t e = hipMalloc(&d_steps, n_snap * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpyAsync(d_steps, snap_step, n_snap * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(sample_kernel, dim3(blocks_for(n)), dim3(256), 0, s, d_inst, n_inst, d_k, G, snap, d_steps,
                           n_snap, seed, n, Q, T);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_inst);
    (void)hipFree(d_k);
    if (d_steps) (void)hipFree(d_steps);
    if (e != hipSuccess) return gfail(QS_ERR_HIP, std::string("sample kernel: ") + hipGetErrorString(e));
    return QS_OK;
}

qs_status qs_growth_features(const float *q, int64_t n, float *x, float *baseline, void *hip_stream) {
    if (n < 0 || (n > 0 && (!q || (!x && !baseline)))) return gfail(QS_ERR_ARG, "q and x or baseline are required");
    if (n == 0) return QS_OK;
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), q, n,
                       x, baseline);
    G_HIP(hipGetLastError(), "features kernel");
    return QS_OK;
}

qs_status qs_growth_calibrate(qs_mlp *net, const float *Q, const float *T, int64_t n, float *table) {
    if (!net || !table || n < 0 || (n > 0 && (!Q || !T))) return gfail(QS_ERR_ARG, "net, Q, T and table are required");
    hipStream_t s = qs::mlp_stream(net);
    float *buf = nullptr;  // inputs [n][5], baseline [n], answers [n]
    uint32_t *cnt = nullptr;
    if (n > 0) G_HIP(hipMalloc(&buf, (size_t)n * 7 * sizeof(float)), "allocate calibration buffers");
    if (hipMalloc(&cnt, (size_t)QS_GROWTH_BINS * kBuckets * sizeof(uint32_t)) != hipSuccess) {
        if (buf) (void)hipFree(buf);
        return gfail(QS_ERR_ALLOC, "allocate histogram");
    }
    float *x = buf, *base = buf ? buf + (size_t)n * 5 : nullptr, *y = buf ? buf + (size_t)n * 6 : nullptr;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks_for((int64_t)QS_GROWTH_BINS * kBuckets)), dim3(256), 0, s,
                       reinterpret_cast<float *>(cnt), (int64_t)QS_GROWTH_BINS * kBuckets, 0.0f);
    qs_status st = QS_OK;
    if (n > 0) {
        hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n)), dim3(256), 0, s, Q, n, x, base);
        st = qs_mlp_forward(net, x, n, y);
        if (st == QS_OK) hipLaunchKernelGGL(hist_kernel, dim3(blocks_for(n)), dim3(256), 0, s, Q, y, base, T, n, cnt);
    }
    if (st == QS_OK) hipLaunchKernelGGL(p99_kernel, dim3(blocks_for(QS_GROWTH_BINS)), dim3(256), 0, s, cnt, table);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (buf) (void)hipFree(buf);
    (void)hipFree(cnt);
    if (st != QS_OK) return st;
    if (e != hipSuccess) return gfail(QS_ERR_HIP, std::string("calibration: ") + hipGetErrorString(e));
    return QS_OK;
}

qs_status qs_growth_map_noalloc(qs_mlp *net, const float *table, float tol, const float *q, int64_t n, float *out,
                                uint8_t *needs_solver) {
    if (!net) return gfail(QS_ERR_ARG, "the network is required");
    if (n < 0 || (n > 0 && (!q || !out || !needs_solver))) return gfail(QS_ERR_ARG, "q, out and needs_solver are required");
    if (n > QS_GROWTH_NOALLOC_MAX)
        return gfail(QS_ERR_ARG, "n = " + std::to_string(n) + " queries exceed the scratch of this entry point (at most " +
                                     std::to_string((long long)QS_GROWTH_NOALLOC_MAX) + " per call)");
    const int dev = qs::mlp_device(net);
    G_HIP(hipSetDevice(dev), "hipSetDevice");
    if (n == 0) return QS_OK;
    float *x = nullptr;
    qs_status st = scratch_for_device(dev, &x);
    if (st != QS_OK) return st;
    float *base = x + (size_t)n * 5;
    hipStream_t s = qs::mlp_stream(net);
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n)), dim3(256), 0, s, q, n, x, base);
    G_HIP(hipGetLastError(), "features kernel");
    st = qs_mlp_forward(net, x, n, out);
    if (st != QS_OK) return st;
    hipLaunchKernelGGL(finish_kernel, dim3(blocks_for(n)), dim3(256), 0, s, q, n, base, out, table, tol, needs_solver);
    G_HIP(hipGetLastError(), "finishing kernel");
    return QS_OK;
}

qs_status qs_growth_map(qs_mlp *net, const float *table, float tol, const float *q, int64_t n, int32_t mode,
                        float *out, uint8_t *used_solver, void *hip_stream) {
    if (n < 0 || (n > 0 && (!q || !out))) return gfail(QS_ERR_ARG, "q and out are required");
    if (mode != QS_GROWTH_SURROGATE && mode != QS_GROWTH_SOLVER && mode != QS_GROWTH_AUTO)
        return gfail(QS_ERR_ARG, "unknown mode");
    if (mode != QS_GROWTH_SOLVER && !net) return gfail(QS_ERR_ARG, "the surrogate modes need a network");
    if (n == 0) return QS_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    float *x = nullptr;
    uint8_t *flag = nullptr;
    qs_status st = QS_OK;
    auto cleanup = [&]() {
        if (x) (void)hipFree(x);
        if (flag && flag != used_solver) (void)hipFree(flag);
    };
    float *base = nullptr;
    if (mode != QS_GROWTH_SOLVER) {
        G_HIP(hipMalloc(&x, (size_t)n * 6 * sizeof(float)), "allocate features");
        base = x + (size_t)n * 5;
        hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n)), dim3(256), 0, s, q, n, x, base);
        if (hipStreamSynchronize(s) != hipSuccess) { cleanup(); return gfail(QS_ERR_HIP, "features kernel"); }
        st = qs_mlp_forward(net, x, n, out);
        if (st == QS_OK && hipStreamSynchronize(qs::mlp_stream(net)) != hipSuccess) st = gfail(QS_ERR_HIP, "network");
        if (st != QS_OK) { cleanup(); return st; }
    }
    if (mode == QS_GROWTH_SURROGATE) {
        hipLaunchKernelGGL(finish_kernel, dim3(blocks_for(n)), dim3(256), 0, s, q, n, base, out, nullptr, 0.0f, nullptr);
        if (used_solver && hipMemsetAsync(used_solver, 0, (size_t)n, s) != hipSuccess) { cleanup(); return gfail(QS_ERR_HIP, "clear flags"); }
        cleanup();
        G_HIP(hipStreamSynchronize(s), "synchronize");
        return QS_OK;
    }
    // which queries go to the solver, with their rows, in the order of their positions
    std::vector<int64_t> sel;
    std::vector<float> rows;
    if (mode == QS_GROWTH_AUTO) {
        flag = used_solver;
        if (!flag && hipMalloc(&flag, (size_t)n) != hipSuccess) { cleanup(); return gfail(QS_ERR_ALLOC, "allocate flags"); }
        hipLaunchKernelGGL(finish_kernel, dim3(blocks_for(n)), dim3(256), 0, s, q, n, base, out, table, tol, flag);
        // the flagged queries are compacted on the device: a first pass counts them into a
        // buffer for up to 65536, a second pass fills one of the counted size if they are more
        int64_t cap = std::min<int64_t>(n, 65536), cnt = 0;
        for (int pass = 0; pass < 2; ++pass) {
            char *sb = nullptr;
            const size_t bytes = 256 + (size_t)cap * (sizeof(int64_t) + 5 * sizeof(float));
            if (hipMalloc(&sb, bytes) != hipSuccess) { (void)hipGetLastError(); cleanup(); return gfail(QS_ERR_ALLOC, "allocate selection"); }
            auto *d_cnt = reinterpret_cast<unsigned long long *>(sb);
            auto *d_idx = reinterpret_cast<int64_t *>(sb + 256);
            auto *d_rows = reinterpret_cast<float *>(sb + 256 + (size_t)cap * sizeof(int64_t));
            unsigned long long hc = 0;
            hipError_t e = hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long), s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(select_kernel, dim3(blocks_for(n)), dim3(256), 0, s, q, flag, n, d_cnt, d_idx, d_rows, cap);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipMemcpyAsync(&hc, d_cnt, sizeof(hc), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            cnt = (int64_t)hc;
            std::vector<int64_t> hi;
            std::vector<float> hr;
            if (e == hipSuccess && cnt <= cap) {
                hi.resize((size_t)cnt);
                hr.resize((size_t)cnt * 5);
                if (cnt > 0) e = hipMemcpyAsync(hi.data(), d_idx, hi.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess && cnt > 0) e = hipMemcpyAsync(hr.data(), d_rows, hr.size() * sizeof(float), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
            }
            (void)hipFree(sb);
            if (e != hipSuccess) { cleanup(); return gfail(QS_ERR_HIP, std::string("select solver queries: ") + hipGetErrorString(e)); }
            if (cnt > cap) { cap = cnt; continue; }
            std::vector<int64_t> order((size_t)cnt);
            for (int64_t i = 0; i < cnt; ++i) order[i] = i;
            std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return hi[x] < hi[y]; });
            sel.resize((size_t)cnt);
            rows.resize((size_t)cnt * 5);
            for (int64_t i = 0; i < cnt; ++i) {
                sel[i] = hi[order[i]];
                for (int d = 0; d < 5; ++d) rows[5 * i + d] = hr[5 * order[i] + d];
            }
            break;
        }
    } else {
        rows.resize((size_t)n * 5);
        G_HIP(hipMemcpyAsync(rows.data(), q, rows.size() * sizeof(float), hipMemcpyDeviceToHost, s), "copy queries");
        G_HIP(hipStreamSynchronize(s), "synchronize");
        sel.resize((size_t)n);
        for (int64_t i = 0; i < n; ++i) sel[i] = i;
    }
    if (!sel.empty()) {
        std::vector<float> vals;
        st = solve_queries(rows.data(), sel, s, &vals);
        if (st == QS_OK) {
            int64_t *d_idx = nullptr;
            float *d_val = nullptr;
            hipError_t e = hipMalloc(&d_idx, sel.size() * sizeof(int64_t));
            if (e == hipSuccess) e = hipMalloc(&d_val, sel.size() * sizeof(float));
            if (e == hipSuccess) e = hipMemcpyAsync(d_idx, sel.data(), sel.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(d_val, vals.data(), vals.size() * sizeof(float), hipMemcpyHostToDevice, s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for((int64_t)sel.size())), dim3(256), 0, s, d_idx, d_val,
                                   (int64_t)sel.size(), out, mode == QS_GROWTH_SOLVER ? used_solver : nullptr);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (d_idx) (void)hipFree(d_idx);
            if (d_val) (void)hipFree(d_val);
            if (e != hipSuccess) st = gfail(QS_ERR_HIP, std::string("scatter solver answers: ") + hipGetErrorString(e));
        }
    }
    cleanup();
    return st;
}

}  // extern "C"
