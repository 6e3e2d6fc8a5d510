// Growth maps (include/qs_growth.h): windowed-growth targets from solver snapshots, training
// examples drawn from them, the surrogate's feature map, the held-out error table, and the
// query entry point with its solver fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/qs_growth.h"
#include "qs_internal.h"

// Scratch of the allocation-free query entry point: the features of at most
// QS_GROWTH_NOALLOC_MAX queries (5 MiB).  Each device holds its own copy, from the library's
// load until the process ends; every call on a device shares it.
static __device__ __align__(256) float scratch[(size_t)QS_GROWTH_NOALLOC_MAX * 5];

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kBinsPerFeature = 8;

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
    float f_nb, f_gamma;  // features 0 and 1
    double tau_f;
};

// cells in one plasma wavelength 2 pi (at least one)
int window_cells(double h) { return std::max(1, (int)std::lround(kTwoPi / h)); }

__host__ __device__ inline float feat_nb(double nb) { return (float)(log10(nb) + 2.0); }
__host__ __device__ inline float feat_gamma(double g) { return (float)((log10(g) - 2.5) / 1.5); }
__host__ __device__ inline float feat_k(double k) { return (float)((k - 2.025) / 1.975); }
__host__ __device__ inline float feat_xi(double xi) { return (float)(xi / 100.0 - 1.0); }
__host__ __device__ inline double tau_final(double nb, double g) { return 10.0 * sqrt(g / nb); }

// A^2 / S^2 of one entry from ln|E| and ln|B| (exp of -inf is 0)
__device__ inline double a2_rel(float le, float lb, double ln_s) {
    return exp(2.0 * ((double)le - ln_s)) + exp(2.0 * ((double)lb - ln_s));
}

// One thread per (snapshot, column): sliding window over the cells, recomputed exactly at
// every multiple of the window length so that rounding does not accumulate.
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
    const int M = I.n_modes, W = I.win;
    double sum = 0.0;
    for (int j = 0; j < I.n_xi; ++j) {
        if (j % W == 0 && j > 0) {  // exact re-summation of the window ending at j - 1
            sum = 0.0;
            for (int i = j - W; i < j; ++i) sum += a2_rel(le[base + (int64_t)i * M], lb[base + (int64_t)i * M], I.ln_s);
        }
        sum += a2_rel(le[base + (int64_t)j * M], lb[base + (int64_t)j * M], I.ln_s);
        if (j >= W) sum -= a2_rel(le[base + (int64_t)(j - W) * M], lb[base + (int64_t)(j - W) * M], I.ln_s);
        const int cnt = min(j + 1, W);
        G[base + (int64_t)j * M] = (float)(0.5 * log(fmax(sum, 0.0) / cnt));
    }
}

__device__ inline uint64_t sm64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) sample_kernel(const GInst *__restrict__ inst, int n_inst,
                                                     const double *__restrict__ kt, const float *__restrict__ G,
                                                     int64_t snap_elems, const int32_t *__restrict__ steps, int n_snap,
                                                     uint64_t seed, int64_t n, float *__restrict__ X,
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
    const int64_t q = r - I.off;
    const int j = (int)(q / I.n_modes), m = (int)(q % I.n_modes);
    const double xi = (j + 0.5) * I.h;
    const double tau = steps[t] * I.d_tau;
    X[5 * i + 0] = I.f_nb;
    X[5 * i + 1] = I.f_gamma;
    X[5 * i + 2] = feat_k(kt[I.k0 + m]);
    X[5 * i + 3] = feat_xi(xi);
    X[5 * i + 4] = (float)(2.0 * tau / I.tau_f - 1.0);
    T[i] = G[e];
}

__global__ void __launch_bounds__(256) features_kernel(const float *__restrict__ q, int64_t n, float *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double nb = exp((double)q[5 * i]), g = exp((double)q[5 * i + 1]);
    x[5 * i + 0] = feat_nb(nb);
    x[5 * i + 1] = feat_gamma(g);
    x[5 * i + 2] = feat_k(q[5 * i + 2]);
    x[5 * i + 3] = feat_xi(q[5 * i + 3]);
    x[5 * i + 4] = (float)(2.0 * (double)q[5 * i + 4] / tau_final(nb, g) - 1.0);
}

__device__ inline int bin_of(const float *x) {
    int b = 0;
    for (int d = 0; d < 5; ++d) {
        int c = (int)floorf((x[d] + 1.0f) * (kBinsPerFeature / 2));
        c = min(kBinsPerFeature - 1, max(0, c));
        b = b * kBinsPerFeature + c;
    }
    return b;
}

__global__ void __launch_bounds__(256) fill_kernel(float *p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Held-out error histogram: bucket 0 holds |y - t| <= e0, bucket b >= 1 the range
// (e0 2^((b-1)/4), e0 2^(b/4)], the last bucket everything above (and non-finite errors).
constexpr int kBuckets = 64;
constexpr float kE0 = 1e-4f;
constexpr int kMinCount = 32;  // fewer held-out examples in a bin: no estimate

__host__ __device__ inline float bucket_edge(int b) {
    return b >= kBuckets - 1 ? 3.0e38f : kE0 * exp2f(0.25f * (float)b);
}

__global__ void __launch_bounds__(256) hist_kernel(const float *__restrict__ x, const float *__restrict__ y,
                                                   const float *__restrict__ t, int64_t n, uint32_t *__restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float e = fabsf(y[i] - t[i]);
    int b;
    if (!(e <= 3.0e38f)) b = kBuckets - 1;
    else if (e <= kE0) b = 0;
    else b = min(kBuckets - 1, 1 + (int)floorf(4.0f * log2f(e / kE0)));
    atomicAdd(cnt + (int64_t)bin_of(x + 5 * i) * kBuckets + b, 1u);
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

// 1 where the solver must answer: outside the box, no held-out data in the bin, or the
// bin's held-out error above tol
__global__ void __launch_bounds__(256) route_kernel(const float *__restrict__ x, int64_t n,
                                                    const float *__restrict__ table, float tol,
                                                    uint8_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool inside = true;
    for (int d = 0; d < 5; ++d) inside = inside && x[5 * i + d] >= -1.0f && x[5 * i + d] <= 1.0f;
    const float e = table ? table[bin_of(x + 5 * i)] : -1.0f;
    flag[i] = (inside && e >= 0.0f && e <= tol) ? 0 : 1;
}

__global__ void __launch_bounds__(256) scatter_kernel(const int64_t *__restrict__ idx, const float *__restrict__ val,
                                                      int64_t n, float *__restrict__ out, uint8_t *__restrict__ used) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[idx[i]] = val[i];
    if (used) used[idx[i]] = 1;
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
        d.f_nb = feat_nb(g.nb_over_np);
        d.f_gamma = feat_gamma(g.gamma_b);
        d.tau_f = tau_final(g.nb_over_np, g.gamma_b);
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

// cells of the batched sweep's discretization for a beam of length L
int cells_for(double L) {
    if (L >= 5.0) return (int)std::lround(128.0 + 8064.0 * (L - 5.0) / 195.0);
    return std::max(1, (int)std::lround(128.0 * L / 5.0));
}

// Solver answers for the queries hq[5 i..] at positions sel; values returned in vals.
struct Group {
    double nb, g, L = 0.0;
    std::vector<double> ks;
    std::vector<int64_t> members;  // positions in the selection
};

// Solver answers for the selected queries of groups [g0, g1): one batched context, one
// instance per group, marched to each distinct step in turn.
qs_status solve_groups(const std::vector<float> &hq, const std::vector<int64_t> &sel,
                       const std::vector<Group> &groups, size_t g0, size_t g1, hipStream_t s,
                       std::vector<float> *vals) {
    const double S = 1e-6;
    const int n_steps_max = 200;  // steps of tau_f
    const size_t ng = g1 - g0;
    std::vector<qs_params> params(ng);
    std::vector<double> qv(1, -1.0), mv(1, 1.0);
    std::vector<std::vector<double>> nbv(ng);
    std::vector<qs_growth_instance> gis(ng);
    for (size_t i = 0; i < ng; ++i) {
        const Group &G = groups[g0 + i];
        nbv[i] = {G.nb};
        qs_params &p = params[i];
        std::memset(&p, 0, sizeof(p));
        p.n_species = 1;
        p.q = qv.data();
        p.m = mv.data();
        p.nb_over_np = nbv[i].data();
        p.gamma_b = G.g;
        p.length = G.L;
        p.profile = QS_PROFILE_FLATTOP;
        p.geometry = QS_GEOM_SPECTRAL;
        p.n_modes = (int64_t)G.ks.size();
        p.kx = const_cast<double *>(G.ks.data());
        p.n_xi = cells_for(G.L);
        p.d_tau = tau_final(G.nb, G.g) / n_steps_max;
        p.precision = QS_FP32;
        p.seed_kind = QS_SEED_UNIFORM;
        p.seed_amp = S;
        gis[i] = qs_growth_instance{G.nb, G.g, G.L, p.d_tau, S, p.n_xi, (int32_t)p.n_modes, p.kx};
    }
    qs_ctx *ctx = nullptr;
    qs_status st = qs_init(params.data(), (int32_t)params.size(), s, nullptr, 0, &ctx);
    if (st != QS_OK) return st;
    int64_t snap = 0;
    for (const qs_growth_instance &g : gis) snap += (int64_t)g.n_xi * g.n_modes;
    float *buf = nullptr;
    if (hipMalloc(&buf, (size_t)snap * 3 * sizeof(float)) != hipSuccess) {
        qs_free(ctx);
        return gfail(QS_ERR_ALLOC, "growth map: snapshot buffers");
    }
    float *le = buf, *lb = buf + snap, *Gd = buf + 2 * snap;
    // queries by step
    std::vector<std::pair<int, int64_t>> order;  // (step, position in sel)
    std::map<int64_t, int> gof;  // position in sel -> local group
    for (size_t i = 0; i < ng; ++i)
        for (int64_t p : groups[g0 + i].members) {
            gof[p] = (int)i;
            const float *q = &hq[5 * (size_t)sel[p]];
            const int stp = (int)std::lround((double)q[4] / params[i].d_tau);  // tau >= 0 (checked)
            order.push_back({stp, p});
        }
    std::sort(order.begin(), order.end());
    std::vector<int64_t> goff(ng);
    {
        int64_t o = 0;
        for (size_t i = 0; i < ng; ++i) { goff[i] = o; o += (int64_t)gis[i].n_xi * gis[i].n_modes; }
    }
    std::vector<float> hG(snap);
    int done = 0;
    size_t a = 0;
    while (a < order.size() && st == QS_OK) {
        const int stp = order[a].first;
        if (stp > done) st = qs_step_tau(ctx, stp - done, 1, nullptr, nullptr, nullptr);
        done = stp;
        if (st == QS_OK) st = qs_step_tau(ctx, 0, 1, le, lb, nullptr);
        if (st == QS_OK) st = qs_growth_targets(gis.data(), (int32_t)gis.size(), le, lb, 1, Gd, s);
        if (st == QS_OK && hipMemcpyAsync(hG.data(), Gd, (size_t)snap * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
            st = gfail(QS_ERR_HIP, "growth map: copy targets");
        if (st == QS_OK && hipStreamSynchronize(s) != hipSuccess) st = gfail(QS_ERR_HIP, "growth map: synchronize");
        for (; st == QS_OK && a < order.size() && order[a].first == stp; ++a) {
            const int64_t p = order[a].second;
            const int i = gof.at(p);
            const float *q = &hq[5 * (size_t)sel[p]];
            const double h = gis[i].length / gis[i].n_xi;
            const int j = std::min(gis[i].n_xi - 1, std::max(0, (int)std::ceil((double)q[3] / h) - 1));
            const auto &ks = groups[g0 + i].ks;
            const int m = (int)(std::lower_bound(ks.begin(), ks.end(), (double)q[2]) - ks.begin());
            (*vals)[p] = hG[goff[i] + (int64_t)j * gis[i].n_modes + m];
        }
    }
    if (st == QS_OK) st = qs_sync_check(ctx);
    (void)hipFree(buf);
    qs_free(ctx);
    return st;
}


qs_status solve_queries(const std::vector<float> &hq, const std::vector<int64_t> &sel, hipStream_t s,
                        std::vector<float> *vals) {
    // the solver needs a physical beam and a point on or behind its front at tau >= 0; the
    // step count follows tau (tau_f/200 per step), so tau beyond tau_f marches further
    for (int64_t p : sel) {
        const float *q = &hq[5 * (size_t)p];
        bool ok = true;
        for (int d = 0; d < 5; ++d) ok = ok && std::isfinite(q[d]);
        ok = ok && q[1] > 0.0f && q[2] >= 0.0f && q[3] >= 0.0f && q[4] >= 0.0f;
        if (ok) ok = (double)q[4] / (tau_final(std::exp((double)q[0]), std::exp((double)q[1])) / 200.0) < 2.0e6;
        if (!ok)
            return gfail(QS_ERR_ARG, "query " + std::to_string(p) +
                                         " cannot go to the solver: it needs finite values, gamma > 1, k >= 0, "
                                         "xi >= 0 and 0 <= tau <= 1e4 tau_f");
    }
    std::map<std::pair<uint32_t, uint32_t>, int> gid;
    std::vector<Group> groups;
    for (size_t p = 0; p < sel.size(); ++p) {
        const float *q = &hq[5 * (size_t)sel[p]];
        const auto key = std::make_pair(__builtin_bit_cast(uint32_t, q[0]), __builtin_bit_cast(uint32_t, q[1]));
        auto it = gid.find(key);
        int id;
        if (it == gid.end()) {
            id = (int)groups.size();
            gid[key] = id;
            groups.emplace_back();
            groups.back().nb = std::exp((double)q[0]);
            groups.back().g = std::exp((double)q[1]);
        } else {
            id = it->second;
        }
        Group &G = groups[id];
        G.L = std::max(G.L, (double)q[3]);
        G.ks.push_back((double)q[2]);
        G.members.push_back((int64_t)p);
    }
    vals->assign(sel.size(), 0.f);
    for (Group &G : groups) {
        std::sort(G.ks.begin(), G.ks.end());
        G.ks.erase(std::unique(G.ks.begin(), G.ks.end()), G.ks.end());
        G.L = std::max(G.L, 1e-3);
    }
    // run the groups in chunks whose solver state stays within a fixed budget
    const size_t kBudget = size_t(8) << 30;  // bytes of FP32 state per chunk
    size_t g0 = 0;
    while (g0 < groups.size()) {
        size_t g1 = g0, bytes = 0;
        while (g1 < groups.size()) {
            const size_t blocks = (groups[g1].ks.size() + 31) / 32;
            const size_t b = blocks * (size_t)cells_for(groups[g1].L) * 3 * 64 * 4;
            if (g1 > g0 && (bytes + b > kBudget || g1 - g0 >= 65536)) break;
            bytes += b;
            ++g1;
        }
        qs_status st = solve_groups(hq, sel, groups, g0, g1, s, vals);
        if (st != QS_OK) return st;
        g0 = g1;
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
                           const int32_t *snap_step, uint64_t seed, int64_t n, float *X, float *T, void *hip_stream) {
    qs_status st = check_insts(inst, n_inst);
    if (st != QS_OK) return st;
    if (!G || !snap_step || n_snap < 1 || n < 0 || (n > 0 && (!X || !T)))
        return gfail(QS_ERR_ARG, "G, snap_step, n_snap >= 1, n >= 0, X and T are required");
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
                           n_snap, seed, n, X, T);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_inst);
    (void)hipFree(d_k);
    if (d_steps) (void)hipFree(d_steps);
    if (e != hipSuccess) return gfail(QS_ERR_HIP, std::string("sample kernel: ") + hipGetErrorString(e));
    return QS_OK;
}

qs_status qs_growth_features(const float *q, int64_t n, float *x, void *hip_stream) {
    if (n < 0 || (n > 0 && (!q || !x))) return gfail(QS_ERR_ARG, "q and x are required");
    if (n == 0) return QS_OK;
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n)), dim3(256), 0, static_cast<hipStream_t>(hip_stream), q, n, x);
    G_HIP(hipGetLastError(), "features kernel");
    return QS_OK;
}

qs_status qs_growth_calibrate(qs_mlp *net, const float *X, const float *T, int64_t n, float *table) {
    if (!net || !table || n < 0 || (n > 0 && (!X || !T))) return gfail(QS_ERR_ARG, "net, X, T and table are required");
    hipStream_t s = qs::mlp_stream(net);
    float *y = nullptr;
    uint32_t *cnt = nullptr;
    if (n > 0) G_HIP(hipMalloc(&y, n * sizeof(float)), "allocate predictions");
    if (hipMalloc(&cnt, (size_t)QS_GROWTH_BINS * kBuckets * sizeof(uint32_t)) != hipSuccess) {
        if (y) (void)hipFree(y);
        return gfail(QS_ERR_ALLOC, "allocate histogram");
    }
    hipLaunchKernelGGL(fill_kernel, dim3(blocks_for((int64_t)QS_GROWTH_BINS * kBuckets)), dim3(256), 0, s,
                       reinterpret_cast<float *>(cnt), (int64_t)QS_GROWTH_BINS * kBuckets, 0.0f);
    qs_status st = QS_OK;
    if (n > 0) {
        st = qs_mlp_forward(net, X, n, y);
        if (st == QS_OK) hipLaunchKernelGGL(hist_kernel, dim3(blocks_for(n)), dim3(256), 0, s, X, y, T, n, cnt);
    }
    if (st == QS_OK) hipLaunchKernelGGL(p99_kernel, dim3(blocks_for(QS_GROWTH_BINS)), dim3(256), 0, s, cnt, table);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (y) (void)hipFree(y);
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
    hipStream_t s = qs::mlp_stream(net);
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n)), dim3(256), 0, s, q, n, x);
    G_HIP(hipGetLastError(), "features kernel");
    st = qs_mlp_forward(net, x, n, out);
    if (st != QS_OK) return st;
    hipLaunchKernelGGL(route_kernel, dim3(blocks_for(n)), dim3(256), 0, s, x, n, table, tol, needs_solver);
    G_HIP(hipGetLastError(), "routing kernel");
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
    if (mode != QS_GROWTH_SOLVER) {
        G_HIP(hipMalloc(&x, (size_t)n * 5 * sizeof(float)), "allocate features");
        hipLaunchKernelGGL(features_kernel, dim3(blocks_for(n)), dim3(256), 0, s, q, n, x);
        if (hipStreamSynchronize(s) != hipSuccess) { cleanup(); return gfail(QS_ERR_HIP, "features kernel"); }
        st = qs_mlp_forward(net, x, n, out);
        if (st == QS_OK && hipStreamSynchronize(qs::mlp_stream(net)) != hipSuccess) st = gfail(QS_ERR_HIP, "network");
        if (st != QS_OK) { cleanup(); return st; }
    }
    if (mode == QS_GROWTH_SURROGATE) {
        if (used_solver && hipMemsetAsync(used_solver, 0, (size_t)n, s) != hipSuccess) { cleanup(); return gfail(QS_ERR_HIP, "clear flags"); }
        cleanup();
        G_HIP(hipStreamSynchronize(s), "synchronize");
        return QS_OK;
    }
    // which queries go to the solver
    std::vector<float> hq((size_t)n * 5);
    G_HIP(hipMemcpyAsync(hq.data(), q, hq.size() * sizeof(float), hipMemcpyDeviceToHost, s), "copy queries");
    std::vector<int64_t> sel;
    if (mode == QS_GROWTH_AUTO) {
        flag = used_solver;
        if (!flag && hipMalloc(&flag, (size_t)n) != hipSuccess) { cleanup(); return gfail(QS_ERR_ALLOC, "allocate flags"); }
        hipLaunchKernelGGL(route_kernel, dim3(blocks_for(n)), dim3(256), 0, s, x, n, table, tol, flag);
        std::vector<uint8_t> hf((size_t)n);
        if (hipMemcpyAsync(hf.data(), flag, (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { cleanup(); return gfail(QS_ERR_HIP, "copy flags"); }
        for (int64_t i = 0; i < n; ++i) if (hf[i]) sel.push_back(i);
    } else {
        G_HIP(hipStreamSynchronize(s), "synchronize");
        sel.resize((size_t)n);
        for (int64_t i = 0; i < n; ++i) sel[i] = i;
    }
    if (!sel.empty()) {
        std::vector<float> vals;
        st = solve_queries(hq, sel, s, &vals);
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
