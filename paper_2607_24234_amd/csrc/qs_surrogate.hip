// Surrogate training and persistence (include/qs_surrogate.h): the whole pipeline -- batched
// solver sweeps, windowed growth targets, example draws, the network's training on the
// device and its held-out error table -- as one library call, and the file that holds the
// result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qs_surrogate.h"
#include "qs_internal.h"

struct qs_surrogate {
    qs_mlp *net = nullptr;
    float *table = nullptr;  // device [QS_GROWTH_BINS]
    int device = 0;
};

namespace {

qs_status sfail(qs_status st, const std::string &m) {
    qs::set_last_error(m);
    return st;
}
#define S_HIP(call, what)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return sfail(QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ configuration
struct Cfg {
    int train_instances = 256, heldout_instances = 1024, modes = 128, heldout_modes = 32, steps = 200;
    int train_dense_steps = 10, train_snap_every = 5, heldout_snap_every = 10;
    double samples = 1e7, heldout_samples = 4e6;
    double heldout_length = 200.0;
    int chunk_instances = 64;
    int epochs = 60, batch = 8192;
    double lr = 1e-3, lr_min = 1e-5, weight_decay = 0.01;
    double seed = 0;
};

struct Key {
    const char *name;
    double *d;
    int *i;
};

// A flat JSON object of numbers ({"epochs": 40, ...}); unknown keys are errors.
qs_status parse_cfg(const char *text, Cfg *c) {
    if (!text) return QS_OK;
    std::vector<Key> keys = {
        {"train_instances", nullptr, &c->train_instances}, {"heldout_instances", nullptr, &c->heldout_instances},
        {"modes", nullptr, &c->modes}, {"heldout_modes", nullptr, &c->heldout_modes}, {"steps", nullptr, &c->steps},
        {"train_dense_steps", nullptr, &c->train_dense_steps}, {"train_snap_every", nullptr, &c->train_snap_every},
        {"heldout_snap_every", nullptr, &c->heldout_snap_every}, {"samples", &c->samples, nullptr},
        {"heldout_samples", &c->heldout_samples, nullptr}, {"heldout_length", &c->heldout_length, nullptr},
        {"chunk_instances", nullptr, &c->chunk_instances},
        {"epochs", nullptr, &c->epochs}, {"batch", nullptr, &c->batch}, {"lr", &c->lr, nullptr},
        {"lr_min", &c->lr_min, nullptr}, {"weight_decay", &c->weight_decay, nullptr}, {"seed", &c->seed, nullptr}};
    const char *p = text;
    auto ws = [&]() { while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r') ++p; };
    ws();
    if (*p == '\0') return QS_OK;
    if (*p != '{') return sfail(QS_ERR_ARG, "configuration: a JSON object of numbers is expected");
    ++p;
    ws();
    if (*p == '}') return QS_OK;
    for (;;) {
        ws();
        if (*p != '"') return sfail(QS_ERR_ARG, "configuration: a quoted key is expected");
        const char *k0 = ++p;
        while (*p && *p != '"') ++p;
        if (*p != '"') return sfail(QS_ERR_ARG, "configuration: unterminated key");
        const std::string key(k0, p - k0);
        ++p;
        ws();
        if (*p != ':') return sfail(QS_ERR_ARG, "configuration: ':' expected after \"" + key + "\"");
        ++p;
        ws();
        char *end = nullptr;
        const double v = std::strtod(p, &end);
        if (end == p || !std::isfinite(v)) return sfail(QS_ERR_ARG, "configuration: a number is expected for \"" + key + "\"");
        p = end;
        bool found = false;
        for (const Key &kk : keys) {
            if (key != kk.name) continue;
            found = true;
            if (kk.d) *kk.d = v;
            else {
                if (v != std::floor(v) || std::fabs(v) > 2e9) return sfail(QS_ERR_ARG, "configuration: \"" + key + "\" must be an integer");
                *kk.i = (int)v;
            }
        }
        if (!found) return sfail(QS_ERR_ARG, "configuration: unknown key \"" + key + "\"");
        ws();
        if (*p == ',') { ++p; continue; }
        if (*p == '}') { ++p; break; }
        return sfail(QS_ERR_ARG, "configuration: ',' or '}' expected");
    }
    ws();
    if (*p != '\0') return sfail(QS_ERR_ARG, "configuration: text after the object");
    return QS_OK;
}

qs_status check_cfg(const Cfg &c) {
    const bool ok = c.train_instances >= 1 && c.heldout_instances >= 1 && c.modes >= 1 && c.heldout_modes >= 1 &&
                    c.steps >= 1 &&
                    c.train_snap_every >= 1 && c.heldout_snap_every >= 1 && c.heldout_snap_every <= c.steps &&
                    c.train_dense_steps >= 0 && c.train_dense_steps < c.steps && c.samples >= c.batch &&
                    c.heldout_samples >= 1 &&
                    c.heldout_length >= 5.0 && c.heldout_length <= 200.0 &&
                    c.chunk_instances >= 1 && c.epochs >= 1 && c.batch >= 128 && c.batch % 128 == 0 &&
                    c.batch <= (1 << 20) && c.lr > 0 && c.lr_min > 0 && c.lr_min <= c.lr && c.weight_decay >= 0 &&
                    c.seed >= 0 && c.samples <= 2e9 && c.heldout_samples <= 2e9;
    return ok ? QS_OK : sfail(QS_ERR_ARG, "configuration: a value is out of its range");
}

// ------------------------------------------------------------------ draws
uint64_t sm64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
double u53(uint64_t seed, uint64_t i) { return (double)(sm64(seed, i) >> 11) * (1.0 / 9007199254740992.0); }

struct Inst {
    double nb, g, L, d_tau;
    int n_xi;
    std::vector<double> k;
};

// cells of the growth map's width h0 = 200/8192 (the finest of the batched sweep) for every
// beam: a beam of drawn length L takes N = round(L/h0) cells and the length N h0
constexpr double kCellWidth = 200.0 / 8192.0;

// n instances with (log10 n_b, log10 gamma) stratified over a near-square grid of the square
// [-3, -1] x [1, 4] (one uniform point per cell: log-uniform marginals, no empty corner of the
// plane), L uniform in [5, 200] (or fixed), d_tau = tau_f / steps; `modes` wavenumbers,
// uniform in [0.05, 4] (jittered: k_m = 0.05 + 3.95 (m + u)/modes with one u per instance),
// from the stream `seed`
std::vector<Inst> draw_instances(int n, uint64_t seed, double fixed_length, int modes, bool jitter_k, const Cfg &c) {
    std::vector<Inst> out(n);
    const int cols = (int)std::ceil(std::sqrt((double)n));
    const int rows = (n + cols - 1) / cols;
    for (int i = 0; i < n; ++i) {
        Inst &d = out[i];
        const int a = i % cols, b = i / cols;
        d.nb = std::pow(10.0, -3.0 + 2.0 * (a + u53(seed, 4 * (uint64_t)i)) / cols);
        d.g = std::pow(10.0, 1.0 + 3.0 * (b + u53(seed, 4 * (uint64_t)i + 1)) / rows);
        const double L = fixed_length > 0 ? fixed_length : 5.0 + 195.0 * u53(seed, 4 * (uint64_t)i + 2);
        d.n_xi = std::max(1, (int)std::lround(L / kCellWidth));
        d.L = d.n_xi * kCellWidth;
        d.d_tau = 10.0 * std::sqrt(d.g / d.nb) / c.steps;
        const double u = jitter_k ? u53(seed, 4 * (uint64_t)i + 3) : 0.0;
        d.k.resize(modes);
        for (int m = 0; m < modes; ++m)
            d.k[m] = jitter_k ? 0.05 + 3.95 * (m + u) / modes
                              : (modes == 1 ? 0.05 : 0.05 + 3.95 * m / (modes - 1));
    }
    return out;
}

__global__ void residual_kernel(const float *__restrict__ t, const float *__restrict__ base, int64_t n,
                                float *__restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = t[i] - base[i];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Snapshot schedule of a sweep: every step below `dense`, then first, first + every, ... below
// the step count, and the last step when `with_final` (first >= dense).
struct Sched {
    int dense, first, every;
    bool with_final;
};

std::vector<int32_t> snap_steps(const Sched &sc, int steps) {
    std::vector<int32_t> out;
    for (int st = 0; st < sc.dense; ++st) out.push_back(st);
    for (int st = sc.first; st < steps; st += sc.every) out.push_back(st);
    if (sc.with_final) out.push_back(steps);
    return out;
}

// Solver runs over `inst` (in chunks of c.chunk_instances; chunk j snapshots by sched(j)),
// windowed targets, and n examples (queries Q, targets T) drawn over all their entries.
template <class SchedFn>
qs_status examples(const std::vector<Inst> &inst, const Cfg &c, SchedFn sched, uint64_t sample_seed, int64_t n,
                   float *Q, float *T, hipStream_t s) {
    // entries of every chunk (cells x modes x snapshots): the examples are shared out in
    // proportion to them
    std::vector<int64_t> chunk_entries;
    int64_t total = 0;
    for (size_t i0 = 0, j = 0; i0 < inst.size(); i0 += c.chunk_instances, ++j) {
        int64_t e = 0;
        for (size_t i = i0; i < std::min(inst.size(), i0 + (size_t)c.chunk_instances); ++i)
            e += (int64_t)inst[i].n_xi * (int64_t)inst[i].k.size();
        e *= (int64_t)snap_steps(sched(j), c.steps).size();
        chunk_entries.push_back(e);
        total += e;
    }
    int64_t done = 0, seen = 0;
    const double q[1] = {-1.0}, ms[1] = {1.0};
    for (size_t i0 = 0, j = 0; i0 < inst.size(); i0 += c.chunk_instances, ++j) {
        const size_t i1 = std::min(inst.size(), i0 + (size_t)c.chunk_instances);
        const Sched sc = sched(j);
        const std::vector<int32_t> steps = snap_steps(sc, c.steps);
        const int n_snap = (int)steps.size();
        std::vector<qs_params> params(i1 - i0);
        std::vector<double> nbs(i1 - i0);
        std::vector<qs_growth_instance> gis(i1 - i0);
        int64_t snap = 0;
        for (size_t i = i0; i < i1; ++i) {
            const Inst &d = inst[i];
            qs_params &p = params[i - i0];
            std::memset(&p, 0, sizeof(p));
            nbs[i - i0] = d.nb;
            p.n_species = 1;
            p.q = q;
            p.m = ms;
            p.nb_over_np = &nbs[i - i0];
            p.gamma_b = d.g;
            p.length = d.L;
            p.profile = QS_PROFILE_FLATTOP;
            p.geometry = QS_GEOM_SPECTRAL;
            p.n_modes = (int64_t)d.k.size();
            p.kx = d.k.data();
            p.n_xi = d.n_xi;
            p.d_tau = d.d_tau;
            p.precision = QS_FP32;
            p.seed_kind = QS_SEED_UNIFORM;
            p.seed_amp = 1e-6;
            gis[i - i0] = qs_growth_instance{d.nb, d.g, d.L, d.d_tau, 1e-6, d.n_xi, (int32_t)d.k.size(), d.k.data()};
            snap += (int64_t)d.n_xi * (int64_t)d.k.size();
        }
        seen += chunk_entries[j];
        // examples of this chunk: its share of all entries (the last chunk takes the rest)
        const int64_t upto = i1 == inst.size() ? n : (int64_t)std::llround((double)n * (double)seen / (double)total);
        const int64_t nc = upto - done;
        qs_ctx *ctx = nullptr;
        qs_status st = qs_init(params.data(), (int32_t)params.size(), s, nullptr, 0, &ctx);
        if (st != QS_OK) return st;
        float *buf = nullptr;
        if (hipMalloc(&buf, (size_t)snap * n_snap * 3 * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            qs_free(ctx);
            return sfail(QS_ERR_ALLOC, "surrogate data: snapshot buffers");
        }
        float *le = buf, *lb = buf + (size_t)snap * n_snap, *G = buf + 2 * (size_t)snap * n_snap;
        // stepping: the dense steps with a snapshot each, the steps up to `first` without, then
        // the regular snapshots, then the final state
        const size_t reg0 = (size_t)sc.dense * snap;
        const size_t fin = (size_t)(n_snap - 1) * snap;
        if (sc.dense > 0) st = qs_step_tau(ctx, sc.dense, 1, le, lb, nullptr);
        if (st == QS_OK && sc.first > sc.dense) st = qs_step_tau(ctx, sc.first - sc.dense, 1, nullptr, nullptr, nullptr);
        if (st == QS_OK && sc.first < c.steps) st = qs_step_tau(ctx, c.steps - sc.first, sc.every, le + reg0, lb + reg0, nullptr);
        if (st == QS_OK && sc.with_final) st = qs_step_tau(ctx, 0, 1, le + fin, lb + fin, nullptr);
        if (st == QS_OK) st = qs_sync_check(ctx);
        if (st == QS_OK) st = qs_growth_targets(gis.data(), (int32_t)gis.size(), le, lb, n_snap, G, s);
        if (st == QS_OK && nc > 0)
            st = qs_growth_sample(gis.data(), (int32_t)gis.size(), G, n_snap, steps.data(), sample_seed + i0, nc,
                                  Q + 5 * done, T + done, s);
        if (st == QS_OK && hipStreamSynchronize(s) != hipSuccess) st = sfail(QS_ERR_HIP, "surrogate data: synchronize");
        (void)hipFree(buf);
        qs_free(ctx);
        if (st != QS_OK) return st;
        done = upto;
    }
    return QS_OK;
}

constexpr int D = 512;
const int kDims[6] = {5, D, D, D, D, 1};

// uniform in +-1/sqrt(fan_in) from the stream `seed`; the output layer scaled by `scale`
// with bias `mean` (initial outputs with the targets' centre and spread)
std::vector<float> init_params(uint64_t seed, double mean, double scale) {
    std::vector<float> p;
    uint64_t ctr = 0;
    for (int l = 0; l < 5; ++l) {
        const double b = 1.0 / std::sqrt((double)kDims[l]);
        const size_t nw = (size_t)kDims[l + 1] * kDims[l], nb = kDims[l + 1];
        for (size_t i = 0; i < nw; ++i) p.push_back((float)((2.0 * u53(seed, ctr++) - 1.0) * b * (l == 4 ? scale : 1.0)));
        for (size_t i = 0; i < nb; ++i) p.push_back((float)(l == 4 ? mean : (2.0 * u53(seed, ctr++) - 1.0) * b));
    }
    return p;
}

constexpr char kMagic[8] = {'Q', 'S', 'S', 'U', 'R', 'R', '0', '1'};

struct FileHeader {
    char magic[8];
    uint32_t version, n_params, n_bins, meta_len;
};

std::string json_escape(const std::string &s) {
    std::string o;
    for (char ch : s) {
        if (ch == '"' || ch == '\\') o += '\\';
        o += ch;
    }
    return o;
}

}  // namespace

extern "C" {

qs_status qs_surrogate_train(const char *cfg_json, const char *out_path, void *hip_stream, double *stats) {
    if (!out_path || !*out_path) return sfail(QS_ERR_ARG, "out_path is required");
    Cfg c;
    qs_status st = parse_cfg(cfg_json, &c);
    if (st != QS_OK) return st;
    st = check_cfg(c);
    if (st != QS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const auto t0 = std::chrono::steady_clock::now();
    const uint64_t seed = (uint64_t)c.seed;
    const int64_t n = ((int64_t)c.samples / c.batch) * c.batch, nh = (int64_t)c.heldout_samples;
    // data: training sweep (lengths uniform), held-out sweep (independent draws, every length
    // heldout_length so that xi is uniform, snapshots between the training ones)
    float *mem = nullptr;  // Q, T, X, base/residual for training; Qh, Th for held-out
    const size_t bytes = ((size_t)n * 12 + (size_t)nh * 6) * sizeof(float);
    if (hipMalloc(&mem, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return sfail(QS_ERR_ALLOC, "surrogate data: example buffers");
    }
    float *Q = mem, *T = Q + 5 * n, *X = T + n, *R = X + 5 * n, *Qh = R + n, *Th = Qh + 5 * nh;
    const std::vector<Inst> tr = draw_instances(c.train_instances, sm64(seed, 0x7261696e), 0.0, c.modes, false, c);
    const std::vector<Inst> ho = draw_instances(c.heldout_instances, sm64(seed, 0x68656c64), c.heldout_length,
                                                c.heldout_modes, true, c);
    // training: every step of the first train_dense_steps (the fast start of the growth),
    // then every train_snap_every-th, and the last; held-out: every heldout_snap_every-th
    // step from an offset that cycles with the chunk, so that the held-out examples fall on
    // every step, between the training snapshots as well as on them
    const Sched train_sched{c.train_dense_steps, c.train_dense_steps, c.train_snap_every, true};
    st = examples(tr, c, [&](size_t) { return train_sched; }, sm64(seed, 1), n, Q, T, s);
    if (st == QS_OK)
        st = examples(ho, c, [&](size_t j) { return Sched{0, (int)(j % (size_t)c.heldout_snap_every), c.heldout_snap_every, false}; },
                      sm64(seed, 2), nh, Qh, Th, s);
    // residual targets over the baseline, and the network inputs
    if (st == QS_OK) st = qs_growth_features(Q, n, X, R, s);
    if (st == QS_OK) {
        hipLaunchKernelGGL(residual_kernel, dim3(blocks_for(n)), dim3(256), 0, s, T, R, n, R);
        if (hipGetLastError() != hipSuccess) st = sfail(QS_ERR_HIP, "residual kernel");
    }
    std::vector<float> hr;
    if (st == QS_OK) {
        hr.resize((size_t)n);
        if (hipMemcpyAsync(hr.data(), R, (size_t)n * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = sfail(QS_ERR_HIP, "surrogate data: copy targets");
    }
    const auto t1 = std::chrono::steady_clock::now();
    qs_mlp *net = nullptr;
    float *table = nullptr;
    double last_loss = 0.0;
    if (st == QS_OK) {
        double sum = 0.0, sq = 0.0;
        for (float v : hr) { sum += v; sq += (double)v * v; }
        const double mean = sum / n, sd = std::sqrt(std::max(sq / n - mean * mean, 1e-12));
        st = qs_mlp_create(c.batch, hip_stream, &net);
        std::vector<float> p0 = init_params(sm64(seed, 3), mean, sd);
        if (st == QS_OK) st = qs_mlp_set_params(net, p0.data());
    }
    // AdamW over contiguous batches of the (already random) examples, a different batch
    // order each epoch, cosine learning rate from lr to lr_min
    const int64_t batches = n / c.batch;
    const int64_t total_steps = (int64_t)c.epochs * batches;
    int64_t k = 0;
    for (int ep = 0; ep < c.epochs && st == QS_OK; ++ep) {
        const int64_t shift = ((int64_t)ep * 7919) % batches;
        for (int64_t i = 0; i < batches && st == QS_OK; ++i) {
            const int64_t b = (i + shift) % batches;
            const double tt = (double)k / (double)std::max<int64_t>(1, total_steps - 1);
            const double lr = c.lr_min + 0.5 * (c.lr - c.lr_min) * (1.0 + std::cos(M_PI * tt));
            const bool want = (ep == c.epochs - 1 && i == batches - 1);
            st = qs_mlp_grads(net, X + 5 * b * c.batch, R + b * c.batch, c.batch, want ? &last_loss : nullptr);
            if (st == QS_OK) st = qs_mlp_adamw(net, lr, 0.9, 0.999, 1e-8, c.weight_decay);
            ++k;
        }
    }
    const auto t2 = std::chrono::steady_clock::now();
    // held-out: error table and error statistics of the full answer (baseline + network)
    double hs[5] = {0, 0, 0, 0, 0};
    if (st == QS_OK && hipMalloc(&table, (size_t)QS_GROWTH_BINS * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        st = sfail(QS_ERR_ALLOC, "error table");
    }
    if (st == QS_OK) st = qs_growth_calibrate(net, Qh, Th, nh, table);
    std::vector<float> htab(QS_GROWTH_BINS);
    if (st == QS_OK) {
        // reuse the training buffers: inputs X[0 .. 5 nh), answers R[0 .. nh), baselines R[nh .. 2 nh)
        // (n >= nh is not required: fall back to a fresh buffer)
        float *x = X, *y = R, *bb = R + nh;
        float *own = nullptr;
        if (nh * 2 > n) {
            if (hipMalloc(&own, (size_t)nh * 7 * sizeof(float)) != hipSuccess) { (void)hipGetLastError(); st = sfail(QS_ERR_ALLOC, "held-out buffers"); }
            x = own; y = own + 5 * nh; bb = own + 6 * nh;
        }
        if (st == QS_OK) st = qs_growth_features(Qh, nh, x, bb, s);
        if (st == QS_OK && hipStreamSynchronize(s) != hipSuccess) st = sfail(QS_ERR_HIP, "synchronize");
        if (st == QS_OK) st = qs_mlp_forward(net, x, nh, y);
        std::vector<float> hy((size_t)nh), hb((size_t)nh), ht((size_t)nh);
        if (st == QS_OK) {
            hipStream_t ns = qs::mlp_stream(net);
            if (hipMemcpyAsync(hy.data(), y, nh * 4, hipMemcpyDeviceToHost, ns) != hipSuccess ||
                hipMemcpyAsync(hb.data(), bb, nh * 4, hipMemcpyDeviceToHost, ns) != hipSuccess ||
                hipMemcpyAsync(ht.data(), Th, nh * 4, hipMemcpyDeviceToHost, ns) != hipSuccess ||
                hipMemcpyAsync(htab.data(), table, htab.size() * 4, hipMemcpyDeviceToHost, ns) != hipSuccess ||
                hipStreamSynchronize(ns) != hipSuccess)
                st = sfail(QS_ERR_HIP, "copy held-out results");
        }
        if (own) (void)hipFree(own);
        if (st == QS_OK) {
            std::vector<double> e((size_t)nh);
            double sq = 0.0, mx = 0.0;
            int64_t within = 0;
            for (int64_t i = 0; i < nh; ++i) {
                e[i] = std::fabs((double)hy[i] + hb[i] - ht[i]);
                if (!std::isfinite(e[i])) e[i] = 1e30;
                sq += e[i] * e[i];
                mx = std::max(mx, e[i]);
                within += e[i] <= 1e-2;
            }
            const int64_t r99 = std::max<int64_t>(0, (int64_t)std::ceil(0.99 * nh) - 1);
            std::nth_element(e.begin(), e.begin() + r99, e.end());
            hs[0] = std::sqrt(sq / nh);
            hs[1] = e[r99];
            hs[2] = mx;
            hs[3] = (double)within / nh;
            int64_t trusted = 0;
            for (float v : htab) trusted += (v >= 0.0f && v <= 1e-2f);
            hs[4] = (double)trusted / QS_GROWTH_BINS;
        }
    }
    const auto t3 = std::chrono::steady_clock::now();
    const double sec_data = std::chrono::duration<double>(t1 - t0).count();
    const double sec_train = std::chrono::duration<double>(t2 - t1).count();
    const double sec_cal = std::chrono::duration<double>(t3 - t2).count();
    // the file: header, parameters, table, and a JSON record of the configuration and results
    std::vector<float> params((size_t)qs_mlp_param_count());
    if (st == QS_OK) st = qs_mlp_get_params(net, params.data());
    if (st == QS_OK) {
        char meta[1024];
        std::snprintf(meta, sizeof(meta),
                      "{\"train_instances\": %d, \"heldout_instances\": %d, \"modes\": %d, \"heldout_modes\": %d, \"steps\": %d, "
                      "\"train_dense_steps\": %d, \"train_snap_every\": %d, \"heldout_snap_every\": %d, "
                      "\"samples\": %lld, \"heldout_samples\": %lld, \"heldout_length\": %g, "
                      "\"epochs\": %d, \"batch\": %d, \"lr\": %g, \"lr_min\": %g, \"weight_decay\": %g, \"seed\": %llu, "
                      "\"heldout_rms\": %.6g, \"heldout_p99\": %.6g, \"heldout_max\": %.6g, \"heldout_within_1e-2\": %.6g, "
                      "\"bins_trusted_1e-2\": %.6g, \"final_loss\": %.6g, \"seconds_data\": %.3f, \"seconds_train\": %.3f, "
                      "\"seconds_calibrate\": %.3f}",
                      c.train_instances, c.heldout_instances, c.modes, c.heldout_modes, c.steps, c.train_dense_steps, c.train_snap_every,
                      c.heldout_snap_every, (long long)n, (long long)nh, c.heldout_length, c.epochs,
                      c.batch, c.lr, c.lr_min, c.weight_decay, (unsigned long long)seed, hs[0], hs[1], hs[2], hs[3],
                      hs[4], last_loss, sec_data, sec_train, sec_cal);
        FileHeader hd;
        std::memcpy(hd.magic, kMagic, 8);
        hd.version = 1;
        hd.n_params = (uint32_t)params.size();
        hd.n_bins = QS_GROWTH_BINS;
        hd.meta_len = (uint32_t)std::strlen(meta);
        FILE *f = std::fopen(out_path, "wb");
        if (!f) st = sfail(QS_ERR_ARG, std::string("cannot write ") + out_path);
        else {
            bool ok = std::fwrite(&hd, sizeof(hd), 1, f) == 1 &&
                      std::fwrite(params.data(), 4, params.size(), f) == params.size() &&
                      std::fwrite(htab.data(), 4, htab.size(), f) == htab.size() &&
                      std::fwrite(meta, 1, hd.meta_len, f) == hd.meta_len;
            ok = (std::fclose(f) == 0) && ok;
            if (!ok) st = sfail(QS_ERR_ARG, std::string("writing ") + out_path + " failed");
        }
    }
    if (st == QS_OK && stats) {
        stats[0] = hs[0]; stats[1] = hs[1]; stats[2] = hs[2]; stats[3] = hs[3]; stats[4] = hs[4];
        stats[5] = last_loss; stats[6] = sec_data; stats[7] = sec_train;
    }
    if (table) (void)hipFree(table);
    if (net) qs_mlp_free(net);
    (void)hipFree(mem);
    return st;
}

qs_status qs_surrogate_load(const char *path, void *hip_stream, qs_surrogate **out) {
    if (!path || !out) return sfail(QS_ERR_ARG, "path and out are required");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return sfail(QS_ERR_ARG, std::string("cannot open ") + path);
    FileHeader hd;
    std::vector<float> params, table;
    bool ok = std::fread(&hd, sizeof(hd), 1, f) == 1 && std::memcmp(hd.magic, kMagic, 8) == 0 && hd.version == 1 &&
              hd.n_params == (uint32_t)qs_mlp_param_count() && hd.n_bins == (uint32_t)QS_GROWTH_BINS;
    if (ok) {
        params.resize(hd.n_params);
        table.resize(hd.n_bins);
        ok = std::fread(params.data(), 4, params.size(), f) == params.size() &&
             std::fread(table.data(), 4, table.size(), f) == table.size();
    }
    std::fclose(f);
    if (!ok) return sfail(QS_ERR_ARG, std::string(path) + " is not a surrogate file of this library");
    qs_surrogate *sur = new (std::nothrow) qs_surrogate;
    if (!sur) return sfail(QS_ERR_ALLOC, "host allocation failed");
    S_HIP(hipGetDevice(&sur->device), "hipGetDevice");
    qs_status st = qs_mlp_create(128, hip_stream, &sur->net);
    if (st == QS_OK) st = qs_mlp_set_params(sur->net, params.data());
    if (st == QS_OK && hipMalloc(&sur->table, table.size() * 4) != hipSuccess) {
        (void)hipGetLastError();
        st = sfail(QS_ERR_ALLOC, "error table");
    }
    if (st == QS_OK && hipMemcpy(sur->table, table.data(), table.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        st = sfail(QS_ERR_HIP, "copy error table");
    if (st != QS_OK) {
        qs_surrogate_free(sur);
        return st;
    }
    *out = sur;
    return QS_OK;
}

qs_mlp *qs_surrogate_net(const qs_surrogate *s) { return s ? s->net : nullptr; }

const float *qs_surrogate_table(const qs_surrogate *s) { return s ? s->table : nullptr; }

void qs_surrogate_free(qs_surrogate *s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->net) qs_mlp_free(s->net);
    if (s->table) (void)hipFree(s->table);
    delete s;
}

}  // extern "C"
