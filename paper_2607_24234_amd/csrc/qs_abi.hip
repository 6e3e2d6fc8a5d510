// Host side of libqs: argument validation, per-instance tables, workspace layout, launch
// sequencing and state import/export.  Every entry point is declared in include/qs.h.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qs_internal.h"

namespace qs {
namespace {

thread_local std::string g_err;

qs_status fail(qs_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

}  // namespace

void set_last_error(const std::string &msg) { g_err = msg; }

namespace {

qs_status hip_fail(hipError_t e, const char *what) {
    return fail(QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define QS_HIP(call, what)                           \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// real columns per lane of the step kernel: 1 (the two parts of a mode in adjacent lanes,
// the default) or 2 (one mode per lane); QS_COLUMNS_PER_LANE overrides the default
int env_nc() {
    const char *s = std::getenv("QS_COLUMNS_PER_LANE");
    if (s && (std::atoi(s) == 1 || std::atoi(s) == 2)) return std::atoi(s);
    return 1;
}

// Sizes derived from validated parameters.
struct Plan {
    int precision = QS_FP32;
    int nc = 1;                    // real columns per lane
    size_t ts = 4;                 // bytes per state element
    std::vector<InstDev> inst;
    std::vector<int32_t> blk_inst;
    int64_t state_elems = 0;
    int64_t table_elems = 0;       // Omega centres+faces (and shape) elements
    int64_t total_modes = 0;
    int64_t total_pmodes = 0;
    int64_t snap_elems = 0;        // elements of one snapshot over all instances
    int32_t max_n_xi = 0;
    int32_t seg_target = 0;        // target cells per xi-segment
    int32_t wg_waves = 16;         // wave slots per workgroup of the march kernel
    int32_t n_wg = 0;              // workgroups of the march kernel
    int32_t max_seg = 1;           // largest segment count of any instance
    int32_t max_seg_len = 0;       // longest segment of any segmented instance (cells)
    int64_t n_scale = 0;           // entries of the per-(segment, mode) scale arrays
    std::vector<int2> wave_table;  // [n_wg][wg_waves]: (global block, segment) or (-1, -1)
    // workspace offsets (bytes)
    size_t off_state, off_omega, off_shape, off_k, off_coef, off_log2s, off_epend, off_inst, off_blk,
        off_iidx, off_err, off_wtab, off_front, total;
    int64_t n_blocks = 0;
};

// 32-bit words of the error region: see StepArgs::err
constexpr int kErrWords = 8;

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        return cus;
    (void)hipGetLastError();
    return 256;  // MI355X
}

// Segment each instance into ceil(N/seg) pieces (at most max_seg) and pack the (block,
// segment) waves into workgroups of W slots, first fit by decreasing segment count; a
// block's segments take consecutive slots of one workgroup.  Returns the workgroup count.
// Segments of an instance of N cells for a target of seg cells and at most max_seg pieces:
// equal lengths ceil(N/count), and no empty segment.
int segments_of(int N, int seg, int max_seg) {
    const int c = std::min(max_seg, std::max(1, (N + seg - 1) / seg));
    const int len = (N + c - 1) / c;
    return (N + len - 1) / len;
}

int pack(const std::vector<InstDev> &inst, int seg, int W, int max_seg, std::vector<int> *nseg_out,
         std::vector<int2> *table) {
    const int n = (int)inst.size();
    std::vector<int> nseg(n);
    for (int i = 0; i < n; ++i) nseg[i] = segments_of(inst[i].n_xi, seg, max_seg);
    std::vector<std::pair<int, int>> items;  // (segments, global block)
    for (int i = 0; i < n; ++i)
        for (int b = 0; b < inst[i].n_blocks; ++b) items.push_back({nseg[i], inst[i].block0 + b});
    std::stable_sort(items.begin(), items.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    std::vector<int> freeslots;  // per workgroup
    std::vector<std::vector<int2>> wgs;
    // workgroups with free slots, bucketed by free count, for a near-linear first fit
    std::vector<std::vector<int>> by_free(W + 1);
    for (const auto &it : items) {
        const int need = it.first;
        int g = -1;
        for (int f = need; f <= W && g < 0; ++f) {
            while (!by_free[f].empty()) {
                const int cand = by_free[f].back();
                if (freeslots[cand] != f) { by_free[f].pop_back(); continue; }  // stale entry
                g = cand;
                by_free[f].pop_back();
                break;
            }
        }
        if (g < 0) {
            g = (int)wgs.size();
            wgs.emplace_back();
            freeslots.push_back(W);
        }
        for (int s = 0; s < need; ++s) wgs[g].push_back(make_int2(it.second, s));
        freeslots[g] -= need;
        by_free[freeslots[g]].push_back(g);
    }
    if (nseg_out) *nseg_out = nseg;
    if (table) {
        table->assign((size_t)wgs.size() * W, make_int2(-1, -1));
        for (size_t g = 0; g < wgs.size(); ++g)
            for (size_t s = 0; s < wgs[g].size(); ++s) (*table)[g * W + s] = wgs[g][s];
    }
    return (int)wgs.size();
}

bool finite(double x) { return std::isfinite(x); }

// Offset inside one cell of a block of the value (var, part) of the block's local mode q,
// for NC real columns per lane (column lane*NC + c holds part (lane*NC+c) & 1 of local
// mode (lane*NC+c)/2, stored at row var*NC + c, lane).
int64_t elem_of(int NC, int q, int var, int part) {
    const int col = 2 * q + part;
    const int lane = col / NC, c = col % NC;
    return (int64_t)(var * NC + c) * kWave + lane;
}

qs_status validate_one(const qs_params &p, int i) {
    const std::string at = "instance " + std::to_string(i) + ": ";
    if (p.geometry != QS_GEOM_SPECTRAL && p.geometry != QS_GEOM_TRANSVERSE_GRID)
        return fail(QS_ERR_ARG, at + "unknown geometry");
    if (p.n_species < 1 || p.n_species > 64) return fail(QS_ERR_ARG, at + "n_species must be in [1, 64]");
    if (!p.q || !p.m || !p.nb_over_np) return fail(QS_ERR_ARG, at + "q, m and nb_over_np are required");
    for (int s = 0; s < p.n_species; ++s) {
        if (!finite(p.q[s]) || !finite(p.m[s]) || !(p.m[s] > 0.0))
            return fail(QS_ERR_ARG, at + "species " + std::to_string(s) + ": need finite q and m > 0");
        if (!finite(p.nb_over_np[s]) || p.nb_over_np[s] < 0.0)
            return fail(QS_ERR_ARG, at + "species " + std::to_string(s) + ": need finite nb_over_np >= 0");
    }
    if (!finite(p.gamma_b) || !(p.gamma_b > 1.0)) return fail(QS_ERR_ARG, at + "gamma_b must be finite and > 1");
    if (!finite(p.length) || !(p.length > 0.0)) return fail(QS_ERR_ARG, at + "length must be finite and > 0");
    if (p.n_xi < 1 || p.n_xi > (1 << 20)) return fail(QS_ERR_ARG, at + "n_xi must be in [1, 2^20]");
    if (!finite(p.d_tau) || !(p.d_tau > 0.0)) return fail(QS_ERR_ARG, at + "d_tau must be finite and > 0");
    if (p.precision != QS_FP64 && p.precision != QS_FP32) return fail(QS_ERR_ARG, at + "unknown precision");
    if (p.geometry == QS_GEOM_TRANSVERSE_GRID) {
        auto pow2 = [](int v) { return v >= 2 && v <= 256 && (v & (v - 1)) == 0; };
        if (!pow2(p.nx) || !pow2(p.ny)) return fail(QS_ERR_ARG, at + "nx and ny must be powers of two in [2, 256]");
        if (p.n_xi > 65535) return fail(QS_ERR_ARG, at + "n_xi must be at most 65535 on the transverse grid");
        if (!finite(p.lx) || !(p.lx > 0.0) || !finite(p.ly) || !(p.ly > 0.0))
            return fail(QS_ERR_ARG, at + "lx and ly must be finite and > 0");
        if (!finite(p.sigma_r) || p.sigma_r < 0.0) return fail(QS_ERR_ARG, at + "sigma_r must be finite and >= 0");
        if (!finite(p.centroid_offset)) return fail(QS_ERR_ARG, at + "centroid_offset must be finite");
        if ((int64_t)p.nx * p.ny * (int64_t)p.n_xi > (int64_t(1) << 31))
            return fail(QS_ERR_ARG, at + "nx * ny * n_xi must be at most 2^31");
        if (p.precision != QS_FP32) return fail(QS_ERR_UNSUPPORTED, at + "the transverse grid runs in FP32 only");
        if (p.flags & QS_FLAG_STEADY_INFLOW) return fail(QS_ERR_UNSUPPORTED, at + "STEADY_INFLOW is spectral only");
        if (p.flags & QS_FLAG_FPERP_SNAPSHOTS) return fail(QS_ERR_UNSUPPORTED, at + "FPERP_SNAPSHOTS is spectral only");
        if (p.flags & QS_FLAG_STATIONARY_FRONT) return fail(QS_ERR_UNSUPPORTED, at + "STATIONARY_FRONT is spectral only");
    } else {
        if (p.n_modes < 1 || p.n_modes > (int64_t(1) << 26)) return fail(QS_ERR_ARG, at + "n_modes must be in [1, 2^26]");
        if (!p.kx) return fail(QS_ERR_ARG, at + "kx is required");
        for (int64_t m = 0; m < p.n_modes; ++m) {
            if (!finite(p.kx[m]) || (p.ky && !finite(p.ky[m])))
                return fail(QS_ERR_ARG, at + "non-finite wavenumber at mode " + std::to_string(m));
        }
    }
    switch (p.profile) {
    case QS_PROFILE_FLATTOP: break;
    case QS_PROFILE_GAUSSIAN:
        if (!finite(p.sigma_xi) || !(p.sigma_xi > 0.0) || !finite(p.xi_center))
            return fail(QS_ERR_ARG, at + "GAUSSIAN profile needs sigma_xi > 0 and a finite xi_center");
        break;
    case QS_PROFILE_TABLE:
        if (!p.profile_table) return fail(QS_ERR_ARG, at + "TABLE profile needs profile_table");
        for (int j = 0; j < p.n_xi; ++j)
            if (!finite(p.profile_table[j]) || p.profile_table[j] < 0.0)
                return fail(QS_ERR_ARG, at + "profile_table entries must be finite and >= 0");
        break;
    default: return fail(QS_ERR_ARG, at + "unknown profile");
    }
    if (p.seed_kind == QS_SEED_CENTROID && p.geometry != QS_GEOM_TRANSVERSE_GRID)
        return fail(QS_ERR_UNSUPPORTED, at + "CENTROID seed needs the transverse-grid geometry");
    if (p.seed_kind == QS_SEED_FRONT_IMPULSE && p.geometry == QS_GEOM_TRANSVERSE_GRID)
        return fail(QS_ERR_UNSUPPORTED, at + "FRONT_IMPULSE seed is spectral only");
    if (p.seed_kind != QS_SEED_NOISE && p.seed_kind != QS_SEED_UNIFORM && p.seed_kind != QS_SEED_CENTROID &&
        p.seed_kind != QS_SEED_FRONT_IMPULSE && p.seed_kind != QS_SEED_NONE)
        return fail(QS_ERR_ARG, at + "unknown seed_kind");
    if (!finite(p.seed_amp)) return fail(QS_ERR_ARG, at + "seed_amp must be finite");
    if (p.seed_kind == QS_SEED_FRONT_IMPULSE && p.geometry == QS_GEOM_SPECTRAL) {
        for (int64_t m = 0; m < p.n_modes; ++m) {
            double k2 = p.kx[m] * p.kx[m] + (p.ky ? p.ky[m] * p.ky[m] : 0.0);
            if (k2 == 0.0) return fail(QS_ERR_ARG, at + "FRONT_IMPULSE seed needs k != 0 for every mode");
        }
    }
    if (p.flags & ~(QS_FLAG_DROP_LONGITUDINAL | QS_FLAG_NO_RESTORING | QS_FLAG_STEADY_INFLOW | QS_FLAG_FPERP_SNAPSHOTS |
                    QS_FLAG_STATIONARY_FRONT))
        return fail(QS_ERR_ARG, at + "unknown flag bits");
    if ((p.flags & QS_FLAG_STEADY_INFLOW) && (p.flags & QS_FLAG_STATIONARY_FRONT))
        return fail(QS_ERR_ARG, at + "STEADY_INFLOW and STATIONARY_FRONT are exclusive");
    return QS_OK;
}

qs_status make_plan(const qs_params *params, int32_t n, const qs_plan *plan, Plan &pl) {
    if (!params) return fail(QS_ERR_ARG, "params is NULL");
    if (n < 1 || n > (1 << 20)) return fail(QS_ERR_ARG, "n_instances must be in [1, 2^20]");
    for (int i = 0; i < n; ++i) {
        qs_status st = validate_one(params[i], i);
        if (st != QS_OK) return st;
        if (params[i].geometry != QS_GEOM_SPECTRAL)
            return fail(QS_ERR_ARG, "a TRANSVERSE_GRID instance must be the only instance of its context");
        if (params[i].precision != params[0].precision)
            return fail(QS_ERR_ARG, "all instances must share one precision");
        if ((params[i].flags & QS_FLAG_NO_RESTORING) != (params[0].flags & QS_FLAG_NO_RESTORING))
            return fail(QS_ERR_ARG, "all instances must share QS_FLAG_NO_RESTORING");
    }
    pl.precision = params[0].precision;
    pl.nc = env_nc();
    if (plan && plan->columns_per_lane != 0) {
        if (plan->columns_per_lane != 1 && plan->columns_per_lane != 2)
            return fail(QS_ERR_ARG, "plan.columns_per_lane must be 0, 1 or 2");
        pl.nc = plan->columns_per_lane;
    }
    if (plan && plan->segment_cells < 0) return fail(QS_ERR_ARG, "plan.segment_cells must be >= 0");
    pl.ts = pl.precision == QS_FP64 ? 8 : 4;
    const int lanes_modes = 32 * pl.nc;  // modes per 64-lane block
    int64_t blocks = 0, pmodes = 0, modes = 0, state = 0, table = 0, snap = 0;
    pl.inst.resize(n);
    for (int i = 0; i < n; ++i) {
        const qs_params &p = params[i];
        InstDev &d = pl.inst[i];
        std::memset(&d, 0, sizeof(d));
        d.n_xi = p.n_xi;
        d.n_modes = (int32_t)p.n_modes;
        d.n_blocks = (int32_t)((p.n_modes + lanes_modes - 1) / lanes_modes);
        d.block0 = (int32_t)blocks;
        d.pmode0 = (int32_t)pmodes;
        d.mode0 = (int32_t)modes;
        d.flags = p.flags | (p.profile == QS_PROFILE_FLATTOP ? kFlatProfile : 0);
        d.state_off = state;
        d.omega_off = table;
        d.snap_off = snap;
        d.snap_ld = (int32_t)p.n_modes;
        const double h = p.length / p.n_xi;
        const bool drop = (p.flags & QS_FLAG_DROP_LONGITUDINAL) != 0;
        d.h = h;
        d.ih = 1.0 / h;
        d.dtau = p.d_tau;
        d.ginv = 1.0 / p.gamma_b;
        d.g3inv = drop ? 0.0 : 1.0 / (p.gamma_b * p.gamma_b * p.gamma_b);
        d.c1 = std::cos(h);
        d.s1 = std::sin(h);
        d.c2 = std::cos(0.5 * h);
        d.s2 = std::sin(0.5 * h);
        blocks += d.n_blocks;
        pmodes += (int64_t)d.n_blocks * lanes_modes;
        modes += p.n_modes;
        state += (int64_t)d.n_blocks * p.n_xi * 3 * pl.nc * kWave;
        table += 2 * (int64_t)p.n_xi;
        snap += (int64_t)p.n_xi * p.n_modes;
        pl.max_n_xi = std::max(pl.max_n_xi, p.n_xi);
    }
    if (blocks > (int64_t(1) << 31) - 1) return fail(QS_ERR_ARG, "too many blocks");
    pl.blk_inst.resize(blocks);
    for (int i = 0; i < n; ++i)
        for (int b = 0; b < pl.inst[i].n_blocks; ++b) pl.blk_inst[pl.inst[i].block0 + b] = i;
    pl.state_elems = state;
    pl.table_elems = table;
    pl.total_modes = modes;
    pl.total_pmodes = pmodes;
    pl.snap_elems = snap;

    // xi-segmentation and workgroup packing.  Segments of one block share a workgroup; its
    // size W (>= the largest segment count) is the one that keeps the most waves resident
    // per CU for the kernel's register and LDS footprint.
    const int Wmax = march_wg_waves(pl.precision, pl.nc);
    const bool restoring = !(params[0].flags & QS_FLAG_NO_RESTORING);
    bool flat = true;
    for (const InstDev &d : pl.inst) flat = flat && (d.flags & kFlatProfile);
    std::vector<int> wpc(Wmax + 1, -1);  // resident workgroups per CU by size
    auto wgs_per_cu = [&](int W, bool segmented) {
        const int key = segmented ? W : 0;
        if (key > 0 && wpc[key] >= 0) return wpc[key];
        int r = march_wgs_per_cu(pl.precision, pl.nc, restoring, flat, W, segmented);
        if (r <= 0) {
            // no device to ask: the register budgets the kernels are built for
            const int per_simd = pl.nc == 1 ? (pl.precision == QS_FP64 ? 4 : 6) : (pl.precision == QS_FP64 ? 2 : 4);
            r = std::max(1, 4 * per_simd / W);
        }
        if (key > 0) wpc[key] = r;
        return r;
    };
    auto pick_w = [&](int mseg, int *per_cu) {
        int best_w = mseg, best_res = -1;
        for (int W = mseg; W <= Wmax; ++W) {
            const int r = wgs_per_cu(W, mseg > 1);
            if (r * W > best_res) { best_res = r * W; best_w = W; }
        }
        *per_cu = std::max(1, best_res / best_w);
        return best_w;
    };
    auto max_segs = [&](int seg) {
        int m = 1;
        for (const InstDev &d : pl.inst) m = std::max(m, segments_of(d.n_xi, seg, Wmax));
        return m;
    };
    int seg = 0;
    if (plan && plan->segment_cells > 0) {
        seg = plan->segment_cells;
    } else {
        // estimated makespan of a long launch: rounds of resident workgroups x longest
        // segment x (1 + pipeline fill of the tau-skew over ~100 steps)
        const int cus = device_cus();
        double best = 1e300;
        for (int div = 1; div <= Wmax; ++div) {
            const int cand = (pl.max_n_xi + div - 1) / div;
            if (cand < 32 && div > 1) break;
            const int mseg = max_segs(cand);
            int per_cu = 1;
            const int W = pick_w(mseg, &per_cu);
            std::vector<int> ns;
            const int nwg = pack(pl.inst, cand, W, Wmax, &ns, nullptr);
            int mlen = 0;
            for (int i = 0; i < n; ++i) mlen = std::max(mlen, (pl.inst[i].n_xi + ns[i] - 1) / ns[i]);
            const int64_t conc = (int64_t)cus * per_cu;
            const double est = (double)((nwg + conc - 1) / conc) * mlen * (1.0 + (mseg - 1) / 100.0);
            if (est < best * (1.0 - 1e-9)) { best = est; seg = cand; }
        }
    }
    {
        int per_cu = 1;
        pl.wg_waves = pick_w(max_segs(seg), &per_cu);
    }
    const int W = pl.wg_waves;
    pl.seg_target = seg;
    std::vector<int> nseg;
    pl.n_wg = pack(pl.inst, seg, W, Wmax, &nseg, &pl.wave_table);
    int64_t nscale = 0;
    pl.max_seg = 1;
    for (int i = 0; i < n; ++i) {
        InstDev &d = pl.inst[i];
        d.n_seg = nseg[i];
        d.seg_len = (d.n_xi + d.n_seg - 1) / d.n_seg;  // (n_seg - 1) * seg_len < n_xi
        d.scale_off = nscale;
        nscale += (int64_t)d.n_seg * d.n_blocks * lanes_modes;
        pl.max_seg = std::max(pl.max_seg, d.n_seg);
        if (d.n_seg > 1) pl.max_seg_len = std::max(pl.max_seg_len, d.seg_len);
    }
    pl.n_scale = nscale;
    size_t o = 0;
    pl.off_state = o; o = align_up(o + (size_t)state * pl.ts);
    pl.off_omega = o; o = align_up(o + (size_t)table * pl.ts);
    pl.off_shape = o; o = align_up(o + (size_t)table * sizeof(double));
    pl.off_k = o; o = align_up(o + (size_t)pmodes * sizeof(double));
    pl.off_coef = o; o = align_up(o + (size_t)pmodes * 2 * sizeof(double));
    pl.off_log2s = o; o = align_up(o + (size_t)nscale * sizeof(int32_t));
    pl.off_epend = o; o = align_up(o + (size_t)nscale * sizeof(int32_t));
    pl.off_inst = o; o = align_up(o + (size_t)n * sizeof(InstDev));
    pl.off_blk = o; o = align_up(o + (size_t)blocks * sizeof(int32_t));
    pl.off_iidx = o; o = align_up(o + (size_t)n * sizeof(int32_t));
    pl.off_err = o; o = align_up(o + sizeof(uint32_t) * kErrWords);
    pl.off_wtab = o; o = align_up(o + pl.wave_table.size() * sizeof(int2));
    pl.off_front = o; o = align_up(o + (size_t)blocks * pl.nc * kWave * sizeof(double));
    pl.n_blocks = blocks;
    pl.total = o;
    return QS_OK;
}

}  // namespace
}  // namespace qs

using namespace qs;

struct qs_ctx {
    Plan pl;
    GridCtx *grid = nullptr;   // finite-width context (then pl is unused)
    int device = 0;
    double wall_clock_hz = 1e8;  // rate of the device's constant wall clock
    double wait_seconds = -1.0;  // test hook: hand-off wait budget (< 0: the default)
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    bool owns_ws = false;
    int64_t steps_done = 0;
    int32_t graphs = 0;   // live graphs (they read the instance table, snapshot layout included)
    // the state holds invalid results (a reported failure with no rollback copy); stepping is
    // refused until qs_set_state or qs_load_checkpoint replaces it
    bool poisoned = false;
    std::string poison_why;
    // rollback guard (qs_set_rollback): state, scales, then an int64 step count (-1: empty)
    char *guard = nullptr;
    size_t guard_bytes = 0;
    char *at(size_t off) const { return ws + off; }
};

namespace {

// the three state regions and their copies in the rollback guard
GuardArgs guard_args(qs_ctx *c) {
    const Plan &pl = c->pl;
    const size_t sb = (size_t)pl.state_elems * pl.ts, nb = (size_t)pl.n_scale * sizeof(int32_t);
    GuardArgs g{};
    const size_t off[3] = {pl.off_state, pl.off_log2s, pl.off_epend};
    const size_t gof[3] = {0, sb, sb + nb};
    const size_t len[3] = {sb, nb, nb};
    for (int r = 0; r < 3; ++r) {
        g.src[r] = reinterpret_cast<const uint4 *>(c->at(off[r]));
        g.dst[r] = reinterpret_cast<uint4 *>(c->guard + gof[r]);
        g.n16[r] = (int64_t)(len[r] / 16);
    }
    g.err = reinterpret_cast<const uint32_t *>(c->at(pl.off_err));
    g.meta = reinterpret_cast<int64_t *>(c->guard + c->guard_bytes - sizeof(int64_t));
    return g;
}

qs_status upload_tables(qs_ctx *c, const qs_params *params) {
    const Plan &pl = c->pl;
    const int n = (int)pl.inst.size();
    std::vector<double> kmode(pl.total_pmodes, 0.0);
    std::vector<double> coef(2 * (size_t)pl.total_pmodes, 0.0);
    std::vector<int32_t> iidx(n);
    // tables: a flat-top instance's are constants, filled on the device; the others are built
    // here and copied per instance
    std::vector<FlatTable> flat;
    std::vector<std::vector<double>> shapes, oms;
    std::vector<std::vector<float>> om32s;
    for (int i = 0; i < n; ++i) {
        const qs_params &p = params[i];
        const InstDev &d = pl.inst[i];
        const int N = p.n_xi;
        const double h = p.length / N;
        double q2nm = 0.0;  // sum_s q_s^2 nb_s / m_s
        for (int s = 0; s < p.n_species; ++s) q2nm += p.q[s] * p.q[s] * p.nb_over_np[s] / p.m[s];
        if (p.profile == QS_PROFILE_FLATTOP) {
            FlatTable ft;
            ft.off = d.omega_off;
            ft.n = N;
            ft.pad = 0;
            ft.q2nm = q2nm;
            flat.push_back(ft);
        } else {
            shapes.emplace_back(2 * (size_t)N, 0.0);
            oms.emplace_back(2 * (size_t)N, 0.0);
            double *f = shapes.back().data();
            double *oc = oms.back().data();
            double *of = oc + N;
            for (int j = 0; j < N; ++j) {
                const double xi = (j + 0.5) * h;
                if (p.profile == QS_PROFILE_GAUSSIAN) {
                    const double z = (xi - p.xi_center) / p.sigma_xi;
                    f[j] = std::exp(-0.5 * z * z);
                } else f[j] = p.profile_table[j];
                oc[j] = q2nm * f[j];
            }
            for (int j = 0; j < N; ++j) of[j] = (j + 1 < N) ? 0.5 * (oc[j] + oc[j + 1]) : 0.0;
            QS_HIP(hipMemcpyAsync(reinterpret_cast<double *>(c->at(pl.off_shape)) + d.omega_off, f,
                                  2 * (size_t)N * sizeof(double), hipMemcpyHostToDevice, c->stream), "copy profile");
            if (pl.precision == QS_FP64) {
                QS_HIP(hipMemcpyAsync(reinterpret_cast<double *>(c->at(pl.off_omega)) + d.omega_off, oc,
                                      2 * (size_t)N * sizeof(double), hipMemcpyHostToDevice, c->stream),
                       "copy Omega tables");
            } else {
                om32s.emplace_back(oms.back().begin(), oms.back().end());
                QS_HIP(hipMemcpyAsync(reinterpret_cast<float *>(c->at(pl.off_omega)) + d.omega_off, om32s.back().data(),
                                      2 * (size_t)N * sizeof(float), hipMemcpyHostToDevice, c->stream),
                       "copy Omega tables");
            }
        }
        for (int64_t m = 0; m < p.n_modes; ++m) {
            const double kx = p.kx[m], ky = p.ky ? p.ky[m] : 0.0;
            const double k = std::sqrt(kx * kx + ky * ky), kp = 1.0 / (1.0 + k * k);
            kmode[d.pmode0 + m] = k;
            // push coefficients: d_tau T' = (k^2 kappa/gamma) Omega n_p,
            // d_tau P' = -(kappa/(gamma^3 h)) Omega d_xi n_p
            coef[2 * (d.pmode0 + m)] = k * k * kp * d.ginv;
            coef[2 * (d.pmode0 + m) + 1] = -kp * d.g3inv * d.ih;
        }
        iidx[i] = i;
    }
    if (!flat.empty()) {
        // the descriptions are staged in the state array, which seeding clears next (it holds
        // at least 3 x 64 elements per cell of every instance, far more than one description)
        if (flat.size() * sizeof(FlatTable) > (size_t)pl.state_elems * pl.ts)
            return fail(QS_ERR_HIP, "flat tables: staging does not fit");
        auto *d_flat = reinterpret_cast<FlatTable *>(c->at(pl.off_state));
        QS_HIP(hipMemcpyAsync(d_flat, flat.data(), flat.size() * sizeof(FlatTable), hipMemcpyHostToDevice, c->stream),
               "copy flat tables");
        QS_HIP(launch_flat_tables(pl.precision, d_flat, (int)flat.size(), reinterpret_cast<double *>(c->at(pl.off_shape)),
                                  c->at(pl.off_omega), c->stream),
               "flat tables");
    }
    QS_HIP(hipMemcpyAsync(c->at(pl.off_k), kmode.data(), kmode.size() * sizeof(double),
                          hipMemcpyHostToDevice, c->stream), "copy wavenumbers");
    QS_HIP(hipMemcpyAsync(c->at(pl.off_coef), coef.data(), coef.size() * sizeof(double),
                          hipMemcpyHostToDevice, c->stream), "copy push coefficients");
    QS_HIP(hipMemcpyAsync(c->at(pl.off_inst), pl.inst.data(), pl.inst.size() * sizeof(InstDev),
                          hipMemcpyHostToDevice, c->stream), "copy instance table");
    QS_HIP(hipMemcpyAsync(c->at(pl.off_blk), pl.blk_inst.data(), pl.blk_inst.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, c->stream), "copy block table");
    QS_HIP(hipMemcpyAsync(c->at(pl.off_iidx), iidx.data(), iidx.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, c->stream), "copy instance index");
    QS_HIP(hipMemcpyAsync(c->at(pl.off_wtab), pl.wave_table.data(), pl.wave_table.size() * sizeof(int2),
                          hipMemcpyHostToDevice, c->stream), "copy wave table");
    QS_HIP(hipMemsetAsync(c->at(pl.off_err), 0, sizeof(uint32_t) * kErrWords, c->stream), "clear error flag");
    // the host vectors die here: make the copies complete first
    QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
    return QS_OK;
}

qs_status seed_state(qs_ctx *c, const qs_params *params) {
    const Plan &pl = c->pl;
    // every instance must share the seed kind/amp/rng_seed within one launch: launch per group
    const int n = (int)pl.inst.size();
    QS_HIP(hipMemsetAsync(c->at(pl.off_state), 0, (size_t)pl.state_elems * pl.ts, c->stream), "clear state");
    QS_HIP(hipMemsetAsync(c->at(pl.off_log2s), 0, (size_t)pl.n_scale * sizeof(int32_t), c->stream), "clear scales");
    QS_HIP(hipMemsetAsync(c->at(pl.off_epend), 0, (size_t)pl.n_scale * sizeof(int32_t), c->stream), "clear scales");
    int i0 = 0;
    while (i0 < n) {
        int i1 = i0 + 1;
        while (i1 < n && params[i1].seed_kind == params[i0].seed_kind &&
               params[i1].seed_amp == params[i0].seed_amp && params[i1].rng_seed == params[i0].rng_seed)
            ++i1;
        if (params[i0].seed_kind != QS_SEED_NONE) {
            int b0 = pl.inst[i0].block0;
            int nb = pl.inst[i1 - 1].block0 + pl.inst[i1 - 1].n_blocks - b0;
            int mx = 0;
            for (int i = i0; i < i1; ++i) mx = std::max(mx, pl.inst[i].n_xi);
            SeedArgs a{};
            a.state = c->at(pl.off_state);
            a.blk_inst = reinterpret_cast<const int32_t *>(c->at(pl.off_blk));
            a.block_base = b0;
            a.inst = reinterpret_cast<const InstDev *>(c->at(pl.off_inst));
            a.shape = reinterpret_cast<const double *>(c->at(pl.off_shape));
            a.kmode = reinterpret_cast<const double *>(c->at(pl.off_k));
            a.log2s = reinterpret_cast<int32_t *>(c->at(pl.off_log2s));
            a.epend = reinterpret_cast<int32_t *>(c->at(pl.off_epend));
            a.kind = params[i0].seed_kind;
            a.amp = params[i0].seed_amp;
            a.rng_seed = params[i0].rng_seed;
            a.inst_index = reinterpret_cast<const int32_t *>(c->at(pl.off_iidx));
            QS_HIP(launch_seed(pl.precision, pl.nc, nb, mx, a, c->stream), "seed kernel");
        }
        i0 = i1;
    }
    // the stationary front's values: cell 0's charge density of the seeded (tau = 0) state
    QS_HIP(launch_front_capture(pl.precision, pl.nc, c->at(pl.off_state),
                                reinterpret_cast<const int32_t *>(c->at(pl.off_blk)),
                                reinterpret_cast<const InstDev *>(c->at(pl.off_inst)), (int)pl.n_blocks,
                                reinterpret_cast<double *>(c->at(pl.off_front)), c->stream),
           "front capture");
    return QS_OK;
}

}  // namespace

qs_status qs::set_mode_coefficients(qs_ctx *c, const double *cT, const double *cP) {
    if (!c || !cT || !cP) return fail(QS_ERR_ARG, "set_mode_coefficients: arguments are required");
    if (c->grid) return fail(QS_ERR_UNSUPPORTED, "set_mode_coefficients: spectral contexts only");
    const Plan &pl = c->pl;
    std::vector<double> coef(2 * (size_t)pl.total_pmodes, 0.0);
    for (const InstDev &d : pl.inst)
        for (int m = 0; m < d.n_modes; ++m) {
            coef[2 * ((size_t)d.pmode0 + m)] = cT[d.mode0 + m];
            coef[2 * ((size_t)d.pmode0 + m) + 1] = cP[d.mode0 + m];
        }
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    QS_HIP(hipMemcpyAsync(c->at(pl.off_coef), coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice,
                          c->stream),
           "copy push coefficients");
    QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
    return QS_OK;
}

qs_status qs::set_snapshot_cells(qs_ctx *c, const int32_t *first, int64_t *snap_elems) {
    if (!c || !first || !snap_elems) return fail(QS_ERR_ARG, "set_snapshot_cells: arguments are required");
    if (c->grid) return fail(QS_ERR_UNSUPPORTED, "set_snapshot_cells: spectral contexts only");
    Plan &pl = c->pl;
    for (size_t i = 0; i < pl.inst.size(); ++i)
        if (first[i] < 0 || first[i] >= pl.inst[i].n_xi)
            return fail(QS_ERR_ARG, "set_snapshot_cells: first cell of instance " + std::to_string(i) + " out of range");
    int64_t snap = 0;
    for (size_t i = 0; i < pl.inst.size(); ++i) {
        InstDev &d = pl.inst[i];
        d.snap_first = first[i];
        d.snap_off = snap;
        snap += (int64_t)(d.n_xi - d.snap_first) * d.snap_ld;
    }
    pl.snap_elems = snap;
    *snap_elems = snap;
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    QS_HIP(hipMemcpyAsync(c->at(pl.off_inst), pl.inst.data(), pl.inst.size() * sizeof(InstDev), hipMemcpyHostToDevice,
                          c->stream),
           "copy instance table");
    QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
    return QS_OK;
}

namespace {

bool is_grid(const qs_params *params, int32_t n) {
    return params && n >= 1 && params[0].geometry == QS_GEOM_TRANSVERSE_GRID;
}

qs_status check_grid(const qs_params *params, int32_t n) {
    if (n != 1) return fail(QS_ERR_ARG, "a TRANSVERSE_GRID instance must be the only instance of its context");
    return validate_one(params[0], 0);
}

}  // namespace

extern "C" {

int32_t qs_abi_version(void) { return QS_ABI_VERSION; }

const char *qs_last_error(void) { return g_err.c_str(); }

size_t qs_workspace_size_ex(const qs_params *params, int32_t n_instances, const qs_plan *plan) {
    if (is_grid(params, n_instances)) return check_grid(params, n_instances) == QS_OK ? grid_workspace_size(params[0]) : 0;
    Plan pl;
    if (make_plan(params, n_instances, plan, pl) != QS_OK) return 0;
    return pl.total;
}

size_t qs_workspace_size(const qs_params *params, int32_t n_instances) {
    return qs_workspace_size_ex(params, n_instances, nullptr);
}

qs_status qs_init_ex(const qs_params *params, int32_t n_instances, const qs_plan *plan, void *hip_stream,
                     void *workspace, size_t workspace_bytes, qs_ctx **out) {
    g_err.clear();
    if (!out) return fail(QS_ERR_ARG, "out is NULL");
    if (is_grid(params, n_instances)) {
        qs_status st = check_grid(params, n_instances);
        if (st != QS_OK) return st;
        if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
            return fail(QS_ERR_ARG, "workspace must be 256-byte aligned");
        qs_ctx *c = new (std::nothrow) qs_ctx;
        if (!c) return fail(QS_ERR_ALLOC, "host allocation of the context failed");
        c->stream = static_cast<hipStream_t>(hip_stream);
        if (hipGetDevice(&c->device) != hipSuccess) { delete c; return fail(QS_ERR_HIP, "hipGetDevice failed"); }
        std::string msg;
        st = grid_create(params[0], workspace, workspace_bytes, c->stream, &c->grid, &msg);
        if (st != QS_OK) { delete c; return fail(st, msg); }
        *out = c;
        return QS_OK;
    }
    Plan pl;
    qs_status st = make_plan(params, n_instances, plan, pl);
    if (st != QS_OK) return st;
    if (workspace && workspace_bytes < pl.total)
        return fail(QS_ERR_ALLOC, "workspace too small: need " + std::to_string(pl.total) + " bytes");
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
        return fail(QS_ERR_ARG, "workspace must be 256-byte aligned");
    qs_ctx *c = new (std::nothrow) qs_ctx;
    if (!c) return fail(QS_ERR_ALLOC, "host allocation of the context failed");
    c->pl = std::move(pl);
    c->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) { delete c; return hip_fail(e, "hipGetDevice"); }
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && khz > 0)
        c->wall_clock_hz = 1e3 * khz;
    (void)hipGetLastError();
    const size_t lds = march_lds_bytes(c->pl.precision, c->pl.nc, c->pl.wg_waves, c->pl.max_seg > 1);
    e = allow_march_lds(c->pl.precision, c->pl.nc, lds);
    if (e != hipSuccess) { delete c; return hip_fail(e, "allow march kernel LDS"); }
    if (workspace) {
        c->ws = static_cast<char *>(workspace);
    } else {
        void *p = nullptr;
        e = hipMalloc(&p, c->pl.total);
        if (e != hipSuccess) { delete c; return fail(QS_ERR_ALLOC, "hipMalloc of the workspace failed"); }
        c->ws = static_cast<char *>(p);
        c->owns_ws = true;
    }
    st = upload_tables(c, params);
    if (st == QS_OK) st = seed_state(c, params);
    if (st != QS_OK) { qs_free(c); return st; }
    *out = c;
    return QS_OK;
}

qs_status qs_init(const qs_params *params, int32_t n_instances, void *hip_stream, void *workspace,
                  size_t workspace_bytes, qs_ctx **out) {
    return qs_init_ex(params, n_instances, nullptr, hip_stream, workspace, workspace_bytes, out);
}

qs_status qs_get_plan(const qs_ctx *c, qs_plan *plan, int32_t *n_workgroups, int32_t *waves_per_workgroup) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    if (c->grid) return fail(QS_ERR_UNSUPPORTED, "transverse-grid contexts have no march plan");
    if (plan) {
        plan->columns_per_lane = c->pl.nc;
        plan->segment_cells = c->pl.seg_target;
        plan->max_segments = c->pl.max_seg;
        plan->reserved = 0;
    }
    if (n_workgroups) *n_workgroups = c->pl.n_wg;
    if (waves_per_workgroup) *waves_per_workgroup = c->pl.wg_waves;
    return QS_OK;
}

qs_status qs_step_tau(qs_ctx *c, int32_t n_steps, int32_t out_every, void *out_ln_e, void *out_ln_b,
                      void *out_max_ln_a) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    if (n_steps < 0) return fail(QS_ERR_ARG, "n_steps must be >= 0");
    if ((out_ln_e == nullptr) != (out_ln_b == nullptr))
        return fail(QS_ERR_ARG, "out_ln_e and out_ln_b must both be given or both be NULL");
    const bool snaps = out_ln_e != nullptr;
    if (snaps && out_every < 1) return fail(QS_ERR_ARG, "out_every must be >= 1");
    if (n_steps == 0 && !snaps) return QS_OK;
    if (c->poisoned && n_steps > 0)
        return fail(QS_ERR_STATE, "the context's state is invalid (" + c->poison_why +
                                      "); replace it with qs_set_state or qs_load_checkpoint");
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    if (c->grid) {
        std::string msg;
        qs_status st = grid_step(c->grid, n_steps, out_every, out_ln_e, out_ln_b, out_max_ln_a, c->stream, &msg);
        if (st != QS_OK) return fail(st, msg);
        c->steps_done += n_steps;
        return QS_OK;
    }
    const Plan &pl = c->pl;
    StepArgs a{};
    a.state = c->at(pl.off_state);
    a.blk_inst = reinterpret_cast<const int32_t *>(c->at(pl.off_blk));
    a.inst = reinterpret_cast<const InstDev *>(c->at(pl.off_inst));
    a.omega = c->at(pl.off_omega);
    a.kmode = reinterpret_cast<const double *>(c->at(pl.off_k));
    a.coef = reinterpret_cast<const double *>(c->at(pl.off_coef));
    a.log2s = reinterpret_cast<int32_t *>(c->at(pl.off_log2s));
    a.epend = reinterpret_cast<int32_t *>(c->at(pl.off_epend));
    a.total_modes = (int32_t)pl.total_modes;
    a.err = reinterpret_cast<uint32_t *>(c->at(pl.off_err));
    a.wave_table = reinterpret_cast<const int2 *>(c->at(pl.off_wtab));
    a.front0 = reinterpret_cast<const double *>(c->at(pl.off_front));
    // a segment waits for its predecessor to finish one step of its own cells: allow 2 s
    // plus 20 us per cell before the wait reports a stall
    a.wait_ticks = (uint64_t)(c->wall_clock_hz * (c->wait_seconds >= 0.0 ? c->wait_seconds
                                                                         : 2.0 + 20e-6 * pl.max_seg_len));
    const bool restoring = !(pl.inst[0].flags & QS_FLAG_NO_RESTORING);
    bool flat = true;
    for (const InstDev &d : pl.inst) flat = flat && (d.flags & kFlatProfile);
    auto launch = [&](bool fields, bool snap_first_only) {
        return launch_march(pl.precision, pl.nc, restoring, fields, flat, pl.n_wg, pl.wg_waves, pl.max_seg > 1,
                            snap_first_only, a, c->stream);
    };
    if (n_steps == 0) {
        a.ln_e = out_ln_e;
        a.ln_b = out_ln_b;
        a.update = 0;
        a.n_steps = 1;
        QS_HIP(launch(true, false), "march kernel");
        return QS_OK;
    }
    if (c->guard) QS_HIP(launch_guard_copy(guard_args(c), c->stream), "rollback copy");
    // segments of one mode combine their per-step maxima with order-independent atomics
    const bool keyed = out_max_ln_a != nullptr && pl.max_seg > 1;
    if (keyed)
        QS_HIP(launch_key_fill(pl.precision, out_max_ln_a, (int64_t)n_steps * pl.total_modes, c->stream), "key fill");
    a.max_ln_a = out_max_ln_a;
    a.keyed = keyed ? 1 : 0;
    a.update = 1;
    // one launch per snapshot interval: with one column per lane the stepping kernel writes
    // the snapshot of the interval's first step itself, keeping its two-step sweeps; with two
    // columns per lane the snapshot step runs as a one-step launch and the steps up to the
    // next snapshot as another; a snapshot at every step runs as one launch of snapshot steps
    const bool first_form = pl.nc == 1 && out_every > 1;
    int s0 = 0;
    while (s0 < n_steps) {
        const bool snap = snaps && (s0 % out_every == 0);
        int s1 = s0 + 1;
        if (!snap || first_form) {
            s1 = n_steps;
            if (snaps) s1 = std::min(n_steps, (s0 / out_every + 1) * out_every);
        } else if (out_every == 1) {
            s1 = n_steps;
        }
        a.ln_e = snap ? out_ln_e : nullptr;
        a.ln_b = snap ? out_ln_b : nullptr;
        a.snap_base = snap ? (int64_t)(s0 / out_every) * pl.snap_elems : 0;
        a.snap_stride = snap ? pl.snap_elems : 0;
        a.max_base = (int64_t)s0 * pl.total_modes;
        a.n_steps = s1 - s0;
        QS_HIP(launch(snap || out_max_ln_a != nullptr, snap && first_form), "march kernel");
        QS_HIP(launch_advance_steps(a.err, s1 - s0, c->stream), "step counter");
        c->steps_done += s1 - s0;
        s0 = s1;
    }
    if (keyed)
        QS_HIP(launch_key_decode(pl.precision, out_max_ln_a, (int64_t)n_steps * pl.total_modes, c->stream), "key decode");
    return QS_OK;
}

qs_status qs_sync_check(qs_ctx *c) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    if (c->grid) {
        std::string msg;
        qs_status st = grid_sync_check(c->grid, c->stream, &msg);
        if (st == QS_OK) return QS_OK;
        c->poisoned = true;
        c->poison_why = msg;
        return fail(st, msg + " after step " + std::to_string(c->steps_done) +
                            "; the state is invalid until replaced (qs_grid_set_state)");
    }
    QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
    const Plan &pl = c->pl;
    uint32_t err[kErrWords];
    QS_HIP(hipMemcpy(err, c->at(pl.off_err), sizeof(err), hipMemcpyDeviceToHost), "read error flags");
    if (!err[0] && !err[1]) return QS_OK;
    qs_status st;
    std::string msg;
    if (err[1]) {
        st = QS_ERR_HIP;
        msg = "a xi-segment hand-off wait gave up (the results of that launch are invalid)";
    } else {
        st = QS_ERR_NUMERIC;
        uint64_t key;
        std::memcpy(&key, err + 2, sizeof(key));
        key = ~key;
        const int64_t step = (int64_t)(key >> 32);
        const int64_t pm = (int64_t)(key & 0xffffffffu);
        msg = "non-finite state at renormalization";
        const int lm = 32 * pl.nc;  // padded modes per block
        for (size_t i = 0; i < pl.inst.size(); ++i) {
            const InstDev &d = pl.inst[i];
            if (pm >= d.pmode0 && pm < d.pmode0 + (int64_t)d.n_blocks * lm) {
                msg += " in instance " + std::to_string(i) + ", mode " + std::to_string(pm - d.pmode0);
                break;
            }
        }
        msg += ", after tau-step " + std::to_string(step);
    }
    // clear the flags, the first-failure key and nothing else (the step counter stays)
    QS_HIP(hipMemset(c->at(pl.off_err), 0, 4 * sizeof(uint32_t)), "clear error flags");
    int64_t good = -1;
    if (c->guard)
        QS_HIP(hipMemcpy(&good, c->guard + c->guard_bytes - sizeof(int64_t), sizeof(good), hipMemcpyDeviceToHost),
               "read rollback step");
    if (good >= 0) {
        const size_t sb = (size_t)pl.state_elems * pl.ts, nb = (size_t)pl.n_scale * sizeof(int32_t);
        QS_HIP(hipMemcpy(c->at(pl.off_state), c->guard, sb, hipMemcpyDeviceToDevice), "restore state");
        QS_HIP(hipMemcpy(c->at(pl.off_log2s), c->guard + sb, nb, hipMemcpyDeviceToDevice), "restore scales");
        QS_HIP(hipMemcpy(c->at(pl.off_epend), c->guard + sb + nb, nb, hipMemcpyDeviceToDevice), "restore scales");
        QS_HIP(hipMemcpy(c->at(pl.off_err) + 4 * sizeof(uint32_t), &good, sizeof(good), hipMemcpyHostToDevice),
               "restore step counter");
        c->steps_done = good;
        return fail(st, msg + "; the state was rolled back to tau-step " + std::to_string(good));
    }
    c->poisoned = true;
    c->poison_why = msg;
    return fail(st, msg + "; the state is invalid until replaced (qs_set_state or qs_load_checkpoint)");
}

qs_status qs_set_snapshot_align(qs_ctx *c, int32_t align, int64_t *snapshot_elems) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    if (c->grid) return fail(QS_ERR_UNSUPPORTED, "transverse-grid contexts have their own snapshot layout");
    if (align < 1 || align > 1024 || (align & (align - 1)) != 0)
        return fail(QS_ERR_ARG, "align must be a power of two in [1, 1024]");
    if (c->graphs > 0) return fail(QS_ERR_STATE, "the context has live graphs, which keep its snapshot layout");
    Plan &pl = c->pl;
    int64_t snap = 0;
    for (InstDev &d : pl.inst) {
        d.snap_first = 0;
        d.snap_ld = (int32_t)(((int64_t)d.n_modes + align - 1) / align * align);
        d.snap_off = snap;
        snap += (int64_t)d.n_xi * d.snap_ld;
    }
    pl.snap_elems = snap;
    if (snapshot_elems) *snapshot_elems = snap;
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    QS_HIP(hipMemcpyAsync(c->at(pl.off_inst), pl.inst.data(), pl.inst.size() * sizeof(InstDev), hipMemcpyHostToDevice,
                          c->stream),
           "copy instance table");
    QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
    return QS_OK;
}

qs_status qs_set_rollback(qs_ctx *c, int32_t enable) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    if (c->grid) return fail(QS_ERR_UNSUPPORTED, "transverse-grid contexts have no rollback copy");
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    if (!enable) {
        if (c->guard) {
            QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
            (void)hipFree(c->guard);
            c->guard = nullptr;
            c->guard_bytes = 0;
        }
        return QS_OK;
    }
    if (c->guard) return QS_OK;
    const Plan &pl = c->pl;
    const size_t bytes = (size_t)pl.state_elems * pl.ts + 2 * (size_t)pl.n_scale * sizeof(int32_t) + sizeof(int64_t);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(QS_ERR_ALLOC, "hipMalloc of the rollback copy failed");
    }
    const int64_t empty = -1;
    hipError_t e = hipMemcpy(static_cast<char *>(p) + bytes - sizeof(int64_t), &empty, sizeof(empty), hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(p); return hip_fail(e, "initialize the rollback copy"); }
    c->guard = static_cast<char *>(p);
    c->guard_bytes = bytes;
    return QS_OK;
}

qs_status qs_debug_set_wait_budget(qs_ctx *c, double seconds) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    if (!(seconds >= 0.0) && seconds != -1.0) return fail(QS_ERR_ARG, "seconds must be >= 0, or -1 for the default");
    c->wait_seconds = seconds;
    return QS_OK;
}

int64_t qs_steps_done(const qs_ctx *c) { return c ? c->steps_done : -1; }

qs_status qs_get_state(qs_ctx *c, double *rho, double *j_par, double *j_perp, double *log2_scale) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    if (c->grid) return fail(QS_ERR_UNSUPPORTED, "transverse-grid context: use qs_grid_get_state");
    const Plan &pl = c->pl;
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
    std::vector<char> raw((size_t)pl.state_elems * pl.ts);
    std::vector<int32_t> l2(pl.n_scale), ep(pl.n_scale);
    QS_HIP(hipMemcpy(raw.data(), c->at(pl.off_state), raw.size(), hipMemcpyDeviceToHost), "copy state");
    QS_HIP(hipMemcpy(l2.data(), c->at(pl.off_log2s), l2.size() * 4, hipMemcpyDeviceToHost), "copy scales");
    QS_HIP(hipMemcpy(ep.data(), c->at(pl.off_epend), ep.size() * 4, hipMemcpyDeviceToHost), "copy scales");
    const int NC = pl.nc, ROW = 3 * NC, LM = 32 * NC;
    auto val = [&](int64_t e) -> double {
        return pl.precision == QS_FP64 ? reinterpret_cast<const double *>(raw.data())[e]
                                       : (double)reinterpret_cast<const float *>(raw.data())[e];
    };
    std::vector<double> kmode(pl.total_pmodes);
    QS_HIP(hipMemcpy(kmode.data(), c->at(pl.off_k), kmode.size() * sizeof(double), hipMemcpyDeviceToHost),
           "copy wavenumbers");
    int64_t out0 = 0;
    for (const InstDev &d : pl.inst) {
        const int N = d.n_xi;
        const int64_t pm_inst = (int64_t)d.n_blocks * LM;  // padded modes of the instance
        for (int m = 0; m < d.n_modes; ++m) {
            const int b = m / LM, q = m % LM;
            const double k = kmode[d.pmode0 + m];
            // stored values of segment s are the true ones divided by 2^log2s; report them
            // against the largest applied+pending exponent of the mode (exact rescaling)
            int32_t lmax = INT32_MIN;
            for (int sg = 0; sg < d.n_seg; ++sg) {
                const int64_t si = d.scale_off + sg * pm_inst + m;
                lmax = std::max(lmax, l2[si] + ep[si]);
            }
            if (log2_scale) log2_scale[d.mode0 + m] = (double)lmax;
            for (int j = 0; j < N; ++j) {
                const int64_t si = d.scale_off + (j / d.seg_len) * pm_inst + m;
                const double sc = std::ldexp(1.0, l2[si] - lmax);
                const int64_t cell = d.state_off + ((int64_t)b * N + j) * ROW * kWave;
                auto x = [&](int var, int part) { return val(cell + elem_of(NC, q, var, part)) * sc; };
                const int64_t o = 2 * (out0 + (int64_t)m * N + j);
                if (rho) { rho[o] = x(0, 0); rho[o + 1] = x(0, 1); }
                // stored P' = j_par / h
                if (j_par) { j_par[o] = x(1, 0) * d.h; j_par[o + 1] = x(1, 1) * d.h; }
                // stored T' = k T with T = -i j_perp, i.e. j_perp = i T'/k (identically 0 at k = 0)
                if (j_perp) {
                    j_perp[o] = k != 0.0 ? -x(2, 1) / k : 0.0;
                    j_perp[o + 1] = k != 0.0 ? x(2, 0) / k : 0.0;
                }
            }
        }
        out0 += (int64_t)d.n_modes * N;
    }
    return QS_OK;
}

qs_status qs_set_state(qs_ctx *c, const double *rho, const double *j_par, const double *j_perp,
                       const double *log2_scale) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    if (c->grid) return fail(QS_ERR_UNSUPPORTED, "transverse-grid context: use qs_grid_set_state");
    if (!rho || !j_par || !j_perp || !log2_scale) return fail(QS_ERR_ARG, "all state arrays are required");
    const Plan &pl = c->pl;
    for (int64_t M = 0; M < pl.total_modes; ++M)
        if (!(log2_scale[M] == std::floor(log2_scale[M])) || std::fabs(log2_scale[M]) > 1e9)
            return fail(QS_ERR_ARG, "log2_scale entries must be integers");
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    std::vector<char> raw((size_t)pl.state_elems * pl.ts, 0);
    std::vector<int32_t> l2(pl.n_scale, 0), ep(pl.n_scale, 0);
    const int NC = pl.nc, ROW = 3 * NC, LM = 32 * NC;
    auto put = [&](int64_t e, double v) {
        if (pl.precision == QS_FP64) reinterpret_cast<double *>(raw.data())[e] = v;
        else reinterpret_cast<float *>(raw.data())[e] = (float)v;
    };
    std::vector<double> kmode(pl.total_pmodes);
    QS_HIP(hipMemcpy(kmode.data(), c->at(pl.off_k), kmode.size() * sizeof(double), hipMemcpyDeviceToHost),
           "copy wavenumbers");
    int64_t out0 = 0;
    for (const InstDev &d : pl.inst) {
        const int N = d.n_xi;
        const bool drop = (d.flags & QS_FLAG_DROP_LONGITUDINAL) != 0;
        for (int m = 0; m < d.n_modes; ++m) {
            const int b = m / LM, q = m % LM;
            const double k = kmode[d.pmode0 + m];
            for (int sg = 0; sg < d.n_seg; ++sg)
                l2[d.scale_off + (int64_t)sg * d.n_blocks * LM + m] = (int32_t)log2_scale[d.mode0 + m];
            for (int j = 0; j < N; ++j) {
                const int64_t cell = d.state_off + ((int64_t)b * N + j) * ROW * kWave;
                auto at = [&](int var, int part) { return cell + elem_of(NC, q, var, part); };
                const int64_t o = 2 * (out0 + (int64_t)m * N + j);
                put(at(0, 0), rho[o]); put(at(0, 1), rho[o + 1]);
                // P' = j_par/h; the outer rear face and dropped-longitudinal runs carry none
                const bool zp = drop || j == N - 1;
                put(at(1, 0), zp ? 0.0 : j_par[o] * d.ih); put(at(1, 1), zp ? 0.0 : j_par[o + 1] * d.ih);
                put(at(2, 0), k * j_perp[o + 1]); put(at(2, 1), -k * j_perp[o]);  // T' = -i k j_perp
            }
        }
        out0 += (int64_t)d.n_modes * N;
    }
    QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
    QS_HIP(hipMemcpy(c->at(pl.off_state), raw.data(), raw.size(), hipMemcpyHostToDevice), "copy state");
    QS_HIP(hipMemcpy(c->at(pl.off_log2s), l2.data(), l2.size() * 4, hipMemcpyHostToDevice), "copy scales");
    QS_HIP(hipMemcpy(c->at(pl.off_epend), ep.data(), ep.size() * 4, hipMemcpyHostToDevice), "copy scales");
    c->poisoned = false;
    return QS_OK;
}

namespace {
struct CkptHeader {
    uint64_t magic;        // "QSCKPT01"
    uint64_t state_bytes;  // bytes of the state image
    uint64_t pmodes;       // entries of each scale array
    uint64_t shape_hash;   // hash of the per-instance shapes and constants
    int64_t steps_done;
};
constexpr uint64_t kCkptMagic = 0x3130544B50435351ull;

uint64_t shape_hash(const Plan &pl) {
    // FNV-1a over the instance table (sizes, offsets and step constants; the snapshot layout
    // is no part of the state)
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    };
    for (InstDev d : pl.inst) {
        d.snap_off = 0;
        d.snap_first = 0;
        d.snap_ld = 0;
        mix(&d, sizeof(d));
    }
    mix(&pl.precision, sizeof(pl.precision));
    mix(&pl.nc, sizeof(pl.nc));
    mix(pl.wave_table.data(), pl.wave_table.size() * sizeof(int2));
    return h;
}
}  // namespace

size_t qs_checkpoint_size(const qs_ctx *c) {
    if (!c || c->grid) return 0;
    return sizeof(CkptHeader) + (size_t)c->pl.state_elems * c->pl.ts + 2 * (size_t)c->pl.n_scale * sizeof(int32_t);
}

qs_status qs_save_checkpoint(qs_ctx *c, void *dst, size_t bytes) {
    if (!c || !dst) return fail(QS_ERR_ARG, "ctx and dst are required");
    if (c->grid) return fail(QS_ERR_UNSUPPORTED, "checkpoints of transverse-grid contexts are not supported");
    if (bytes < qs_checkpoint_size(c)) return fail(QS_ERR_ARG, "checkpoint buffer too small");
    const Plan &pl = c->pl;
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
    CkptHeader hd{kCkptMagic, (uint64_t)pl.state_elems * pl.ts, (uint64_t)pl.n_scale, shape_hash(pl), c->steps_done};
    char *o = static_cast<char *>(dst);
    std::memcpy(o, &hd, sizeof(hd));
    o += sizeof(hd);
    QS_HIP(hipMemcpy(o, c->at(pl.off_state), hd.state_bytes, hipMemcpyDeviceToHost), "copy state");
    o += hd.state_bytes;
    QS_HIP(hipMemcpy(o, c->at(pl.off_log2s), pl.n_scale * 4, hipMemcpyDeviceToHost), "copy scales");
    o += pl.n_scale * 4;
    QS_HIP(hipMemcpy(o, c->at(pl.off_epend), pl.n_scale * 4, hipMemcpyDeviceToHost), "copy scales");
    return QS_OK;
}

qs_status qs_load_checkpoint(qs_ctx *c, const void *src, size_t bytes) {
    if (!c || !src) return fail(QS_ERR_ARG, "ctx and src are required");
    if (c->grid) return fail(QS_ERR_UNSUPPORTED, "checkpoints of transverse-grid contexts are not supported");
    if (bytes < qs_checkpoint_size(c)) return fail(QS_ERR_ARG, "checkpoint too small for this context");
    const Plan &pl = c->pl;
    CkptHeader hd;
    std::memcpy(&hd, src, sizeof(hd));
    if (hd.magic != kCkptMagic || hd.state_bytes != (uint64_t)pl.state_elems * pl.ts ||
        hd.pmodes != (uint64_t)pl.n_scale || hd.shape_hash != shape_hash(pl))
        return fail(QS_ERR_ARG, "checkpoint does not match this context's parameters");
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    QS_HIP(hipStreamSynchronize(c->stream), "synchronize");
    const char *o = static_cast<const char *>(src) + sizeof(hd);
    QS_HIP(hipMemcpy(c->at(pl.off_state), o, hd.state_bytes, hipMemcpyHostToDevice), "copy state");
    o += hd.state_bytes;
    QS_HIP(hipMemcpy(c->at(pl.off_log2s), o, pl.n_scale * 4, hipMemcpyHostToDevice), "copy scales");
    o += pl.n_scale * 4;
    QS_HIP(hipMemcpy(c->at(pl.off_epend), o, pl.n_scale * 4, hipMemcpyHostToDevice), "copy scales");
    QS_HIP(hipMemcpy(c->at(pl.off_err) + 4 * sizeof(uint32_t), &hd.steps_done, sizeof(int64_t), hipMemcpyHostToDevice),
           "set step counter");
    c->steps_done = hd.steps_done;
    c->poisoned = false;
    return QS_OK;
}

void qs_free(qs_ctx *c) {
    if (!c) return;
    if (c->grid) {
        (void)hipSetDevice(c->device);
        grid_free(c->grid, c->stream);
        delete c;
        return;
    }
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->guard) (void)hipFree(c->guard);
    if (c->owns_ws && c->ws) (void)hipFree(c->ws);
    delete c;
}

// ----------------------------------------------------------------------------- autotuner
}  // extern "C"

namespace {

uint64_t fnv(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 0x100000001B3ull; }
    return h;
}
template <typename T> uint64_t fnv_v(uint64_t h, const T &v) { return fnv(h, &v, sizeof(v)); }

// Key of a tuning result: everything that changes the work or its shape (not the seed).
uint64_t tune_key(const qs_params *p, int n, int steps) {
    uint64_t h = 0xCBF29CE484222325ull;
    h = fnv_v(h, n);
    h = fnv_v(h, steps);
    for (int i = 0; i < n; ++i) {
        const qs_params &q = p[i];
        h = fnv_v(h, q.n_species);
        h = fnv(h, q.q, sizeof(double) * q.n_species);
        h = fnv(h, q.m, sizeof(double) * q.n_species);
        h = fnv(h, q.nb_over_np, sizeof(double) * q.n_species);
        h = fnv_v(h, q.gamma_b); h = fnv_v(h, q.length); h = fnv_v(h, q.profile);
        h = fnv_v(h, q.n_xi); h = fnv_v(h, q.d_tau); h = fnv_v(h, q.precision);
        h = fnv_v(h, q.flags); h = fnv_v(h, q.n_modes);
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        h = fnv(h, prop.gcnArchName, std::strlen(prop.gcnArchName));
        h = fnv_v(h, prop.multiProcessorCount);
    }
    (void)hipGetLastError();
    return h;
}

bool cache_lookup(const char *path, uint64_t key, qs_plan *plan, double *ms) {
    FILE *f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return false;
    unsigned long long k;
    int nc, seg;
    double t;
    bool hit = false;
    while (std::fscanf(f, "%llx %d %d %lf", &k, &nc, &seg, &t) == 4) {
        if (k == key) { plan->columns_per_lane = nc; plan->segment_cells = seg; *ms = t; hit = true; }
    }
    std::fclose(f);
    return hit;
}

void cache_store(const char *path, uint64_t key, const qs_plan &plan, double ms) {
    FILE *f = path ? std::fopen(path, "a") : nullptr;
    if (!f) return;
    std::fprintf(f, "%016llx %d %d %.17g\n", (unsigned long long)key, plan.columns_per_lane, plan.segment_cells, ms);
    std::fclose(f);
}

}  // namespace

extern "C" {

qs_status qs_tune(const qs_params *params, int32_t n_instances, int32_t steps_per_call, qs_plan *best,
                  double *ms_per_step) {
    g_err.clear();
    if (!best) return fail(QS_ERR_ARG, "best is NULL");
    if (steps_per_call < 1) return fail(QS_ERR_ARG, "steps_per_call must be >= 1");
    if (is_grid(params, n_instances)) return fail(QS_ERR_UNSUPPORTED, "the autotuner plans spectral contexts only");
    Plan base;
    qs_status st = make_plan(params, n_instances, nullptr, base);
    if (st != QS_OK) return st;
    const char *cache = std::getenv("QS_TUNE_CACHE");
    const uint64_t key = tune_key(params, n_instances, steps_per_call);
    double cached_ms = 0.0;
    qs_plan hit{};
    if (cache_lookup(cache, key, &hit, &cached_ms)) {
        *best = hit;
        best->max_segments = 0;
        best->reserved = 0;
        if (ms_per_step) *ms_per_step = cached_ms;
        return QS_OK;
    }
    // candidates: columns per lane x segment counts the workgroup allows, plus the automatic
    // plan of each column count
    struct Cand { qs_plan plan; Plan pl; };
    std::vector<Cand> cands;
    for (int nc = 1; nc <= 2; ++nc) {
        const int Wmax = march_wg_waves(base.precision, nc);
        std::vector<int> segs = {0};
        for (int div : {1, 2, 3, 4, 6, 8, 12, 16})
            if (div <= Wmax) segs.push_back(div == 1 ? (1 << 20) : (base.max_n_xi + div - 1) / div);
        for (int seg : segs) {
            Cand c;
            c.plan = qs_plan{nc, seg, 0, 0};
            if (make_plan(params, n_instances, &c.plan, c.pl) != QS_OK) continue;
            c.plan.segment_cells = c.pl.seg_target;
            bool dup = false;
            for (const Cand &o : cands)
                dup = dup || (o.pl.nc == c.pl.nc && o.pl.wave_table.size() == c.pl.wave_table.size() &&
                              o.pl.seg_target == c.pl.seg_target && o.pl.wg_waves == c.pl.wg_waves);
            if (!dup) cands.push_back(std::move(c));
        }
    }
    size_t ws_bytes = 0;
    for (const Cand &c : cands) ws_bytes = std::max(ws_bytes, c.pl.total);
    // a call of n steps costs a + b n (a: launch and, for segmented plans, the pipeline
    // fill); measured directly for short calls, else fitted from calls of 16 and 96 steps
    // (long enough that the candidates of one run are ranked reliably: with two steps per
    // sweep a call of 96 steps is 48 sweeps)
    const int T1 = 16, T2 = 96;
    const bool direct = steps_per_call <= T2;
    const int T = direct ? steps_per_call : T2;
    const size_t out_bytes = (size_t)T * base.total_modes * base.ts;
    void *ws = nullptr, *outb = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (ws) (void)hipFree(ws);
        if (outb) (void)hipFree(outb);
    };
    if (hipMalloc(&ws, ws_bytes) != hipSuccess || hipMalloc(&outb, out_bytes) != hipSuccess) {
        cleanup();
        return fail(QS_ERR_ALLOC, "autotuner: hipMalloc failed");
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(QS_ERR_HIP, "autotuner: hipEventCreate failed");
    }
    double best_t = 1e300;
    qs_plan best_plan{};
    const bool verbose = std::getenv("QS_TUNE_VERBOSE") != nullptr;
    for (Cand &c : cands) {
        qs_ctx *ctx = nullptr;
        if (qs_init_ex(params, n_instances, &c.plan, nullptr, ws, ws_bytes, &ctx) != QS_OK) continue;
        auto timed = [&](int steps, float *ms) {
            return hipEventRecord(e0, nullptr) == hipSuccess &&
                   qs_step_tau(ctx, steps, 1, nullptr, nullptr, outb) == QS_OK &&
                   hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                   hipEventElapsedTime(ms, e0, e1) == hipSuccess;
        };
        float m1 = 0.f, m2 = 0.f;
        bool ok = qs_step_tau(ctx, 2, 1, nullptr, nullptr, outb) == QS_OK && timed(T, &m2);
        if (ok && !direct) ok = timed(T1, &m1);
        ok = ok && qs_sync_check(ctx) == QS_OK;
        qs_free(ctx);
        if (!ok) continue;
        double per = (double)m2 / T;
        if (!direct) {
            const double b = std::max(0.0, (double)(m2 - m1) / (T2 - T1));
            const double a0 = std::max(0.0, (double)m1 - T1 * b);
            per = (a0 + b * steps_per_call) / steps_per_call;
        }
        if (verbose)
            std::fprintf(stderr, "qs_tune: columns_per_lane %d segment_cells %d (segments %d, waves/workgroup %d): "
                                 "%.4f ms per step\n", c.pl.nc, c.pl.seg_target, c.pl.max_seg, c.pl.wg_waves, per);
        if (per < best_t) { best_t = per; best_plan = c.plan; }
    }
    cleanup();
    (void)hipGetLastError();
    if (best_t >= 1e300) return fail(QS_ERR_HIP, "autotuner: no candidate plan ran");
    best_plan.max_segments = 0;
    best_plan.reserved = 0;
    *best = best_plan;
    if (ms_per_step) *ms_per_step = best_t;
    cache_store(cache, key, best_plan, best_t);
    return QS_OK;
}

qs_status qs_grid_get_state(qs_ctx *c, double *rho, double *j_par, double *j_x, double *j_y) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    if (!c->grid) return fail(QS_ERR_UNSUPPORTED, "not a transverse-grid context");
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    std::string msg;
    qs_status st = grid_get_state(c->grid, rho, j_par, j_x, j_y, c->stream, &msg);
    return st == QS_OK ? QS_OK : fail(st, msg);
}

qs_status qs_grid_set_state(qs_ctx *c, const double *rho, const double *j_par, const double *j_x, const double *j_y) {
    if (!c) return fail(QS_ERR_ARG, "ctx is NULL");
    if (!c->grid) return fail(QS_ERR_UNSUPPORTED, "not a transverse-grid context");
    if (!rho || !j_par || !j_x || !j_y) return fail(QS_ERR_ARG, "all state arrays are required");
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    std::string msg;
    qs_status st = grid_set_state(c->grid, rho, j_par, j_x, j_y, c->stream, &msg);
    if (st != QS_OK) return fail(st, msg);
    c->poisoned = false;
    return QS_OK;
}

// ----------------------------------------------------------------------------- graphs
struct qs_graph {
    qs_ctx *ctx = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t n_steps = 0;
};

qs_status qs_graph_create(qs_ctx *c, int32_t n_steps, int32_t out_every, void *out_ln_e, void *out_ln_b,
                          void *out_max_ln_a, qs_graph **out) {
    if (!c || !out) return fail(QS_ERR_ARG, "ctx and out are required");
    if (n_steps < 1) return fail(QS_ERR_ARG, "n_steps must be >= 1");
    *out = nullptr;
    QS_HIP(hipSetDevice(c->device), "hipSetDevice");
    // capture the launches of one qs_step_tau call on a private stream (the context's own
    // stream may be the null stream, which cannot be captured)
    hipStream_t cap = nullptr;
    QS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "create capture stream");
    hipStream_t keep = c->stream;
    const int64_t done = c->steps_done;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    qs_status st = QS_OK;
    if (e == hipSuccess) {
        c->stream = cap;
        st = qs_step_tau(c, n_steps, out_every, out_ln_e, out_ln_b, out_max_ln_a);
        c->stream = keep;
        c->steps_done = done;  // nothing ran
        e = hipStreamEndCapture(cap, &g);
    }
    std::string msg = g_err;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess && st == QS_OK) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (st != QS_OK) return fail(st, msg);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    qs_graph *q = new (std::nothrow) qs_graph;
    if (!q) { (void)hipGraphExecDestroy(exec); return fail(QS_ERR_ALLOC, "host allocation failed"); }
    q->ctx = c;
    q->exec = exec;
    q->n_steps = n_steps;
    ++c->graphs;
    *out = q;
    return QS_OK;
}

qs_status qs_graph_launch(qs_graph *g) {
    if (!g) return fail(QS_ERR_ARG, "graph is NULL");
    if (g->ctx->poisoned)
        return fail(QS_ERR_STATE, "the context's state is invalid (" + g->ctx->poison_why +
                                      "); replace it with qs_set_state or qs_load_checkpoint");
    QS_HIP(hipSetDevice(g->ctx->device), "hipSetDevice");
    QS_HIP(hipGraphLaunch(g->exec, g->ctx->stream), "graph launch");
    g->ctx->steps_done += g->n_steps;
    return QS_OK;
}

void qs_graph_free(qs_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    (void)hipGraphExecDestroy(g->exec);
    --g->ctx->graphs;
    delete g;
}

// Host evaluation of the device's SplitMix64 (used by the generator cross-check tests).
uint64_t qs_debug_splitmix64(uint64_t seed, uint64_t i) { return splitmix64_host(seed, i); }

}  // extern "C"
