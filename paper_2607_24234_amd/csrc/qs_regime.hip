// E/B regime diagnostic over field snapshots (include/qs_regime.h; Sec. III.B and III.C):
// per (cell, mode) the ratio of the electric to the magnetic field energy summed over a
// window of 2w + 1 cells, and per mode the first electrically dominated cell.
//
// Windows are summed a sub-tile of T consecutive outputs at a time.  With the span
// s[i] = cell j0 - w + i of outputs j0 + r (r < T), the window of output r is s[r .. r + 2w];
// when 2w + 1 >= T it splits into a suffix of the head s[0 .. T-1], the middle s[T .. 2w]
// common to all T outputs, and a prefix of the tail s[2w+1 ..], so each output costs a few
// adds and nothing is ever subtracted (a running sum that drops the cell leaving the window
// loses the small terms of a field spanning many decades along xi).  Each field's terms are
// exp(2 (ln - m)) with m that field's largest value over a span around the outputs; an
// output whose sum falls below Tiny (its window far below m) is summed again over its own
// window, and a field with no finite value in the span gives -inf (NaN where a value is
// NaN) without that.  Narrow windows (2w + 1 < kTile) are summed directly.  Three forms:
// FP32 windows of 8..64 cells stream each 64-mode block down xi through LDS, the middles
// from 8-row block sums (regime_stream); other windows that fit stage 64-mode tiles in LDS
// (regime_tile); the rest walk global memory one lane per mode (regime_map).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>

#include "../../include/qs_regime.h"
#include "qs_internal.h"

namespace {

constexpr int kTile = 16;

template <typename T>
struct Tiny;
template <>
struct Tiny<float> {
    static constexpr float v = 1e-25f;   // FP32 terms below ~1e-38 vanish: < 1e-11 of such a sum
};
template <>
struct Tiny<double> {
    static constexpr double v = 1e-250;
};

// FP32 uses the hardware base-2 exponential and logarithm (about 1 ulp each; an argument
// 2 (ln - m) of magnitude up to ~60 carries a relative rounding of ~1e-6 into a term, far
// inside the FP32 bar of R); FP64 the library's correctly rounded-to-1-ulp exp and log
__device__ __forceinline__ float ex(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
__device__ __forceinline__ double ex(double x) { return exp(x); }
__device__ __forceinline__ float lg(float x) { return __builtin_amdgcn_logf(x) * 0.69314718055994531f; }
__device__ __forceinline__ double lg(double x) { return log(x); }

// 1/2 ln sum_{i=lo..hi} e^{2 v_i} over one window, relative to the window's own largest value:
// NaN if the window holds a NaN, -inf if every value is -inf
template <typename T>
__device__ __attribute__((noinline)) T window_log_energy(const T *__restrict__ v, int64_t stride, int lo, int hi) {
    T top = -INFINITY;
    bool nan = false;
    for (int i = lo; i <= hi; ++i) {
        const T x = v[(int64_t)i * stride];
        nan |= x != x;
        top = fmax(top, x);
    }
    if (nan) return (T)NAN;
    if (top == -INFINITY) return -INFINITY;
    T s = 0;
    for (int i = lo; i <= hi; ++i) s += ex(T(2) * (v[(int64_t)i * stride] - top));
    return top + T(0.5) * lg(s);
}

// Terms exp(2 (ln - m)) are taken against r = ref(m): m itself, or 0 when m = -inf (no
// finite value in the span: the terms are then 0, or NaN for a NaN).  A window's 1/2 ln of its
// energy from its term sum: -inf (or NaN) when m = -inf; m + 1/2 ln(sum) while the sum stays
// above Tiny; else, or when m = +inf, summed again over the window's own values in G.
template <typename T>
__device__ __forceinline__ T ref(T m) { return m == -INFINITY ? T(0) : m; }

template <typename T>
__device__ __forceinline__ T window_L(T m, T sum, const T *G, int64_t gst, int lo, int hi) {
    if (m == -INFINITY) return sum != sum ? (T)NAN : -INFINITY;
    if (m < INFINITY && !(sum < Tiny<T>::v)) return m + T(0.5) * lg(sum);
    return window_log_energy(G, gst, lo, hi);
}

// Outputs j = ja .. jb-1 (all valid: w <= j < n - w) of one mode, read from global memory.
// E, B address that mode's column with E[(c - cell0) * st] = cell c; R (may be null) is the
// column of the output, rst apart; first = the first j with R_j > 0 here (-1 if none).  Per
// kTile outputs the span maximum, the terms, and the head / middle / tail sums.
template <typename T>
__device__ __forceinline__ void run_outputs(const T *E, const T *B, int64_t st, int cell0, int ja, int jb, int w,
                                            T *__restrict__ R, int64_t rst, int &first) {
    first = -1;
    auto emit = [&](int j, T le, T lb) {
        const T r = le - lb;
        if (R) R[(int64_t)j * rst] = r;
        if (first < 0 && r > T(0)) first = j;
    };
    if (2 * w + 1 < kTile) {
        for (int j = ja; j < jb; ++j)
            emit(j, window_log_energy(E, st, j - w - cell0, j + w - cell0),
                 window_log_energy(B, st, j - w - cell0, j + w - cell0));
        return;
    }
    for (int j0 = ja; j0 < jb; j0 += kTile) {
        const int c = min(kTile, jb - j0);
        const T *Es = E + (int64_t)(j0 - w - cell0) * st, *Bs = B + (int64_t)(j0 - w - cell0) * st;   // s[0]
        const int len = 2 * w + c;                                                                     // span cells
        T mE = -INFINITY, mB = -INFINITY;
#pragma unroll 8
        for (int i = 0; i < len; ++i) {
            mE = fmax(mE, Es[(int64_t)i * st]);
            mB = fmax(mB, Bs[(int64_t)i * st]);
        }
        const T rE = ref(mE), rB = ref(mB);
        // head suffix sums, middle sum, then the outputs with the tail prefix
        T hE[kTile], hB[kTile];
#pragma unroll
        for (int r = 0; r < kTile; ++r) {
            hE[r] = ex(T(2) * (Es[(int64_t)r * st] - rE));
            hB[r] = ex(T(2) * (Bs[(int64_t)r * st] - rB));
        }
#pragma unroll
        for (int r = kTile - 2; r >= 0; --r) {
            hE[r] += hE[r + 1];
            hB[r] += hB[r + 1];
        }
        T sE = 0, sB = 0;
#pragma unroll 8
        for (int i = kTile; i <= 2 * w; ++i) {
            sE += ex(T(2) * (Es[(int64_t)i * st] - rE));
            sB += ex(T(2) * (Bs[(int64_t)i * st] - rB));
        }
        T pE = 0, pB = 0;
#pragma unroll
        for (int r = 0; r < kTile; ++r) {
            if (r < c) {
                const int j = j0 + r;
                const T se = hE[r] + sE + pE, sb = hB[r] + sB + pB;
                emit(j, window_L(mE, se, E, st, j - w - cell0, j + w - cell0),
                     window_L(mB, sb, B, st, j - w - cell0, j + w - cell0));
                if (r + 1 < c) {
                    pE += ex(T(2) * (Es[(int64_t)(2 * w + 1 + r) * st] - rE));
                    pB += ex(T(2) * (Bs[(int64_t)(2 * w + 1 + r) * st] - rB));
                }
            }
        }
    }
}

// General form: one lane per mode walks its whole column in global memory (any window).
template <typename T>
__global__ void __launch_bounds__(256) regime_map(const T *__restrict__ ln_e, const T *__restrict__ ln_b, int64_t n_modes,
                                                  int n, int w, T *__restrict__ out, int32_t *__restrict__ first_out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_modes) return;
    const int64_t st = n_modes;
    T *R = out ? out + k : nullptr;
    // cells whose window would leave [0, n)
    const int jbeg = w < n ? w : n, jend = n - w > jbeg ? n - w : jbeg;   // valid outputs: [jbeg, jend)
    if (R) {
        for (int j = 0; j < jbeg; ++j) R[(int64_t)j * st] = (T)NAN;
        for (int j = jend; j < n; ++j) R[(int64_t)j * st] = (T)NAN;
    }
    int first;
    run_outputs(ln_e + k, ln_b + k, st, 0, jbeg, jend, w, R, st, first);
    if (first_out) first_out[k] = first;
}

// Window sums for outputs ja .. jb-1 from terms already in LDS: X[(c - cell0) * 64] holds
// exp(2 (ln_c - m)) for one field of one mode (m its largest value over the staged span), so
// each output costs a few adds: the head suffix, the middle common to kTile outputs and the
// tail prefix (nothing subtracted).  Windows whose sum falls below Tiny (far below m), and
// every window when m is not finite, are summed again from the raw column G (global memory,
// G[c * gst] = ln of cell c).  L[r] = 1/2 ln sum |F|^2 of output ja + r (r < kTile).
template <typename T>
__device__ __forceinline__ void window_energies(const T *X, int cell0, int ja, int c, int w, T m, const T *G,
                                                int64_t gst, T (&L)[kTile]) {
    const T *Xs = X + (ja - w - cell0) * 64;   // s[0]
    if (2 * w + 1 < kTile) {
#pragma unroll
        for (int r = 0; r < kTile; ++r) {
            if (r < c) {
                T sum = 0;
                for (int i = 0; i <= 2 * w; ++i) sum += Xs[(r + i) * 64];
                L[r] = window_L(m, sum, G, gst, ja + r - w, ja + r + w);
            }
        }
        return;
    }
    T h[kTile];
#pragma unroll
    for (int r = 0; r < kTile; ++r) h[r] = Xs[r * 64];
#pragma unroll
    for (int r = kTile - 2; r >= 0; --r) h[r] += h[r + 1];
    T mid = 0;
#pragma unroll 8
    for (int i = kTile; i <= 2 * w; ++i) mid += Xs[i * 64];
    T pre = 0;
#pragma unroll
    for (int r = 0; r < kTile; ++r) {
        if (r < c) {
            const T sum = h[r] + mid + pre;
            L[r] = window_L(m, sum, G, gst, ja + r - w, ja + r + w);
            if (r + 1 < c) pre += Xs[(2 * w + 1 + r) * 64];
        }
    }
}

// Staged form: a workgroup takes 64 modes and `to` consecutive outputs.  Its 256 threads copy
// the span of those outputs (to + 2w cells of both fields, one 64-mode row per wave and
// load) into LDS once, find each mode's largest value of each field over the span, and turn
// every staged value into its term exp(2 (ln - m)) in place; wave v then sums the windows of
// quarter v of the tile from LDS (lane = mode, rows read without bank conflicts).  Each cell
// is read from memory (to + 2w) / to times and exponentiated as often, instead of once per
// window.  The first electrically dominated cell combines over the tile's waves, then over
// tiles with atomicMin (first_out starts at INT32_MAX; regime_first_finish maps what is left
// to -1).
template <typename T>
__global__ void __launch_bounds__(256) regime_tile(const T *__restrict__ ln_e, const T *__restrict__ ln_b, int64_t n_modes,
                                                   int n, int w, int to, T *__restrict__ out, int32_t *__restrict__ first_out) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __shared__ int fw[4][64];
    __shared__ T pm[2][4][64];
    T *sE = reinterpret_cast<T *>(smem);
    T *sB = sE + (size_t)(to + 2 * w) * 64;
    const int jbeg = w, jend = n - w;   // the host launches this form only when jend > jbeg
    const int o0 = jbeg + (int)blockIdx.y * to, o1 = min(o0 + to, jend);
    const int rows = (o1 - o0) + 2 * w, c0 = o0 - w;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t k = (int64_t)blockIdx.x * 64 + lane;
    const bool live = k < n_modes;
    const int64_t kk = live ? k : 0;
    constexpr int U = 40;  // rows in flight per wave before their LDS stores
    T mE = -INFINITY, mB = -INFINITY;
    for (int r0 = wv; r0 < rows; r0 += 4 * U) {
        T ve[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = min(r0 + 4 * u, rows - 1);
            const int64_t g = (int64_t)(c0 + r) * n_modes + kk;
            ve[u] = ln_e[g];
            vb[u] = ln_b[g];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = r0 + 4 * u;
            if (r < rows) {
                sE[r * 64 + lane] = ve[u];
                sB[r * 64 + lane] = vb[u];
                mE = fmax(mE, ve[u]);
                mB = fmax(mB, vb[u]);
            }
        }
    }
    pm[0][wv][lane] = mE;
    pm[1][wv][lane] = mB;
    __syncthreads();
    mE = fmax(fmax(pm[0][0][lane], pm[0][1][lane]), fmax(pm[0][2][lane], pm[0][3][lane]));
    mB = fmax(fmax(pm[1][0][lane], pm[1][1][lane]), fmax(pm[1][2][lane], pm[1][3][lane]));
    // each wave turns the rows it staged into terms (its own writes: no barrier needed before)
    const T rE = ref(mE), rB = ref(mB);
    for (int r = wv; r < rows; r += 4) {
        sE[r * 64 + lane] = ex(T(2) * (sE[r * 64 + lane] - rE));
        sB[r * 64 + lane] = ex(T(2) * (sB[r * 64 + lane] - rB));
    }
    __syncthreads();
    const int q = (o1 - o0 + 3) / 4;
    const int ja = o0 + wv * q, jb = min(ja + q, o1);
    T *R = out && live ? out + k : nullptr;
    int first = -1;
    if (live) {
        for (int j0 = ja; j0 < jb; j0 += kTile) {
            const int c = min(kTile, jb - j0);
            T le[kTile], lb[kTile];
            window_energies(sE + lane, c0, j0, c, w, mE, ln_e + k, n_modes, le);
            window_energies(sB + lane, c0, j0, c, w, mB, ln_b + k, n_modes, lb);
#pragma unroll
            for (int r = 0; r < kTile; ++r) {
                if (r < c) {
                    const T v = le[r] - lb[r];
                    if (R) R[(int64_t)(j0 + r) * n_modes] = v;
                    if (first < 0 && v > T(0)) first = j0 + r;
                }
            }
        }
    }
    if (R) {
        if (blockIdx.y == 0)
            for (int j = wv; j < jbeg; j += 4) R[(int64_t)j * n_modes] = (T)NAN;
        if (blockIdx.y == gridDim.y - 1)
            for (int j = jend + wv; j < n; j += 4) R[(int64_t)j * n_modes] = (T)NAN;
    }
    fw[wv][lane] = first < 0 ? INT32_MAX : first;
    __syncthreads();
    if (wv == 0 && live && first_out) {
        const int f = min(min(fw[0][lane], fw[1][lane]), min(fw[2][lane], fw[3][lane]));
        if (f != INT32_MAX) atomicMin(first_out + k, f);
    }
}

// Streaming form (FP32, kTile <= 2w + 1, 2w + kChunk <= kSpan): a workgroup of 16 waves takes
// 64 modes and walks its share of the outputs in chunks of kChunk = 128 (8 per wave).  LDS
// holds the raw ln values of both fields over the current chunk's span, row i = cell
// o0 - w + i (o0 the chunk's first output), so every access is a fixed offset from the
// wave's first row.  Per chunk: each mode's largest value of each field over the span
// (from the values the threads staged, exchanged through LDS); the raw halo rows the next
// chunk keeps into registers; every staged value turned into its term in place, once, with
// the 8-row block sums; then each wave's windows from the terms (head and tail term by term,
// the middle from block sums).  Meanwhile the rows of the next chunk are in flight into
// registers; once the chunk is done the halo rows go to the front and the new rows follow
// them.  Every cell is read from memory once (plus a 2w halo where a mode block's outputs
// are split between workgroups) and exponentiated (kChunk + 2w) / kChunk times.
constexpr int kChunk = 128;
constexpr int kSpan = 256;
constexpr int kWaves = 16;               // waves per streaming workgroup
constexpr int kSub = kChunk / kWaves;    // outputs (and block rows) per wave and chunk

// Outputs ja .. ja+c-1 (c <= TS) of one wave against the chunk's references mE, mB.  E, B
// point at the wave's first span row (s[0] = cell ja - w), rows 64 apart, holding the terms
// exp(2 (ln - ref(m))) of the span; bE, bB at the block sums of that row's block (block TS
// rows, 64 apart), so the middle s[TS .. 2w] is q = (2w + 1 - TS) / TS whole blocks plus a
// remainder; head and tail terms one by one.
template <int TS, typename T>
__device__ __forceinline__ void span_outputs(const T *E, const T *B, const T *bE, const T *bB, int ja, int c, int w,
                                             T mE, T mB, const T *GE, const T *GB, int64_t gst, T *__restrict__ R,
                                             int &first) {
    T hE[TS], hB[TS];
#pragma unroll
    for (int r = 0; r < TS; ++r) {
        hE[r] = E[r * 64];
        hB[r] = B[r * 64];
    }
#pragma unroll
    for (int r = TS - 2; r >= 0; --r) {
        hE[r] += hE[r + 1];
        hB[r] += hB[r + 1];
    }
    const int q = (2 * w + 1 - TS) / TS;
    T sE = 0, sB = 0;
    for (int b = 1; b <= q; ++b) {
        sE += bE[b * 64];
        sB += bB[b * 64];
    }
    for (int i = TS * (q + 1); i <= 2 * w; ++i) {
        sE += E[i * 64];
        sB += B[i * 64];
    }
    const T *Et = E + (2 * w + 1) * 64, *Bt = B + (2 * w + 1) * 64;   // the tail
    // the quick form of window_L; outputs that need their own window's sum are marked and
    // done after the loop (written out there: the kernel makes no calls)
    auto quick = [&](T m, T sum, bool &again) -> T {
        if (m == -INFINITY) return sum != sum ? (T)NAN : -INFINITY;
        if (m < INFINITY && !(sum < Tiny<T>::v)) return m + T(0.5) * lg(sum);
        again = true;
        return T(0);
    };
    unsigned again = 0, pos = 0;   // bit r: output r redone below / R > 0
    T pE = 0, pB = 0;
#pragma unroll
    for (int r = 0; r < TS; ++r) {
        if (r < c) {
            bool a = false;
            const T v = quick(mE, hE[r] + sE + pE, a) - quick(mB, hB[r] + sB + pB, a);
            if (!a) {
                if (R) R[(int64_t)(ja + r) * gst] = v;
                pos |= (unsigned)(v > T(0)) << r;
            } else {
                again |= 1u << r;
            }
            if (r + 1 < c) {
                pE += Et[r * 64];
                pB += Bt[r * 64];
            }
        }
    }
    if (again) {
        // rare: 1/2 ln sum over the output's own window from global memory, against that
        // window's own largest value (as window_log_energy)
        auto own = [&](const T *G, int lo, int hi) -> T {
            T top = -INFINITY;
            bool nan = false;
            for (int i = lo; i <= hi; ++i) {
                const T x = G[(int64_t)i * gst];
                nan |= x != x;
                top = fmax(top, x);
            }
            if (nan) return (T)NAN;
            if (top == -INFINITY) return -INFINITY;
            T sum = 0;
            for (int i = lo; i <= hi; ++i) sum += ex(T(2) * (G[(int64_t)i * gst] - top));
            return top + T(0.5) * lg(sum);
        };
        for (int r = 0; r < c; ++r) {
            if ((again >> r) & 1u) {
                const int j = ja + r;
                const T v = own(GE, j - w, j + w) - own(GB, j - w, j + w);
                if (R) R[(int64_t)j * gst] = v;
                pos |= (unsigned)(v > T(0)) << r;
            }
        }
    }
    if (first < 0 && pos) first = ja + __builtin_ctz(pos);
}

template <typename T>
__global__ void __launch_bounds__(64 * kWaves) regime_stream(const T *__restrict__ ln_e, const T *__restrict__ ln_b,
                                                             int64_t n_modes, int n, int w, int chunks_per_group,
                                                             T *__restrict__ out, int32_t *__restrict__ first_out) {
    __shared__ T span[2][kSpan * 64];
    __shared__ int fw[kWaves][64];
    __shared__ T pm[2][kWaves][64];
    __shared__ T bsum[2][kSpan / kSub][64];
    const int jbeg = w, jend = n - w;   // the host launches this form only when jend > jbeg and 2w + kChunk <= kSpan
    const int n_chunks = (jend - jbeg + kChunk - 1) / kChunk;
    const int ca = (int)blockIdx.y * chunks_per_group, cb = min(ca + chunks_per_group, n_chunks);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // Workgroups are dealt to the eight XCDs in turn; XCD x takes a contiguous range of mode
    // blocks, so the blocks that run side by side on one XCD are neighbours in memory and
    // share, in that XCD's L2, the cache lines their rows straddle (a row of n_modes values
    // is in general not line-aligned).
    const unsigned nb = gridDim.x, q8 = nb / 8, r8 = nb % 8, x8 = blockIdx.x % 8;
    const unsigned mb = x8 * q8 + min(x8, r8) + blockIdx.x / 8;
    const int64_t k = (int64_t)mb * 64 + lane;
    const bool live = k < n_modes;
    const int64_t kk = live ? k : 0;
    const T *GE = ln_e + kk, *GB = ln_b + kk;
    T *R = out && live ? out + k : nullptr;
    T *sE = span[0] + lane, *sB = span[1] + lane;
    if (R) {
        if (blockIdx.y == 0)
            for (int j = wv; j < jbeg; j += kWaves) R[(int64_t)j * n_modes] = (T)NAN;
        if (blockIdx.y == gridDim.y - 1)
            for (int j = jend + wv; j < n; j += kWaves) R[(int64_t)j * n_modes] = (T)NAN;
    }
    int first = -1;
    if (ca < cb) {   // uniform over the workgroup
        // the first chunk's span: cells [o0 - w, min(o0 + kChunk, jend) + w) into rows 0 ..
        {
            const int c0 = jbeg + ca * kChunk - w;
            const int rows = min(kChunk, jend - (jbeg + ca * kChunk)) + 2 * w;
            T a = -INFINITY, bb = -INFINITY;
            constexpr int U = kSpan / kWaves / 2;   // two rounds of loads in flight
            for (int r0 = wv; r0 < rows; r0 += kWaves * U) {
                T ve[U], vb[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int r = min(r0 + kWaves * u, rows - 1);
                    ve[u] = GE[(int64_t)(c0 + r) * n_modes];
                    vb[u] = GB[(int64_t)(c0 + r) * n_modes];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int r = r0 + kWaves * u;
                    if (r < rows) {
                        sE[r * 64] = ve[u];
                        sB[r * 64] = vb[u];
                        a = fmax(a, ve[u]);
                        bb = fmax(bb, vb[u]);
                    }
                }
            }
            pm[0][wv][lane] = a;
            pm[1][wv][lane] = bb;
        }
        __syncthreads();
        for (int ch = ca; ch < cb; ++ch) {
            const int o0 = jbeg + ch * kChunk, o1 = min(o0 + kChunk, jend);
            // rows of the next chunk: cells [o1 + w, o1 + w + nn), in flight during this chunk
            const int nn = ch + 1 < cb ? min(o1 + kChunk, jend) - o1 : 0;
            constexpr int P = kChunk / kWaves;
            T pe[P], pb[P];
#pragma unroll
            for (int u = 0; u < P; ++u) {
                const int r = min(wv + kWaves * u, max(nn - 1, 0));
                const int64_t g = (int64_t)(nn > 0 ? o1 + w + r : o0) * n_modes;
                pe[u] = GE[g];
                pb[u] = GB[g];
            }
            T mE = pm[0][0][lane], mB = pm[1][0][lane];
#pragma unroll
            for (int v = 1; v < kWaves; ++v) {
                mE = fmax(mE, pm[0][v][lane]);
                mB = fmax(mB, pm[1][v][lane]);
            }
            // the last 2w rows move to the front of the next chunk's span as raw values: this
            // thread's halo rows into registers before the span turns into terms
            constexpr int H = kChunk / kWaves;   // 2w <= kChunk rows of halo
            T he[H], hb[H];
            T a = -INFINITY, bb = -INFINITY;
            if (nn > 0) {
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    const int r = wv + kWaves * u;
                    if (r < 2 * w) {
                        he[u] = sE[(kChunk + r) * 64];
                        hb[u] = sB[(kChunk + r) * 64];
                        a = fmax(a, he[u]);
                        bb = fmax(bb, hb[u]);
                    }
                }
            }
            __syncthreads();   // every halo row is read
            // every span value into its term exp(2 (ln - ref(m))) in place (each value
            // exponentiated once per chunk), with the sums over kSub-row blocks
            {
                const T rE = ref(mE), rB = ref(mB);
                const int len = (o1 - o0) + 2 * w, nblk = (len + kSub - 1) / kSub;
                for (int b = wv; b < nblk; b += kWaves) {
                    T sa = 0, sb = 0;
#pragma unroll
                    for (int i = 0; i < kSub; ++i) {
                        const int rr = b * kSub + i;
                        if (rr < len) {
                            const T te = ex(T(2) * (sE[rr * 64] - rE)), tb = ex(T(2) * (sB[rr * 64] - rB));
                            sE[rr * 64] = te;
                            sB[rr * 64] = tb;
                            sa += te;
                            sb += tb;
                        }
                    }
                    bsum[0][b][lane] = sa;
                    bsum[1][b][lane] = sb;
                }
            }
            __syncthreads();
            const int ja = o0 + kSub * wv, c = min(kSub, o1 - ja);
            if (live && c > 0) {
                int f = -1;
                span_outputs<kSub>(sE + kSub * wv * 64, sB + kSub * wv * 64, &bsum[0][wv][lane], &bsum[1][wv][lane], ja,
                                   c, w, mE, mB, GE, GB, n_modes, R, f);
                if (first < 0) first = f;
            }
            __syncthreads();   // the chunk's windows are summed
            if (nn > 0) {      // uniform; then o1 - o0 = kChunk
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    const int r = wv + kWaves * u;
                    if (r < 2 * w) {
                        sE[r * 64] = he[u];
                        sB[r * 64] = hb[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < P; ++u) {
                    const int r = wv + kWaves * u;
                    if (r < nn) {
                        sE[(2 * w + r) * 64] = pe[u];
                        sB[(2 * w + r) * 64] = pb[u];
                        a = fmax(a, pe[u]);
                        bb = fmax(bb, pb[u]);
                    }
                }
                pm[0][wv][lane] = a;
                pm[1][wv][lane] = bb;
                __syncthreads();
            }
        }
    }
    fw[wv][lane] = first < 0 ? INT32_MAX : first;
    __syncthreads();
    if (wv == 0 && live && first_out) {
        int f = fw[0][lane];
#pragma unroll
        for (int v = 1; v < kWaves; ++v) f = min(f, fw[v][lane]);
        if (f != INT32_MAX) atomicMin(first_out + k, f);
    }
}

__global__ void __launch_bounds__(256) regime_first_fill(int32_t *__restrict__ f, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] = INT32_MAX;
}

__global__ void __launch_bounds__(256) regime_first_finish(int32_t *__restrict__ f, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && f[i] == INT32_MAX) f[i] = -1;
}

// Tile length of the staged form for a window of w cells, and its LDS bytes: the longest
// tile (at least 64 outputs) whose span fits 74 KiB (two workgroups per compute unit), else
// 152 KiB (one); 0 if neither fits (the general form runs instead).
template <typename T>
int tile_outputs(int w, int n_valid, size_t *lds) {
    const size_t row = 64 * 2 * sizeof(T);
    for (const size_t lim : {(size_t)74 * 1024, (size_t)152 * 1024}) {
        const int64_t rmax = (int64_t)(lim / row);
        if (rmax >= 2 * (int64_t)w + 64) {
            // whole sub-tiles of kTile outputs for each of the four waves
            const int to = (int)std::min<int64_t>((rmax - 2 * (int64_t)w) / (4 * kTile) * (4 * kTile), n_valid);
            *lds = (size_t)(to + 2 * w) * row;
            return to;
        }
    }
    return 0;
}

template <typename T>
hipError_t launch(const T *e, const T *b, int64_t n_modes, int n, int w, T *R, int32_t *F, hipStream_t s) {
    const int n_valid = n - 2 * w;
    const int64_t mblocks = (n_modes + 63) / 64;
    // (windows narrower than a sub-tile, 2w + 1 < kTile, take the tile form's direct sums)
    if constexpr (sizeof(T) == 4) if (n_valid > 0 && 2 * w + 1 >= kTile && 2 * w + kChunk <= kSpan && mblocks <= 0x7fffffff) {
        // split the chunks of a mode block over workgroups until there are ~2048 of them
        const int n_chunks = (n_valid + kChunk - 1) / kChunk;
        const int64_t want = std::max<int64_t>(1, std::min<int64_t>(n_chunks, (2048 + mblocks - 1) / mblocks));
        const int cpg = (int)((n_chunks + want - 1) / want);
        const int groups = (n_chunks + cpg - 1) / cpg;
        const dim3 g1((unsigned)((n_modes + 255) / 256));
        if (F) hipLaunchKernelGGL(regime_first_fill, g1, dim3(256), 0, s, F, n_modes);
        hipLaunchKernelGGL(regime_stream<T>, dim3((unsigned)mblocks, (unsigned)groups), dim3(64 * kWaves), 0, s, e, b, n_modes, n,
                           w, cpg, R, F);
        if (F) hipLaunchKernelGGL(regime_first_finish, g1, dim3(256), 0, s, F, n_modes);
        return hipGetLastError();
    }
    size_t lds = 0;
    const int to = n_valid > 0 ? tile_outputs<T>(w, n_valid, &lds) : 0;
    const int64_t tiles = to > 0 ? (n_valid + to - 1) / to : 0;
    if (to == 0 || tiles > 65535 || mblocks > 0x7fffffff) {
        hipLaunchKernelGGL(regime_map<T>, dim3((unsigned)((n_modes + 255) / 256)), dim3(256), 0, s, e, b, n_modes, n, w,
                           R, F);
        return hipGetLastError();
    }
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(&regime_tile<T>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    const dim3 g1((unsigned)((n_modes + 255) / 256));
    if (F) hipLaunchKernelGGL(regime_first_fill, g1, dim3(256), 0, s, F, n_modes);
    hipLaunchKernelGGL(regime_tile<T>, dim3((unsigned)mblocks, (unsigned)tiles), dim3(256), lds, s, e, b, n_modes, n, w, to,
                       R, F);
    if (F) hipLaunchKernelGGL(regime_first_finish, g1, dim3(256), 0, s, F, n_modes);
    return hipGetLastError();
}

qs_status rfail(qs_status s, const std::string &m) {
    qs::set_last_error(m);
    return s;
}

}  // namespace

extern "C" {

qs_status qs_regime_map(const void *ln_e, const void *ln_b, int64_t n_modes, int32_t n_xi, int32_t half_window,
                        int32_t precision, void *log_ratio, int32_t *first_e_cell, void *hip_stream) {
    if (n_modes < 1 || n_xi < 1 || half_window < 0) return rfail(QS_ERR_ARG, "n_modes >= 1, n_xi >= 1, half_window >= 0");
    if (precision != QS_FP32 && precision != QS_FP64) return rfail(QS_ERR_ARG, "precision must be QS_FP32 or QS_FP64");
    if (!ln_e || !ln_b) return rfail(QS_ERR_ARG, "ln_e and ln_b are required");
    if (!log_ratio && !first_e_cell) return rfail(QS_ERR_ARG, "at least one of log_ratio and first_e_cell is required");
    if ((n_modes + 255) / 256 > 0x7fffffff) return rfail(QS_ERR_ARG, "too many modes");
    const int w = (int)std::min<int64_t>(half_window, n_xi);   // a longer window leaves no valid cell either way
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const hipError_t e =
        precision == QS_FP32
            ? launch(static_cast<const float *>(ln_e), static_cast<const float *>(ln_b), n_modes, (int)n_xi, w,
                     static_cast<float *>(log_ratio), first_e_cell, s)
            : launch(static_cast<const double *>(ln_e), static_cast<const double *>(ln_b), n_modes, (int)n_xi, w,
                     static_cast<double *>(log_ratio), first_e_cell, s);
    return e == hipSuccess ? QS_OK : rfail(QS_ERR_HIP, std::string("regime map: ") + hipGetErrorString(e));
}

}  // extern "C"
