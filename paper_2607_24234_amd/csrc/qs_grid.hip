// Finite-width (transverse-grid) path for gfx950: the beam perturbations live on a periodic
// nx x ny grid in each xi cell (Sec. IV.B, the full transverse Laplacian of Eq.
// poisson_QSA), FP32 state with FP64 oscillator carries.
//
// One application of the model operator A to a state W = (rho, j_par, j_x, j_y) runs as
// four fully parallel passes instead of a sequential slice-by-slice chain:
//   march    : (d_xi^2 + 1) n_p = rho down every transverse column (65,536 independent
//              columns for 256^2), exact cell propagator, FP64 carries: n_p at centres,
//              d_xi n_p at the rear faces (and at centres for the fields);
//   rows     : per xi slice, FFT along x of z1 = n_p + i d_xi n_p and z2 = j_x + i j_y,
//              written transposed ([slice][kx][y]) through LDS so the next pass reads
//              contiguous columns;
//   columns  : per slice and column pair (kx, -kx): FFT along y, the spectral operators
//              (Helmholtz inverse 1/(1 + k^2), gradient, divergence) using the conjugate
//              partner at -k to split the two real fields packed in each complex transform,
//              inverse FFT along y, in place;
//   rows^-1  : inverse FFT along x and the pointwise rates
//                d_tau rho = d_xi j_par - div j_perp,  d_tau j_par = -gamma^-3 Omega d_xi Psi,
//                d_tau j_perp = gamma^-1 Omega grad Psi,
//              fused with the Runge-Kutta stage update (Horner form W_{m+1} = U + c_m A W_m).
// The fields for snapshots and per-step maxima take the same three transform passes on
// (rho - n_p) + i rho and d_xi n_p.  FFTs are radix-4 Stockham (Govindaraju et al., SC'08)
// in LDS with a twiddle table computed in FP64 on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kRows = 8;  // rows per workgroup of the row passes

struct GridArgs {
    int nx, ny, n_xi, log_nx, log_ny;
    int64_t P, T;          // points per slice, points in all
    double lx, ly, h, ih;
    double C1, S1, C2, S2;
    bool restoring;
    float om0;             // sum q^2 n_b / m
    float ginv, g3inv;
    const float *f;        // longitudinal profile [n_xi]
    const float *g;        // transverse profile [P]
    const float2 *twx, *twy;  // exp(-2 pi i m / n), m < n
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Stockham FFTs (Govindaraju et al., SC'08) of `cnt` transforms of length N = 2^LOGN stored
// back to back in b0, ping-ponging with b1, by all threads of the workgroup: one radix-2
// stage first when LOGN is odd, then radix-4 stages (4 points, 3 twiddles per butterfly,
// half the passes and barriers of radix 2).  Forward uses exp(-2 pi i k / N) from the
// table tw[N].  Returns 1 if the result is in b1, else 0.
template <int LOGN>
__device__ int fft_stockham(float2 *__restrict__ b0, float2 *__restrict__ b1, int cnt,
                            const float2 *__restrict__ tw, bool inverse) {
    constexpr int N = 1 << LOGN;
    float2 *in = b0, *out = b1;
    int res = 0;
    if (LOGN & 1) {
        constexpr int H = N / 2;
        for (int t = threadIdx.x; t < cnt * H; t += blockDim.x) {
            const int tr = t >> (LOGN - 1), j = t & (H - 1);
            const float2 x0 = in[tr * N + j], x1 = in[tr * N + j + H];
            out[tr * N + 2 * j] = cadd(x0, x1);
            out[tr * N + 2 * j + 1] = csub(x0, x1);
        }
        __syncthreads();
        float2 *tmp = in; in = out; out = tmp;
        res ^= 1;
    }
    if (LOGN >= 2) {
        constexpr int Q = N / 4;
#pragma unroll
        for (int s = (LOGN & 1); s < LOGN; s += 2) {
            const int Ns = 1 << s;
            for (int t = threadIdx.x; t < cnt * Q; t += blockDim.x) {
                const int tr = t >> (LOGN - 2), j = t & (Q - 1);
                const int k = j & (Ns - 1);
                const float2 *src = in + tr * N;
                float2 *dst = out + tr * N;
                float2 v0 = src[j], v1 = src[j + Q], v2 = src[j + 2 * Q], v3 = src[j + 3 * Q];
                if (k) {
                    const int ts = k * (N >> (s + 2));   // k N / (4 Ns)
                    float2 w1 = tw[ts], w2 = tw[2 * ts], w3 = tw[3 * ts];
                    if (inverse) { w1.y = -w1.y; w2.y = -w2.y; w3.y = -w3.y; }
                    v1 = cmul(v1, w1);
                    v2 = cmul(v2, w2);
                    v3 = cmul(v3, w3);
                }
                const float2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), d = csub(v1, v3);
                // forward: -i d; inverse: +i d
                const float2 a3 = inverse ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
                const int o = ((j - k) << 2) + k;
                dst[o] = cadd(a0, a2);
                dst[o + Ns] = cadd(a1, a3);
                dst[o + 2 * Ns] = csub(a0, a2);
                dst[o + 3 * Ns] = csub(a1, a3);
            }
            __syncthreads();
            float2 *tmp = in; in = out; out = tmp;
            res ^= 1;
        }
    }
    return res;
}

__device__ int block_fft(float2 *__restrict__ b0, float2 *__restrict__ b1, int n, int logn, int cnt,
                         const float2 *__restrict__ tw, bool inverse) {
    switch (logn) {
    case 1: return fft_stockham<1>(b0, b1, cnt, tw, inverse);
    case 2: return fft_stockham<2>(b0, b1, cnt, tw, inverse);
    case 3: return fft_stockham<3>(b0, b1, cnt, tw, inverse);
    case 4: return fft_stockham<4>(b0, b1, cnt, tw, inverse);
    case 5: return fft_stockham<5>(b0, b1, cnt, tw, inverse);
    case 6: return fft_stockham<6>(b0, b1, cnt, tw, inverse);
    case 7: return fft_stockham<7>(b0, b1, cnt, tw, inverse);
    default: return fft_stockham<8>(b0, b1, cnt, tw, inverse);
    }
}

// ----------------------------------------------------------------------------- march
// One thread per transverse point: FP64 carries down the column.  The 65,536 columns of a
// 256^2 grid are one wave per SIMD, so the loads run kMarchAhead cells ahead in a register
// ring (slot j % kMarchAhead; no copies at the loop edge) to keep enough bytes in flight.
constexpr int kMarchAhead = 16;

__global__ void __launch_bounds__(256) grid_march(GridArgs a, const float *__restrict__ rho, float *__restrict__ np_c,
                                                  float *__restrict__ v_f, float *__restrict__ v_c) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    double y = 0.0, v = 0.0;
    auto cell = [&](int j, float rf) {
        const double r = (double)rf;
        double nc, yn, vn, vc;
        if (a.restoring) {
            const double w = y - r;
            nc = r + a.C2 * w + a.S2 * v;
            vc = a.C2 * v - a.S2 * w;
            yn = r + a.C1 * w + a.S1 * v;
            vn = a.C1 * v - a.S1 * w;
        } else {
            nc = y + 0.5 * a.h * v + 0.125 * a.h * a.h * r;
            vc = v + 0.5 * a.h * r;
            yn = y + a.h * v + 0.5 * a.h * a.h * r;
            vn = v + a.h * r;
        }
        y = yn;
        v = vn;
        const int64_t o = (int64_t)j * a.P + p;
        np_c[o] = (float)nc;
        if (v_f) v_f[o] = (float)vn;   // the field pass needs only n_p and the centre derivative
        if (v_c) v_c[o] = (float)vc;
    };
    const int last = a.n_xi - 1;
    float ring[kMarchAhead];
#pragma unroll
    for (int d = 0; d < kMarchAhead; ++d) ring[d] = rho[(int64_t)min(d, last) * a.P + p];
    int jb = 0;
    for (; jb + kMarchAhead <= a.n_xi; jb += kMarchAhead) {
#pragma unroll
        for (int u = 0; u < kMarchAhead; ++u) {
            const float r = ring[u];
            ring[u] = rho[(int64_t)min(jb + u + kMarchAhead, last) * a.P + p];   // the end reloads the last cell
            cell(jb + u, r);
        }
    }
#pragma unroll
    for (int u = 0; u < kMarchAhead; ++u)
        if (jb + u < a.n_xi) cell(jb + u, ring[u]);
}

// ----------------------------------------------------------------------------- rows
// mode 0 (stage): z1 = np_c + i v_f, z2 = jx + i jy
// mode 1 (fields): z1 = (rho - np_c) + i rho, z2 = v_c
// Output Z1, Z2: [slice][kx][y] complex.
__global__ void __launch_bounds__(256) grid_rows_fwd(GridArgs a, int mode, const float *__restrict__ A0,
                                                     const float *__restrict__ A1, const float *__restrict__ B0,
                                                     const float *__restrict__ B1, float2 *__restrict__ Z1,
                                                     float2 *__restrict__ Z2) {
    extern __shared__ float2 sm[];
    const int nx = a.nx, ny = a.ny;
    const int R = min(kRows, ny);
    const int j = blockIdx.y;
    const int y0 = blockIdx.x * R;
    float2 *b0 = sm, *b1 = sm + 2 * R * nx;
    float2 *tw = sm + 4 * R * nx;
    for (int t = threadIdx.x; t < nx; t += blockDim.x) tw[t] = a.twx[t];
    const int64_t base = (int64_t)j * a.P + (int64_t)y0 * nx;
    for (int t = threadIdx.x; t < R * nx; t += blockDim.x) {
        const int64_t o = base + t;
        float2 z1, z2;
        if (mode == 0) {
            z1 = make_float2(A0[o], A1[o]);
            z2 = make_float2(B0[o], B1[o]);
        } else {
            const float r = A1[o];
            z1 = make_float2(r - A0[o], r);
            z2 = make_float2(B0[o], 0.f);
        }
        b0[t] = z1;
        b0[R * nx + t] = z2;
    }
    __syncthreads();
    const int res = block_fft(b0, b1, nx, a.log_nx, 2 * R, tw, false);
    const float2 *o = res ? b1 : b0;
    // transposed store: for each kx the R consecutive y values are contiguous
    for (int t = threadIdx.x; t < nx * R; t += blockDim.x) {
        const int kx = t / R, r = t % R;
        const int64_t d = ((int64_t)j * nx + kx) * ny + y0 + r;
        Z1[d] = o[r * nx + kx];
        Z2[d] = o[(R + r) * nx + kx];
    }
}

// ----------------------------------------------------------------------------- columns
__device__ __forceinline__ float wavenum(int i, int n, double l) {
    return (float)(6.283185307179586 * (double)(i <= n / 2 ? i : i - n) / l);
}
__device__ __forceinline__ float dwavenum(int i, int n, double l) { return i == n / 2 ? 0.f : wavenum(i, n, l); }

// One workgroup per (slice, column pair kx, nx - kx), in place over Z1, Z2.  mode 0:
// O1 = d_xi Psi + i div j, O2 = d_x Psi + i d_y Psi; mode 1: O1 = grad phi_E, O2 = grad
// phi_B (as x + i y components), phi_E = H(rho - n_p), phi_B = H rho (all still transformed
// along x).
__global__ void __launch_bounds__(256) grid_cols(GridArgs a, int mode, float2 *__restrict__ Z1,
                                                 float2 *__restrict__ Z2) {
    extern __shared__ float2 sm[];
    const int nx = a.nx, ny = a.ny;
    const int j = blockIdx.y;
    const int kxa = blockIdx.x;                 // 0 .. nx/2
    const int kxb = (nx - kxa) % nx;            // its conjugate partner column
    const int ncol = (kxb == kxa) ? 1 : 2;
    float2 *b0 = sm, *b1 = sm + 4 * ny;
    float2 *tw = sm + 8 * ny;
    for (int t = threadIdx.x; t < ny; t += blockDim.x) tw[t] = a.twy[t];
    // transforms: [col 0 Z1][col 0 Z2][col 1 Z1][col 1 Z2]
    for (int t = threadIdx.x; t < 2 * ncol * ny; t += blockDim.x) {
        const int tr = t / ny, y = t % ny;
        const int kx = (tr >> 1) ? kxb : kxa;
        const int64_t d = ((int64_t)j * nx + kx) * ny + y;
        b0[t] = (tr & 1) ? Z2[d] : Z1[d];
    }
    __syncthreads();
    int res = block_fft(b0, b1, ny, a.log_ny, 2 * ncol, tw, false);
    float2 *F = res ? b1 : b0;   // spectra
    float2 *G = res ? b0 : b1;   // outputs
    const float inv = 1.0f / ((float)nx * (float)ny);
    for (int t = threadIdx.x; t < ncol * ny; t += blockDim.x) {
        const int c = t / ny, ky = t % ny;
        const int kx = c ? kxb : kxa;
        const int cp = (ncol == 1) ? 0 : 1 - c;          // column holding -kx
        const int kyp = (ny - ky) % ny;
        const float2 z1 = F[(2 * c) * ny + ky], z1p = cconj(F[(2 * cp) * ny + kyp]);
        const float2 z2 = F[(2 * c + 1) * ny + ky], z2p = cconj(F[(2 * cp + 1) * ny + kyp]);
        const float kxv = wavenum(kx, nx, a.lx), kyv = wavenum(ky, ny, a.ly);
        const float kap = 1.0f / (1.0f + kxv * kxv + kyv * kyv);
        const float dx = dwavenum(kx, nx, a.lx), dy = dwavenum(ky, ny, a.ly);
        // the two real fields packed in z: F(re) = (z + conj z(-k))/2, F(im) = (z - conj z(-k))/(2i)
        const float2 re1 = make_float2(0.5f * (z1.x + z1p.x), 0.5f * (z1.y + z1p.y));
        const float2 im1 = make_float2(0.5f * (z1.y - z1p.y), -0.5f * (z1.x - z1p.x));
        float2 o1, o2;
        if (mode == 0) {
            const float2 jxh = make_float2(0.5f * (z2.x + z2p.x), 0.5f * (z2.y + z2p.y));
            const float2 jyh = make_float2(0.5f * (z2.y - z2p.y), -0.5f * (z2.x - z2p.x));
            // kappa F(v_f) + i (i dx Jx + i dy Jy) = kappa V - (dx Jx + dy Jy)
            o1 = make_float2(kap * im1.x - (dx * jxh.x + dy * jyh.x), kap * im1.y - (dx * jxh.y + dy * jyh.y));
            // (i dx - dy) kappa N
            const float2 nk = make_float2(kap * re1.x, kap * re1.y);
            o2 = make_float2(-dx * nk.y - dy * nk.x, dx * nk.x - dy * nk.y);
        } else {
            const float2 dk = make_float2(kap * re1.x, kap * re1.y);   // kappa F(rho - n_p)
            const float2 rk = make_float2(kap * im1.x, kap * im1.y);   // kappa F(rho)
            o1 = make_float2(-dx * dk.y - dy * dk.x, dx * dk.x - dy * dk.y);
            o2 = make_float2(-dx * rk.y - dy * rk.x, dx * rk.x - dy * rk.y);
        }
        G[(2 * c) * ny + ky] = make_float2(o1.x * inv, o1.y * inv);
        G[(2 * c + 1) * ny + ky] = make_float2(o2.x * inv, o2.y * inv);
    }
    __syncthreads();
    // inverse along y, in place over the inputs
    res = block_fft(G, F, ny, a.log_ny, 2 * ncol, tw, true);
    const float2 *R0 = res ? F : G;
    for (int t = threadIdx.x; t < 2 * ncol * ny; t += blockDim.x) {
        const int tr = t / ny, y = t % ny;
        const int kx = (tr >> 1) ? kxb : kxa;
        const int64_t d = ((int64_t)j * nx + kx) * ny + y;
        if (tr & 1) Z2[d] = R0[t];
        else Z1[d] = R0[t];
    }
}

// Fields: O3 = (y-transform, kappa / (nx ny), inverse y-transform) of one x-transformed column
// of v_c, before grid_cols reuses that buffer.
// mode-1 helper: O3 columns were kept in F slots; a separate small pass transforms them.
__global__ void __launch_bounds__(256) grid_cols_o3(GridArgs a, const float2 *__restrict__ Z2in, float2 *__restrict__ Z3) {
    extern __shared__ float2 sm[];
    const int nx = a.nx, ny = a.ny;
    const int j = blockIdx.y, kx = blockIdx.x;
    float2 *b0 = sm, *b1 = sm + ny, *tw = sm + 2 * ny;
    for (int t = threadIdx.x; t < ny; t += blockDim.x) tw[t] = a.twy[t];
    const int64_t base = ((int64_t)j * nx + kx) * ny;
    for (int t = threadIdx.x; t < ny; t += blockDim.x) b0[t] = Z2in[base + t];
    __syncthreads();
    int res = block_fft(b0, b1, ny, a.log_ny, 1, tw, false);
    float2 *F = res ? b1 : b0, *G = res ? b0 : b1;
    const float inv = 1.0f / ((float)nx * (float)ny);
    for (int ky = threadIdx.x; ky < ny; ky += blockDim.x) {
        const float kxv = wavenum(kx, nx, a.lx), kyv = wavenum(ky, ny, a.ly);
        const float kap = inv / (1.0f + kxv * kxv + kyv * kyv);
        G[ky] = make_float2(kap * F[ky].x, kap * F[ky].y);
    }
    __syncthreads();
    res = block_fft(G, F, ny, a.log_ny, 1, tw, true);
    const float2 *R0 = res ? F : G;
    for (int t = threadIdx.x; t < ny; t += blockDim.x) Z3[base + t] = R0[t];
}

// ----------------------------------------------------------------------------- rows^-1
__device__ __forceinline__ uint32_t fkey_pos(float x) { return __builtin_bit_cast(uint32_t, x); }

// The box maximum of a field pass is folded with atomicMax over non-negative float keys
// (they order as unsigned ints).  Hundreds of thousands of atomics on one address per pass
// queue up in one L2 channel and stall the traffic behind them, so each workgroup first
// reduces its own maximum and the workgroups spread over kKeySlots keys per step, kept
// key_stride entries apart; grid_max_finish folds the slots.
constexpr int kKeySlots = 32;

__device__ __forceinline__ float nan_max(float a, float b) { return (b > a || !(b <= b)) ? b : a; }

// workgroup maximum of amax (every thread of the block calls it), one atomic per block
__device__ __forceinline__ void block_max_to_key(float amax, uint32_t *key, int key_stride) {
    __shared__ float red[4];
    for (int off = 32; off >= 1; off >>= 1) amax = nan_max(amax, __shfl_xor(amax, off));
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wv] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; ++w) amax = nan_max(amax, red[w]);
        const int slot = (int)((blockIdx.x + blockIdx.y) & (kKeySlots - 1));
        atomicMax(key + (int64_t)slot * key_stride, fkey_pos(amax));
    }
}

// mode 0: rates and the stage update.  W_in: the stage input (its j_par for the face
// difference); U: the step's start state; W_out = U + c A W_in, or (final) U += dtau A W_in.
// mode 1: fields: snapshot ln|E|, ln|B| and the box maximum of |E|^2 + |B|^2.
struct RowInvArgs {
    int mode;
    const float2 *O1, *O2, *O3;
    const float *in_jpar;
    const float *U[4];
    float *out[4];
    float coef;
    int final_update;
    float *ln_e, *ln_b;        // snapshot (mode 1) or null
    uint32_t *max_key;         // the step's first key slot (mode 1) or null
    int key_stride;            // entries between two slots of one step
    uint32_t *err;             // non-finite flag (final update)
};

__global__ void __launch_bounds__(256) grid_rows_inv(GridArgs a, RowInvArgs r) {
    extern __shared__ float2 sm[];
    const int nx = a.nx, ny = a.ny;
    const int R = min(kRows, ny);
    const int j = blockIdx.y;
    const int y0 = blockIdx.x * R;
    const int ntr = r.mode == 1 ? 3 : 2;
    float2 *b0 = sm, *b1 = sm + ntr * R * nx, *tw = sm + 2 * ntr * R * nx;
    for (int t = threadIdx.x; t < nx; t += blockDim.x) tw[t] = a.twx[t];
    for (int t = threadIdx.x; t < nx * R; t += blockDim.x) {
        const int kx = t / R, rr = t % R;
        const int64_t d = ((int64_t)j * nx + kx) * ny + y0 + rr;
        b0[rr * nx + kx] = r.O1[d];
        b0[(R + rr) * nx + kx] = r.O2[d];
        if (ntr == 3) b0[(2 * R + rr) * nx + kx] = r.O3[d];
    }
    __syncthreads();
    const int res = block_fft(b0, b1, nx, a.log_nx, ntr * R, tw, true);
    const float2 *o = res ? b1 : b0;
    float amax = 0.f;
    const float fj = a.f[j];
    const float fn = j + 1 < a.n_xi ? a.f[j + 1] : 0.f;
    for (int t = threadIdx.x; t < R * nx; t += blockDim.x) {
        const int rr = t / nx, x = t % nx;
        const int64_t pt = (int64_t)(y0 + rr) * nx + x;
        const int64_t e = (int64_t)j * a.P + pt;
        const float2 v1 = o[rr * nx + x], v2 = o[(R + rr) * nx + x];
        if (r.mode == 0) {
            const float gp = a.g[pt];
            const float om_c = a.om0 * fj * gp;
            const float om_f = j + 1 < a.n_xi ? a.om0 * gp * 0.5f * (fj + fn) : 0.f;
            const float pin = r.in_jpar[e];
            const float pprev = j > 0 ? r.in_jpar[e - a.P] : 0.f;
            float rate[4];
            rate[0] = (pin - pprev) * (float)a.ih - v1.y;
            rate[1] = j + 1 < a.n_xi ? -a.g3inv * om_f * v1.x : 0.f;
            rate[2] = a.ginv * om_c * v2.x;
            rate[3] = a.ginv * om_c * v2.y;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float nv = r.U[q][e] + r.coef * rate[q];
                r.out[q][e] = nv;
                if (q == 0 && r.final_update && !(fabsf(nv) <= 3.0e38f)) r.err[0] = 1u;
            }
        } else {
            const float2 v3 = o[(2 * R + rr) * nx + x];
            const float e2 = v3.x * v3.x + v1.x * v1.x + v1.y * v1.y;
            const float b2 = v2.x * v2.x + v2.y * v2.y;
            if (r.ln_e) {
                r.ln_e[e] = 0.5f * logf(e2);
                r.ln_b[e] = 0.5f * logf(b2);
            }
            const float a2 = e2 + b2;
            amax = (a2 > amax || !(a2 <= a2)) ? a2 : amax;
        }
    }
    if (r.mode == 1 && r.max_key) block_max_to_key(amax, r.max_key, r.key_stride);
}

// ----------------------------------------------------------------------------- 256-point passes
// For 256 x 256 grids every transform runs in registers.  The 16 lanes of a group hold a
// transform as x[q + 16 r] in v[r] (lane q); the split 256 = 16 x 16 (four-step FFT) takes a
// 16-point FFT in registers, the twiddle W256^(q k), one exchange through LDS inside the
// wave, and a second 16-point FFT, after which lane q holds X[q + 16 r] in v[r] again.  The
// passes keep the data layouts of the general kernels above; the transposed loads and
// stores go through LDS in runs of 16 rows (128 B).

// cos(2 pi k / 16)
__host__ __device__ constexpr float cos16(int k) {
    constexpr float c[5] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f, 0.0f};
    k &= 15;
    return k <= 4 ? c[k] : k <= 8 ? -c[8 - k] : k <= 12 ? -c[k - 8] : c[16 - k];
}

// t W16^e, W16 = exp(-2 pi i / 16) (its conjugate for the inverse), 0 <= e < 8
template <bool INV> __device__ __forceinline__ float2 rot16(float2 t, int e) {
    if (e == 0) return t;
    if (e == 4) return INV ? make_float2(-t.y, t.x) : make_float2(t.y, -t.x);
    const float c = cos16(e), sn = INV ? cos16(e + 12) : -cos16(e + 12);
    return make_float2(t.x * c - t.y * sn, t.x * sn + t.y * c);
}

__host__ __device__ constexpr int brev4(int i) { return ((i & 1) << 3) | ((i & 2) << 1) | ((i & 4) >> 1) | ((i & 8) >> 3); }

// 16-point FFT in registers, natural order in and out (radix-2, decimation in time)
template <bool INV> __device__ __forceinline__ void fft16(float2 (&v)[16]) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int k = brev4(i);
        if (i < k) {
            const float2 t = v[i];
            v[i] = v[k];
            v[k] = t;
        }
    }
#pragma unroll
    for (int len = 2; len <= 16; len <<= 1)
#pragma unroll
        for (int i = 0; i < 16; i += len)
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const float2 t = rot16<INV>(v[i + k + len / 2], k * (16 / len));
                const float2 u = v[i + k];
                v[i + k] = cadd(u, t);
                v[i + k + len / 2] = csub(u, t);
            }
}

// LDS written by lanes of this wave is visible to its other lanes after this point
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 256-point FFT by a group of 16 lanes (lane q); ex: the group's 16 x 17 exchange area;
// tw: W256^m, m < 256
template <bool INV>
__device__ __forceinline__ void fft256(float2 (&v)[16], int q, float2 *ex, const float2 *tw) {
    fft16<INV>(v);                      // over r: Y[q][k] in v[k]
#pragma unroll
    for (int k = 1; k < 16; ++k) {
        float2 w = tw[q * k];
        if (INV) w.y = -w.y;
        v[k] = cmul(v[k], w);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) ex[k * 17 + q] = v[k];
    wave_sync();
#pragma unroll
    for (int n = 0; n < 16; ++n) v[n] = ex[q * 17 + n];   // column k = q: Y[n][q]
    wave_sync();
    fft16<INV>(v);                      // X[16 k1 + q] in v[k1]
}

// rows: as grid_rows_fwd for 256 x 256; 16 rows per workgroup, a 16-lane group per row
// holding both transforms
template <int MODE>
__global__ void __launch_bounds__(256) grid_rows_fwd256(GridArgs a, const float *__restrict__ A0,
                                                        const float *__restrict__ A1, const float *__restrict__ B0,
                                                        const float *__restrict__ B1, float2 *__restrict__ Z1,
                                                        float2 *__restrict__ Z2) {
    constexpr int R = 16, XP = R + 1;
    __shared__ float2 tw[256];
    __shared__ float2 sm[2 * 256 * XP];   // [transform][kx][row]; the exchange areas alias it
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, q = lane & 15, grp = lane >> 4;
    const int rr = 4 * wv + grp;
    const int j = blockIdx.y, y0 = blockIdx.x * R;
    tw[tid] = a.twx[tid];
    const int64_t rowb = (int64_t)j * a.P + (int64_t)(y0 + rr) * 256;
    float2 z1[16], z2[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t o = rowb + q + 16 * r;
        if (MODE == 0) {
            z1[r] = make_float2(A0[o], A1[o]);
            z2[r] = make_float2(B0[o], B1[o]);
        } else {
            const float rho = A1[o];
            z1[r] = make_float2(rho - A0[o], rho);
            z2[r] = make_float2(B0[o], 0.f);
        }
    }
    __syncthreads();
    float2 *ex = sm + (4 * wv + grp) * 272;
    fft256<false>(z1, q, ex, tw);
    fft256<false>(z2, q, ex, tw);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int kx = q + 16 * r;
        sm[kx * XP + rr] = z1[r];
        sm[(256 + kx) * XP + rr] = z2[r];
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 2 * R; ++it) {
        const int t = tid + 256 * it;
        const int f = t / (256 * R), kx = (t / R) & 255, r = t % R;
        const int64_t d = ((int64_t)j * 256 + kx) * a.ny + y0 + r;
        (f ? Z2 : Z1)[d] = sm[(f * 256 + kx) * XP + r];
    }
}

// columns: as grid_cols for 256 x 256; a workgroup takes 8 column pairs (kx, -kx) of a
// slice, pair 0 being the two self-conjugate columns 0 and 128; a 16-lane group per column
// holding both transforms; the partner column is in the same wave.  MODE 1 (fields) also
// writes Z3 = H v_c (the work of grid_cols_o3) from the Z2 spectrum it replaces.
template <int MODE>
__global__ void __launch_bounds__(256) grid_cols256(GridArgs a, float2 *__restrict__ Z1, float2 *__restrict__ Z2,
                                                    float2 *__restrict__ Z3) {
    __shared__ float2 tw[256];
    __shared__ float2 spec[16][2][256];   // the 16 columns' spectra; each group's exchange area aliases its own
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, q = lane & 15, grp = lane >> 4;
    const int slot = 4 * wv + grp;
    const int s = blockIdx.x * 8 + (slot >> 1);
    const int kx = s == 0 ? (slot & 1) * 128 : ((slot & 1) ? 256 - s : s);
    const int ps = s == 0 ? slot : (slot ^ 1);
    const int j = blockIdx.y;
    tw[tid] = a.twy[tid];
    const int64_t cb = ((int64_t)j * 256 + kx) * 256;
    float2 z1[16], z2[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        z1[r] = Z1[cb + q + 16 * r];
        z2[r] = Z2[cb + q + 16 * r];
    }
    __syncthreads();
    float2 *ex = &spec[slot][0][0];
    fft256<false>(z1, q, ex, tw);
    fft256<false>(z2, q, ex, tw);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        spec[slot][0][q + 16 * r] = z1[r];
        spec[slot][1][q + 16 * r] = z2[r];
    }
    wave_sync();
    const float inv = 1.0f / 65536.0f;
    const float kxv = wavenum(kx, 256, a.lx), dx = dwavenum(kx, 256, a.lx);
    float2 z3[MODE == 1 ? 16 : 1];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int ky = q + 16 * r, kyp = (256 - ky) & 255;
        const float2 z1p = cconj(spec[ps][0][kyp]), z2p = cconj(spec[ps][1][kyp]);
        const float kyv = wavenum(ky, 256, a.ly), dy = dwavenum(ky, 256, a.ly);
        const float kap = 1.0f / (1.0f + kxv * kxv + kyv * kyv);
        const float2 re1 = make_float2(0.5f * (z1[r].x + z1p.x), 0.5f * (z1[r].y + z1p.y));
        const float2 im1 = make_float2(0.5f * (z1[r].y - z1p.y), -0.5f * (z1[r].x - z1p.x));
        float2 o1, o2;
        if (MODE == 0) {
            const float2 jxh = make_float2(0.5f * (z2[r].x + z2p.x), 0.5f * (z2[r].y + z2p.y));
            const float2 jyh = make_float2(0.5f * (z2[r].y - z2p.y), -0.5f * (z2[r].x - z2p.x));
            o1 = make_float2(kap * im1.x - (dx * jxh.x + dy * jyh.x), kap * im1.y - (dx * jxh.y + dy * jyh.y));
            const float2 nk = make_float2(kap * re1.x, kap * re1.y);
            o2 = make_float2(-dx * nk.y - dy * nk.x, dx * nk.x - dy * nk.y);
        } else {
            const float2 dk = make_float2(kap * re1.x, kap * re1.y);
            const float2 rk = make_float2(kap * im1.x, kap * im1.y);
            o1 = make_float2(-dx * dk.y - dy * dk.x, dx * dk.x - dy * dk.y);
            o2 = make_float2(-dx * rk.y - dy * rk.x, dx * rk.x - dy * rk.y);
            if constexpr (MODE == 1) z3[r] = make_float2(kap * inv * z2[r].x, kap * inv * z2[r].y);
        }
        z1[r] = make_float2(o1.x * inv, o1.y * inv);
        z2[r] = make_float2(o2.x * inv, o2.y * inv);
    }
    wave_sync();   // the partner's spectrum is read before the exchange areas are reused
    fft256<true>(z1, q, ex, tw);
    fft256<true>(z2, q, ex, tw);
    if constexpr (MODE == 1) fft256<true>(z3, q, ex, tw);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        Z1[cb + q + 16 * r] = z1[r];
        Z2[cb + q + 16 * r] = z2[r];
        if constexpr (MODE == 1) Z3[cb + q + 16 * r] = z3[r];
    }
}

// inverse rows: as grid_rows_inv for 256 x 256 (NTR = 2: rates and stage update; 3: fields)
template <int NTR>
__global__ void __launch_bounds__(256) grid_rows_inv256(GridArgs a, RowInvArgs r) {
    constexpr int R = 16, XP = R + 1;
    __shared__ float2 tw[256];
    __shared__ float2 sm[2 * 256 * XP];   // [transform][kx][row], two at a time; the exchange areas alias it
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, q = lane & 15, grp = lane >> 4;
    const int rr = 4 * wv + grp;
    const int j = blockIdx.y, y0 = blockIdx.x * R;
    tw[tid] = a.twx[tid];
    float2 v[NTR][16];
#pragma unroll
    for (int f0 = 0; f0 < NTR; f0 += 2) {
        const int nf = NTR - f0 < 2 ? NTR - f0 : 2;
#pragma unroll
        for (int it = 0; it < nf * R; ++it) {   // all loads in flight before the LDS stores
            const int t = tid + 256 * it;
            const int f = t / (256 * R), kx = (t / R) & 255, rw = t % R;
            const int64_t d = ((int64_t)j * 256 + kx) * a.ny + y0 + rw;
            const int fi = f0 + f;
            sm[(f * 256 + kx) * XP + rw] = fi == 0 ? r.O1[d] : (fi == 1 ? r.O2[d] : r.O3[d]);
        }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < 2; ++f)
            if (f < nf)
#pragma unroll
                for (int i = 0; i < 16; ++i) v[f0 + f][i] = sm[(f * 256 + q + 16 * i) * XP + rr];
        __syncthreads();
    }
    float2 *ex = sm + (4 * wv + grp) * 272;
#pragma unroll
    for (int f = 0; f < NTR; ++f) fft256<true>(v[f], q, ex, tw);
    const int64_t rowp = (int64_t)(y0 + rr) * 256;
    float amax = 0.f;
    const float fj = a.f[j];
    const float fn = j + 1 < a.n_xi ? a.f[j + 1] : 0.f;
    if (NTR == 2) {
        // the update may write where it reads (the last stage updates U in place): each half
        // of the row's points loads all its inputs before any of its stores
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float u[4][8], pin[8], pprev[8], gp[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int64_t pt = rowp + q + 16 * (8 * h + i);
                const int64_t e = (int64_t)j * a.P + pt;
#pragma unroll
                for (int c = 0; c < 4; ++c) u[c][i] = r.U[c][e];
                pin[i] = r.in_jpar[e];
                pprev[i] = j > 0 ? r.in_jpar[e - a.P] : 0.f;
                gp[i] = a.g[pt];
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int64_t e = (int64_t)j * a.P + rowp + q + 16 * (8 * h + i);
                const float2 v1 = v[0][8 * h + i], v2 = v[1][8 * h + i];
                const float om_c = a.om0 * fj * gp[i];
                const float om_f = j + 1 < a.n_xi ? a.om0 * gp[i] * 0.5f * (fj + fn) : 0.f;
                float rate[4];
                rate[0] = (pin[i] - pprev[i]) * (float)a.ih - v1.y;
                rate[1] = j + 1 < a.n_xi ? -a.g3inv * om_f * v1.x : 0.f;
                rate[2] = a.ginv * om_c * v2.x;
                rate[3] = a.ginv * om_c * v2.y;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float nv = u[c][i] + r.coef * rate[c];
                    r.out[c][e] = nv;
                    if (c == 0 && r.final_update && !(fabsf(nv) <= 3.0e38f)) r.err[0] = 1u;
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t e = (int64_t)j * a.P + rowp + q + 16 * i;
            const float2 v1 = v[0][i], v2 = v[1][i], v3 = v[NTR - 1][i];
            const float e2 = v3.x * v3.x + v1.x * v1.x + v1.y * v1.y;
            const float b2 = v2.x * v2.x + v2.y * v2.y;
            if (r.ln_e) {
                r.ln_e[e] = 0.5f * logf(e2);
                r.ln_b[e] = 0.5f * logf(b2);
            }
            const float a2 = e2 + b2;
            amax = (a2 > amax || !(a2 <= a2)) ? a2 : amax;
        }
    }
    if (NTR == 3 && r.max_key) block_max_to_key(amax, r.max_key, r.key_stride);
}

// out[i] = ln sqrt of the largest key over the kKeySlots slots of step i
__global__ void grid_max_finish(const uint32_t *keys, int key_stride, float *out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t m = 0u;
    for (int sl = 0; sl < kKeySlots; ++sl) m = max(m, keys[(int64_t)sl * key_stride + i]);
    out[i] = 0.5f * logf(__builtin_bit_cast(float, m));
}

__global__ void __launch_bounds__(256) grid_zero_u32(uint32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__device__ inline uint64_t gsm64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// seeds: 0 noise amp (2u-1) f g, 1 uniform amp f g, 3 centroid offset x/sigma^2 f g + noise
__global__ void __launch_bounds__(256) grid_seed(GridArgs a, int kind, double amp, double offset, double sigma_r,
                                                 uint64_t seed, float *__restrict__ rho) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.T) return;
    const int j = (int)(i / a.P);
    const int64_t pt = i % a.P;
    const int ix = (int)(pt % a.nx);
    const double x = (double)(ix - a.nx / 2) * a.lx / a.nx;
    const double fg = (double)a.f[j] * (double)a.g[pt];
    const double u = (double)(gsm64(seed, (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
    double r = 0.0;
    if (kind == QS_SEED_NOISE) r = amp * (2.0 * u - 1.0) * fg;
    else if (kind == QS_SEED_UNIFORM) r = amp * fg;
    else if (kind == QS_SEED_CENTROID) r = (sigma_r > 0.0 ? offset * x / (sigma_r * sigma_r) : 0.0) * fg + amp * (2.0 * u - 1.0) * fg;
    rho[i] = (float)r;
}

}  // namespace

// ----------------------------------------------------------------------------- host
struct GridCtx {
    GridArgs a{};
    double dtau = 0.0;
    void *mem = nullptr;
    bool owns = false;
    float *U[4], *Wa[4], *Wb[4];
    float *np_c, *v_f, *v_c;
    float2 *Z1, *Z2, *Z3;
    float *f, *g;
    float2 *twx, *twy;
    uint32_t *err, *keys;
    int max_keys = 0;
};

namespace {

unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

size_t grid_bytes(int64_t T, int64_t P, int n_xi, int nx, int ny, size_t *offs) {
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += (b + 255) / 256 * 256; return r; };
    int k = 0;
    for (int i = 0; i < 12; ++i) offs[k++] = take((size_t)T * 4);        // U, Wa, Wb
    for (int i = 0; i < 3; ++i) offs[k++] = take((size_t)T * 4);         // np_c, v_f, v_c
    for (int i = 0; i < 3; ++i) offs[k++] = take((size_t)T * 8);         // Z1, Z2, Z3
    offs[k++] = take((size_t)n_xi * 4);                                  // f
    offs[k++] = take((size_t)P * 4);                                     // g
    offs[k++] = take((size_t)nx * 8);                                    // twx
    offs[k++] = take((size_t)ny * 8);                                    // twy
    offs[k++] = take(16);                                                // err
    offs[k++] = take((size_t)kKeySlots * 4096 * 4);                      // keys [slot][step] (per-step maxima)
    return o;
}

int ilog2(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }

size_t lds_rows(const GridArgs &a, int ntr) {
    const int R = std::min(kRows, a.ny);
    return (size_t)(2 * ntr * R * a.nx + a.nx) * sizeof(float2);
}
size_t lds_cols(const GridArgs &a) { return (size_t)(8 * a.ny + a.ny) * sizeof(float2); }

// 256 x 256 grids take the register-FFT passes
bool is256(const GridArgs &a) { return a.nx == 256 && a.ny == 256; }

// one application of A to W_in, combined with the stage update
hipError_t apply(GridCtx *c, float *const *Win, float *const *Wout, float coef, bool final_update, hipStream_t s) {
    const GridArgs &a = c->a;
    const int R = std::min(kRows, a.ny);
    const bool r256 = is256(a);
    hipLaunchKernelGGL(grid_march, dim3(nblk(a.P)), dim3(256), 0, s, a, Win[0], c->np_c, c->v_f, (float *)nullptr);
    if (r256) {
        hipLaunchKernelGGL(grid_rows_fwd256<0>, dim3(16, a.n_xi), dim3(256), 0, s, a, c->np_c, c->v_f, Win[2], Win[3],
                           c->Z1, c->Z2);
        hipLaunchKernelGGL(grid_cols256<0>, dim3(16, a.n_xi), dim3(256), 0, s, a, c->Z1, c->Z2, (float2 *)nullptr);
    } else {
        hipLaunchKernelGGL(grid_rows_fwd, dim3(a.ny / R, a.n_xi), dim3(256), lds_rows(a, 2), s, a, 0, c->np_c, c->v_f,
                           Win[2], Win[3], c->Z1, c->Z2);
        hipLaunchKernelGGL(grid_cols, dim3(a.nx / 2 + 1, a.n_xi), dim3(256), lds_cols(a), s, a, 0, c->Z1, c->Z2);
    }
    RowInvArgs r{};
    r.mode = 0;
    r.O1 = c->Z1;
    r.O2 = c->Z2;
    r.in_jpar = Win[1];
    for (int q = 0; q < 4; ++q) { r.U[q] = c->U[q]; r.out[q] = Wout[q]; }
    r.coef = coef;
    r.final_update = final_update ? 1 : 0;
    r.err = c->err;
    if (r256) hipLaunchKernelGGL(grid_rows_inv256<2>, dim3(16, a.n_xi), dim3(256), 0, s, a, r);
    else hipLaunchKernelGGL(grid_rows_inv, dim3(a.ny / R, a.n_xi), dim3(256), lds_rows(a, 2), s, a, r);
    return hipGetLastError();
}

// fields of the state U: snapshot (ln_e/ln_b may be null) and/or the maximum into key
hipError_t fields(GridCtx *c, float *ln_e, float *ln_b, uint32_t *key, hipStream_t s) {
    const GridArgs &a = c->a;
    const int R = std::min(kRows, a.ny);
    const bool r256 = is256(a);
    hipLaunchKernelGGL(grid_march, dim3(nblk(a.P)), dim3(256), 0, s, a, c->U[0], c->np_c, (float *)nullptr, c->v_c);
    if (r256)
        hipLaunchKernelGGL(grid_rows_fwd256<1>, dim3(16, a.n_xi), dim3(256), 0, s, a, c->np_c, c->U[0], c->v_c,
                           (const float *)nullptr, c->Z1, c->Z2);
    else
        hipLaunchKernelGGL(grid_rows_fwd, dim3(a.ny / R, a.n_xi), dim3(256), lds_rows(a, 2), s, a, 1, c->np_c, c->U[0],
                           c->v_c, (const float *)nullptr, c->Z1, c->Z2);
    // O3 = H v_c from the untouched Z2 spectrum column by column, before the column pass
    // overwrites Z2 (the 256-point column pass does both)
    if (r256) {
        hipLaunchKernelGGL(grid_cols256<1>, dim3(16, a.n_xi), dim3(256), 0, s, a, c->Z1, c->Z2, c->Z3);
    } else {
        hipLaunchKernelGGL(grid_cols_o3, dim3(a.nx, a.n_xi), dim3(256), (size_t)3 * a.ny * sizeof(float2), s, a,
                           c->Z2, c->Z3);
        hipLaunchKernelGGL(grid_cols, dim3(a.nx / 2 + 1, a.n_xi), dim3(256), lds_cols(a), s, a, 1, c->Z1, c->Z2);
    }
    RowInvArgs r{};
    r.mode = 1;
    r.O1 = c->Z1;
    r.O2 = c->Z2;
    r.O3 = c->Z3;
    r.ln_e = ln_e;
    r.ln_b = ln_b;
    r.max_key = key;
    r.key_stride = c->max_keys;
    if (r256) hipLaunchKernelGGL(grid_rows_inv256<3>, dim3(16, a.n_xi), dim3(256), 0, s, a, r);
    else hipLaunchKernelGGL(grid_rows_inv, dim3(a.ny / R, a.n_xi), dim3(256), lds_rows(a, 3), s, a, r);
    return hipGetLastError();
}

}  // namespace

hipError_t grid_allow_lds(const GridCtx *c) {
    const size_t rows = lds_rows(c->a, 3), cols = lds_cols(c->a);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&grid_rows_fwd),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)rows);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&grid_rows_inv), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)rows);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&grid_cols), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)cols);
    return e;
}

size_t grid_workspace_size(const qs_params &p) {
    size_t offs[32];
    const int64_t P = (int64_t)p.nx * p.ny;
    return grid_bytes(P * p.n_xi, P, p.n_xi, p.nx, p.ny, offs);
}

qs_status grid_create(const qs_params &p, void *workspace, size_t ws_bytes, hipStream_t s, GridCtx **out,
                      std::string *err) {
    GridCtx *c = new (std::nothrow) GridCtx;
    if (!c) { *err = "host allocation failed"; return QS_ERR_ALLOC; }
    GridArgs &a = c->a;
    a.nx = p.nx;
    a.ny = p.ny;
    a.n_xi = p.n_xi;
    a.log_nx = ilog2(p.nx);
    a.log_ny = ilog2(p.ny);
    a.P = (int64_t)p.nx * p.ny;
    a.T = a.P * p.n_xi;
    a.lx = p.lx;
    a.ly = p.ly;
    a.h = p.length / p.n_xi;
    a.ih = 1.0 / a.h;
    a.C1 = std::cos(a.h);
    a.S1 = std::sin(a.h);
    a.C2 = std::cos(0.5 * a.h);
    a.S2 = std::sin(0.5 * a.h);
    a.restoring = !(p.flags & QS_FLAG_NO_RESTORING);
    double om0 = 0.0;
    for (int sp = 0; sp < p.n_species; ++sp) om0 += p.q[sp] * p.q[sp] * p.nb_over_np[sp] / p.m[sp];
    a.om0 = (float)om0;
    a.ginv = (float)(1.0 / p.gamma_b);
    a.g3inv = (p.flags & QS_FLAG_DROP_LONGITUDINAL) ? 0.f : (float)(1.0 / (p.gamma_b * p.gamma_b * p.gamma_b));
    c->dtau = p.d_tau;
    size_t offs[32];
    const size_t bytes = grid_bytes(a.T, a.P, a.n_xi, a.nx, a.ny, offs);
    if (workspace) {
        if (ws_bytes < bytes) { delete c; *err = "workspace too small"; return QS_ERR_ALLOC; }
        c->mem = workspace;
    } else {
        if (hipMalloc(&c->mem, bytes) != hipSuccess) { delete c; *err = "hipMalloc of the grid buffers failed"; return QS_ERR_ALLOC; }
        c->owns = true;
    }
    char *b = static_cast<char *>(c->mem);
    int k = 0;
    for (int q = 0; q < 4; ++q) c->U[q] = (float *)(b + offs[k++]);
    for (int q = 0; q < 4; ++q) c->Wa[q] = (float *)(b + offs[k++]);
    for (int q = 0; q < 4; ++q) c->Wb[q] = (float *)(b + offs[k++]);
    c->np_c = (float *)(b + offs[k++]);
    c->v_f = (float *)(b + offs[k++]);
    c->v_c = (float *)(b + offs[k++]);
    c->Z1 = (float2 *)(b + offs[k++]);
    c->Z2 = (float2 *)(b + offs[k++]);
    c->Z3 = (float2 *)(b + offs[k++]);
    c->f = (float *)(b + offs[k++]);
    c->g = (float *)(b + offs[k++]);
    c->twx = (float2 *)(b + offs[k++]);
    c->twy = (float2 *)(b + offs[k++]);
    c->err = (uint32_t *)(b + offs[k++]);
    c->keys = (uint32_t *)(b + offs[k++]);
    c->max_keys = 4096;
    a.f = c->f;
    a.g = c->g;
    a.twx = c->twx;
    a.twy = c->twy;
    // tables
    std::vector<float> f(p.n_xi), g(a.P);
    for (int j = 0; j < p.n_xi; ++j) {
        const double xi = (j + 0.5) * a.h;
        if (p.profile == QS_PROFILE_FLATTOP) f[j] = 1.f;
        else if (p.profile == QS_PROFILE_GAUSSIAN) {
            const double z = (xi - p.xi_center) / p.sigma_xi;
            f[j] = (float)std::exp(-0.5 * z * z);
        } else f[j] = (float)p.profile_table[j];
    }
    for (int iy = 0; iy < p.ny; ++iy)
        for (int ix = 0; ix < p.nx; ++ix) {
            const double x = (ix - p.nx / 2) * p.lx / p.nx, y = (iy - p.ny / 2) * p.ly / p.ny;
            g[(size_t)iy * p.nx + ix] =
                p.sigma_r > 0.0 ? (float)std::exp(-(x * x + y * y) / (2.0 * p.sigma_r * p.sigma_r)) : 1.f;
        }
    auto table = [](int n) {
        std::vector<float2> t(n);
        for (int m = 0; m < n; ++m) t[m] = make_float2((float)std::cos(-2.0 * M_PI * m / n), (float)std::sin(-2.0 * M_PI * m / n));
        return t;
    };
    const std::vector<float2> tx = table(p.nx), ty = table(p.ny);
    hipError_t e = hipMemcpyAsync(c->f, f.data(), f.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->g, g.data(), g.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->twx, tx.data(), tx.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->twy, ty.data(), ty.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(c->err, 0, 16, s);
    for (int q = 0; q < 4 && e == hipSuccess; ++q) e = hipMemsetAsync(c->U[q], 0, (size_t)a.T * 4, s);
    if (e == hipSuccess) e = grid_allow_lds(c);
    if (e == hipSuccess && p.seed_kind != QS_SEED_NONE) {
        hipLaunchKernelGGL(grid_seed, dim3(nblk(a.T)), dim3(256), 0, s, a, p.seed_kind, p.seed_amp, p.centroid_offset,
                           p.sigma_r, p.rng_seed, c->U[0]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host tables die here
    if (e != hipSuccess) {
        if (c->owns) (void)hipFree(c->mem);
        delete c;
        *err = std::string("grid set-up: ") + hipGetErrorString(e);
        return QS_ERR_HIP;
    }
    *out = c;
    return QS_OK;
}

void grid_free(GridCtx *c, hipStream_t s) {
    if (!c) return;
    (void)hipStreamSynchronize(s);
    if (c->owns) (void)hipFree(c->mem);
    delete c;
}

qs_status grid_step(GridCtx *c, int32_t n_steps, int32_t out_every, void *ln_e, void *ln_b, void *max_ln_a,
                    hipStream_t s, std::string *err) {
    const GridArgs &a = c->a;
    const float dt = (float)c->dtau;
    const float cm[3] = {(float)(0.25 * c->dtau), (float)(c->dtau / 3.0), (float)(0.5 * c->dtau)};
    hipError_t e = hipSuccess;
    if (n_steps == 0) {
        e = fields(c, static_cast<float *>(ln_e), static_cast<float *>(ln_b), nullptr, s);
        if (e != hipSuccess) { *err = std::string("grid fields: ") + hipGetErrorString(e); return QS_ERR_HIP; }
        return QS_OK;
    }
    for (int s0 = 0; s0 < n_steps && e == hipSuccess; s0 += c->max_keys) {
        const int cnt = std::min(c->max_keys, n_steps - s0);
        if (max_ln_a)
            hipLaunchKernelGGL(grid_zero_u32, dim3(nblk(kKeySlots * c->max_keys)), dim3(256), 0, s, c->keys,
                               kKeySlots * c->max_keys);
        for (int i = 0; i < cnt && e == hipSuccess; ++i) {
            const int st = s0 + i;
            const bool snap = ln_e && (st % out_every == 0);
            if (snap || max_ln_a) {
                const int64_t so = snap ? (int64_t)(st / out_every) * a.T : 0;
                e = fields(c, snap ? static_cast<float *>(ln_e) + so : nullptr, snap ? static_cast<float *>(ln_b) + so : nullptr,
                           max_ln_a ? c->keys + i : nullptr, s);
            }
            // Horner-form RK4: W1 = U, W_{m+1} = U + c_m A W_m, U' = U + dtau A W4
            if (e == hipSuccess) e = apply(c, c->U, c->Wa, cm[0], false, s);
            if (e == hipSuccess) e = apply(c, c->Wa, c->Wb, cm[1], false, s);
            if (e == hipSuccess) e = apply(c, c->Wb, c->Wa, cm[2], false, s);
            if (e == hipSuccess) e = apply(c, c->Wa, c->U, dt, true, s);
        }
        if (e == hipSuccess && max_ln_a) {
            hipLaunchKernelGGL(grid_max_finish, dim3(nblk(cnt)), dim3(256), 0, s, c->keys, c->max_keys,
                               static_cast<float *>(max_ln_a) + s0, cnt);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) { *err = std::string("grid step: ") + hipGetErrorString(e); return QS_ERR_HIP; }
    return QS_OK;
}

qs_status grid_sync_check(GridCtx *c, hipStream_t s, std::string *err) {
    uint32_t flag = 0;
    if (hipStreamSynchronize(s) != hipSuccess || hipMemcpy(&flag, c->err, 4, hipMemcpyDeviceToHost) != hipSuccess) {
        *err = "grid: synchronize";
        return QS_ERR_HIP;
    }
    if (flag) {
        (void)hipMemset(c->err, 0, 4);
        *err = "non-finite state on the transverse grid";
        return QS_ERR_NUMERIC;
    }
    return QS_OK;
}

qs_status grid_get_state(GridCtx *c, double *rho, double *jpar, double *jx, double *jy, hipStream_t s, std::string *err) {
    double *dst[4] = {rho, jpar, jx, jy};
    std::vector<float> tmp(c->a.T);
    if (hipStreamSynchronize(s) != hipSuccess) { *err = "synchronize"; return QS_ERR_HIP; }
    for (int q = 0; q < 4; ++q) {
        if (!dst[q]) continue;
        if (hipMemcpy(tmp.data(), c->U[q], tmp.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) { *err = "copy state"; return QS_ERR_HIP; }
        for (int64_t i = 0; i < c->a.T; ++i) dst[q][i] = tmp[i];
    }
    return QS_OK;
}

qs_status grid_set_state(GridCtx *c, const double *rho, const double *jpar, const double *jx, const double *jy,
                         hipStream_t s, std::string *err) {
    const double *src[4] = {rho, jpar, jx, jy};
    std::vector<float> tmp(c->a.T);
    if (hipStreamSynchronize(s) != hipSuccess) { *err = "synchronize"; return QS_ERR_HIP; }
    for (int q = 0; q < 4; ++q) {
        for (int64_t i = 0; i < c->a.T; ++i) tmp[i] = (float)src[q][i];
        if (q == 1)  // no flux through the rear face of the beam
            for (int64_t i = (int64_t)(c->a.n_xi - 1) * c->a.P; i < c->a.T; ++i) tmp[i] = 0.f;
        if (hipMemcpy(c->U[q], tmp.data(), tmp.size() * 4, hipMemcpyHostToDevice) != hipSuccess) { *err = "copy state"; return QS_ERR_HIP; }
    }
    return QS_OK;
}

}  // namespace qs
