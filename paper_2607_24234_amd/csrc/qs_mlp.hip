// Growth-map surrogate network (include/qs_mlp.h): 5 -> 512 x4 -> 1 MLP with exact GELU,
// MSE loss and AdamW, for gfx950.
//
// The three 512 x 512 layers and their backward products are one kernel, gemm_nt:
// C[M][N] = A[M][K] B[N][K]^T with bfloat16 operands (both K-contiguous) on the matrix cores
// (v_mfma_f32_32x32x16_bf16, float32 accumulation), 128 x 128 tiles per workgroup of eight
// waves (two per SIMD), each wave 64 x 32 (2 x 1 MFMA tiles).  The workgroup stages its 128 rows of A and
// of B through LDS in chunks of 64 reduction indices (double buffered; eight threads read
// each row's 128 contiguous bytes) and the waves read their fragments there.  The three
// uses differ only in operands and epilogue:
//   forward      z = h W^T + b             A = h [rows][in],      B = W [out][in]
//   input grad   dh = dz W                 A = dz [rows][out],    B = W^T [in][out]
//   weight grad  dW = dz^T h (split over rows) A = dz^T [out][rows], B = h^T [in][rows]
// so the forward pass also stores h^T and the backward pass dz^T (bfloat16) for the weight
// gradients.  The first layer (5 inputs) and the last (1 output) are float32 VALU kernels.
// Reductions over rows (bias and first/last-layer weight gradients, the loss) write
// per-tile partial sums that a second kernel adds in a fixed order: the gradients are
// deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/qs_mlp.h"
#include "qs_internal.h"

namespace {

constexpr int D = 512;   // hidden width
constexpr int DIN = 5;   // inputs
constexpr int kWave = 64;

// flat parameter layout
constexpr int64_t OFF_W1 = 0;
constexpr int64_t OFF_B1 = OFF_W1 + (int64_t)D * DIN;
constexpr int64_t OFF_W2 = OFF_B1 + D;
constexpr int64_t OFF_B2 = OFF_W2 + (int64_t)D * D;
constexpr int64_t OFF_W3 = OFF_B2 + D;
constexpr int64_t OFF_B3 = OFF_W3 + (int64_t)D * D;
constexpr int64_t OFF_W4 = OFF_B3 + D;
constexpr int64_t OFF_B4 = OFF_W4 + (int64_t)D * D;
constexpr int64_t OFF_W5 = OFF_B4 + D;
constexpr int64_t OFF_B5 = OFF_W5 + D;
constexpr int64_t N_PARAMS = OFF_B5 + 1;
// W2..W4 and b2..b4 are evenly spaced
__host__ __device__ constexpr int64_t off_w(int l) { return OFF_W2 + (int64_t)l * (OFF_W3 - OFF_W2); }
__host__ __device__ constexpr int64_t off_b(int l) { return OFF_B2 + (int64_t)l * (OFF_W3 - OFF_W2); }
static_assert(off_w(2) == OFF_W4 && off_b(2) == OFF_B4, "layer spacing");

using bf16_t = uint16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));


// float32 -> bfloat16, round to nearest, ties to even (NaN kept quiet)
__device__ __forceinline__ bf16_t f2bf(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (bf16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// exact GELU x Phi(x) and its derivative Phi(x) + x phi(x)
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// ----------------------------------------------------------------------------- layer 1
// z1 = W1 x + b1 for a tile of 64 rows x 64 outputs per 256 threads: thread t owns output
// o0 + t%64 and 16 consecutive rows, so both h (row-major) and h^T rows are contiguous.
__global__ void __launch_bounds__(256) l1_fwd(const float *__restrict__ x, int64_t n_valid, const float *__restrict__ P,
                                              float *__restrict__ z, bf16_t *__restrict__ h, bf16_t *__restrict__ hT,
                                              int64_t ldT) {
    const int o = blockIdx.x * 64 + (threadIdx.x & 63);
    const int64_t r0 = (int64_t)blockIdx.y * 64 + 16 * (threadIdx.x >> 6);
    float w[DIN];
#pragma unroll
    for (int i = 0; i < DIN; ++i) w[i] = P[OFF_W1 + (int64_t)o * DIN + i];
    const float b = P[OFF_B1 + o];
    bf16_t col[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t m = r0 + r;
        float s = b;
        if (m < n_valid) {
#pragma unroll
            for (int i = 0; i < DIN; ++i) s += w[i] * x[m * DIN + i];
        }
        if (z) z[m * D + o] = s;
        const bf16_t hb = f2bf(gelu(s));
        h[m * D + o] = hb;
        col[r] = hb;
    }
    if (hT) {
        uint4 *dst = reinterpret_cast<uint4 *>(hT + (int64_t)o * ldT + r0);
        uint32_t p[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) p[q] = (uint32_t)col[2 * q] | ((uint32_t)col[2 * q + 1] << 16);
        dst[0] = make_uint4(p[0], p[1], p[2], p[3]);
        dst[1] = make_uint4(p[4], p[5], p[6], p[7]);
    }
}

// dW1[o][i] = sum_m dz1[m][o] x[m][i] and db1[o] = sum_m dz1[m][o]: partial sums per tile of
// 64 rows, part[tile][o][6]
__global__ void __launch_bounds__(256) l1_wgrad(const float *__restrict__ dz1, const float *__restrict__ x,
                                                float *__restrict__ part) {
    __shared__ float red[4][64][DIN + 1];
    const int ol = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + ol;
    const int64_t r0 = (int64_t)blockIdx.y * 64 + 16 * g;
    float acc[DIN + 1] = {};
    for (int r = 0; r < 16; ++r) {
        const int64_t m = r0 + r;
        const float d = dz1[m * D + o];
#pragma unroll
        for (int i = 0; i < DIN; ++i) acc[i] += d * x[m * DIN + i];
        acc[DIN] += d;
    }
#pragma unroll
    for (int i = 0; i <= DIN; ++i) red[g][ol][i] = acc[i];
    __syncthreads();
    if (g == 0) {
#pragma unroll
        for (int i = 0; i <= DIN; ++i)
            part[((int64_t)blockIdx.y * D + o) * (DIN + 1) + i] = ((red[0][ol][i] + red[1][ol][i]) + red[2][ol][i]) + red[3][ol][i];
    }
}

// ----------------------------------------------------------------------------- layer 5
// y[m] = W5 . h4[m] + b5: one wave per row (8 bfloat16 per lane); with targets also
// dy[m] = 2 (y - t)/batch and per-block partials of sum (y - t)^2 and sum dy.
__global__ void __launch_bounds__(256) l5_fwd(const bf16_t *__restrict__ h4, const float *__restrict__ P,
                                              int64_t n_valid, float *__restrict__ y, const float *__restrict__ t,
                                              float inv_batch2, float *__restrict__ dy, float *__restrict__ lossp) {
    __shared__ float sl[4], sd[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t m = (int64_t)blockIdx.x * 4 + wv;
    const uint4 v = *reinterpret_cast<const uint4 *>(h4 + m * D + 8 * lane);
    const uint32_t u[4] = {v.x, v.y, v.z, v.w};
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        s += bf2f((bf16_t)(u[q] & 0xFFFFu)) * P[OFF_W5 + 8 * lane + 2 * q];
        s += bf2f((bf16_t)(u[q] >> 16)) * P[OFF_W5 + 8 * lane + 2 * q + 1];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    s += P[OFF_B5];
    float e2 = 0.f, d = 0.f;
    if (lane == 0) {
        if (m < n_valid) y[m] = s;
        if (t) {
            const float e = s - t[m];
            d = e * inv_batch2;
            dy[m] = d;
            e2 = e * e;
        }
    }
    if (t) {
        if (lane == 0) { sl[wv] = e2; sd[wv] = d; }
        __syncthreads();
        if (threadIdx.x == 0) {
            lossp[2 * blockIdx.x] = ((sl[0] + sl[1]) + sl[2]) + sl[3];
            lossp[2 * blockIdx.x + 1] = ((sd[0] + sd[1]) + sd[2]) + sd[3];
        }
    }
}

// dz4 = (dy W5) * GELU'(z4), stored as bfloat16 (row-major and transposed); partials per
// 64-row tile of db4 = sum dz4 (colpart) and dW5 = sum dy h4 (w5part)
__global__ void __launch_bounds__(256) l5_bwd(const float *__restrict__ dy, const float *__restrict__ P,
                                              const float *__restrict__ z4, const bf16_t *__restrict__ h4,
                                              bf16_t *__restrict__ dzb, bf16_t *__restrict__ dzT, int64_t ldT,
                                              float *__restrict__ colpart, float *__restrict__ w5part) {
    __shared__ float red[2][4][64];
    const int ol = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + ol;
    const int64_t r0 = (int64_t)blockIdx.y * 64 + 16 * g;
    const float w = P[OFF_W5 + o];
    bf16_t col[16];
    float sb = 0.f, sw = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t m = r0 + r;
        const float dyv = dy[m];
        const float d = dyv * w * gelu_d(z4[m * D + o]);
        const bf16_t b = f2bf(d);
        dzb[m * D + o] = b;
        col[r] = b;
        sb += d;
        sw += dyv * bf2f(h4[m * D + o]);
    }
    uint4 *dst = reinterpret_cast<uint4 *>(dzT + (int64_t)o * ldT + r0);
    uint32_t p[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) p[q] = (uint32_t)col[2 * q] | ((uint32_t)col[2 * q + 1] << 16);
    dst[0] = make_uint4(p[0], p[1], p[2], p[3]);
    dst[1] = make_uint4(p[4], p[5], p[6], p[7]);
    red[0][g][ol] = sb;
    red[1][g][ol] = sw;
    __syncthreads();
    if (g == 0) {
        colpart[(int64_t)blockIdx.y * D + o] = ((red[0][0][ol] + red[0][1][ol]) + red[0][2][ol]) + red[0][3][ol];
        w5part[(int64_t)blockIdx.y * D + o] = ((red[1][0][ol] + red[1][1][ol]) + red[1][2][ol]) + red[1][3][ol];
    }
}

// ----------------------------------------------------------------------------- gemm_nt
enum Epi { EPI_FWD = 0, EPI_BWD = 1, EPI_PART = 2 };

struct GemmArgs {
    const bf16_t *A;
    int64_t lda;
    const bf16_t *B;
    int64_t ldb;
    int64_t k_len;        // reduction length per split (multiple of 64)
    int64_t M, N;         // C extent (multiples of 128)
    // EPI_FWD
    const float *bias;    // [N]
    float *z;             // [M][N] or null
    bf16_t *h;            // [M][N]
    bf16_t *hT;           // [N][ldT] or null
    int64_t ldT;
    // EPI_BWD
    const float *zprev;   // [M][N]
    float *dzf;           // [M][N] float32 or null
    bf16_t *dzb;          // [M][N] or null
    bf16_t *dzT;          // [N][ldT] or null
    float *colpart;       // [M/64][N] or null
    // EPI_PART
    float *part;          // [split][M][N]
};

__device__ __forceinline__ bf16x8 frag(const bf16_t *p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

constexpr int KC = 64;         // reduction chunk staged through LDS
constexpr int SLD = KC + 8;    // LDS row pitch of a staged chunk (bfloat16 elements)
constexpr int NJ = 1;          // 32-column MFMA tiles per wave

template <int EPI>
__global__ void __launch_bounds__(512) gemm_nt(GemmArgs g) {
    // the workgroup's 128 rows of A and of B for one chunk of 64 reduction indices, double
    // buffered; the 8-element pad puts the rows a fragment read touches on distinct banks
    __shared__ __attribute__((aligned(16))) bf16_t sa[2][128 * SLD];
    __shared__ __attribute__((aligned(16))) bf16_t sb[2][128 * SLD];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 2, wn = wv & 3;
    const int64_t m0 = (int64_t)blockIdx.y * 128 + 64 * wm;
    const int64_t n0 = (int64_t)blockIdx.x * 128 + 32 * NJ * wn;
    const int64_t kb = (int64_t)blockIdx.z * g.k_len;
    // staging: thread t moves 16 bytes of rows t/8 + 64 i (i < 2) at chunk columns 8 (t%8),
    // so eight threads read one row's 128 contiguous bytes
    const int sr = tid >> 3, sc = 8 * (tid & 7);
    const bf16_t *ga = g.A + ((int64_t)blockIdx.y * 128 + sr) * g.lda + kb + sc;
    const bf16_t *gb = g.B + ((int64_t)blockIdx.x * 128 + sr) * g.ldb + kb + sc;
    u32x4 stA[2], stB[2];
    auto fetch = [&](int64_t k) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            stA[i] = *reinterpret_cast<const u32x4 *>(ga + 64 * i * g.lda + k);
            stB[i] = *reinterpret_cast<const u32x4 *>(gb + 64 * i * g.ldb + k);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            *reinterpret_cast<u32x4 *>(&sa[buf][(sr + 64 * i) * SLD + sc]) = stA[i];
            *reinterpret_cast<u32x4 *>(&sb[buf][(sr + 64 * i) * SLD + sc]) = stB[i];
        }
    };
    // fragments: lane reads 8 reduction indices 16 s + 8 (lane/32) .. of row lane%32 (+ 32)
    const int lr = lane & 31, lk = 8 * (lane >> 5);
    f32x16 acc[2][NJ];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    const int chunks = (int)(g.k_len / KC);
    fetch(0);
    put(0);
    __syncthreads();
    for (int c = 0; c < chunks; ++c) {
        const int cur = c & 1;
        if (c + 1 < chunks) fetch((int64_t)(c + 1) * KC);   // in flight during this chunk's products
        const bf16_t *pa = &sa[cur][(64 * wm + lr) * SLD + lk];
        const bf16_t *pb = &sb[cur][(32 * NJ * wn + lr) * SLD + lk];
#pragma unroll
        for (int s = 0; s < KC / 16; ++s) {
            const bf16x8 a0 = frag(pa + 16 * s), a1 = frag(pa + 32 * SLD + 16 * s);
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const bf16x8 b = frag(pb + 32 * j * SLD + 16 * s);
                acc[0][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b, acc[0][j], 0, 0, 0);
                acc[1][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b, acc[1][j], 0, 0, 0);
            }
        }
        if (c + 1 < chunks) put(cur ^ 1);   // that buffer's last readers passed the previous barrier
        __syncthreads();
    }

    // result element r of lane: row 8(r/4) + 4(lane/32) + r%4, column lane%32 of each tile
    const int rb = 4 * (lane >> 5);
    float csum[NJ] = {};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int64_t n = n0 + 32 * j + lr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t mq = m0 + 32 * i + 8 * q + rb;  // four consecutive rows mq..mq+3
                bf16_t t4[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t m = mq + e;
                    const float v = acc[i][j][4 * q + e];
                    if (EPI == EPI_FWD) {
                        const float zz = v + g.bias[n];
                        if (g.z) g.z[m * g.N + n] = zz;
                        const bf16_t hb = f2bf(gelu(zz));
                        g.h[m * g.N + n] = hb;
                        t4[e] = hb;
                    } else if (EPI == EPI_BWD) {
                        const float d = v * gelu_d(g.zprev[m * g.N + n]);
                        if (g.dzf) g.dzf[m * g.N + n] = d;
                        const bf16_t db = f2bf(d);
                        if (g.dzb) g.dzb[m * g.N + n] = db;
                        t4[e] = db;
                        csum[j] += d;
                    } else {
                        g.part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = v;
                        t4[e] = 0;
                    }
                }
                bf16_t *tr = EPI == EPI_FWD ? g.hT : (EPI == EPI_BWD ? g.dzT : nullptr);
                if (tr) {
                    const uint2 pk = make_uint2((uint32_t)t4[0] | ((uint32_t)t4[1] << 16),
                                                (uint32_t)t4[2] | ((uint32_t)t4[3] << 16));
                    *reinterpret_cast<uint2 *>(tr + n * g.ldT + mq) = pk;
                }
            }
        }
    if (EPI == EPI_BWD && g.colpart) {
        // this wave's 64 rows: lanes l and l + 32 hold the two halves of each column
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const float s = csum[j] + __shfl_xor(csum[j], 32);
            if (lane < 32) g.colpart[((m0 >> 6)) * g.N + n0 + 32 * j + lr] = s;
        }
    }
}

// Reductions of per-tile partials.  Every sum runs in a fixed order (gradients are
// deterministic), with all of a thread's loads issued before its adds.

// out[i] = sum_{s < S} part[s * stride + i * step], S <= 16: one thread per output, the S terms
// added in order
__global__ void __launch_bounds__(256) reduce_parts(const float *__restrict__ part, int S, int64_t stride,
                                                    int64_t count, int64_t step, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = k < S ? part[(int64_t)k * stride + i * step] : 0.f;
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (k < S) s += v[k];
    out[i] = s;
}

// sum over 64 lanes, each lane's value in a fixed butterfly order; lane 0's result is used
__device__ __forceinline__ float wave_sum(float s) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    return s;
}

// out[o] = sum_{s < S} part[s * stride + o * step] for many partials: one wave per output,
// lane l adding s = l, l + 64, ... in order, then the wave's fixed butterfly
__global__ void __launch_bounds__(256) reduce_parts_wide(const float *__restrict__ part, int S, int64_t stride,
                                                         int64_t count, int64_t step, float *__restrict__ out) {
    const int64_t o = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (o >= count) return;   // whole waves
    float s = 0.f;
    for (int k = lane; k < S; k += 64) s += part[(int64_t)k * stride + o * step];
    s = wave_sum(s);
    if (lane == 0) out[o] = s;
}

// first-layer partials [tiles][o][6] -> dW1 [o][5], db1 [o]: one wave per (o, c)
__global__ void __launch_bounds__(256) reduce_l1(const float *__restrict__ part, int tiles, float *__restrict__ G) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= D * (DIN + 1)) return;   // whole waves
    const int o = i / (DIN + 1), c = i % (DIN + 1);
    float s = 0.f;
    for (int k = lane; k < tiles; k += 64) s += part[((int64_t)k * D + o) * (DIN + 1) + c];
    s = wave_sum(s);
    if (lane == 0) {
        if (c < DIN) G[OFF_W1 + (int64_t)o * DIN + c] = s;
        else G[OFF_B1 + o] = s;
    }
}

// sum over blocks of the (loss, dy) partial pairs -> db5 (device); the loss is read by the host.
// One workgroup: thread t adds blocks t, t + 256, ... in order, then a fixed tree over the
// four waves.
__global__ void __launch_bounds__(256) reduce_db5(const float *__restrict__ lossp, int blocks, float *__restrict__ G,
                                                  float *__restrict__ loss_out) {
    __shared__ float red[2][4];
    float sl = 0.f, sd = 0.f;
    for (int b = threadIdx.x; b < blocks; b += 256) {
        sl += lossp[2 * b];
        sd += lossp[2 * b + 1];
    }
    sl = wave_sum(sl);
    sd = wave_sum(sd);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = sl;
        red[1][wv] = sd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        G[OFF_B5] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        loss_out[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    }
}

// ----------------------------------------------------------------------------- optimizer
__global__ void __launch_bounds__(256) adamw(float *__restrict__ w, const float *__restrict__ gr, float *__restrict__ m,
                                             float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                                             float wd, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    w[i] = w[i] - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * w[i]);
}

// bfloat16 copies of W2..W4 ([out][in]) and their transposes ([in][out])
__global__ void __launch_bounds__(256) convert_weights(const float *__restrict__ P, bf16_t *__restrict__ Wb,
                                                       bf16_t *__restrict__ WTb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * (int64_t)D * D) return;
    const int l = (int)(i / ((int64_t)D * D));
    const int64_t e = i % ((int64_t)D * D);
    const int o = (int)(e / D), in = (int)(e % D);
    const bf16_t b = f2bf(P[off_w(l) + e]);
    Wb[(int64_t)l * D * D + e] = b;
    WTb[(int64_t)l * D * D + (int64_t)in * D + o] = b;
}


// bfloat16 W2..W4 in matrix-core A-fragment order, [3][16][32][64][8]: block (fb, ks) holds
// W[32 fb + lane%32][16 ks + 8 (lane/32) + i] for lane < 64, i < 8, one contiguous KiB
__global__ void __launch_bounds__(256) pack_weights(const float *__restrict__ P, bf16_t *__restrict__ Wp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * (int64_t)D * D) return;
    const int l = (int)(i / ((int64_t)D * D));
    const int64_t e = i % ((int64_t)D * D);
    const int o = (int)(e / D), in = (int)(e % D);
    const int fb = o / 32, ks = in / 16, lane = o % 32 + 32 * ((in % 16) / 8);
    Wp[((((int64_t)l * 16 + fb) * 32 + ks) * 64 + lane) * 8 + in % 8] = f2bf(P[off_w(l) + e]);
}

// ----------------------------------------------------------------------------- fused inference
// One persistent kernel runs the whole network on tiles of 64 queries; only x and y touch
// memory outside the workgroup.  A tile's activations stay in LDS as bfloat16
// [64 queries][512 features] with a row pitch of 520 elements (the 32 rows of a fragment
// read then fall on distinct banks).  Wave w of a group of four computes output features
// 128 w .. 128 w + 127 of each layer for all 64 queries as the transposed product
// z^T = W h^T: the weights are the A operand, read from L2 in fragment order (Wp), the
// activations the B operand, read from LDS.  The first layer is a float32 matrix-core
// product with the bias as a sixth input of value 1; the last layer is a float32 dot
// product per query, summed over the four waves in a fixed order.  GELU takes Phi from a
// table of cubic Hermite pieces (phi_table below).
//
// A workgroup holds two such groups, each with a tile of its own, on one compute unit.  A
// tile's work is a chain of seven items separated by workgroup barriers: the first layer
// and its GELU; the products of each 512 x 512 layer, each but the last followed by its
// GELU into the tile; the last GELU with the dot product.  Group 1 runs one item behind
// group 0, so between two barriers one group's waves issue matrix products while the
// other's (on the same SIMDs) do GELU work.  What bounds the kernel is then the weight
// stream of the product items: each tile reads all 1.5 MB of W2..W4 from L2, about 64 bytes
// per clock per compute unit at the matrix-core rate, which is the order of what L2 delivers.
constexpr int FT = 64;              // queries per tile
constexpr int ALD = D + 8;          // LDS row pitch of the activation tile (bfloat16 elements)
constexpr int KS = D / 16;          // k-steps of a 512-long product
constexpr int PHI_N = 192;          // cubic pieces of Phi on [-6, 6], 16 per unit of x

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

struct InferArgs {
    const float *x;       // [n][5], n <= kInferChunk
    int32_t n;
    const float *P;       // float32 parameters
    const bf16x8 *Wp;     // packed W2..W4
    const f32x4 *phi;     // [PHI_N] (c0, c1, c2, c3) per piece
    float *y;             // [n]
};
constexpr int32_t kInferChunk = 1 << 25;   // queries per launch (byte offsets stay 32-bit)

// raw buffer access: a 128-bit descriptor (base, size in bytes), a per-lane VGPR offset and a
// wave-uniform SGPR offset; where the per-lane offset (which the range check covers) is past
// the size, loads return 0 and stores are dropped
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}

// x Phi(x): t = 16 x + 96 clamped to [0, 192 - 1/64], piece floor(t), position f = t - floor(t),
// Phi = c0 + f (c1 + f (c2 + f c3)).  Beyond [-6, 6] Phi is taken at the end of the range
// (|Phi - 0| or |Phi - 1| < 1e-9 there); a NaN input clamps to piece 0 and propagates
// through the final product.
__device__ __forceinline__ float gelu_tab(float v, const f32x4 *tab) {
    const float t = fminf(fmaxf(fmaf(v, 16.f, 0.5f * PHI_N), 0.f), PHI_N - 0.015625f);
    const float f = __builtin_amdgcn_fractf(t);
    const f32x4 c = tab[(int)t];
    return v * fmaf(f, fmaf(f, fmaf(f, c.w, c.z), c.y), c.x);
}

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    const f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ float bf_lo(uint32_t p) { return __builtin_bit_cast(float, p << 16); }
__device__ __forceinline__ float bf_hi(uint32_t p) { return __builtin_bit_cast(float, p & 0xFFFF0000u); }

__global__ void __launch_bounds__(512, 1) mlp_infer(InferArgs a) {
    __shared__ __attribute__((aligned(16))) bf16_t act[2][FT * ALD];
    __shared__ f32x4 tab[PHI_N];
    __shared__ f32x4 bw[D];              // b2, b3, b4, W5: four rows of 512 floats
    __shared__ float red[2][4][FT];
    __shared__ float w1s[D * (DIN + 1)];     // [feature][W1 row, b1]
    __shared__ float xs[2][FT * DIN];        // each group's inputs of its coming tile
    const int tid = threadIdx.x, lane = tid & 63, lr = lane & 31, lh = lane >> 5;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int grp = wid >> 2, w = wid & 3, gt = tid & 255;
    for (int i = tid; i < PHI_N; i += 512) tab[i] = a.phi[i];
    for (int i = tid; i < D * (DIN + 1); i += 512) {
        const int f = i / (DIN + 1), c = i % (DIN + 1);
        w1s[i] = c < DIN ? a.P[OFF_W1 + (int64_t)f * DIN + c] : a.P[OFF_B1 + f];
    }
    for (int i = tid; i < D; i += 512) {
        const int r = i / (D / 4), e = i % (D / 4);
        const float *src = r < 3 ? a.P + off_b(r) : a.P + OFF_W5;
        bw[i] = *reinterpret_cast<const f32x4 *>(src + 4 * e);
    }
    const rsrc_t rx = make_rsrc(a.x, (uint32_t)a.n * DIN * 4);
    const rsrc_t ry = make_rsrc(a.y, (uint32_t)a.n * 4);
    const rsrc_t rw = make_rsrc(a.Wp, 3u * D * D * 2);
    const int tiles = (a.n + FT - 1) / FT;
    // group g of workgroup b takes tiles 2 b + g + 2 G k, k = 0, 1, ... (G workgroups); group 0
    // never has fewer than group 1
    const int stride = 2 * gridDim.x, t0 = 2 * blockIdx.x + grp;
    const int mine = t0 < tiles ? (tiles - 1 - t0) / stride + 1 : 0;
    const int most = 2 * blockIdx.x < tiles ? (tiles - 1 - 2 * (int)blockIdx.x) / stride + 1 : 0;
    bf16_t *const at = act[grp];
    // element e of tile t's inputs ([64][5] float32; the group's thread gt takes e = gt and,
    // below 320, e = gt + 256).  The whole byte offset is in the per-lane operand, which the
    // descriptor's range check covers: queries past n read 0.
    auto load_x = [&](int t, int e) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, (t * FT * DIN + e) * 4, 0, 0));
    };
    constexpr int XE = FT * DIN - 256;   // threads with a second input element
    // bias (or W5) row r for the four consecutive features of accumulator group (fb, j)
    auto brow = [&](int r, int fb, int j) { return bw[r * (D / 4) + (32 * (4 * w + fb) + 8 * j + 4 * lh) / 4]; };
    // GELU of acc as bfloat16 into the activation tile: element 4 j + e of acc[fb][qb] is
    // feature 32 (4 w + fb) + 8 j + 4 (lane/32) + e of query 32 qb + lane%32
    auto store = [&](f32x16 (&acc)[4][2]) {
        bf16_t *row = at + lr * ALD + 128 * w + 4 * lh;
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
#pragma unroll
            for (int fb = 0; fb < 4; ++fb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float h[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) h[e] = gelu_tab(acc[fb][qb][4 * j + e], tab);
                    const uint2 pk = make_uint2(pack_bf16(h[0], h[1]), pack_bf16(h[2], h[3]));
                    *reinterpret_cast<uint2 *>(row + 32 * qb * ALD + 32 * fb + 8 * j) = pk;
                    __builtin_amdgcn_sched_barrier(0);   // bounds the table reads in flight
                }
    };
    // products of hidden layer l + 2 (l = 0, 1, 2) for this wave's 128 features of the tile
    auto layer = [&](int l, f32x16 (&acc)[4][2]) {
        // weight fragment (fb, ks) of this wave: 1 KiB block ((l 16 + 4 w + fb) KS + ks)
        const int wbase = (l * 16 + 4 * w) * KS * 1024;
        auto wload = [&](int fb, int ks) {
            return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rw, lane * 16, wbase + (fb * KS + ks) * 1024, 0));
        };
        auto aload = [&](int qb, int ks) {
            return *reinterpret_cast<const bf16x8 *>(at + (32 * qb + lr) * ALD + 16 * ks + 8 * lh);
        };
        // weight fragments in a ring of four k-steps (slot ks % 4), each loaded two k-steps
        // ahead, activation fragments one k-step ahead (slot ks % 2); the group barriers
        // keep that order.  The first k-step starts the sums from the bias.
        bf16x8 A[4][4], B[2][2];
        auto step = [&](int ks, auto slot, auto first) {
            constexpr int u = decltype(slot)::value;
            const int kn = min(ks + 2, KS - 1), kb = min(ks + 1, KS - 1);   // the end reloads the last step
#pragma unroll
            for (int fb = 0; fb < 4; ++fb) A[(u + 2) % 4][fb] = wload(fb, kn);
#pragma unroll
            for (int qb = 0; qb < 2; ++qb) B[(u + 1) % 2][qb] = aload(qb, kb);
#pragma unroll
            for (int fb = 0; fb < 4; ++fb) {
                if constexpr (decltype(first)::value) {
                    f32x16 bias;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const f32x4 b = brow(l, fb, j);
#pragma unroll
                        for (int e = 0; e < 4; ++e) bias[4 * j + e] = b[e];
                    }
#pragma unroll
                    for (int qb = 0; qb < 2; ++qb)
                        acc[fb][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[u][fb], B[u % 2][qb], bias, 0, 0, 0);
                } else {
#pragma unroll
                    for (int qb = 0; qb < 2; ++qb)
                        acc[fb][qb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[u][fb], B[u % 2][qb], acc[fb][qb], 0, 0, 0);
                }
            }
            if constexpr (!decltype(first)::value) {
                __builtin_amdgcn_sched_group_barrier(0x020, 4, 0);   // 4 global (buffer) reads
                __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // 2 LDS reads
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);   // 8 matrix products
            }
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        using T = std::true_type;
        using F = std::false_type;
#pragma unroll
        for (int fb = 0; fb < 4; ++fb) {
            A[0][fb] = wload(fb, 0);
            A[1][fb] = wload(fb, 1);
        }
        B[0][0] = aload(0, 0);
        B[0][1] = aload(1, 0);
        step(0, I0{}, T{});
#pragma nounroll
        for (int kk = 1; kk < KS - 3; kk += 4) {   // k-steps 1 .. 28
            step(kk, I1{}, F{});
            step(kk + 1, I2{}, F{});
            step(kk + 2, I3{}, F{});
            step(kk + 3, I0{}, F{});
        }
        step(KS - 3, I1{}, F{});
        step(KS - 2, I2{}, F{});
        step(KS - 1, I3{}, F{});
    };
    if (mine > 0) {
        xs[grp][gt] = load_x(t0, gt);
        if (gt < XE) xs[grp][gt + 256] = load_x(t0, gt + 256);
    }
    // output of the group's tile t: the four waves' partial sums in a fixed order, plus b5
    auto put_y = [&](int t) {
        if (gt < FT) {
            const float v = (((red[grp][0][gt] + red[grp][1][gt]) + red[grp][2][gt]) + red[grp][3][gt]) + a.P[OFF_B5];
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), ry, (t * FT + gt) * 4, 0, 0);
        }
    };
    f32x16 acc[4][2];
    __syncthreads();
    // Every item below ends at a workgroup barrier.  Group 1 passes one barrier first, so it
    // runs one item behind group 0; both pass 7 most + 1 barriers.
    if (grp == 1) __syncthreads();
    for (int k = 0; k < most; ++k) {
        const bool live = k < mine;
        const int t = t0 + k * stride;
        if (k >= 1 && k - 1 < mine) put_y(t - stride);   // the previous tile's partial sums are in
        if (live) {
            // first layer (32 x 32 x 2 float32 products, k = inputs 0..4 and the bias): lane
            // holds W1[32 (4 w + fb) + lane%32][2 s + lane/32] (the sixth column is b1) and
            // input 2 s + lane/32 of query 32 qb + lane%32 (the sixth input is 1)
            float w1[4][3], xb[2][3];
#pragma unroll
            for (int s3 = 0; s3 < 3; ++s3) {
#pragma unroll
                for (int fb = 0; fb < 4; ++fb) w1[fb][s3] = w1s[(32 * (4 * w + fb) + lr) * (DIN + 1) + 2 * s3 + lh];
#pragma unroll
                for (int qb = 0; qb < 2; ++qb)
                    xb[qb][s3] = (s3 < 2 || lh == 0) ? xs[grp][(32 * qb + lr) * DIN + 2 * s3 + lh] : 1.f;
            }
#pragma unroll
            for (int fb = 0; fb < 4; ++fb)
#pragma unroll
                for (int qb = 0; qb < 2; ++qb) {
                    f32x16 z = {};
#pragma unroll
                    for (int s3 = 0; s3 < 3; ++s3) z = __builtin_amdgcn_mfma_f32_32x32x2f32(w1[fb][s3], xb[qb][s3], z, 0, 0, 0);
                    acc[fb][qb] = z;
                }
            store(acc);
        }
        __syncthreads();
        for (int l = 0; l < 3; ++l) {
            if (live) layer(l, acc);
            __syncthreads();
            if (live && l < 2) {
                store(acc);
            } else if (live) {
                // last layer: this wave's part of y = W5 . bf16(GELU(z4)); meanwhile the next
                // tile's inputs come into the group's input buffer
                const int tn = t + stride;
                const bool more = tn < tiles;
                const float xv0 = more ? load_x(tn, gt) : 0.f;
                const float xv1 = more && gt < XE ? load_x(tn, gt + 256) : 0.f;
#pragma unroll
                for (int qb = 0; qb < 2; ++qb) {
                    float sum = 0.f;
#pragma unroll
                    for (int fb = 0; fb < 4; ++fb)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const f32x4 w5 = brow(3, fb, j);
                            const uint32_t p0 = pack_bf16(gelu_tab(acc[fb][qb][4 * j], tab), gelu_tab(acc[fb][qb][4 * j + 1], tab));
                            const uint32_t p1 = pack_bf16(gelu_tab(acc[fb][qb][4 * j + 2], tab), gelu_tab(acc[fb][qb][4 * j + 3], tab));
                            sum += w5[0] * bf_lo(p0) + w5[1] * bf_hi(p0) + w5[2] * bf_lo(p1) + w5[3] * bf_hi(p1);
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    sum += __shfl_xor(sum, 32);
                    if (lh == 0) red[grp][w][32 * qb + lr] = sum;
                }
                if (more) {
                    xs[grp][gt] = xv0;
                    if (gt < XE) xs[grp][gt + 256] = xv1;
                }
            }
            __syncthreads();
        }
    }
    if (grp == 0) __syncthreads();
    if (most >= 1 && most - 1 < mine) put_y(t0 + (most - 1) * stride);
}

}  // namespace

// ----------------------------------------------------------------------------- host
struct qs_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t max_batch = 0;
    int64_t t = 0;          // AdamW steps taken
    void *mem = nullptr;    // one allocation for everything below
    float *P, *G, *Mo, *Vo;
    bf16_t *Wb, *WTb;       // [3][D][D]
    bf16_t *Wp;             // [3][D][D] in fragment order (inference)
    bool wp_stale = true;   // Wp lags P: repacked by the next forward call
    float *phi;             // [PHI_N][4] GELU table
    int cus = 0;            // compute units of the device
    float *z[4];            // [B][D]
    bf16_t *h[4];           // [B][D]
    bf16_t *hT[3];          // [D][B]
    bf16_t *dzb[2], *dzT[2];
    float *dz1, *y, *dy;
    float *part;            // split-K partials [16][D][D]
    float *colpart;         // [B/64][D]
    float *w5part;          // [B/64][D]
    float *l1part;          // [B/64][D][6]
    float *lossp;           // [B/4][2]
    float *loss;            // [1]
};

namespace {

qs_status mfail(qs_status st, const std::string &m) {
    qs::set_last_error(m);
    return st;
}
#define MLP_HIP(call, what)                                                                  \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return mfail(QS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t mlp_bytes(int64_t B, std::vector<size_t> *offs) {
    std::vector<size_t> sz = {
        (size_t)N_PARAMS * 4, (size_t)N_PARAMS * 4, (size_t)N_PARAMS * 4, (size_t)N_PARAMS * 4,
        (size_t)3 * D * D * 2, (size_t)3 * D * D * 2, (size_t)3 * D * D * 2, (size_t)PHI_N * 16};
    for (int i = 0; i < 4; ++i) sz.push_back((size_t)B * D * 4);   // z
    for (int i = 0; i < 4; ++i) sz.push_back((size_t)B * D * 2);   // h
    for (int i = 0; i < 3; ++i) sz.push_back((size_t)B * D * 2);   // hT
    for (int i = 0; i < 4; ++i) sz.push_back((size_t)B * D * 2);   // dzb[2], dzT[2]
    sz.push_back((size_t)B * D * 4);                                 // dz1
    sz.push_back((size_t)B * 4);                                     // y
    sz.push_back((size_t)B * 4);                                     // dy
    sz.push_back((size_t)16 * D * D * 4);                            // part
    sz.push_back((size_t)(B / 64) * D * 4);                          // colpart
    sz.push_back((size_t)(B / 64) * D * 4);                          // w5part
    sz.push_back((size_t)(B / 64) * D * (DIN + 1) * 4);              // l1part
    sz.push_back((size_t)(B / 4) * 2 * 4);                           // lossp
    sz.push_back(256);                                               // loss
    size_t o = 0;
    offs->clear();
    for (size_t s : sz) {
        offs->push_back(o);
        o += (s + 255) / 256 * 256;
    }
    return o;
}

// The kernel argument is passed by value: a plain 8-byte-aligned record of pointers and
// extents, far below the kernel-argument limit.
static_assert(sizeof(GemmArgs) == 144 && alignof(GemmArgs) == 8, "GemmArgs layout");
static_assert(std::is_trivially_copyable<GemmArgs>::value, "GemmArgs is copied as bytes");
// static LDS of gemm_nt: two double-buffered 128-row chunks of A and of B
static_assert(2 * 2 * 128 * SLD * sizeof(bf16_t) <= 160 * 1024, "gemm_nt LDS fits a compute unit");

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// What gemm_nt assumes of its launch: whole 128 x 128 output tiles, whole 64-long reduction
// chunks, 16-byte aligned rows of A and B (each thread moves 16 bytes) that hold every split's
// reduction range, a grid inside the device limits, and the outputs its epilogue writes.
// Returns "" when they hold, else what does not.
std::string gemm_check(int epi, const GemmArgs &a, int splits) {
    if (a.M <= 0 || a.N <= 0 || a.M % 128 || a.N % 128) return "output extent not whole 128 x 128 tiles";
    if (a.M / 128 > 65535 || a.N / 128 > 2147483647LL) return "grid beyond the device limits";
    if (splits < 1 || splits > 1024) return "split count out of range";
    if (a.k_len <= 0 || a.k_len % KC) return "reduction length not whole 64-long chunks";
    if (!a.A || !a.B || !aligned16(a.A) || !aligned16(a.B)) return "A or B missing or not 16-byte aligned";
    if (a.lda % 8 || a.ldb % 8) return "row pitch of A or B not a multiple of 16 bytes";
    if (a.lda < a.k_len * splits || a.ldb < a.k_len * splits) return "rows of A or B shorter than the reduction";
    if (epi == EPI_FWD && (!a.bias || !a.h || (a.hT && a.ldT < a.M))) return "forward epilogue outputs";
    if (epi == EPI_BWD && (!a.zprev || (!a.dzf && !a.dzb) || (a.dzT && a.ldT < a.M)))
        return "backward epilogue inputs or outputs";
    if (epi == EPI_PART && !a.part) return "partial-sum output";
    return "";
}

// the network's buffers inside its one allocation at `b`, at the offsets of mlp_bytes
void assign_buffers(qs_mlp *c, char *b, const std::vector<size_t> &o) {
    int k = 0;
    c->P = (float *)(b + o[k++]); c->G = (float *)(b + o[k++]); c->Mo = (float *)(b + o[k++]); c->Vo = (float *)(b + o[k++]);
    c->Wb = (bf16_t *)(b + o[k++]); c->WTb = (bf16_t *)(b + o[k++]);
    c->Wp = (bf16_t *)(b + o[k++]); c->phi = (float *)(b + o[k++]);
    for (int i = 0; i < 4; ++i) c->z[i] = (float *)(b + o[k++]);
    for (int i = 0; i < 4; ++i) c->h[i] = (bf16_t *)(b + o[k++]);
    for (int i = 0; i < 3; ++i) c->hT[i] = (bf16_t *)(b + o[k++]);
    c->dzb[0] = (bf16_t *)(b + o[k++]); c->dzb[1] = (bf16_t *)(b + o[k++]);
    c->dzT[0] = (bf16_t *)(b + o[k++]); c->dzT[1] = (bf16_t *)(b + o[k++]);
    c->dz1 = (float *)(b + o[k++]); c->y = (float *)(b + o[k++]); c->dy = (float *)(b + o[k++]);
    c->part = (float *)(b + o[k++]); c->colpart = (float *)(b + o[k++]); c->w5part = (float *)(b + o[k++]);
    c->l1part = (float *)(b + o[k++]); c->lossp = (float *)(b + o[k++]); c->loss = (float *)(b + o[k++]);
}

// The GEMMs of a training step on B rows: the forward product of hidden layer l (0..2), and
// for the backward pass of layer l the weight gradient (split over row ranges) and the input
// gradient, reading and writing the ping-pong buffers `cur` / `cur ^ 1`.
GemmArgs fwd_args(const qs_mlp *c, int l, int64_t rows) {
    GemmArgs a{};
    a.A = c->h[l]; a.lda = D;
    a.B = c->Wb + (int64_t)l * D * D; a.ldb = D;
    a.k_len = D; a.M = rows; a.N = D;
    a.bias = c->P + off_b(l);
    a.z = c->z[l + 1];
    a.h = c->h[l + 1];
    a.hT = l < 2 ? c->hT[l + 1] : nullptr;
    a.ldT = c->max_batch;
    return a;
}
// row splits of the weight gradients: at most 16, >= 512 rows each, dividing B/64 (each
// split's rows are whole reduction chunks)
int wgrad_splits(int64_t B) {
    int splits = (int)std::max<int64_t>(1, std::min<int64_t>(16, B / 512));
    while ((B / 64) % splits != 0) --splits;
    return splits;
}
GemmArgs wgrad_args(const qs_mlp *c, int l, int cur, int64_t B, int splits) {
    GemmArgs w{};
    w.A = c->dzT[cur]; w.lda = c->max_batch;
    w.B = c->hT[l]; w.ldb = c->max_batch;
    w.k_len = B / splits; w.M = D; w.N = D;
    w.part = c->part;
    return w;
}
GemmArgs dgrad_args(const qs_mlp *c, int l, int cur, int64_t B) {
    GemmArgs d{};
    d.A = c->dzb[cur]; d.lda = D;
    d.B = c->WTb + (int64_t)l * D * D; d.ldb = D;
    d.k_len = D; d.M = B; d.N = D;
    d.zprev = c->z[l];
    d.ldT = c->max_batch;
    if (l > 0) {
        d.dzb = c->dzb[cur ^ 1];
        d.dzT = c->dzT[cur ^ 1];
        d.colpart = c->colpart;
    } else {
        d.dzf = c->dz1;
    }
    return d;
}

hipError_t gemm_launch(int epi, const GemmArgs &a, int splits, hipStream_t s) {
    const std::string why = gemm_check(epi, a, splits);
    if (!why.empty()) {
        qs::set_last_error("gemm_nt launch: " + why);
        return hipErrorInvalidValue;
    }
    dim3 grid((unsigned)(a.N / 128), (unsigned)(a.M / 128), (unsigned)splits), block(512);
    if (epi == EPI_FWD) hipLaunchKernelGGL(gemm_nt<EPI_FWD>, grid, block, 0, s, a);
    else if (epi == EPI_BWD) hipLaunchKernelGGL(gemm_nt<EPI_BWD>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(gemm_nt<EPI_PART>, grid, block, 0, s, a);
    return hipGetLastError();
}

// training forward pass over a batch of `rows` (multiple of 128) rows: stores z, h and the
// transposes h^T for the weight gradients, the outputs y, dy and the loss partials
hipError_t forward_train(qs_mlp *c, const float *x, int64_t rows, const float *t, float inv_batch2) {
    hipStream_t s = c->stream;
    const int64_t ldT = c->max_batch;
    hipLaunchKernelGGL(l1_fwd, dim3(D / 64, (unsigned)(rows / 64)), dim3(256), 0, s, x, rows, c->P, c->z[0], c->h[0],
                       c->hT[0], ldT);
    for (int l = 0; l < 3; ++l) {
        const hipError_t e = gemm_launch(EPI_FWD, fwd_args(c, l, rows), 1, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(l5_fwd, dim3((unsigned)(rows / 4)), dim3(256), 0, s, c->h[3], c->P, rows, c->y, t, inv_batch2,
                       c->dy, c->lossp);
    return hipGetLastError();
}

// bfloat16 copies of W2..W4 for training (row-major and transposed); the packed inference
// copy follows at the next forward call (training steps do not read it)
void convert(qs_mlp *c) {
    const dim3 grid((unsigned)((3 * D * D + 255) / 256)), block(256);
    hipLaunchKernelGGL(convert_weights, grid, block, 0, c->stream, c->P, c->Wb, c->WTb);
    c->wp_stale = true;
}

// Cubic Hermite pieces of Phi (standard normal distribution function) on [-6, 6], 16 per
// unit: on piece i, x = -6 + (i + f)/16 with f in [0, 1],
//   Phi = c0 + c1 f + c2 f^2 + c3 f^3, matching Phi and its derivative phi at both ends.
// Interpolation error h^4/384 max|Phi''''| < 3e-8 for h = 1/16, plus float32 rounding.
std::vector<float> phi_table() {
    std::vector<float> t(4 * PHI_N);
    const double h = 1.0 / 16.0;
    auto Phi = [](double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); };
    auto phi = [](double x) { return std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI); };
    for (int i = 0; i < PHI_N; ++i) {
        const double x0 = -6.0 + i * h, x1 = x0 + h;
        const double p0 = Phi(x0), p1 = Phi(x1), d0 = h * phi(x0), d1 = h * phi(x1);
        t[4 * i + 0] = (float)p0;
        t[4 * i + 1] = (float)d0;
        t[4 * i + 2] = (float)(3.0 * (p1 - p0) - 2.0 * d0 - d1);
        t[4 * i + 3] = (float)(2.0 * (p0 - p1) + d0 + d1);
    }
    return t;
}

}  // namespace

namespace qs {
hipStream_t mlp_stream(const qs_mlp *net) { return net->stream; }
int mlp_device(const qs_mlp *net) { return net->device; }
}  // namespace qs

extern "C" {

int64_t qs_mlp_param_count(void) { return N_PARAMS; }

qs_status qs_mlp_create(int32_t max_batch, void *hip_stream, qs_mlp **out) {
    if (!out) return mfail(QS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (max_batch < 128 || max_batch % 128 != 0 || max_batch > (1 << 20))
        return mfail(QS_ERR_ARG, "max_batch must be a positive multiple of 128, at most 2^20");
    qs_mlp *c = new (std::nothrow) qs_mlp;
    if (!c) return mfail(QS_ERR_ALLOC, "host allocation failed");
    c->max_batch = max_batch;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return mfail(QS_ERR_HIP, "hipGetDevice failed"); }
    std::vector<size_t> o;
    const size_t bytes = mlp_bytes(max_batch, &o);
    if (hipMalloc(&c->mem, bytes) != hipSuccess) { delete c; return mfail(QS_ERR_ALLOC, "hipMalloc of the network buffers failed"); }
    assign_buffers(c, static_cast<char *>(c->mem), o);
    hipError_t e = hipMemsetAsync(c->mem, 0, bytes, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) {
        const std::vector<float> tab = phi_table();
        e = hipMemcpy(c->phi, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e != hipSuccess) { (void)hipFree(c->mem); delete c; return mfail(QS_ERR_HIP, "initializing the network buffers failed"); }
    *out = c;
    return QS_OK;
}

qs_status qs_mlp_set_params(qs_mlp *c, const float *host) {
    if (!c || !host) return mfail(QS_ERR_ARG, "net and params are required");
    MLP_HIP(hipSetDevice(c->device), "hipSetDevice");
    MLP_HIP(hipMemcpyAsync(c->P, host, N_PARAMS * 4, hipMemcpyHostToDevice, c->stream), "copy params");
    MLP_HIP(hipMemsetAsync(c->Mo, 0, N_PARAMS * 4, c->stream), "clear moments");
    MLP_HIP(hipMemsetAsync(c->Vo, 0, N_PARAMS * 4, c->stream), "clear moments");
    convert(c);
    MLP_HIP(hipGetLastError(), "convert weights");
    MLP_HIP(hipStreamSynchronize(c->stream), "synchronize");
    c->t = 0;
    return QS_OK;
}

qs_status qs_mlp_get_params(qs_mlp *c, float *host) {
    if (!c || !host) return mfail(QS_ERR_ARG, "net and params are required");
    MLP_HIP(hipSetDevice(c->device), "hipSetDevice");
    MLP_HIP(hipMemcpyAsync(host, c->P, N_PARAMS * 4, hipMemcpyDeviceToHost, c->stream), "copy params");
    MLP_HIP(hipStreamSynchronize(c->stream), "synchronize");
    return QS_OK;
}

qs_status qs_mlp_get_grads(qs_mlp *c, float *host) {
    if (!c || !host) return mfail(QS_ERR_ARG, "net and grads are required");
    MLP_HIP(hipSetDevice(c->device), "hipSetDevice");
    MLP_HIP(hipMemcpyAsync(host, c->G, N_PARAMS * 4, hipMemcpyDeviceToHost, c->stream), "copy grads");
    MLP_HIP(hipStreamSynchronize(c->stream), "synchronize");
    return QS_OK;
}

qs_status qs_mlp_set_grads(qs_mlp *c, const float *host) {
    if (!c || !host) return mfail(QS_ERR_ARG, "net and grads are required");
    MLP_HIP(hipSetDevice(c->device), "hipSetDevice");
    MLP_HIP(hipMemcpyAsync(c->G, host, N_PARAMS * 4, hipMemcpyHostToDevice, c->stream), "copy grads");
    MLP_HIP(hipStreamSynchronize(c->stream), "synchronize");
    return QS_OK;
}

qs_status qs_mlp_forward(qs_mlp *c, const float *x, int64_t n, float *y) {
    if (!c) return mfail(QS_ERR_ARG, "net is NULL");
    if (n < 0) return mfail(QS_ERR_ARG, "n must be >= 0");
    if (n > 0 && (!x || !y)) return mfail(QS_ERR_ARG, "x and y are required");
    MLP_HIP(hipSetDevice(c->device), "hipSetDevice");
    if (n == 0) return QS_OK;
    if (c->wp_stale) {
        hipLaunchKernelGGL(pack_weights, dim3((unsigned)((3 * D * D + 255) / 256)), dim3(256), 0, c->stream, c->P, c->Wp);
        MLP_HIP(hipGetLastError(), "pack weights");
        c->wp_stale = false;
    }
    for (int64_t r0 = 0; r0 < n; r0 += kInferChunk) {
        const int32_t m = (int32_t)std::min<int64_t>(kInferChunk, n - r0);
        const int64_t tiles = (m + FT - 1) / FT;
        const unsigned grid = (unsigned)std::min<int64_t>((tiles + 1) / 2, std::max(c->cus, 1));
        InferArgs a{x + r0 * DIN, m, c->P, reinterpret_cast<const bf16x8 *>(c->Wp),
                    reinterpret_cast<const f32x4 *>(c->phi), y + r0};
        hipLaunchKernelGGL(mlp_infer, dim3(grid), dim3(512), 0, c->stream, a);
    }
    MLP_HIP(hipGetLastError(), "forward kernel");
    return QS_OK;
}

qs_status qs_mlp_grads(qs_mlp *c, const float *x, const float *t, int32_t batch, double *loss) {
    if (!c || !x || !t) return mfail(QS_ERR_ARG, "net, x and t are required");
    if (batch < 128 || batch % 128 != 0 || batch > c->max_batch)
        return mfail(QS_ERR_ARG, "batch must be a positive multiple of 128 and <= max_batch");
    MLP_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = c->stream;
    const int64_t B = batch, ldT = c->max_batch, tiles = B / 64;
    MLP_HIP(forward_train(c, x, B, t, 2.0f / (float)B), "forward kernels");
    // last layer
    hipLaunchKernelGGL(l5_bwd, dim3(D / 64, (unsigned)tiles), dim3(256), 0, s, c->dy, c->P, c->z[3], c->h[3],
                       c->dzb[0], c->dzT[0], ldT, c->colpart, c->w5part);
    hipLaunchKernelGGL(reduce_parts_wide, dim3(D / 4), dim3(256), 0, s, c->colpart, (int)tiles, (int64_t)D, (int64_t)D,
                       (int64_t)1, c->G + OFF_B4);
    hipLaunchKernelGGL(reduce_parts_wide, dim3(D / 4), dim3(256), 0, s, c->w5part, (int)tiles, (int64_t)D, (int64_t)D,
                       (int64_t)1, c->G + OFF_W5);
    hipLaunchKernelGGL(reduce_db5, dim3(1), dim3(256), 0, s, c->lossp, (int)(B / 4), c->G, c->loss);
    // layers 4, 3, 2: weight gradient (split over rows), then the input gradient
    const int splits = wgrad_splits(B);
    int cur = 0;
    for (int l = 2; l >= 0; --l) {
        MLP_HIP(gemm_launch(EPI_PART, wgrad_args(c, l, cur, B, splits), splits, s), "weight-gradient GEMM");
        hipLaunchKernelGGL(reduce_parts, dim3(D * D / 256), dim3(256), 0, s, c->part, splits, (int64_t)D * D,
                           (int64_t)D * D, (int64_t)1, c->G + off_w(l));
        MLP_HIP(gemm_launch(EPI_BWD, dgrad_args(c, l, cur, B), 1, s), "input-gradient GEMM");
        if (l > 0)
            hipLaunchKernelGGL(reduce_parts_wide, dim3(D / 4), dim3(256), 0, s, c->colpart, (int)tiles, (int64_t)D,
                               (int64_t)D, (int64_t)1, c->G + off_b(l - 1));
        cur ^= 1;
    }
    // first layer
    hipLaunchKernelGGL(l1_wgrad, dim3(D / 64, (unsigned)tiles), dim3(256), 0, s, c->dz1, x, c->l1part);
    hipLaunchKernelGGL(reduce_l1, dim3((D * (DIN + 1) + 3) / 4), dim3(256), 0, s, c->l1part, (int)tiles, c->G);
    MLP_HIP(hipGetLastError(), "gradient kernels");
    if (loss) {
        float l = 0.f;
        MLP_HIP(hipMemcpyAsync(&l, c->loss, 4, hipMemcpyDeviceToHost, s), "copy loss");
        MLP_HIP(hipStreamSynchronize(s), "synchronize");
        *loss = (double)l / (double)B;
    }
    return QS_OK;
}

qs_status qs_mlp_adamw(qs_mlp *c, double lr, double beta1, double beta2, double eps, double wd) {
    if (!c) return mfail(QS_ERR_ARG, "net is NULL");
    if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0) || !(wd >= 0))
        return mfail(QS_ERR_ARG, "invalid AdamW hyperparameters");
    MLP_HIP(hipSetDevice(c->device), "hipSetDevice");
    c->t += 1;
    const double c1 = 1.0 - std::pow(beta1, (double)c->t), c2 = 1.0 - std::pow(beta2, (double)c->t);
    hipLaunchKernelGGL(adamw, dim3((unsigned)((N_PARAMS + 255) / 256)), dim3(256), 0, c->stream, c->P, c->G, c->Mo, c->Vo,
                       N_PARAMS, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)wd, (float)c1, (float)c2);
    convert(c);
    MLP_HIP(hipGetLastError(), "optimizer kernels");
    return QS_OK;
}

qs_status qs_mlp_train_step(qs_mlp *c, const float *x, const float *t, int32_t batch, double lr, double *loss) {
    qs_status st = qs_mlp_grads(c, x, t, batch, loss);
    if (st != QS_OK) return st;
    return qs_mlp_adamw(c, lr, 0.9, 0.999, 1e-8, 0.01);
}

void qs_mlp_free(qs_mlp *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->mem);
    delete c;
}

int32_t qs_debug_mlp_gemm_check(int32_t max_batch, int32_t batch, char *msg, int32_t msg_len) {
    auto say = [&](const std::string &m) {
        if (msg && msg_len > 0) {
            std::strncpy(msg, m.c_str(), (size_t)msg_len - 1);
            msg[msg_len - 1] = '\0';
        }
    };
    if (max_batch < 128 || max_batch % 128 != 0 || max_batch > (1 << 20) || batch < 128 || batch % 128 != 0 ||
        batch > max_batch) {
        say("batch sizes outside what qs_mlp_create and qs_mlp_grads accept");
        return -1;
    }
    // the buffers at the offsets of a real network, from a base aligned as hipMalloc aligns
    qs_mlp c;
    c.max_batch = max_batch;
    std::vector<size_t> o;
    (void)mlp_bytes(max_batch, &o);
    assign_buffers(&c, reinterpret_cast<char *>((uintptr_t)1 << 40), o);
    const int64_t B = batch;
    std::string why;
    for (int l = 0; l < 3 && why.empty(); ++l) {
        why = gemm_check(EPI_FWD, fwd_args(&c, l, B), 1);
        if (!why.empty()) why = "forward layer " + std::to_string(l) + ": " + why;
    }
    const int splits = wgrad_splits(B);
    int cur = 0;
    for (int l = 2; l >= 0 && why.empty(); --l) {
        why = gemm_check(EPI_PART, wgrad_args(&c, l, cur, B, splits), splits);
        if (!why.empty()) { why = "weight gradient " + std::to_string(l) + ": " + why; break; }
        why = gemm_check(EPI_BWD, dgrad_args(&c, l, cur, B), 1);
        if (!why.empty()) why = "input gradient " + std::to_string(l) + ": " + why;
        cur ^= 1;
    }
    say(why.empty() ? "ok, " + std::to_string(splits) + " row splits" : why);
    return why.empty() ? 0 : 1;
}

}  // extern "C"
