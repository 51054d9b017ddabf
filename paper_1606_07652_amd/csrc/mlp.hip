// Multilayer perceptron of the learned preconditioner (not part of the paper).
//
// g: R^64 -> R^64, three hidden layers of 256 units with ReLU, affine output layer.
// Parameters are one FP32 vector in the order W1 (256 x 64, row-major [out][in]), b1,
// W2 (256 x 256), b2, W3 (256 x 256), b3, W4 (64 x 256), b4.
//
// Inference (k_mlp_bf16): one workgroup of four waves evaluates 32 rows; activations stay
// in LDS as bfloat16, weights are read as bfloat16 from a copy of the FP32 master
// weights, products run on the gfx950 matrix cores (16x16x32 BF16 MFMA) with FP32
// accumulators initialised with the FP32 bias.  Each wave owns a quarter of the output
// columns of a layer.
//
// Training: FP32 throughout.  A tiled FP32 GEMM (LDS tiles, 4x4 outputs per thread)
// with transpose flags serves the forward layers, the backward data products and the
// weight gradients; weight gradients reduce over rows in fixed 256-row chunks whose
// partial sums are added in order, so a gradient is deterministic.  The loss is
// sum_r w_r ||g(x_r) - t_r||^2 / sum_r w_r; Adam (Kingma and Ba, 2015) updates the FP32
// master weights.  The training loop keeps the parameters with the lowest loss on the
// held-out rows.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace rbf {
namespace {

constexpr int IN = RBF_MLP_IN, HID = RBF_MLP_HIDDEN, OUT = RBF_MLP_IN;
constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + (int64_t)HID * IN, OFF_W2 = OFF_B1 + HID,
                  OFF_B2 = OFF_W2 + (int64_t)HID * HID, OFF_W3 = OFF_B2 + HID,
                  OFF_B3 = OFF_W3 + (int64_t)HID * HID, OFF_W4 = OFF_B3 + HID,
                  OFF_B4 = OFF_W4 + (int64_t)OUT * HID, NPARAM = OFF_B4 + OUT;
static_assert(NPARAM == RBF_MLP_NPARAMS, "parameter count");
// bfloat16 copy of the weight matrices only
constexpr int64_t BF_W1 = 0, BF_W2 = BF_W1 + (int64_t)HID * IN, BF_W3 = BF_W2 + (int64_t)HID * HID,
                  BF_W4 = BF_W3 + (int64_t)HID * HID, NBF = BF_W4 + (int64_t)OUT * HID;

struct Layer {
    int in, out;
    int64_t w, b, bf;
};
constexpr Layer kLayers[4] = {{IN, HID, OFF_W1, OFF_B1, BF_W1},
                              {HID, HID, OFF_W2, OFF_B2, BF_W2},
                              {HID, HID, OFF_W3, OFF_B3, BF_W3},
                              {HID, OUT, OFF_W4, OFF_B4, BF_W4}};

constexpr int kT = 256;          // threads per workgroup
constexpr int kChunkRows = 256;  // rows per partial sum of a weight gradient

// FP32 -> bfloat16, round to nearest even; NaN stays NaN
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ReLU that lets NaN through (so a broken network is seen by the caller's guard)
__device__ __forceinline__ float relu(float v) { return (v > 0.f || v != v) ? v : 0.f; }

__global__ void k_to_bf16(const float *__restrict__ src, uint16_t *__restrict__ dst, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i < n) dst[i] = f2bf(src[i]);
}

// ---- inference: BF16 MFMA ------------------------------------------------------------

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TM = 32;            // rows per workgroup
constexpr int LDSW = HID + 8;     // LDS row stride in bfloat16 (528 bytes, 16-byte aligned)

// One layer for the workgroup's TM rows.  MFMA 16x16x32: lane l supplies A[l % 16][8 (l / 16) + e]
// and B[8 (l / 16) + e][l % 16] (e = 0..7), and receives C[4 (l / 16) + q][l % 16] (q = 0..3).
template <int K, int N, bool LAST>
__device__ __forceinline__ void mlp_layer(const uint16_t *act_in, uint16_t *act_out, const uint16_t *__restrict__ W,
                                          const float *__restrict__ bias, float *__restrict__ y, int64_t row0,
                                          int64_t rows) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = N / 4;     // output columns of this wave
    constexpr int NT = NW / 16;   // 16-wide column tiles
    constexpr int MT = TM / 16;   // 16-high row tiles
    const int col0 = wave * NW;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const float bv = bias[col0 + 16 * j + lr];
#pragma unroll
        for (int i = 0; i < MT; ++i) acc[i][j] = f32x4{bv, bv, bv, bv};
    }
#pragma unroll 2
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a[MT], b[NT];
#pragma unroll
        for (int i = 0; i < MT; ++i)
            a[i] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(act_in + (16 * i + lr) * LDSW + k0 + lk));
#pragma unroll
        for (int j = 0; j < NT; ++j)
            b[j] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(W + (int64_t)(col0 + 16 * j + lr) * K + k0 + lk));
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    const int rq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * i + rq + q, c = col0 + 16 * j + lr;
                const float v = acc[i][j][q];
                if (!LAST) act_out[r * LDSW + c] = f2bf(relu(v));
                else if (row0 + r < rows) y[(row0 + r) * OUT + c] = v;
            }
}

__global__ void __launch_bounds__(kT) k_mlp_bf16(const float *__restrict__ x, int64_t rows,
                                                 const uint16_t *__restrict__ wbf, const float *__restrict__ params,
                                                 float *__restrict__ y) {
    __shared__ __attribute__((aligned(16))) uint16_t bufA[TM * LDSW];
    __shared__ __attribute__((aligned(16))) uint16_t bufB[TM * LDSW];
    const int64_t row0 = (int64_t)blockIdx.x * TM;
    for (int e = threadIdx.x; e < TM * IN; e += kT) {
        const int r = e / IN, c = e % IN;
        const float v = (row0 + r < rows) ? x[(row0 + r) * IN + c] : 0.f;
        bufA[r * LDSW + c] = f2bf(v);
    }
    __syncthreads();
    mlp_layer<IN, HID, false>(bufA, bufB, wbf + BF_W1, params + OFF_B1, nullptr, row0, rows);
    __syncthreads();
    mlp_layer<HID, HID, false>(bufB, bufA, wbf + BF_W2, params + OFF_B2, nullptr, row0, rows);
    __syncthreads();
    mlp_layer<HID, HID, false>(bufA, bufB, wbf + BF_W3, params + OFF_B3, nullptr, row0, rows);
    __syncthreads();
    mlp_layer<HID, OUT, true>(bufB, nullptr, wbf + BF_W4, params + OFF_B4, y, row0, rows);
}

// ---- training: FP32 -------------------------------------------------------------------

// C (+ blockIdx.z * cslab) = op(A) op(B) over k in the z-th chunk of kchunk.
// op(A)(m, k) = TA ? A[k lda + m] : A[m lda + k];  op(B)(k, n) = TB ? B[n ldb + k] : B[k ldb + n].
// EPI 0: store; 1: + bias[n], ReLU; 2: + bias[n]; 3: zero where mask[m ldm + n] <= 0.
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(kT) k_gemm(int M, int N, int K, int kchunk, const float *__restrict__ A, int lda,
                                             const float *__restrict__ B, int ldb, float *__restrict__ C, int ldc,
                                             int64_t cslab, const float *__restrict__ bias,
                                             const float *__restrict__ mask, int ldm) {
    __shared__ float As[16][64 + 4];
    __shared__ float Bs[16][64 + 4];
    const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int mm = TA ? (t & 15) * 4 + e : t >> 2;
            const int kk = TA ? t >> 4 : (t & 3) * 4 + e;
            const int m = m0 + mm, k = k0 + kk;
            float v = 0.f;
            if (m < M && k < ke) v = TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
            As[kk][mm] = v;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int nn = TB ? t >> 2 : (t & 15) * 4 + e;
            const int kk = TB ? (t & 3) * 4 + e : t >> 4;
            const int n = n0 + nn, k = k0 + kk;
            float v = 0.f;
            if (n < N && k < ke) v = TB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n];
            Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    float *Cz = C + blockIdx.z * cslab;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
            if (m >= M || n >= N) continue;
            float v = acc[i][j];
            if (EPI == 1 || EPI == 2) v += bias[n];
            if (EPI == 1) v = relu(v);
            if (EPI == 3) v = mask[(int64_t)m * ldm + n] > 0.f ? v : 0.f;
            Cz[(int64_t)m * ldc + n] = v;
        }
}

// part[z * N + n] = sum of D[r][n] over rows r of chunk z
__global__ void k_colsum_part(const float *__restrict__ D, int64_t rows, int N, float *__restrict__ part) {
    const int n = blockIdx.x * kT + threadIdx.x;
    if (n >= N) return;
    const int64_t r0 = (int64_t)blockIdx.y * kChunkRows, r1 = min(rows, r0 + kChunkRows);
    float s = 0.f;
    for (int64_t r = r0; r < r1; ++r) s += D[r * N + n];
    part[(int64_t)blockIdx.y * N + n] = s;
}

// out[i] = sum_z part[z * len + i], z in order
__global__ void k_sum_parts(const float *__restrict__ part, int S, int64_t len, float *__restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[z * len + i];
    out[i] = s;
}

__device__ double block_sum_d(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// out[slot] = sum of w[0..n)  (one workgroup, fixed order)
__global__ void __launch_bounds__(kT) k_sum_f(const float *__restrict__ w, int64_t n, double *__restrict__ out) {
    __shared__ double sh[kT];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kT) s += (double)w[i];
    s = block_sum_d(s, sh);
    if (threadIdx.x == 0) *out = s;
}

__global__ void __launch_bounds__(kT) k_sum_d(const double *__restrict__ v, int64_t n, double *__restrict__ out) {
    __shared__ double sh[kT];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kT) s += v[i];
    s = block_sum_d(s, sh);
    if (threadIdx.x == 0) *out = s;
}

// dG = 2 w_r (G - T) / W and part[block] = sum of w_r (G - T)^2 over the block's elements
__global__ void __launch_bounds__(kT) k_loss(const float *__restrict__ G, const float *__restrict__ T,
                                             const float *__restrict__ w, int64_t rows,
                                             const double *__restrict__ wsum, float *__restrict__ dG,
                                             double *__restrict__ part) {
    __shared__ double sh[kT];
    const int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x;
    const double W = *wsum;
    double c = 0.0;
    if (e < rows * OUT) {
        const double wr = w[e / OUT];
        const double d = (double)G[e] - (double)T[e];
        dG[e] = W > 0.0 ? (float)(2.0 * wr * d / W) : 0.f;
        c = wr * d * d;
    }
    c = block_sum_d(c, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = c;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_gather_rows(const float *__restrict__ src, const int *__restrict__ idx, int64_t nrows, int width,
                              float *__restrict__ dst) {
    const int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (e >= nrows * width) return;
    const int64_t r = e / width;
    dst[e] = src[(int64_t)idx[r] * width + e % width];
}

unsigned nblk(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace
}  // namespace rbf

struct rbf_mlp {
    rbf::Arena arena;
    float *params = nullptr;   // FP32 master parameters [NPARAM]
    uint16_t *wbf = nullptr;   // bfloat16 weights [NBF]
    float *adam_m = nullptr, *adam_v = nullptr;
    int64_t step = 0;
    // training workspace, sized for cap rows
    rbf::Arena ws;
    int64_t cap = 0;
    float *xb = nullptr, *tb = nullptr, *wb = nullptr, *h[3] = {}, *g = nullptr, *dg = nullptr, *da = nullptr,
          *db = nullptr, *grad = nullptr, *part = nullptr, *best = nullptr;
    double *lpart = nullptr, *dsc = nullptr;
};

namespace rbf {
namespace {

int refresh_bf16(rbf_mlp *m, hipStream_t s) {
    for (const Layer &L : kLayers) {
        const int64_t n = (int64_t)L.in * L.out;
        k_to_bf16<<<nblk(n), kT, 0, s>>>(m->params + L.w, m->wbf + L.bf, n);
        RBF_HIP(hipGetLastError());
    }
    return RBF_OK;
}

int ensure_ws(rbf_mlp *m, int64_t rows) {
    if (m->cap >= rows) return RBF_OK;
    m->ws.release();
    m->cap = 0;
    Arena &a = m->ws;
    const int64_t S = (rows + kChunkRows - 1) / kChunkRows;
    RBF_TRY(a.alloc((void **)&m->xb, sizeof(float) * rows * IN));
    RBF_TRY(a.alloc((void **)&m->tb, sizeof(float) * rows * OUT));
    RBF_TRY(a.alloc((void **)&m->wb, sizeof(float) * rows));
    for (int l = 0; l < 3; ++l) RBF_TRY(a.alloc((void **)&m->h[l], sizeof(float) * rows * HID));
    RBF_TRY(a.alloc((void **)&m->g, sizeof(float) * rows * OUT));
    RBF_TRY(a.alloc((void **)&m->dg, sizeof(float) * rows * OUT));
    RBF_TRY(a.alloc((void **)&m->da, sizeof(float) * rows * HID));
    RBF_TRY(a.alloc((void **)&m->db, sizeof(float) * rows * HID));
    RBF_TRY(a.alloc((void **)&m->grad, sizeof(float) * NPARAM));
    RBF_TRY(a.alloc((void **)&m->part, sizeof(float) * S * (int64_t)HID * HID));
    RBF_TRY(a.alloc((void **)&m->best, sizeof(float) * NPARAM));
    RBF_TRY(a.alloc((void **)&m->lpart, sizeof(double) * ((rows * OUT + kT - 1) / kT + 1)));
    RBF_TRY(a.alloc((void **)&m->dsc, sizeof(double) * 8));
    m->cap = rows;
    return RBF_OK;
}

template <bool TA, bool TB, int EPI>
int gemm(hipStream_t s, int M, int N, int K, int kchunk, const float *A, int lda, const float *B, int ldb, float *C,
         int ldc, int64_t cslab, const float *bias, const float *mask, int ldm) {
    const int S = (K + kchunk - 1) / kchunk;
    dim3 grid((N + 63) / 64, (M + 63) / 64, S);
    k_gemm<TA, TB, EPI><<<grid, kT, 0, s>>>(M, N, K, kchunk, A, lda, B, ldb, C, ldc, cslab, bias, mask, ldm);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

// FP32 forward of rows x (in the workspace layout): h[0..2], g
int forward32(rbf_mlp *m, const float *x, int64_t rows, hipStream_t s) {
    const float *in = x;
    for (int l = 0; l < 4; ++l) {
        const Layer &L = kLayers[l];
        float *out = l < 3 ? m->h[l] : m->g;
        if (l < 3)
            RBF_TRY((gemm<false, true, 1>(s, (int)rows, L.out, L.in, L.in, in, L.in, m->params + L.w, L.in, out, L.out,
                                         0, m->params + L.b, nullptr, 0)));
        else
            RBF_TRY((gemm<false, true, 2>(s, (int)rows, L.out, L.in, L.in, in, L.in, m->params + L.w, L.in, out, L.out,
                                         0, m->params + L.b, nullptr, 0)));
        in = out;
    }
    return RBF_OK;
}

// loss numerator and weight sum of the rows just forwarded (device scalars dsc[0], dsc[1]),
// and dG
int loss_grad_out(rbf_mlp *m, const float *t, const float *w, int64_t rows, hipStream_t s) {
    k_sum_f<<<1, kT, 0, s>>>(w, rows, m->dsc + 1);
    RBF_HIP(hipGetLastError());
    const int64_t nb = (rows * OUT + kT - 1) / kT;
    k_loss<<<(unsigned)nb, kT, 0, s>>>(m->g, t, w, rows, m->dsc + 1, m->dg, m->lpart);
    RBF_HIP(hipGetLastError());
    k_sum_d<<<1, kT, 0, s>>>(m->lpart, nb, m->dsc);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

// gradient of the loss of the rows just forwarded into m->grad
int backward32(rbf_mlp *m, const float *x, int64_t rows, hipStream_t s) {
    const int S = (int)((rows + kChunkRows - 1) / kChunkRows);
    const float *delta = m->dg;
    float *bufs[2] = {m->da, m->db};
    for (int l = 3; l >= 0; --l) {
        const Layer &L = kLayers[l];
        const float *act = l > 0 ? m->h[l - 1] : x;
        // dW = delta^T act over row chunks, then the chunks in order
        RBF_TRY((gemm<true, false, 0>(s, L.out, L.in, (int)rows, kChunkRows, delta, L.out, act, L.in, m->part, L.in,
                                     (int64_t)L.out * L.in, nullptr, nullptr, 0)));
        k_sum_parts<<<nblk((int64_t)L.out * L.in), kT, 0, s>>>(m->part, S, (int64_t)L.out * L.in, m->grad + L.w);
        RBF_HIP(hipGetLastError());
        dim3 cg((L.out + kT - 1) / kT, S);
        k_colsum_part<<<cg, kT, 0, s>>>(delta, rows, L.out, m->part);
        RBF_HIP(hipGetLastError());
        k_sum_parts<<<nblk(L.out), kT, 0, s>>>(m->part, S, L.out, m->grad + L.b);
        RBF_HIP(hipGetLastError());
        if (l > 0) {
            // delta_{l-1} = (delta W) masked by the ReLU of the layer below
            float *nd = bufs[l & 1];
            RBF_TRY((gemm<false, false, 3>(s, (int)rows, L.in, L.out, L.out, delta, L.out, m->params + L.w, L.in, nd,
                                          L.in, 0, nullptr, act, L.in)));
            delta = nd;
        }
    }
    return RBF_OK;
}

int read_scalars(rbf_mlp *m, hipStream_t s, double *num, double *den) {
    double h[2];
    RBF_HIP(hipMemcpyAsync(h, m->dsc, sizeof(h), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    *num = h[0];
    *den = h[1];
    return RBF_OK;
}

// weighted loss of rows [0, rows) of (x, t, w), in chunks of the workspace size
int eval_loss(rbf_mlp *m, const float *x, const float *t, const float *w, int64_t rows, hipStream_t s,
              double *loss) {
    double num = 0, den = 0;
    for (int64_t r0 = 0; r0 < rows; r0 += m->cap) {
        const int64_t nr = std::min(m->cap, rows - r0);
        RBF_TRY(forward32(m, x + r0 * IN, nr, s));
        RBF_TRY(loss_grad_out(m, t + r0 * OUT, w + r0, nr, s));
        double a, b;
        RBF_TRY(read_scalars(m, s, &a, &b));
        num += a;
        den += b;
    }
    *loss = den > 0 ? num / den : 0.0;
    return RBF_OK;
}

}  // namespace

int mlp_infer_bf16(rbf_mlp *m, const float *x, int64_t rows, float *y, hipStream_t s) {
    if (rows <= 0) return RBF_OK;
    k_mlp_bf16<<<(unsigned)((rows + TM - 1) / TM), kT, 0, s>>>(x, rows, m->wbf, m->params, y);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

}  // namespace rbf

using namespace rbf;

namespace {
const char kMagic[8] = {'R', 'B', 'F', '-', 'M', 'L', 'P', '\0'};
const uint32_t kVersion = 1;

int mlp_new(const float *host_params, uint64_t seed, rbf_mlp **out) {
    rbf_mlp *m = new rbf_mlp();
    auto fail = [&](int rc) {
        m->ws.release();
        m->arena.release();
        delete m;
        return rc;
    };
    int rc;
    if ((rc = m->arena.alloc((void **)&m->params, sizeof(float) * NPARAM)) != RBF_OK) return fail(rc);
    if ((rc = m->arena.alloc((void **)&m->wbf, sizeof(uint16_t) * NBF)) != RBF_OK) return fail(rc);
    if ((rc = m->arena.alloc((void **)&m->adam_m, sizeof(float) * NPARAM)) != RBF_OK) return fail(rc);
    if ((rc = m->arena.alloc((void **)&m->adam_v, sizeof(float) * NPARAM)) != RBF_OK) return fail(rc);
    std::vector<float> p(NPARAM, 0.f);
    if (host_params) {
        std::memcpy(p.data(), host_params, sizeof(float) * NPARAM);
    } else {
        // He-uniform hidden layers, zero biases, zero output layer (g = 0 at the start)
        uint64_t st = seed;
        for (int l = 0; l < 3; ++l) {
            const Layer &L = kLayers[l];
            const double a = std::sqrt(6.0 / L.in);
            for (int64_t i = 0; i < (int64_t)L.in * L.out; ++i) {
                const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
                p[L.w + i] = (float)((2.0 * u - 1.0) * a);
            }
        }
    }
    if (hipMemcpy(m->params, p.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->adam_m, 0, sizeof(float) * NPARAM) != hipSuccess ||
        hipMemset(m->adam_v, 0, sizeof(float) * NPARAM) != hipSuccess) {
        set_error("rbf_mlp_create: device copy failed");
        return fail(RBF_EHIP);
    }
    if ((rc = refresh_bf16(m, nullptr)) != RBF_OK) return fail(rc);
    if (hipDeviceSynchronize() != hipSuccess) {
        set_error("rbf_mlp_create: device error");
        return fail(RBF_EHIP);
    }
    *out = m;
    return RBF_OK;
}
}  // namespace

extern "C" int rbf_mlp_create(const float *params, uint64_t seed, rbf_mlp **out) {
    if (!out) { set_error("rbf_mlp_create: null output"); return RBF_EINVAL; }
    return mlp_new(params, seed, out);
}

extern "C" int rbf_mlp_destroy(rbf_mlp *m) {
    if (!m) return RBF_OK;
    (void)hipDeviceSynchronize();
    m->ws.release();
    m->arena.release();
    delete m;
    return RBF_OK;
}

extern "C" int rbf_mlp_get_params(const rbf_mlp *m, float *params) {
    if (!m || !params) { set_error("rbf_mlp_get_params: null argument"); return RBF_EINVAL; }
    RBF_HIP(hipDeviceSynchronize());
    RBF_HIP(hipMemcpy(params, m->params, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    return RBF_OK;
}

extern "C" int rbf_mlp_save(const rbf_mlp *m, const char *path) {
    if (!m || !path) { set_error("rbf_mlp_save: null argument"); return RBF_EINVAL; }
    std::vector<float> p(NPARAM);
    RBF_TRY(rbf_mlp_get_params(m, p.data()));
    FILE *f = std::fopen(path, "wb");
    if (!f) { set_error("rbf_mlp_save: cannot open %s", path); return RBF_EINVAL; }
    const uint32_t hdr[8] = {kVersion, 4, (uint32_t)IN, (uint32_t)HID, (uint32_t)HID, (uint32_t)HID, (uint32_t)OUT, 1};
    const uint64_t np = (uint64_t)NPARAM;
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
              std::fwrite(&np, sizeof(np), 1, f) == 1 && std::fwrite(p.data(), sizeof(float), NPARAM, f) == (size_t)NPARAM;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) { set_error("rbf_mlp_save: write to %s failed", path); return RBF_EINVAL; }
    return RBF_OK;
}

extern "C" int rbf_mlp_load(const char *path, rbf_mlp **out) {
    if (!path || !out) { set_error("rbf_mlp_load: null argument"); return RBF_EINVAL; }
    FILE *f = std::fopen(path, "rb");
    if (!f) { set_error("rbf_mlp_load: cannot open %s", path); return RBF_EINVAL; }
    char magic[8];
    uint32_t hdr[8];
    uint64_t np = 0;
    std::vector<float> p(NPARAM);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::fread(hdr, sizeof(hdr), 1, f) == 1 &&
              std::fread(&np, sizeof(np), 1, f) == 1;
    const uint32_t want[8] = {kVersion, 4, (uint32_t)IN, (uint32_t)HID, (uint32_t)HID, (uint32_t)HID, (uint32_t)OUT, 1};
    ok = ok && std::memcmp(magic, kMagic, 8) == 0 && std::memcmp(hdr, want, sizeof(want)) == 0 &&
         np == (uint64_t)NPARAM;
    ok = ok && std::fread(p.data(), sizeof(float), NPARAM, f) == (size_t)NPARAM;
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;   // nothing after the parameters
    std::fclose(f);
    if (!ok) {
        set_error("rbf_mlp_load: %s is not a version-%u weight file of the 64-256-256-256-64 network", path, kVersion);
        return RBF_EINVAL;
    }
    return mlp_new(p.data(), 0, out);
}

extern "C" int rbf_mlp_forward(rbf_mlp *m, const float *x, int64_t rows, float *y, int precision, void *stream) {
    if (!m || rows < 0 || (rows > 0 && (!x || !y))) { set_error("rbf_mlp_forward: bad arguments"); return RBF_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (precision == RBF_MLP_BF16) return mlp_infer_bf16(m, x, rows, y, s);
    if (precision != RBF_MLP_F32) { set_error("rbf_mlp_forward: unknown precision %d", precision); return RBF_EINVAL; }
    const int64_t chunk = 4096;
    RBF_TRY(ensure_ws(m, std::min<int64_t>(std::max<int64_t>(rows, 1), chunk)));
    for (int64_t r0 = 0; r0 < rows; r0 += m->cap) {
        const int64_t nr = std::min(m->cap, rows - r0);
        RBF_TRY(forward32(m, x + r0 * IN, nr, s));
        RBF_HIP(hipMemcpyAsync(y + r0 * OUT, m->g, sizeof(float) * nr * OUT, hipMemcpyDeviceToDevice, s));
    }
    return RBF_OK;
}

extern "C" int rbf_mlp_loss_grad(rbf_mlp *m, const float *x, const float *t, const float *w, int64_t rows,
                                 double *loss, float *grad, void *stream) {
    if (!m || !x || !t || !w || rows <= 0 || rows > (1 << 20)) {
        set_error("rbf_mlp_loss_grad: bad arguments (1 <= rows <= 2^20)");
        return RBF_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    RBF_TRY(ensure_ws(m, rows));
    RBF_TRY(forward32(m, x, rows, s));
    RBF_TRY(loss_grad_out(m, t, w, rows, s));
    RBF_TRY(backward32(m, x, rows, s));
    double num, den;
    RBF_TRY(read_scalars(m, s, &num, &den));
    if (loss) *loss = den > 0 ? num / den : 0.0;
    if (grad) RBF_HIP(hipMemcpy(grad, m->grad, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
    return RBF_OK;
}

extern "C" int rbf_mlp_train(rbf_mlp *m, const float *x, const float *t, const float *w, int64_t rows,
                             const rbf_train_opts *o, void *stream, rbf_train_info *info) {
    if (!m || !x || !t || !w || rows <= 0) { set_error("rbf_mlp_train: bad arguments"); return RBF_EINVAL; }
    auto t0 = std::chrono::steady_clock::now();
    rbf_train_opts opt;
    std::memset(&opt, 0, sizeof(opt));
    if (o) opt = *o;
    const int epochs = opt.epochs > 0 ? opt.epochs : 100;
    const int patience = opt.patience;
    const double lr = opt.lr > 0 ? opt.lr : 1e-3, b1 = opt.beta1 > 0 ? opt.beta1 : 0.9,
                 b2 = opt.beta2 > 0 ? opt.beta2 : 0.999, eps = opt.eps > 0 ? opt.eps : 1e-8;
    const double vf = opt.val_frac;
    if (vf < 0 || vf >= 1) { set_error("rbf_mlp_train: val_frac must lie in [0, 1)"); return RBF_EINVAL; }
    const int64_t nval = (int64_t)std::floor(vf * (double)rows);
    const int64_t ntr = rows - nval;
    if (ntr <= 0) { set_error("rbf_mlp_train: no training rows"); return RBF_EINVAL; }
    const int64_t batch = std::min<int64_t>(opt.batch > 0 ? opt.batch : 512, ntr);
    hipStream_t s = (hipStream_t)stream;
    RBF_TRY(ensure_ws(m, std::max<int64_t>(batch, 1)));
    int *idx = nullptr;
    RBF_HIP(hipMalloc(&idx, sizeof(int) * ntr));
    struct Free { int *p; ~Free() { if (p) (void)hipFree(p); } } fr{idx};

    rbf_train_info inf;
    std::memset(&inf, 0, sizeof(inf));
    double best = INFINITY;
    if (nval > 0) {
        RBF_TRY(eval_loss(m, x + ntr * IN, t + ntr * OUT, w + ntr, nval, s, &best));
        inf.init_val_loss = best;
        RBF_HIP(hipMemcpyAsync(m->best, m->params, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, s));
    }
    inf.best_val_loss = best;
    uint64_t st = opt.seed;
    std::vector<int> order(ntr);
    int since = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t i = 0; i < ntr; ++i) order[i] = (int)i;
        for (int64_t i = ntr - 1; i > 0; --i) std::swap(order[i], order[splitmix64(st) % (uint64_t)(i + 1)]);
        RBF_HIP(hipMemcpyAsync(idx, order.data(), sizeof(int) * ntr, hipMemcpyHostToDevice, s));
        double num = 0, den = 0;
        for (int64_t b0 = 0; b0 < ntr; b0 += batch) {
            const int64_t nr = std::min(batch, ntr - b0);
            k_gather_rows<<<nblk(nr * IN), kT, 0, s>>>(x, idx + b0, nr, IN, m->xb);
            k_gather_rows<<<nblk(nr * OUT), kT, 0, s>>>(t, idx + b0, nr, OUT, m->tb);
            k_gather_rows<<<nblk(nr), kT, 0, s>>>(w, idx + b0, nr, 1, m->wb);
            RBF_HIP(hipGetLastError());
            RBF_TRY(forward32(m, m->xb, nr, s));
            RBF_TRY(loss_grad_out(m, m->tb, m->wb, nr, s));
            RBF_TRY(backward32(m, m->xb, nr, s));
            ++m->step;
            const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)m->step)));
            const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)m->step)));
            k_adam<<<nblk(NPARAM), kT, 0, s>>>(m->params, m->grad, m->adam_m, m->adam_v, NPARAM, (float)lr, (float)b1,
                                               (float)b2, (float)eps, c1, c2);
            RBF_HIP(hipGetLastError());
            double a, b;
            RBF_TRY(read_scalars(m, s, &a, &b));   // loss of the batch before the update
            num += a;
            den += b;
        }
        const double tr = den > 0 ? num / den : 0.0;
        double vl = tr;
        if (nval > 0) RBF_TRY(eval_loss(m, x + ntr * IN, t + ntr * OUT, w + ntr, nval, s, &vl));
        if (inf.nhist < 256) {
            inf.train_loss[inf.nhist] = tr;
            inf.val_loss[inf.nhist] = vl;
            ++inf.nhist;
        }
        inf.epochs_run = ep + 1;
        inf.final_train_loss = tr;
        if (nval > 0) {
            if (vl < best) {
                best = vl;
                inf.best_epoch = ep + 1;
                since = 0;
                RBF_HIP(hipMemcpyAsync(m->best, m->params, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, s));
            } else if (patience > 0 && ++since >= patience) {
                break;
            }
        }
    }
    if (nval > 0) {
        RBF_HIP(hipMemcpyAsync(m->params, m->best, sizeof(float) * NPARAM, hipMemcpyDeviceToDevice, s));
        inf.best_val_loss = best;
    } else {
        inf.best_epoch = inf.epochs_run;
    }
    RBF_TRY(refresh_bf16(m, s));
    RBF_HIP(hipStreamSynchronize(s));
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return RBF_OK;
}

// ---------------------------------------------------------------------------------------
// FP32 forward without allocation.  The two hidden activation buffers of a call live in
// `scratch`, a file-scope device array of fixed size; every device the library runs on
// holds its own copy for the life of the process.  Host code never passes the array's
// name to a kernel (on the host it only stands for the symbol): the device address comes
// from hipGetSymbolAddress, taken once per device with that device current.
namespace {

constexpr int64_t kStaticRows = RBF_MLP_STATIC_MAX_ROWS;
__device__ __align__(256) float scratch[2 * kStaticRows * HID];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(float **out) {
    int dev = -1;
    RBF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("rbf_mlp_forward_static: device %d out of range", dev);
        return RBF_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        RBF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("rbf_mlp_forward_static: no device address for the scratch array on device %d", dev);
            return RBF_EHIP;
        }
        g_scratch_ptr[dev] = (float *)p;
    }
    *out = g_scratch_ptr[dev];
    return RBF_OK;
}

}  // namespace

extern "C" int rbf_mlp_forward_static(rbf_mlp *m, const float *x, int64_t rows, float *y, void *stream) {
    if (!m || rows < 0 || (rows > 0 && (!x || !y))) {
        set_error("rbf_mlp_forward_static: bad arguments");
        return RBF_EINVAL;
    }
    if (rows > kStaticRows) {
        set_error("rbf_mlp_forward_static: %lld rows exceed the static workspace of %lld rows; "
                  "split the call", (long long)rows, (long long)kStaticRows);
        return RBF_EINVAL;
    }
    float *ws = nullptr;
    RBF_TRY(scratch_for_current_device(&ws));
    if (rows == 0) return RBF_OK;
    hipStream_t s = (hipStream_t)stream;
    // h0 -> buffer A, h1 -> buffer B, h2 -> buffer A (h0 is dead once h1 is written),
    // output layer straight into y.  Every row is written before it is read, so nothing
    // needs clearing; the kernels and their summation order are those of rbf_mlp_forward.
    float *bufA = ws, *bufB = ws + kStaticRows * HID;
    const float *in = x;
    float *outs[3] = {bufA, bufB, bufA};
    for (int l = 0; l < 3; ++l) {
        const Layer &L = kLayers[l];
        RBF_TRY((gemm<false, true, 1>(s, (int)rows, L.out, L.in, L.in, in, L.in, m->params + L.w, L.in, outs[l],
                                     L.out, 0, m->params + L.b, nullptr, 0)));
        in = outs[l];
    }
    const Layer &L = kLayers[3];
    RBF_TRY((gemm<false, true, 2>(s, (int)rows, L.out, L.in, L.in, in, L.in, m->params + L.w, L.in, y, L.out, 0,
                                 m->params + L.b, nullptr, 0)));
    return RBF_OK;
}
