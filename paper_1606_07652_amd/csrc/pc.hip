// Right preconditioners of the GMRES solve (not part of the paper): block-Jacobi over
// 64-point blocks of the Morton order, and a learned correction of its output.
//
// Block factorisation (k_bj_setup): one wave per block.  The block's kernel matrix
// A_bb + reg I is formed in FP64 in LDS (column-major, lane i owns row i) and inverted in
// place by Gauss-Jordan elimination with partial pivoting (the blocks of the multiquadric are
// indefinite, and Wendland's function is positive definite only in one dimension): at step k
// the wave finds the row of largest |a_ik|, i >= k, swaps it with row k (lane j swaps the
// two entries of column j), every lane updates its own row with row k read as a broadcast,
// then row and column k are rescaled; at the end the columns are swapped back in reverse
// order of the row swaps.  Rows beyond a short last block are padded with the identity.  The
// inverse is stored column-major, so the apply (lane i forms row i of the product) reads each
// column with one coalesced load.
//
// Apply (k_bj_rows): four waves per workgroup, one block per wave.  The block's entries of
// v are gathered through the permutation into LDS, y_b = inv_b v_b, and either written back
// in caller order (block-Jacobi) or kept in Morton order with the block norm and the
// normalised row that the network reads (learned).
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace rbf {
namespace {

constexpr int BS = RBF_PC_BLOCK;
constexpr int kT = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The kernels with block preconditioners, in FP64: the Gaussian exp(-r^2/(2 s^2)), the
// multiquadric sqrt(r^2 + c^2), the inverse multiquadric 1/sqrt(r^2 + c^2) and Wendland's
// (1 - e r)_+^3 (3 e r + 1).
__device__ double block_phi(int kernel, double r2, double shape) {
    if (kernel == RBF_GAUSSIAN) return exp(-r2 / (2.0 * shape * shape));
    if (kernel == RBF_MULTIQUADRIC) return sqrt(r2 + shape * shape);
    if (kernel == RBF_INVERSE_MULTIQUADRIC) return 1.0 / sqrt(r2 + shape * shape);
    const double er = shape * sqrt(r2);
    const double t = fmax(1.0 - er, 0.0);
    return t * t * t * (3.0 * er + 1.0);
}

template <class T>
__global__ void __launch_bounds__(BS) k_bj_setup(const T *__restrict__ xs, int64_t n, int d, int kernel, double shape,
                                                 double reg, double *__restrict__ inv, int *__restrict__ flag) {
    __shared__ double L[BS * BS];
    __shared__ double px[kMaxDim][BS];
    const int i = threadIdx.x;
    const int64_t b = blockIdx.x, g = b * BS + i;
    const int m = (int)min<int64_t>(BS, n - b * BS);
    for (int k = 0; k < d; ++k) px[k][i] = i < m ? (double)xs[(int64_t)k * n + g] : 0.0;
    __syncthreads();
    for (int j = 0; j < BS; ++j) {
        double a;
        if (i < m && j < m) {
            double r2 = 0.0;
            for (int k = 0; k < d; ++k) {
                const double t = px[k][i] - px[k][j];
                r2 += t * t;
            }
            a = block_phi(kernel, r2, shape) + (i == j ? reg : 0.0);
        } else {
            a = i == j ? 1.0 : 0.0;
        }
        L[j * BS + i] = a;
    }
    __syncthreads();
    __shared__ int ipiv[BS];
    for (int k = 0; k < BS; ++k) {
        // pivot: the row of largest |a_ik| among i >= k (lowest index on ties)
        double best = i >= k ? fabs(L[k * BS + i]) : -1.0;
        int bi = i;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (i == 0) ipiv[k] = bi;
        if (bi != k) {   // uniform over the wave: lane j swaps rows k and bi of column j
            const double t = L[i * BS + k];
            L[i * BS + k] = L[i * BS + bi];
            L[i * BS + bi] = t;
        }
        __syncthreads();
        const double piv = L[k * BS + k];
        if (!(fabs(piv) > 0.0) || !isfinite(piv)) {   // uniform over the wave
            if (i == 0) flag[0] = 1;
            return;
        }
        const double p = 1.0 / piv;
        const double aik = L[k * BS + i];
        __syncthreads();
        if (i != k) {
            const double f = aik * p;
            for (int j = 0; j < BS; ++j)
                if (j != k) L[j * BS + i] -= f * L[j * BS + k];
        }
        __syncthreads();
        if (i != k) {
            L[i * BS + k] *= p;          // row k
            L[k * BS + i] = -aik * p;    // column k
        } else {
            L[k * BS + k] = p;
        }
        __syncthreads();
    }
    // the row swaps of the factorisation become column swaps of the inverse, in reverse order
    for (int k = BS - 1; k >= 0; --k) {
        const int q = ipiv[k];
        if (q != k) {
            const double t = L[k * BS + i];
            L[k * BS + i] = L[q * BS + i];
            L[q * BS + i] = t;
        }
        __syncthreads();
    }
    double *out = inv + b * BS * BS;
    for (int j = 0; j < BS; ++j) out[j * BS + i] = L[j * BS + i];
}

// y_b = inv_b v_b.  MODE 0: z[perm] = y.  MODE 1: y (Morton order), s_b = ||y_b||, x_b = y_b / s_b.
template <int MODE>
__global__ void __launch_bounds__(kT) k_bj_rows(const double *__restrict__ inv, const int *__restrict__ perm,
                                                int64_t n, int64_t nblk, const double *__restrict__ v,
                                                double *__restrict__ z, double *__restrict__ y_out,
                                                double *__restrict__ s_out, float *__restrict__ x_out) {
    __shared__ double vs[kT / BS][BS];
    const int lane = threadIdx.x & (BS - 1), w = threadIdx.x / BS;
    const int64_t b = blockIdx.x * (int64_t)(kT / BS) + w;
    const int64_t g = b * BS + lane;
    const bool valid = b < nblk && g < n;
    vs[w][lane] = valid ? v[perm[g]] : 0.0;
    __syncthreads();
    if (b >= nblk) return;
    const double *col = inv + b * BS * BS + lane;
    double y = 0.0;
#pragma unroll 8
    for (int j = 0; j < BS; ++j) y = fma(col[j * BS], vs[w][j], y);
    if (MODE == 0) {
        if (valid) z[perm[g]] = y;
        return;
    }
    if (!valid) y = 0.0;
    const double s = sqrt(wave_sum(y * y));
    if (valid) y_out[g] = y;
    if (lane == 0) s_out[b] = s;
    x_out[b * BS + lane] = s > 0.0 ? (float)(y / s) : 0.f;
}

// Block-Jacobi over a batch: wave = one global block; its problem by binary search over the
// first-block table, then as k_bj_rows<0> on that problem's slice of v and z.
__global__ void __launch_bounds__(kT) k_bj_rows_batch(BatchBj bj, const double *__restrict__ v,
                                                      double *__restrict__ z) {
    __shared__ double vs[kT / BS][BS];
    const int lane = threadIdx.x & (BS - 1), w = threadIdx.x / BS;
    const int64_t b = blockIdx.x * (int64_t)(kT / BS) + w;
    int q = 0;
    if (b < bj.nblk) {
        int lo = 0, hi = bj.nprob;   // largest q with bfirst[q] <= b
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (bj.bfirst[mid] <= b) lo = mid; else hi = mid;
        }
        q = lo;
    }
    const int64_t lb = b - bj.bfirst[q], off = bj.off[q], nq = bj.off[q + 1] - off;
    const int64_t g = lb * BS + lane;
    const bool valid = b < bj.nblk && g < nq;
    const int *perm = bj.perm[q];
    vs[w][lane] = valid ? v[off + perm[g]] : 0.0;
    __syncthreads();
    if (b >= bj.nblk) return;
    const double *col = bj.inv[q] + lb * BS * BS + lane;
    double y = 0.0;
#pragma unroll 8
    for (int j = 0; j < BS; ++j) y = fma(col[j * BS], vs[w][j], y);
    if (valid) z[off + perm[g]] = y;
}

// z[perm[g]] = y_g + s_b G[b][g - 64 b]   (0 when s_b = 0)
__global__ void k_pc_combine(const double *__restrict__ y, const double *__restrict__ s, const float *__restrict__ G,
                             const int *__restrict__ perm, int64_t n, double *__restrict__ z) {
    const int64_t g = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (g >= n) return;
    const int64_t b = g / BS;
    const double sb = s[b];
    z[perm[g]] = sb > 0.0 ? y[g] + sb * (double)G[g] : 0.0;
}

// training rows of one (r, e) pair; enorm2 = ||e||^2 (device)
__global__ void __launch_bounds__(kT) k_pc_pairs(const double *__restrict__ inv, const int *__restrict__ perm,
                                                 int64_t n, int64_t nblk, const double *__restrict__ r,
                                                 const double *__restrict__ e, const double *__restrict__ enorm2,
                                                 float *__restrict__ X, float *__restrict__ T,
                                                 float *__restrict__ W) {
    __shared__ double vs[kT / BS][BS];
    const int lane = threadIdx.x & (BS - 1), w = threadIdx.x / BS;
    const int64_t b = blockIdx.x * (int64_t)(kT / BS) + w;
    const int64_t g = b * BS + lane;
    const bool valid = b < nblk && g < n;
    vs[w][lane] = valid ? r[perm[g]] : 0.0;
    __syncthreads();
    if (b >= nblk) return;
    const double *col = inv + b * BS * BS + lane;
    double y = 0.0;
#pragma unroll 8
    for (int j = 0; j < BS; ++j) y = fma(col[j * BS], vs[w][j], y);
    if (!valid) y = 0.0;
    const double eb = valid ? e[perm[g]] : 0.0;
    const double s = sqrt(wave_sum(y * y));
    const bool ok = s > 0.0;
    X[b * BS + lane] = ok ? (float)(y / s) : 0.f;
    T[b * BS + lane] = ok ? (float)((eb - y) / s) : 0.f;
    if (lane == 0) {
        const double en = *enorm2;
        const bool full = (b + 1) * BS <= n;
        W[b] = (ok && full && en > 0.0) ? (float)(s * s / en) : 0.f;
    }
}

__global__ void __launch_bounds__(kT) k_dot_self(const double *__restrict__ v, int64_t n, double *__restrict__ out) {
    __shared__ double sh[kT];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kT) s += v[i] * v[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// out = a - b, formed in T (so an F32 difference is exact in FP64 and converts back exactly)
template <class T>
__global__ void k_diff64(const T *__restrict__ a, const T *__restrict__ b, double *__restrict__ out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i < n) out[i] = (double)(T)(a[i] - b[i]);
}

__global__ void k_to32(const double *__restrict__ a, float *__restrict__ out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i < n) out[i] = (float)a[i];
}

template <class T>
__global__ void k_to64(const T *__restrict__ a, double *__restrict__ out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i < n) out[i] = (double)a[i];
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

int ensure_pc_buffers(rbf_plan *p) {
    if (p->pc_y) return RBF_OK;
    const int64_t nb = (p->n + BS - 1) / BS;
    Arena &a = p->pc_arena;
    RBF_TRY(a.alloc((void **)&p->pc_y, sizeof(double) * p->n));
    RBF_TRY(a.alloc((void **)&p->pc_s, sizeof(double) * nb));
    RBF_TRY(a.alloc((void **)&p->pc_x, sizeof(float) * nb * BS));
    RBF_TRY(a.alloc((void **)&p->pc_g, sizeof(float) * nb * BS));
    RBF_TRY(a.alloc((void **)&p->pc_flag, sizeof(int) * 4));
    RBF_TRY(a.alloc((void **)&p->pc_scal, sizeof(double) * 4));
    p->nblk = nb;
    return RBF_OK;
}

// factorise every block of (A_bb + reg I) into inv (nblk 64 x 64 doubles)
int factor_blocks(rbf_plan *p, double reg, double *inv) {
    hipStream_t s = p->stream;
    RBF_HIP(hipMemsetAsync(p->pc_flag, 0, sizeof(int), s));
    if (p->dtype == RBF_F32)
        k_bj_setup<float><<<(unsigned)p->nblk, BS, 0, s>>>((const float *)p->xs, p->n, p->d, p->kernel, p->shape,
                                                            reg, inv, p->pc_flag);
    else
        k_bj_setup<double><<<(unsigned)p->nblk, BS, 0, s>>>((const double *)p->xs, p->n, p->d, p->kernel, p->shape,
                                                             reg, inv, p->pc_flag);
    RBF_HIP(hipGetLastError());
    int flag = 0;
    RBF_HIP(hipMemcpyAsync(&flag, p->pc_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    if (flag) {
        set_error("block factorisation: a block is numerically singular at reg = %g (a property of the kernel "
                  "and the points: coincident points, or an eigenvalue of a block at -reg)", reg);
        return RBF_EINVAL;
    }
    return RBF_OK;
}

// Block preconditioners for the Gaussian, the multiquadric kernels and Wendland's function (the
// thin-plate spline and r^5 need the polynomial terms of the augmented solve, which has none);
// the network's features and training pairs for the Gaussian and the multiquadric kernels.
int check_bj_kernel(const rbf_plan *p) {
    if (p->kernel != RBF_GAUSSIAN && p->kernel != RBF_MULTIQUADRIC && p->kernel != RBF_INVERSE_MULTIQUADRIC &&
        p->kernel != RBF_WENDLAND) {
        set_error("block-Jacobi: Gaussian, multiquadric, inverse multiquadric and Wendland kernels are supported");
        return RBF_EUNSUPPORTED;
    }
    return RBF_OK;
}

int check_learned_kernel(const rbf_plan *p) {
    if (p->kernel != RBF_GAUSSIAN && p->kernel != RBF_MULTIQUADRIC && p->kernel != RBF_INVERSE_MULTIQUADRIC) {
        set_error("learned preconditioner: the Gaussian and the multiquadric kernels are supported");
        return RBF_EUNSUPPORTED;
    }
    return RBF_OK;
}

// Phi(0), the scale of the default regularisations
double phi_zero(const rbf_plan *p) {
    if (p->kernel == RBF_INVERSE_MULTIQUADRIC) return 1.0 / p->shape;
    if (p->kernel == RBF_MULTIQUADRIC) return p->shape;
    return 1.0;
}

int build_lp(rbf_plan *p, double reg);

// block-Jacobi inverses at reg
int build_bj(rbf_plan *p, double reg) {
    RBF_TRY(check_bj_kernel(p));
    RBF_TRY(ensure_pc_buffers(p));
    if (!p->bj_inv) RBF_TRY(p->pc_arena.alloc((void **)&p->bj_inv, sizeof(double) * p->nblk * BS * BS));
    // feature inverses that share this storage keep their reg: they move to their own
    const double shared_lp = (p->lp_inv == p->bj_inv && p->lp_reg >= 0) ? p->lp_reg : -1.0;
    if (p->lp_inv == p->bj_inv) { p->lp_inv = nullptr; p->lp_reg = -1.0; }
    p->bj_reg = -1.0;
    RBF_TRY(factor_blocks(p, reg, p->bj_inv));
    p->bj_reg = reg;
    if (shared_lp >= 0) return build_lp(p, shared_lp);
    return RBF_OK;
}

// feature inverses of the learned map at reg (shares the block-Jacobi storage when the regs agree)
int build_lp(rbf_plan *p, double reg) {
    RBF_TRY(check_learned_kernel(p));
    RBF_TRY(ensure_pc_buffers(p));
    p->lp_reg = -1.0;
    p->lp_inv = nullptr;
    if (p->bj_reg == reg) {
        p->lp_inv = p->bj_inv;
    } else {
        if (!p->lp_own) RBF_TRY(p->pc_arena.alloc((void **)&p->lp_own, sizeof(double) * p->nblk * BS * BS));
        RBF_TRY(factor_blocks(p, reg, p->lp_own));
        p->lp_inv = p->lp_own;
    }
    p->lp_reg = reg;
    return RBF_OK;
}

// 1e-2 Phi(0) (Phi(0) = 1 for the Gaussian): the best of 1e-8 .. 1e-1 in GMRES(50) solves of
// 3-D mixed, 3-D uniform and 2-D jittered Gaussian systems
constexpr double kDefaultBjReg = 1e-2;
// near-exact local solves: the features keep the small-eigenvalue components of the block
// error that the network has to see (at 1e-2 it learned nothing on the same data)
constexpr double kDefaultLpReg = 1e-6;

// y = A x in FP64 through the plan's dtype (tmp: two plan-dtype vectors of n)
int product64(rbf_plan *p, const double *x, double *y, void *tmp) {
    hipStream_t s = p->stream;
    if (p->dtype == RBF_F64) return launch_matvec(p, x, y);
    float *tin = (float *)tmp, *tout = tin + p->n;
    // the harvest forms F32 errors in F32, so this narrowing copy is exact
    k_to32<<<grid_of(p->n), kT, 0, s>>>(x, tin, p->n);
    RBF_HIP(hipGetLastError());
    RBF_TRY(launch_matvec(p, tin, tout));
    k_to64<float><<<grid_of(p->n), kT, 0, s>>>(tout, y, p->n);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

}  // namespace

int pc_ready(rbf_plan *p, int kind) {
    if (kind == RBF_PC_NONE) return RBF_OK;
    if (kind != RBF_PC_BLOCK_JACOBI && kind != RBF_PC_LEARNED) {
        set_error("unknown preconditioner %d", kind);
        return RBF_EINVAL;
    }
    if (p->bj_reg < 0) RBF_TRY(build_bj(p, kDefaultBjReg * phi_zero(p)));
    if (kind == RBF_PC_LEARNED) {
        if (!p->mlp) {
            set_error("learned preconditioner: no network attached (rbf_pc_set_learned)");
            return RBF_ESTATE;
        }
        if (p->lp_reg < 0) RBF_TRY(build_lp(p, kDefaultLpReg * phi_zero(p)));
    }
    return RBF_OK;
}

int pc_apply(rbf_plan *p, int kind, const double *v, double *z) {
    hipStream_t s = p->stream;
    const unsigned nb = (unsigned)((p->nblk + kT / BS - 1) / (kT / BS));
    if (kind == RBF_PC_BLOCK_JACOBI) {
        k_bj_rows<0><<<nb, kT, 0, s>>>(p->bj_inv, p->perm, p->n, p->nblk, v, z, nullptr, nullptr, nullptr);
        RBF_HIP(hipGetLastError());
        return RBF_OK;
    }
    if (kind == RBF_PC_LEARNED) {
        k_bj_rows<1><<<nb, kT, 0, s>>>(p->lp_inv, p->perm, p->n, p->nblk, v, nullptr, p->pc_y, p->pc_s, p->pc_x);
        RBF_HIP(hipGetLastError());
        RBF_TRY(mlp_infer_bf16(p->mlp, p->pc_x, p->nblk, p->pc_g, s));
        k_pc_combine<<<grid_of(p->n), kT, 0, s>>>(p->pc_y, p->pc_s, p->pc_g, p->perm, p->n, z);
        RBF_HIP(hipGetLastError());
        return RBF_OK;
    }
    set_error("pc_apply: preconditioner %d cannot be applied", kind);
    return RBF_EINVAL;
}

int batch_bj_prepare(const std::vector<rbf_plan *> &plans, const std::vector<int64_t> &offsets, Arena &ar,
                     hipStream_t s, BatchBj *bj) {
    const int P = (int)plans.size();
    std::vector<const double *> inv(P);
    std::vector<const int *> perm(P);
    std::vector<int64_t> bfirst(P + 1, 0);
    for (int q = 0; q < P; ++q) {
        rbf_plan *p = plans[q];
        if (p->n != offsets[q + 1] - offsets[q]) {
            set_error("batched block-Jacobi: problem %d has %lld points, its plan %lld", q,
                      (long long)(offsets[q + 1] - offsets[q]), (long long)p->n);
            return RBF_EINVAL;
        }
        RBF_TRY(check_bj_kernel(p));
        if (p->bj_reg < 0) RBF_TRY(build_bj(p, kDefaultBjReg * phi_zero(p)));
        inv[q] = p->bj_inv;
        perm[q] = p->perm;
        bfirst[q + 1] = bfirst[q] + p->nblk;
    }
    const double **dinv = nullptr;
    const int **dperm = nullptr;
    int64_t *doff = nullptr, *dbf = nullptr;
    RBF_TRY(ar.alloc((void **)&dinv, sizeof(double *) * P));
    RBF_TRY(ar.alloc((void **)&dperm, sizeof(int *) * P));
    RBF_TRY(ar.alloc((void **)&doff, sizeof(int64_t) * (P + 1)));
    RBF_TRY(ar.alloc((void **)&dbf, sizeof(int64_t) * (P + 1)));
    RBF_HIP(hipMemcpyAsync(dinv, inv.data(), sizeof(double *) * P, hipMemcpyHostToDevice, s));
    RBF_HIP(hipMemcpyAsync(dperm, perm.data(), sizeof(int *) * P, hipMemcpyHostToDevice, s));
    RBF_HIP(hipMemcpyAsync(doff, offsets.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice, s));
    RBF_HIP(hipMemcpyAsync(dbf, bfirst.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice, s));
    RBF_HIP(hipStreamSynchronize(s));   // the host tables above go out of scope
    *bj = BatchBj{dinv, dperm, doff, dbf, P, bfirst[P]};
    return RBF_OK;
}

int batch_bj_apply(const BatchBj &bj, const double *v, double *z, hipStream_t s) {
    if (bj.nblk <= 0) return RBF_OK;
    const unsigned nb = (unsigned)((bj.nblk + kT / BS - 1) / (kT / BS));
    k_bj_rows_batch<<<nb, kT, 0, s>>>(bj, v, z);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

}  // namespace rbf

using namespace rbf;

extern "C" int rbf_pc_block_jacobi(rbf_plan *plan, double reg) {
    if (!plan) { set_error("rbf_pc_block_jacobi: null plan"); return RBF_EINVAL; }
    RBF_TRY(reject_eval_plan(plan, "rbf_pc_block_jacobi"));
    if (!std::isfinite(reg)) { set_error("rbf_pc_block_jacobi: reg must be finite"); return RBF_EINVAL; }
    return build_bj(plan, reg < 0 ? kDefaultBjReg * phi_zero(plan) : reg);
}

extern "C" int rbf_pc_learned_features(rbf_plan *plan, double reg) {
    if (!plan) { set_error("rbf_pc_learned_features: null plan"); return RBF_EINVAL; }
    RBF_TRY(reject_eval_plan(plan, "rbf_pc_learned_features"));
    if (!std::isfinite(reg)) { set_error("rbf_pc_learned_features: reg must be finite"); return RBF_EINVAL; }
    return build_lp(plan, reg < 0 ? kDefaultLpReg * phi_zero(plan) : reg);
}

extern "C" int rbf_pc_apply(rbf_plan *plan, int kind, const double *v, double *z) {
    if (!plan || !v || !z) { set_error("rbf_pc_apply: null argument"); return RBF_EINVAL; }
    RBF_TRY(reject_eval_plan(plan, "rbf_pc_apply"));
    if (kind != RBF_PC_BLOCK_JACOBI && kind != RBF_PC_LEARNED) {
        set_error("rbf_pc_apply: kind must be RBF_PC_BLOCK_JACOBI or RBF_PC_LEARNED");
        return RBF_EINVAL;
    }
    RBF_TRY(pc_ready(plan, kind));
    return pc_apply(plan, kind, v, z);
}

extern "C" int rbf_pc_set_learned(rbf_plan *plan, rbf_mlp *mlp) {
    if (!plan) { set_error("rbf_pc_set_learned: null plan"); return RBF_EINVAL; }
    plan->mlp = mlp;
    return RBF_OK;
}

extern "C" int rbf_pc_pairs(rbf_plan *plan, const double *r, const double *e, float *x, float *t, float *w) {
    if (!plan || !r || !e || !x || !t || !w) { set_error("rbf_pc_pairs: null argument"); return RBF_EINVAL; }
    RBF_TRY(reject_eval_plan(plan, "rbf_pc_pairs"));
    if (plan->lp_reg < 0) RBF_TRY(build_lp(plan, kDefaultLpReg * phi_zero(plan)));
    hipStream_t s = plan->stream;
    k_dot_self<<<1, kT, 0, s>>>(e, plan->n, plan->pc_scal);
    const unsigned nb = (unsigned)((plan->nblk + kT / BS - 1) / (kT / BS));
    k_pc_pairs<<<nb, kT, 0, s>>>(plan->lp_inv, plan->perm, plan->n, plan->nblk, r, e, plan->pc_scal, x, t, w);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

extern "C" int rbf_pc_harvest(rbf_plan *plan, const void *f, double rtol, int max_iters, int precond,
                              const int *caps, int ncaps, float *x, float *t, float *w) {
    if (!plan || !f || !caps || ncaps <= 0 || !x || !t || !w) {
        set_error("rbf_pc_harvest: bad arguments");
        return RBF_EINVAL;
    }
    RBF_TRY(reject_eval_plan(plan, "rbf_pc_harvest"));
    if (precond != RBF_PC_NONE && precond != RBF_PC_BLOCK_JACOBI) {
        set_error("rbf_pc_harvest: the harvesting solves run without a preconditioner or with block-Jacobi");
        return RBF_EINVAL;
    }
    for (int c = 0; c < ncaps; ++c)
        if (caps[c] < 0) { set_error("rbf_pc_harvest: caps must be >= 0"); return RBF_EINVAL; }
    RBF_TRY(pc_ready(plan, precond));
    if (plan->lp_reg < 0) RBF_TRY(build_lp(plan, kDefaultLpReg * phi_zero(plan)));
    const int64_t n = plan->n;
    const size_t tsz = plan->dtype == RBF_F32 ? 4 : 8;
    hipStream_t s = plan->stream;
    // lam*, lam_k (plan dtype), e and r (FP64), and the F32 in/out pair of the product
    Arena tmp;
    void *lstar = nullptr, *lk = nullptr, *pbuf = nullptr;
    double *e64 = nullptr, *r64 = nullptr;
    int rc = RBF_OK;
    if ((rc = tmp.alloc(&lstar, tsz * n)) != RBF_OK || (rc = tmp.alloc(&lk, tsz * n)) != RBF_OK ||
        (rc = tmp.alloc(&pbuf, 2 * sizeof(float) * n)) != RBF_OK ||
        (rc = tmp.alloc((void **)&e64, sizeof(double) * n)) != RBF_OK ||
        (rc = tmp.alloc((void **)&r64, sizeof(double) * n)) != RBF_OK) {
        tmp.release();
        return rc;
    }
    rbf_solve_opts o;
    std::memset(&o, 0, sizeof(o));
    o.restart = 50;
    o.max_iters = max_iters > 0 ? max_iters : 1000;
    o.precond = precond;
    o.zero_init = 1;
    o.fallback = 1;
    rbf_solve_info inf;
    rc = rbf_interp_solve(plan, f, lstar, rtol, &o, &inf);
    if (rc == RBF_ENOCONV) rc = RBF_OK;
    const unsigned nbk = (unsigned)((plan->nblk + kT / BS - 1) / (kT / BS));
    double *en = plan->pc_scal;
    for (int c = 0; c < ncaps && rc == RBF_OK; ++c) {
        if (caps[c] == 0) {
            RBF_HIP(hipMemsetAsync(lk, 0, tsz * n, s));
        } else {
            o.max_iters = caps[c];
            rc = rbf_interp_solve(plan, f, lk, 1e-15, &o, &inf);   // runs to the cap
            if (rc == RBF_ENOCONV) rc = RBF_OK;
            if (rc != RBF_OK) break;
        }
        if (plan->dtype == RBF_F32)
            k_diff64<float><<<grid_of(n), kT, 0, s>>>((const float *)lstar, (const float *)lk, e64, n);
        else
            k_diff64<double><<<grid_of(n), kT, 0, s>>>((const double *)lstar, (const double *)lk, e64, n);
        if (hipGetLastError() != hipSuccess) { set_error("rbf_pc_harvest: launch failed"); rc = RBF_EHIP; break; }
        if ((rc = product64(plan, e64, r64, pbuf)) != RBF_OK) break;
        k_dot_self<<<1, kT, 0, s>>>(e64, n, en);
        k_pc_pairs<<<nbk, kT, 0, s>>>(plan->lp_inv, plan->perm, n, plan->nblk, r64, e64, en,
                                      x + (int64_t)c * plan->nblk * BS, t + (int64_t)c * plan->nblk * BS,
                                      w + (int64_t)c * plan->nblk);
        if (hipGetLastError() != hipSuccess) { set_error("rbf_pc_harvest: launch failed"); rc = RBF_EHIP; break; }
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == RBF_OK) {
        set_error("rbf_pc_harvest: device error");
        rc = RBF_EHIP;
    }
    tmp.release();
    return rc;
}

extern "C" int rbf_pc_train(rbf_plan *const *plans, const void *const *fs, int nplans, double rtol, int max_iters,
                            const int *caps, int ncaps, uint64_t seed, const rbf_train_opts *opts,
                            const char *out_path, rbf_train_info *info) {
    if (!plans || !fs || nplans <= 0 || !out_path) {
        set_error("rbf_pc_train: bad arguments");
        return RBF_EINVAL;
    }
    static const int kCaps[] = {0, 1, 2, 5, 10, 20, 50, 100, 200};
    if (!caps) {
        caps = kCaps;
        ncaps = (int)(sizeof(kCaps) / sizeof(kCaps[0]));
    }
    if (ncaps <= 0) { set_error("rbf_pc_train: ncaps must be positive"); return RBF_EINVAL; }
    int64_t rows = 0;
    for (int q = 0; q < nplans; ++q) {
        if (!plans[q] || !fs[q]) { set_error("rbf_pc_train: null plan or right-hand side %d", q); return RBF_EINVAL; }
        rows += (int64_t)ncaps * ((plans[q]->n + BS - 1) / BS);
    }
    // every plan's rows, one after the other (plan order, then cap order), in one buffer
    Arena tmp;
    float *x = nullptr, *t = nullptr, *w = nullptr;
    int rc = RBF_OK;
    if ((rc = tmp.alloc((void **)&x, sizeof(float) * rows * BS)) != RBF_OK ||
        (rc = tmp.alloc((void **)&t, sizeof(float) * rows * BS)) != RBF_OK ||
        (rc = tmp.alloc((void **)&w, sizeof(float) * rows)) != RBF_OK) {
        tmp.release();
        return rc;
    }
    int64_t at = 0;
    for (int q = 0; q < nplans && rc == RBF_OK; ++q) {
        rc = rbf_pc_harvest(plans[q], fs[q], rtol, max_iters, RBF_PC_NONE, caps, ncaps, x + at * BS, t + at * BS,
                            w + at);
        at += (int64_t)ncaps * ((plans[q]->n + BS - 1) / BS);
    }
    rbf_mlp *m = nullptr;
    if (rc == RBF_OK) rc = rbf_mlp_create(nullptr, seed, &m);
    if (rc == RBF_OK) rc = rbf_mlp_train(m, x, t, w, rows, opts, plans[0]->stream, info);
    if (rc == RBF_OK) rc = rbf_mlp_save(m, out_path);
    if (m) (void)rbf_mlp_destroy(m);
    tmp.release();
    return rc;
}

extern "C" int rbf_pc_load(rbf_plan *plan, const char *path, rbf_mlp **out) {
    if (!plan || !path || !out) { set_error("rbf_pc_load: null argument"); return RBF_EINVAL; }
    RBF_TRY(reject_eval_plan(plan, "rbf_pc_load"));
    RBF_TRY(check_learned_kernel(plan));
    rbf_mlp *m = nullptr;
    RBF_TRY(rbf_mlp_load(path, &m));
    const int rc = rbf_pc_set_learned(plan, m);
    if (rc != RBF_OK) {
        (void)rbf_mlp_destroy(m);
        return rc;
    }
    *out = m;
    return RBF_OK;
}
