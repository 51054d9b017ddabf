// Tree build on the device: bounding cube, quantisation, Morton keys, stable radix
// sort, adaptive boxes level by level, leaves, coarse cells and near lists.
//
// The paper's first FMM step is a hierarchical partition of the domain into groups with
// neighbour groups (section 1, list of FMM steps; section 4, eq. 38).  Definitions used
// here (identical on the CPU reference, so the result can be compared bit for bit):
//  * root cube: lo_k = min x_k, ext = max_k (max x_k - lo_k) (FP64; 1 if degenerate);
//  * q_k = min(floor((x_k - lo_k) * (2^B / ext)), 2^B - 1) in FP64, B = floor(63 / d);
//  * key bit b*d + k = bit b of q_k; stable sort by key;
//  * box at level l = key prefix >> d (B - l); a box exists if its parent is split; it is
//    split if l < maxlev and (l < min_level or count > n_max); unsplit boxes are leaves;
//  * near list of a leaf: every leaf whose closed box meets its closed box.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace rbf {
namespace {

constexpr int kThreads = 256;

template <class T>
__global__ void k_bbox(const T *x, int64_t n, int d, double *part) {
    __shared__ double smin[kThreads * kMaxDim];
    __shared__ double smax[kThreads * kMaxDim];
    double mn[kMaxDim], mx[kMaxDim];
    for (int k = 0; k < d; ++k) { mn[k] = INFINITY; mx[k] = -INFINITY; }
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        for (int k = 0; k < d; ++k) {
            double v = (double)x[i * d + k];
            mn[k] = fmin(mn[k], v);
            mx[k] = fmax(mx[k], v);
        }
    }
    for (int k = 0; k < d; ++k) {
        smin[k * kThreads + threadIdx.x] = mn[k];
        smax[k * kThreads + threadIdx.x] = mx[k];
    }
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int k = 0; k < d; ++k) {
                smin[k * kThreads + threadIdx.x] =
                    fmin(smin[k * kThreads + threadIdx.x], smin[k * kThreads + threadIdx.x + s]);
                smax[k * kThreads + threadIdx.x] =
                    fmax(smax[k * kThreads + threadIdx.x], smax[k * kThreads + threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < d; ++k) {
            part[(blockIdx.x * 2) * kMaxDim + k] = smin[k * kThreads];
            part[(blockIdx.x * 2 + 1) * kMaxDim + k] = smax[k * kThreads];
        }
    }
}

struct QuantArgs {
    double lo[kMaxDim];
    double scale;
    int64_t qmax;
};

template <class T, int D>
__global__ void k_keys(const T *x, int64_t n, QuantArgs qa, int B, uint64_t *keys, int *idx) {
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i >= n) return;
    uint64_t q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double t = (double)x[i * D + k] - qa.lo[k];
        double v = t * qa.scale;
        int64_t qi = (int64_t)floor(v);
        qi = qi < 0 ? 0 : (qi > qa.qmax ? qa.qmax : qi);
        q[k] = (uint64_t)qi;
    }
    uint64_t key = 0;
    for (int b = 0; b < B; ++b) {
#pragma unroll
        for (int k = 0; k < D; ++k) key |= ((q[k] >> b) & 1ull) << (b * D + k);
    }
    keys[i] = key;
    idx[i] = (int)i;
}

// ---- stable LSD radix sort of (key, index), 8-bit digits -------------------------------
constexpr int kSortTile = 4096;

__global__ void __launch_bounds__(kThreads) k_radix_hist(const uint64_t *keys, int n, int shift, int nblocks,
                                                         int *counts) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kSortTile;
    for (int t = threadIdx.x; t < kSortTile; t += kThreads) {
        int i = base + t;
        if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & 255ull)], 1);
    }
    __syncthreads();
    counts[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kThreads) k_radix_scatter(const uint64_t *kin, const int *vin, uint64_t *kout,
                                                            int *vout, int n, int shift, int nblocks,
                                                            const int *offsets) {
    __shared__ int base[256];
    __shared__ int run[256];
    __shared__ int wcnt[kThreads / kWave][256];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    base[threadIdx.x] = offsets[threadIdx.x * nblocks + blockIdx.x];
    run[threadIdx.x] = 0;
    for (int w = 0; w < kThreads / kWave; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const uint64_t gt = (lane == 63) ? 0ull : ((~0ull) << (lane + 1));
    const int tile0 = blockIdx.x * kSortTile;
    for (int c = 0; c < kSortTile; c += kThreads) {
        int i = tile0 + c + threadIdx.x;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0ull;
        int val = valid ? vin[i] : 0;
        int dig = (int)((key >> shift) & 255ull);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            int bit = (dig >> b) & 1;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        int rank = __popcll(peers & lt);
        if (valid && (peers & gt) == 0) wcnt[wave][dig] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pre = 0;
            for (int w = 0; w < wave; ++w) pre += wcnt[w][dig];
            int dst = base[dig] + run[dig] + pre + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        int tot = 0;
        for (int w = 0; w < kThreads / kWave; ++w) {
            tot += wcnt[w][threadIdx.x];
            wcnt[w][threadIdx.x] = 0;
        }
        run[threadIdx.x] += tot;
        __syncthreads();
    }
}

int radix_sort(uint64_t *keys, int *vals, int n, int nbits, hipStream_t s) {
    int nblocks = (n + kSortTile - 1) / kSortTile;
    uint64_t *k2 = nullptr;
    int *v2 = nullptr, *counts = nullptr;
    RBF_HIP(hipMalloc(&k2, sizeof(uint64_t) * (size_t)n));
    RBF_HIP(hipMalloc(&v2, sizeof(int) * (size_t)n));
    RBF_HIP(hipMalloc(&counts, sizeof(int) * 256 * (size_t)nblocks));
    uint64_t *ka = keys, *kb = k2;
    int *va = vals, *vb = v2;
    int passes = (nbits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        k_radix_hist<<<nblocks, kThreads, 0, s>>>(ka, n, shift, nblocks, counts);
        RBF_HIP(hipGetLastError());
        RBF_TRY(exclusive_scan_i32(counts, counts, 256 * nblocks, nullptr, s));
        k_radix_scatter<<<nblocks, kThreads, 0, s>>>(ka, va, kb, vb, n, shift, nblocks, counts);
        RBF_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        RBF_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
        RBF_HIP(hipMemcpyAsync(vals, va, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, s));
    }
    RBF_HIP(hipStreamSynchronize(s));
    RBF_HIP(hipFree(k2));
    RBF_HIP(hipFree(v2));
    RBF_HIP(hipFree(counts));
    return RBF_OK;
}

// ---- levels --------------------------------------------------------------------------
__global__ void k_heads(const uint64_t *keys, int n, int shift, int *head) {
    int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    head[i] = (i == 0) ? 1 : ((keys[i] >> shift) != (keys[i - 1] >> shift));
}

__global__ void k_boxes(const int *head, const int *ex, int n, int *box_start, int *box_of_point) {
    int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    int b = ex[i] + head[i] - 1;
    box_of_point[i] = b;
    if (head[i]) box_start[b] = i;
}

// A box splits while it holds more than nmax points; with separate targets (src_pre: prefix
// counts of sources in sorted order, else null) only its sources count.
__global__ void k_box_status(int nboxes, const int *box_start, int lev, int maxlev, int minlev, int nmax,
                             const int *src_pre, const int *bop_prev, const unsigned char *split_prev,
                             unsigned char *split, int *leafflag, int *leaflev, int *any_split) {
    int b = blockIdx.x * kThreads + threadIdx.x;
    if (b >= nboxes) return;
    int s = box_start[b];
    int cnt = src_pre ? src_pre[box_start[b + 1]] - src_pre[s] : box_start[b + 1] - s;
    int exists = (lev == 0) ? 1 : (int)split_prev[bop_prev[s]];
    int sp = exists && lev < maxlev && (lev < minlev || cnt > nmax);
    split[b] = (unsigned char)sp;
    if (exists && !sp) {
        leafflag[s] = 1;
        leaflev[s] = lev;
    }
    if (sp) atomicOr(any_split, 1);
}

__global__ void k_src_flag(const int *perm, int n, int64_t n_src, int *flag) {
    int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) flag[i] = perm[i] < n_src;
}

__global__ void k_leaves(const int *flag, const int *ex, const int *lev, const uint64_t *keys, int n, int d,
                         int B, int *leaf_begin, int *leaf_level, uint64_t *leaf_prefix, int *leaf_of_point) {
    int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    int a = ex[i] + flag[i] - 1;
    leaf_of_point[i] = a;
    if (flag[i]) {
        int l = lev[i];
        leaf_begin[a] = i;
        leaf_level[a] = l;
        int sh = d * (B - l);
        leaf_prefix[a] = sh >= 64 ? 0ull : (keys[i] >> sh);
    }
}

template <class T>
__global__ void k_gather_points(const T *x, const int *perm, int64_t n, int d, T *xs) {
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    for (int k = 0; k < d; ++k) xs[k * n + i] = x[j * d + k];
}

__global__ void k_leaf_cell(const uint64_t *prefix, const int *level, int nleaves, int d, int lc, int *cell) {
    int a = blockIdx.x * kThreads + threadIdx.x;
    if (a >= nleaves) return;
    cell[a] = (int)(prefix[a] >> (d * (level[a] - lc)));
}

__global__ void k_cell_begin(const int *cell, int nleaves, int64_t ncells, int *cell_begin) {
    int64_t c = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (c > ncells) return;
    int lo = 0, hi = nleaves;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cell[mid] < c) lo = mid + 1; else hi = mid;
    }
    cell_begin[c] = lo;
}

// ---- near lists ----------------------------------------------------------------------
__device__ __forceinline__ int lower_bound_u64(const uint64_t *a, int n, uint64_t v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <int D>
__device__ __forceinline__ void deinterleave(uint64_t prefix, int nbits, int64_t *c) {
#pragma unroll
    for (int k = 0; k < D; ++k) c[k] = 0;
    for (int b = 0; b < nbits; ++b) {
#pragma unroll
        for (int k = 0; k < D; ++k) c[k] |= (int64_t)((prefix >> (b * D + k)) & 1ull) << b;
    }
}

template <int D>
__device__ __forceinline__ uint64_t interleave(const int64_t *c, int nbits) {
    uint64_t key = 0;
    for (int b = 0; b < nbits; ++b) {
#pragma unroll
        for (int k = 0; k < D; ++k) key |= ((uint64_t)(c[k] >> b) & 1ull) << (b * D + k);
    }
    return key;
}

// FILL = false: count list lengths into cnt[a]; FILL = true: write lists at ptr[a].
template <int D, bool FILL>
__global__ void k_near(int nleaves, const uint64_t *keys, int n, int B, const int *leaf_of_point,
                       const int *leaf_level, const uint64_t *leaf_prefix, const int *ptr, int *cnt,
                       int *out) {
    int a = blockIdx.x * kThreads + threadIdx.x;
    if (a >= nleaves) return;
    const int la = leaf_level[a];
    int64_t ca[D];
    deinterleave<D>(leaf_prefix[a], la, ca);
    const int64_t side = (int64_t)1 << la;
    const int64_t sa = (int64_t)1 << (B - la);
    int64_t loa[D], hia[D];
#pragma unroll
    for (int k = 0; k < D; ++k) { loa[k] = ca[k] * sa; hia[k] = loa[k] + sa; }
    int count = 0;
    int *dst = FILL ? out + ptr[a] : nullptr;
    int noff = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) noff *= 3;
    for (int o = 0; o < noff; ++o) {
        int64_t nc[D];
        bool inside = true;
        int t = o;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            nc[k] = ca[k] + (t % 3) - 1;
            t /= 3;
            inside = inside && nc[k] >= 0 && nc[k] < side;
        }
        if (!inside) continue;
        const int sh = D * (B - la);
        uint64_t pf = interleave<D>(nc, la);
        uint64_t k0 = pf << sh;
        uint64_t k1 = (pf + 1) << sh;
        int i0 = lower_bound_u64(keys, n, k0);
        const bool nonempty = (i0 < n && keys[i0] < k1);
        int lb = -1;
        if (nonempty) {
            lb = leaf_of_point[i0];
        } else {
            // an empty cell can still lie inside a coarser leaf: walk up to the first
            // ancestor that holds points; it is inside a leaf iff that leaf is not finer
            for (int l = la - 1; l >= 0; --l) {
                const int sh2 = D * (B - l);
                uint64_t pa = pf >> (D * (la - l));
                int j0 = lower_bound_u64(keys, n, pa << sh2);
                if (j0 < n && keys[j0] < ((pa + 1) << sh2)) {
                    int cand = leaf_of_point[j0];
                    if (leaf_level[cand] <= l) lb = cand;
                    break;
                }
            }
            if (lb < 0) continue;
        }
        int lbl = leaf_level[lb];
        if (lbl <= la) {
            // a coarser (or equal) leaf covers this cell; count it at its first covering offset
            int64_t cb[D];
            deinterleave<D>(leaf_prefix[lb], lbl, cb);
            bool first = true;
            for (int o2 = 0; o2 < o && first; ++o2) {
                int t2 = o2;
                bool in2 = true, cov = true;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    int64_t c2 = ca[k] + (t2 % 3) - 1;
                    t2 /= 3;
                    in2 = in2 && c2 >= 0 && c2 < side;
                    cov = cov && ((c2 >> (la - lbl)) == cb[k]);
                }
                if (in2 && cov) first = false;
            }
            if (first) {
                if (FILL) dst[count] = lb;
                ++count;
            }
        } else {
            int i1 = lower_bound_u64(keys, n, k1);
            int le = leaf_of_point[i1 - 1];
            for (int b = lb; b <= le; ++b) {
                int lv = leaf_level[b];
                int64_t cb[D];
                deinterleave<D>(leaf_prefix[b], lv, cb);
                const int64_t sb = (int64_t)1 << (B - lv);
                bool touch = true;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    int64_t lob = cb[k] * sb, hib = lob + sb;
                    touch = touch && (lob <= hia[k]) && (loa[k] <= hib);
                }
                if (touch) {
                    if (FILL) dst[count] = b;
                    ++count;
                }
            }
        }
    }
    if (FILL) {
        for (int i = 1; i < count; ++i) {
            int v = dst[i], j = i - 1;
            while (j >= 0 && dst[j] > v) { dst[j + 1] = dst[j]; --j; }
            dst[j + 1] = v;
        }
    } else {
        cnt[a] = count;
    }
}

// Merge consecutive near leaves into point ranges for the near-field kernel.
// A leaf's sources are [leaf_begin[b], src_end[b]); near leaves b, b + 1 merge into one range
// when b has no points after its sources.
template <bool FILL>
__global__ void k_ranges(int nleaves, const int *near_ptr, const int *near_idx, const int *leaf_begin,
                         const int *src_end, const int *rptr, int *rcnt, int2 *rng, int *npairs_part) {
    int a = blockIdx.x * kThreads + threadIdx.x;
    if (a >= nleaves) return;
    int c = 0, total = 0;
    int b0 = -1, b1 = -1;
    for (int e = near_ptr[a]; e < near_ptr[a + 1]; ++e) {
        int b = near_idx[e];
        if (b0 >= 0 && b == b1 + 1 && src_end[b1] == leaf_begin[b]) { b1 = b; continue; }
        if (b0 >= 0) {
            if (FILL) rng[rptr[a] + c] = make_int2(leaf_begin[b0], src_end[b1]);
            total += src_end[b1] - leaf_begin[b0];
            ++c;
        }
        b0 = b1 = b;
    }
    if (b0 >= 0) {
        if (FILL) rng[rptr[a] + c] = make_int2(leaf_begin[b0], src_end[b1]);
        total += src_end[b1] - leaf_begin[b0];
        ++c;
    }
    if (!FILL) {
        rcnt[a] = c;
        npairs_part[a] = total;
    }
}

// targets of leaf a: [tgt_begin[a], leaf_begin[a + 1])
__global__ void k_pairs(int nleaves, const int *leaf_begin, const int *tgt_begin, const int *src_total,
                        unsigned long long *acc) {
    int a = blockIdx.x * kThreads + threadIdx.x;
    if (a >= nleaves) return;
    unsigned long long v = (unsigned long long)(leaf_begin[a + 1] - tgt_begin[a]) * (unsigned long long)src_total[a];
    atomicAdd(acc, v);
}

template <class T>
int bbox_typed(rbf_plan *p, const void *points_v) {
    const T *pts = (const T *)points_v;
    const int d = p->d;
    hipStream_t s = p->stream;
    int nbb = (int)std::min<int64_t>(1024, (p->n + kThreads - 1) / kThreads);
    double *part = nullptr;
    RBF_HIP(hipMalloc(&part, sizeof(double) * 2 * kMaxDim * nbb));
    k_bbox<T><<<nbb, kThreads, 0, s>>>(pts, p->n, d, part);
    RBF_HIP(hipGetLastError());
    std::vector<double> hp((size_t)2 * kMaxDim * nbb);
    RBF_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    RBF_HIP(hipFree(part));
    double lo[kMaxDim], hi[kMaxDim];
    for (int k = 0; k < d; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int b = 0; b < nbb; ++b)
        for (int k = 0; k < d; ++k) {
            lo[k] = std::min(lo[k], hp[(b * 2) * kMaxDim + k]);
            hi[k] = std::max(hi[k], hp[(b * 2 + 1) * kMaxDim + k]);
        }
    double ext = 0.0;
    for (int k = 0; k < d; ++k) ext = std::max(ext, hi[k] - lo[k]);
    if (!std::isfinite(ext)) {
        set_error("rbf_fmm_plan: non-finite point coordinates");
        return RBF_EINVAL;
    }
    if (!(ext > 0.0)) ext = 1.0;
    p->ext = ext;
    for (int k = 0; k < d; ++k) p->lo[k] = lo[k];
    p->B = 63 / d;
    return RBF_OK;
}

template <class T>
int tree_typed(rbf_plan *p, const void *points_v) {
    const T *pts = (const T *)points_v;
    const int n = (int)p->n, d = p->d;
    hipStream_t s = p->stream;
    const int B = p->B;
    const double ext = p->ext;
    QuantArgs qa;
    for (int k = 0; k < kMaxDim; ++k) qa.lo[k] = k < d ? p->lo[k] : 0.0;
    qa.scale = std::ldexp(1.0, B) / ext;
    qa.qmax = ((int64_t)1 << B) - 1;

    Arena &ar = p->arena;
    RBF_TRY(ar.alloc((void **)&p->keys, sizeof(uint64_t) * n));
    RBF_TRY(ar.alloc((void **)&p->perm, sizeof(int) * n));
    int nbl = (n + kThreads - 1) / kThreads;
    switch (d) {
        case 2: k_keys<T, 2><<<nbl, kThreads, 0, s>>>(pts, n, qa, B, p->keys, p->perm); break;
        case 3: k_keys<T, 3><<<nbl, kThreads, 0, s>>>(pts, n, qa, B, p->keys, p->perm); break;
        case 5: k_keys<T, 5><<<nbl, kThreads, 0, s>>>(pts, n, qa, B, p->keys, p->perm); break;
        default: set_error("dimension %d not compiled", d); return RBF_EUNSUPPORTED;
    }
    RBF_HIP(hipGetLastError());
    RBF_TRY(radix_sort(p->keys, p->perm, n, d * B, s));

    // sorted coordinates
    RBF_TRY(ar.alloc(&p->xs, sizeof(T) * (size_t)n * d));
    k_gather_points<T><<<nbl, kThreads, 0, s>>>(pts, p->perm, n, d, (T *)p->xs);
    RBF_HIP(hipGetLastError());

    // levels
    int *head = nullptr, *ex = nullptr, *bstart = nullptr, *bop[2] = {nullptr, nullptr};
    unsigned char *spl[2] = {nullptr, nullptr};
    int *leafflag = nullptr, *leaflev = nullptr, *anysplit = nullptr;
    RBF_HIP(hipMalloc(&head, sizeof(int) * n));
    RBF_HIP(hipMalloc(&ex, sizeof(int) * n));
    RBF_HIP(hipMalloc(&bstart, sizeof(int) * (n + 1)));
    RBF_HIP(hipMalloc(&bop[0], sizeof(int) * n));
    RBF_HIP(hipMalloc(&bop[1], sizeof(int) * n));
    RBF_HIP(hipMalloc(&spl[0], n));
    RBF_HIP(hipMalloc(&spl[1], n));
    RBF_HIP(hipMalloc(&leafflag, sizeof(int) * n));
    RBF_HIP(hipMalloc(&leaflev, sizeof(int) * n));
    RBF_HIP(hipMalloc(&anysplit, sizeof(int)));
    RBF_HIP(hipMemsetAsync(leafflag, 0, sizeof(int) * n, s));
    int *srcpre = nullptr;   // separate targets: prefix counts of sources in sorted order [n + 1]
    if (p->n_src > 0) {
        RBF_HIP(hipMalloc(&srcpre, sizeof(int) * (n + 1)));
        k_src_flag<<<nbl, kThreads, 0, s>>>(p->perm, n, p->n_src, head);
        RBF_HIP(hipGetLastError());
        int ns = 0;
        RBF_TRY(exclusive_scan_i32(head, srcpre, n, &ns, s));
        RBF_HIP(hipMemcpyAsync(srcpre + n, &ns, sizeof(int), hipMemcpyHostToDevice, s));
        RBF_HIP(hipStreamSynchronize(s));   // ns is read by the copy
    }
    const int maxlev = std::min(p->max_level, B);
    int cur = 0, lev = 0, nlev = 0;
    for (lev = 0; lev <= maxlev; ++lev) {
        k_heads<<<nbl, kThreads, 0, s>>>(p->keys, n, d * (B - lev), head);
        RBF_HIP(hipGetLastError());
        int nboxes = 0;
        RBF_TRY(exclusive_scan_i32(head, ex, n, &nboxes, s));
        k_boxes<<<nbl, kThreads, 0, s>>>(head, ex, n, bstart, bop[cur]);
        RBF_HIP(hipGetLastError());
        RBF_HIP(hipMemcpyAsync(bstart + nboxes, &n, sizeof(int), hipMemcpyHostToDevice, s));
        RBF_HIP(hipMemsetAsync(anysplit, 0, sizeof(int), s));
        k_box_status<<<(nboxes + kThreads - 1) / kThreads, kThreads, 0, s>>>(
            nboxes, bstart, lev, maxlev, p->min_level, p->n_max, srcpre, bop[cur ^ 1], spl[cur ^ 1], spl[cur],
            leafflag, leaflev, anysplit);
        RBF_HIP(hipGetLastError());
        int hs = 0;
        RBF_HIP(hipMemcpyAsync(&hs, anysplit, sizeof(int), hipMemcpyDeviceToHost, s));
        RBF_HIP(hipStreamSynchronize(s));
        nlev = lev + 1;
        cur ^= 1;
        if (!hs) break;
    }
    p->nlevels = nlev;
    int nleaves = 0;
    RBF_TRY(exclusive_scan_i32(leafflag, ex, n, &nleaves, s));
    p->nleaves = nleaves;
    RBF_TRY(ar.alloc((void **)&p->leaf_begin, sizeof(int) * (nleaves + 1)));
    RBF_TRY(ar.alloc((void **)&p->leaf_level, sizeof(int) * nleaves));
    RBF_TRY(ar.alloc((void **)&p->leaf_prefix, sizeof(uint64_t) * nleaves));
    RBF_TRY(ar.alloc((void **)&p->leaf_cell, sizeof(int) * nleaves));
    int *leaf_of_point = head;  // reuse
    k_leaves<<<nbl, kThreads, 0, s>>>(leafflag, ex, leaflev, p->keys, n, d, B, p->leaf_begin, p->leaf_level,
                                      p->leaf_prefix, leaf_of_point);
    RBF_HIP(hipGetLastError());
    RBF_HIP(hipMemcpyAsync(p->leaf_begin + nleaves, &n, sizeof(int), hipMemcpyHostToDevice, s));

    // coarse cells
    p->ncells = (int64_t)1 << (d * p->lc);
    k_leaf_cell<<<(nleaves + kThreads - 1) / kThreads, kThreads, 0, s>>>(p->leaf_prefix, p->leaf_level, nleaves,
                                                                         d, p->lc, p->leaf_cell);
    RBF_HIP(hipGetLastError());
    RBF_TRY(ar.alloc((void **)&p->cell_leaf_begin, sizeof(int) * (p->ncells + 1)));
    k_cell_begin<<<(int)((p->ncells + 1 + kThreads - 1) / kThreads), kThreads, 0, s>>>(p->leaf_cell, nleaves,
                                                                                       p->ncells, p->cell_leaf_begin);
    RBF_HIP(hipGetLastError());

    // near lists
    int *cnt = ex;  // reuse (nleaves <= n)
    int nlb = (nleaves + kThreads - 1) / kThreads;
    RBF_TRY(ar.alloc((void **)&p->near_ptr, sizeof(int) * (nleaves + 1)));
#define NEAR_LAUNCH(DD, F, PTR, CNT, OUT)                                                                  \
    k_near<DD, F><<<nlb, kThreads, 0, s>>>(nleaves, p->keys, n, B, leaf_of_point, p->leaf_level, p->leaf_prefix, \
                                          PTR, CNT, OUT)
    switch (d) {
        case 2: NEAR_LAUNCH(2, false, nullptr, cnt, nullptr); break;
        case 3: NEAR_LAUNCH(3, false, nullptr, cnt, nullptr); break;
        case 5: NEAR_LAUNCH(5, false, nullptr, cnt, nullptr); break;
    }
    RBF_HIP(hipGetLastError());
    int nnear = 0;
    RBF_TRY(exclusive_scan_i32(cnt, p->near_ptr, nleaves, &nnear, s));
    RBF_HIP(hipMemcpyAsync(p->near_ptr + nleaves, &nnear, sizeof(int), hipMemcpyHostToDevice, s));
    p->nnear = nnear;
    RBF_TRY(ar.alloc((void **)&p->near_idx, sizeof(int) * std::max(nnear, 1)));
    switch (d) {
        case 2: NEAR_LAUNCH(2, true, p->near_ptr, nullptr, p->near_idx); break;
        case 3: NEAR_LAUNCH(3, true, p->near_ptr, nullptr, p->near_idx); break;
        case 5: NEAR_LAUNCH(5, true, p->near_ptr, nullptr, p->near_idx); break;
    }
#undef NEAR_LAUNCH
    RBF_HIP(hipGetLastError());

    // A plan for separate targets orders each leaf's points sources first, targets after (each
    // part keeps its Morton order), and records where the sources end.  The tree and the near
    // lists do not depend on the order inside a leaf.
    std::vector<int> hse;   // host copy of src_end (separate targets only)
    if (p->n_src > 0) {
        std::vector<int> hperm(n), hlb(nleaves + 1), np(n);
        RBF_HIP(hipMemcpyAsync(hperm.data(), p->perm, sizeof(int) * n, hipMemcpyDeviceToHost, s));
        RBF_HIP(hipMemcpyAsync(hlb.data(), p->leaf_begin, sizeof(int) * (nleaves + 1), hipMemcpyDeviceToHost, s));
        RBF_HIP(hipStreamSynchronize(s));
        hse.resize(nleaves);
        for (int a = 0; a < nleaves; ++a) {
            int o = hlb[a];
            for (int i = hlb[a]; i < hlb[a + 1]; ++i)
                if (hperm[i] < p->n_src) np[o++] = hperm[i];
            hse[a] = o;
            for (int i = hlb[a]; i < hlb[a + 1]; ++i)
                if (hperm[i] >= p->n_src) np[o++] = hperm[i];
        }
        RBF_TRY(ar.alloc((void **)&p->src_end, sizeof(int) * nleaves));
        RBF_HIP(hipMemcpyAsync(p->src_end, hse.data(), sizeof(int) * nleaves, hipMemcpyHostToDevice, s));
        RBF_HIP(hipMemcpyAsync(p->perm, np.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
        k_gather_points<T><<<nbl, kThreads, 0, s>>>(pts, p->perm, n, d, (T *)p->xs);
        RBF_HIP(hipGetLastError());
        RBF_HIP(hipStreamSynchronize(s));   // np is freed at the end of this scope
    }
    const int *src_end = p->src_end ? p->src_end : p->leaf_begin + 1;
    const int *tgt_begin = p->src_end ? p->src_end : p->leaf_begin;

    // merged source ranges for the near field
    int *rcnt = leaflev;   // reuse
    int *ptot = leafflag;  // reuse
    k_ranges<false><<<nlb, kThreads, 0, s>>>(nleaves, p->near_ptr, p->near_idx, p->leaf_begin, src_end, nullptr,
                                             rcnt, nullptr, ptot);
    RBF_HIP(hipGetLastError());
    unsigned long long *pacc = nullptr;
    RBF_HIP(hipMalloc(&pacc, sizeof(unsigned long long)));
    RBF_HIP(hipMemsetAsync(pacc, 0, sizeof(unsigned long long), s));
    k_pairs<<<nlb, kThreads, 0, s>>>(nleaves, p->leaf_begin, tgt_begin, ptot, pacc);
    RBF_HIP(hipGetLastError());
    unsigned long long npairs = 0;
    RBF_HIP(hipMemcpyAsync(&npairs, pacc, sizeof(npairs), hipMemcpyDeviceToHost, s));
    RBF_TRY(ar.alloc((void **)&p->src_ptr, sizeof(int) * (nleaves + 1)));
    int nr = 0;
    RBF_TRY(exclusive_scan_i32(rcnt, p->src_ptr, nleaves, &nr, s));
    RBF_HIP(hipMemcpyAsync(p->src_ptr + nleaves, &nr, sizeof(int), hipMemcpyHostToDevice, s));
    p->nranges = nr;
    p->near_pairs = (int64_t)npairs;
    RBF_TRY(ar.alloc((void **)&p->src_rng, sizeof(int2) * std::max(nr, 1)));
    k_ranges<true><<<nlb, kThreads, 0, s>>>(nleaves, p->near_ptr, p->near_idx, p->leaf_begin, src_end, p->src_ptr,
                                            nullptr, p->src_rng, nullptr);
    RBF_HIP(hipGetLastError());
    // wave tasks: (leaf, offset in the leaf) for every 64 consecutive targets of a leaf (all its
    // points, or with separate targets the part after src_end)
    {
        std::vector<int> hb(nleaves + 1), hl(nleaves);
        RBF_HIP(hipMemcpyAsync(hb.data(), p->leaf_begin, sizeof(int) * (nleaves + 1), hipMemcpyDeviceToHost, s));
        RBF_HIP(hipMemcpyAsync(hl.data(), p->leaf_level, sizeof(int) * nleaves, hipMemcpyDeviceToHost, s));
        RBF_HIP(hipStreamSynchronize(s));
        p->min_leaf_level = *std::min_element(hl.begin(), hl.end());
        p->max_leaf_level = *std::max_element(hl.begin(), hl.end());
        std::vector<int2> tk, pk;   // disaggregation tasks (offset in the leaf), near-field tasks
        tk.reserve(nleaves + n / kWave + 1);
        pk.reserve(nleaves + n / kWave + 1);
        for (int a = 0; a < nleaves; ++a) {
            const int t0 = p->n_src > 0 ? hse[a] : hb[a];
            for (int t = t0; t < hb[a + 1]; t += kWave) {
                tk.push_back(make_int2(a, t - hb[a]));
                pk.push_back(make_int2(a, t));
            }
        }
        p->ntasks = (int)tk.size();
        RBF_TRY(ar.alloc((void **)&p->tasks, sizeof(int2) * tk.size()));
        RBF_HIP(hipMemcpyAsync(p->tasks, tk.data(), sizeof(int2) * tk.size(), hipMemcpyHostToDevice, s));
        p->nptasks = (int)pk.size();
        RBF_TRY(ar.alloc((void **)&p->ptasks, sizeof(int2) * pk.size()));
        RBF_HIP(hipMemcpyAsync(p->ptasks, pk.data(), sizeof(int2) * pk.size(), hipMemcpyHostToDevice, s));
        RBF_HIP(hipStreamSynchronize(s));   // tk and pk are freed at the end of this scope
    }
    // sibling groups for the leaf translation
    {
        std::vector<int> hl(nleaves), np(nleaves + 1), ni((size_t)std::max(nnear, 1));
        std::vector<uint64_t> pf(nleaves);
        RBF_HIP(hipMemcpyAsync(hl.data(), p->leaf_level, sizeof(int) * nleaves, hipMemcpyDeviceToHost, s));
        RBF_HIP(hipMemcpyAsync(pf.data(), p->leaf_prefix, sizeof(uint64_t) * nleaves, hipMemcpyDeviceToHost, s));
        RBF_HIP(hipMemcpyAsync(np.data(), p->near_ptr, sizeof(int) * (nleaves + 1), hipMemcpyDeviceToHost, s));
        RBF_HIP(hipMemcpyAsync(ni.data(), p->near_idx, sizeof(int) * std::max(nnear, 1), hipMemcpyDeviceToHost, s));
        RBF_HIP(hipStreamSynchronize(s));
        std::vector<int> gf, up, ui, um;
        std::vector<std::pair<int, int>> ent;
        up.push_back(0);
        for (int a = 0; a < nleaves;) {
            int b = a + 1;
            while (b < nleaves && b - a < 8 && hl[b] == hl[a] && hl[a] > 0 &&
                   (pf[b] >> p->d) == (pf[a] >> p->d))
                ++b;
            gf.push_back(a);
            ent.clear();
            for (int c = a; c < b; ++c)
                for (int e = np[c]; e < np[c + 1]; ++e) ent.emplace_back(ni[e], 1 << (c - a));
            std::sort(ent.begin(), ent.end());
            const size_t u0 = ui.size();
            for (size_t k = 0; k < ent.size();) {
                int m = 0;
                size_t k2 = k;
                while (k2 < ent.size() && ent[k2].first == ent[k].first) m |= ent[k2++].second;
                ui.push_back(ent[k].first);
                um.push_back(m);
                k = k2;
            }
            // pad the group's list to a multiple of 8 entries (a repeat of its first leaf with
            // no members), so the kernel reads whole aligned steps of 8
            while ((ui.size() - u0) % 8 != 0) {
                ui.push_back(ui[u0]);
                um.push_back(0);
            }
            up.push_back((int)ui.size());
            a = b;
        }
        // one more step of 8 past the end: the kernel reads the step after its last one
        for (int k = 0; k < 8; ++k) {
            ui.push_back(0);
            um.push_back(0);
        }
        gf.push_back(nleaves);
        p->ngroups = (int)gf.size() - 1;
        p->nunion = (int64_t)ui.size() - 8;
        RBF_TRY(ar.alloc((void **)&p->grp_first, sizeof(int) * gf.size()));
        RBF_TRY(ar.alloc((void **)&p->uni_ptr, sizeof(int) * up.size()));
        RBF_TRY(ar.alloc((void **)&p->uni_idx, sizeof(int) * ui.size()));
        RBF_TRY(ar.alloc((void **)&p->uni_mask, sizeof(int) * um.size()));
        RBF_HIP(hipMemcpyAsync(p->grp_first, gf.data(), sizeof(int) * gf.size(), hipMemcpyHostToDevice, s));
        RBF_HIP(hipMemcpyAsync(p->uni_ptr, up.data(), sizeof(int) * up.size(), hipMemcpyHostToDevice, s));
        RBF_HIP(hipMemcpyAsync(p->uni_idx, ui.data(), sizeof(int) * ui.size(), hipMemcpyHostToDevice, s));
        RBF_HIP(hipMemcpyAsync(p->uni_mask, um.data(), sizeof(int) * um.size(), hipMemcpyHostToDevice, s));
        RBF_HIP(hipStreamSynchronize(s));
    }
    RBF_HIP(hipStreamSynchronize(s));
    RBF_HIP(hipFree(pacc));
    RBF_HIP(hipFree(head));
    RBF_HIP(hipFree(ex));
    RBF_HIP(hipFree(bstart));
    RBF_HIP(hipFree(bop[0]));
    RBF_HIP(hipFree(bop[1]));
    RBF_HIP(hipFree(spl[0]));
    RBF_HIP(hipFree(spl[1]));
    RBF_HIP(hipFree(leafflag));
    RBF_HIP(hipFree(leaflev));
    RBF_HIP(hipFree(anysplit));
    if (srcpre) RBF_HIP(hipFree(srcpre));
    return RBF_OK;
}

}  // namespace

int compute_bbox(rbf_plan *p, const void *points) {
    if (p->dtype == RBF_F32) return bbox_typed<float>(p, points);
    return bbox_typed<double>(p, points);
}

int build_tree(rbf_plan *p, const void *points) {
    if (p->dtype == RBF_F32) return tree_typed<float>(p, points);
    return tree_typed<double>(p, points);
}

}  // namespace rbf
