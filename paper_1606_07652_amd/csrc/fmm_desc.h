// Per-problem descriptor of the fast product: everything a kernel body reads, as plain
// pointers and scalars, so that one problem or many (a batch) can be launched alike.
#pragma once
#include "internal.h"

namespace rbf {

enum Phase {
    PH_GATHER = 0,
    PH_P2P,
    PH_PHASE_DL,
    PH_P2M,
    PH_M2M,
    PH_M2L_AXIS,
    PH_M2L_LEAF,
    PH_L2P,
    PH_DIRECT,
    PH_COUNT
};

template <class T> struct Desc {
    using C = typename cplx<T>::type;
    const T *xs;            // sorted coordinates, SoA [d][n]
    int64_t n;
    int64_t off;            // offset of this problem in the caller's (concatenated) vectors
    const int *perm, *leaf_begin, *leaf_cell, *near_ptr, *near_idx, *src_ptr, *cell_begin;
    const int *src_end;     // end of each leaf's sources (leaf_begin + 1 unless targets are separate)
    const int2 *src_rng, *tasks, *ptasks;
    int nleaves, ntasks, nptasks;
    int64_t ncells;
    int lc, r;
    int mn, H, HP, R;
    int64_t P;
    double xi0, xiH, dxi;
    const double *wc1;
    T coef;
    T *lam_s, *u_s;
    C *W, *Lx, *Wc, *Lc, *Tmp, *dl;
    int wpl;                // aggregation workgroups per leaf
    int p2m_ch;             // aggregation point chunk
    int far;                // 0: every kept pair is near (no far-field phases)
    const double *wtab;     // w(xi) C(xi) per stored node [P]
    int m2l_sched;          // block order of the leaf translation
    int dim;                // spatial dimension d
    int ngroups;            // sibling groups of the leaf translation
    const int *grp_first, *uni_ptr, *uni_idx, *uni_mask;
    int p2m_lds;            // dynamic LDS bytes of the aggregation kernel
    unsigned mn_magic;      // floor(2^32 / mn) + 1: r / mn = (r * mn_magic) >> 32 for r < 2^22
    // aggregation units: point ranges [p2m_begin[a], p2m_end[a]) written to W[a]
    // (the leaves' sources, or a band's chunks)
    const int *p2m_begin, *p2m_end;
    int p2m_n;
    int l2p_acc;            // 1: the disaggregation adds its far field to u_s (sorted order)
    const double *res_tab;  // residual near-field kernel: polynomial pieces in b [kResCoefs]
    double res_inv;         // pieces per unit of b
    double res_cut2;        // r^2 from which the residual is zero (qmax)
    int *p2p_ctr;           // near-field work queue: per-XCD task counters, kCtrStride ints apart
    int64_t dir_t0, dir_ns; // direct kernel: targets [dir_t0, n), sources [0, dir_ns) of the sorted
                            // points (0 and n, or a one-leaf plan's separate targets and sources)
    int bl_lds;             // band-limited Gaussian: 1 = the direct kernel copies the table (pieces
                            // only, in T) into its dynamic LDS, which the launch sizes for it
};

template <class T> void fill_desc(const rbf_plan *p, Desc<T> *d);
template <class T> void set_p2m_shape(Desc<T> *d, int dim, int64_t R, int mn, int HP);
template <class T> int64_t desc_blocks(const Desc<T> &d, int phase);
template <class T>
int launch_batch_group(int d, int HP, int kernel, const Desc<T> *descs, int nprob, const int *const *bstarts,
                       const int64_t *nblocks, size_t p2m_sh, const T *lam, T *u, hipStream_t s);

}  // namespace rbf
