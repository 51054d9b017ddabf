// Many independent problems in one launch per phase, and a measuring autotuner.
//
// A batch owns one plan per problem (tree, tables and buffers as for a single plan) and
// groups the problems by their padded half grid HP (one kernel instantiation per group).
// For every phase a group launches one grid covering all of its problems: block g finds
// its problem by a binary search over the exclusive prefix of per-problem block counts.
// The whole product (all groups, all phases) is captured once into a HIP graph on the
// batch's own stream and replayed on every call; the graph is captured again only when
// the caller passes different vector pointers.
//
// The autotuner plans each candidate configuration (leaf capacity 64..512, a near-only
// tree whose cells are at least the pruning radius wide, and -- when nothing can be pruned
// -- a single leaf, i.e. the direct sum), times a few products with HIP events and keeps
// the fastest; for a Gaussian far field it then times the coarse levels next to the rule's
// with the best leaf capacity (each level has its own stencil reach and so its own node
// count per dimension) and the other leaf-translation block order.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch.h"

namespace rbf {
namespace {

int pow2i(int l) { return 1 << l; }

// Candidate configurations for the autotuner.
std::vector<rbf_opts> candidates(const rbf_opts *base, int64_t n, int d, int kernel, double shape, double tol,
                                 double ext) {
    std::vector<rbf_opts> out;
    rbf_opts o;
    std::memset(&o, 0, sizeof(o));
    if (base) o = *base;
    o.coarse_level = base ? base->coarse_level : -1;
    o.coarse_radius = base ? base->coarse_radius : -1;
    if (banded_kernel(kernel, d) && !o.exact) {
        // banded far field: the level of the near field's uniform tree around the default
        // (about 256 points per cell), and the exact sum when it stays small enough to time
        const int l0 = (int)std::floor(std::log2(std::max(1.0, (double)n / 256.0)) / d + 0.5);
        for (int l = std::max(1, l0 - 1); l <= std::min(l0 + 1, 18 / d); ++l) {
            rbf_opts c = o;
            c.coarse_level = l;
            out.push_back(c);
        }
        if (n <= (1 << 17)) {
            rbf_opts c = o;
            c.exact = 1;
            out.push_back(c);
        }
        return out;
    }
    for (int nm : {64, 128, 256, 512}) {
        rbf_opts c = o;
        c.n_max = nm;
        out.push_back(c);
        if (n <= nm) break;
    }
    // near-only: uniform tree at the deepest level whose cells are at least R_cut wide
    const double rcut = shape * std::sqrt(2.0 * std::log(4.0 / tol) + 1.0);
    int lstar = 0;
    while (lstar + 1 <= 18 / d && ext / pow2i(lstar + 1) >= rcut) ++lstar;
    if (lstar >= 1) {
        rbf_opts c = o;
        c.coarse_level = lstar;
        c.coarse_radius = 1;
        c.min_level = lstar;
        c.max_level = lstar;
        c.nodes = 4;
        c.n_max = 1 << 30;
        out.push_back(c);
    }
    // one leaf holding every point (the direct sum through the near-field kernel) when no
    // pair can be pruned and the sum stays small enough to time
    if (rcut >= 0.5 * ext && n <= (1 << 19)) {
        rbf_opts c = o;
        c.coarse_level = 0;
        c.coarse_radius = 0;
        c.min_level = 0;
        c.max_level = 0;
        c.nodes = 4;
        c.n_max = 1 << 30;
        out.push_back(c);
    }
    return out;
}

int bbox_ext(const void *points, int64_t n, int d, int dtype, hipStream_t s, double *ext) {
    // reuse the plan machinery: a one-point-per-leaf plan would be wasteful, so read back
    // the coordinates' extent with a tiny host reduction of a device copy
    const size_t tsz = dtype == RBF_F32 ? 4 : 8;
    std::vector<char> h((size_t)n * d * tsz);
    RBF_HIP(hipMemcpyAsync(h.data(), points, h.size(), hipMemcpyDeviceToHost, s));
    RBF_HIP(hipStreamSynchronize(s));
    double lo[kMaxDim], hi[kMaxDim];
    for (int k = 0; k < d; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) {
            double v = dtype == RBF_F32 ? (double)((const float *)h.data())[i * d + k]
                                        : ((const double *)h.data())[i * d + k];
            lo[k] = std::min(lo[k], v);
            hi[k] = std::max(hi[k], v);
        }
    double e = 0;
    for (int k = 0; k < d; ++k) e = std::max(e, hi[k] - lo[k]);
    *ext = e > 0 ? e : 1.0;
    return RBF_OK;
}

// Times reps products of the plan; for_batch: through the per-phase kernels, as a batch runs them
// (a single plan of one leaf would otherwise take the direct kernel).
int time_plan(rbf_plan *p, void *lam, void *u, int reps, bool for_batch, double *ms) {
    auto run = [&]() { return for_batch ? launch_matvec_phases(p, lam, u) : launch_matvec(p, lam, u); };
    hipEvent_t a, b;
    RBF_HIP(hipEventCreate(&a));
    RBF_HIP(hipEventCreate(&b));
    int rc = run();   // warm-up
    if (rc == RBF_OK) rc = (hipEventRecord(a, p->stream) == hipSuccess) ? RBF_OK : RBF_EHIP;
    for (int r = 0; r < reps && rc == RBF_OK; ++r) rc = run();
    if (rc == RBF_OK) rc = (hipEventRecord(b, p->stream) == hipSuccess) ? RBF_OK : RBF_EHIP;
    if (rc == RBF_OK) rc = (hipEventSynchronize(b) == hipSuccess) ? RBF_OK : RBF_EHIP;
    float t = 0;
    if (rc == RBF_OK) rc = (hipEventElapsedTime(&t, a, b) == hipSuccess) ? RBF_OK : RBF_EHIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = t / std::max(reps, 1);
    return rc;
}

__global__ void k_fill_one(void *v, int64_t n, int dtype) {
    int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i >= n) return;
    if (dtype == RBF_F32) ((float *)v)[i] = 1.0f;
    else ((double *)v)[i] = 1.0;
}

int autotune_impl(const void *points, int64_t n, int d, int dtype, int kernel, double shape, double tol,
                  const rbf_opts *base, int reps, hipStream_t s, bool for_batch, rbf_opts *best, double *best_ms) {
    double ext = 1.0;
    RBF_TRY(bbox_ext(points, n, d, dtype, s, &ext));
    auto cands = candidates(base, n, d, kernel, shape, tol, ext);
    const size_t tsz = dtype == RBF_F32 ? 4 : 8;
    void *lam = nullptr, *u = nullptr;
    RBF_HIP(hipMalloc(&lam, tsz * n));
    RBF_HIP(hipMalloc(&u, tsz * n));
    k_fill_one<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(lam, n, dtype);
    double bms = INFINITY;
    int found = 0;
    int best_lc = -1, best_far = 0;   // coarse level and far-field flag of the best plan
    auto try_candidate = [&](const rbf_opts &c) {
        rbf_plan *p = nullptr;
        if (plan_create(points, n, d, dtype, kernel, shape, tol, &c, s, &p) != RBF_OK) return;
        double ms = INFINITY;
        int rc = time_plan(p, lam, u, reps, for_batch, &ms);
        const int lc = p->lc, far = p->far && p->bands.empty();
        rbf_fmm_destroy(p);
        if (rc != RBF_OK) return;
        if (ms < bms) {
            bms = ms;
            *best = c;
            found = 1;
            best_lc = lc;
            best_far = far;
        }
    };
    for (const rbf_opts &c : cands) try_candidate(c);
    // Second stage (Gaussian far field): the quadrature order follows the coarse level through
    // the stencil's reach, so the levels next to the rule's (their node counts differ) and the
    // other leaf-translation block order are timed with the best leaf capacity.
    if (found && best_far && kernel == RBF_GAUSSIAN && best->coarse_level < 0 && best_lc >= 1) {
        const rbf_opts b0 = *best;
        std::vector<rbf_opts> more;
        for (int l : {best_lc - 1, best_lc + 1}) {
            if (l < 1 || l > 18 / d) continue;
            rbf_opts c = b0;
            c.coarse_level = l;
            c.coarse_radius = -1;
            more.push_back(c);
        }
        rbf_opts c = b0;
        c.m2l_schedule = b0.m2l_schedule == 2 ? 0 : 2;
        more.push_back(c);
        for (const rbf_opts &m : more) try_candidate(m);
    }
    (void)hipFree(lam);
    (void)hipFree(u);
    if (!found) {
        set_error("rbf_fmm_autotune: no candidate configuration could be planned");
        return RBF_EUNSUPPORTED;
    }
    if (best_ms) *best_ms = bms;
    return RBF_OK;
}

// Groups touch disjoint problems, so they run concurrently: the largest group (by points) goes
// first to the least-loaded lane.  One lane per group measured faster than fewer lanes even
// though lanes share the process's few hardware queues; the cap bounds the streams a batch holds.
constexpr int kBatchLanes = 8;

int assign_lanes(rbf_batch *b) {
    const int ng = (int)b->groups.size();
    const int nl = std::min(ng, kBatchLanes);
    std::vector<int> order(ng);
    for (int k = 0; k < ng; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->groups[x].points > b->groups[y].points; });
    std::vector<int64_t> load(nl, 0);
    for (int k : order) {
        int best = 0;
        for (int l = 1; l < nl; ++l)
            if (load[l] < load[best]) best = l;
        b->groups[k].lane = best;
        load[best] += b->groups[k].points;
    }
    for (int l = 1; l < nl; ++l) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        RBF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        b->lanes.push_back(s);
        RBF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->lane_done.push_back(e);
    }
    if (nl > 1) RBF_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    return RBF_OK;
}

template <class T> int build_groups(rbf_batch *b) {
    // group problems by padded half grid (one kernel instantiation per group)
    std::vector<int> hps;
    for (rbf_plan *p : b->plans) hps.push_back(p->far ? p->HP : 4);
    std::vector<int> keys = hps;
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    for (int hp : keys) {
        rbf_batch::Group g;
        g.HP = hp;
        std::vector<Desc<T>> ds;
        for (int q = 0; q < b->nprob; ++q) {
            if (hps[q] != hp) continue;
            Desc<T> d;
            std::memset(&d, 0, sizeof(d));
            fill_desc<T>(b->plans[q], &d);
            d.off = b->offsets[q];
            g.points += b->offsets[q + 1] - b->offsets[q];
            // the XCD-range order of the leaf translation (m2l_sched 1) gives every problem a
            // multiple of 8 blocks, so problem-local block ids keep their XCD (id % 8)
            ds.push_back(d);
            g.p2m_sh = std::max(g.p2m_sh, (size_t)d.p2m_lds);
        }
        g.nprob = (int)ds.size();
        RBF_TRY(b->arena.alloc(&g.descs, sizeof(Desc<T>) * ds.size()));
        RBF_HIP(hipMemcpy(g.descs, ds.data(), sizeof(Desc<T>) * ds.size(), hipMemcpyHostToDevice));
        for (int ph = 0; ph < PH_COUNT; ++ph) {
            std::vector<int> pre(ds.size() + 1, 0);
            int64_t tot = 0;
            for (size_t q = 0; q < ds.size(); ++q) {
                pre[q] = (int)tot;
                tot += desc_blocks<T>(ds[q], ph);
            }
            pre[ds.size()] = (int)tot;
            if (tot >= (int64_t)1 << 31) {
                set_error("batch: phase %d needs %lld blocks", ph, (long long)tot);
                return RBF_EUNSUPPORTED;
            }
            g.nblocks[ph] = tot;
            RBF_TRY(b->arena.alloc((void **)&g.bstart[ph], sizeof(int) * pre.size()));
            RBF_HIP(hipMemcpy(g.bstart[ph], pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice));
        }
        b->groups.push_back(g);
    }
    return assign_lanes(b);
}

template <class T> int launch_all(rbf_batch *b, const void *lam, void *u) {
    // Fork the lanes from the batch stream (also inside a graph capture, where the lanes join
    // the capture through this dependency).  Every forked lane is joined back before returning,
    // on the error path too: a capture that ends with a forked stream left unjoined fails, and
    // leaves that stream's capture state behind for the next use of the lane.
    size_t forked = 0;
    int rc = RBF_OK;
    if (!b->lanes.empty()) {
        if (hipEventRecord(b->ev_fork, b->stream) != hipSuccess) {
            set_error("batch: recording the fork event failed");
            return RBF_EHIP;
        }
        for (hipStream_t s : b->lanes) {
            if (hipStreamWaitEvent(s, b->ev_fork, 0) != hipSuccess) {
                set_error("batch: forking lane %zu failed", forked);
                rc = RBF_EHIP;
                break;
            }
            ++forked;
        }
    }
    for (auto &g : b->groups) {
        if (rc != RBF_OK) break;
        const int *bs[PH_COUNT];
        for (int k = 0; k < PH_COUNT; ++k) bs[k] = g.bstart[k];
        hipStream_t s = g.lane ? b->lanes[g.lane - 1] : b->stream;
        rc = launch_batch_group<T>(b->d, g.HP, b->kernel, (const Desc<T> *)g.descs, g.nprob, bs, g.nblocks,
                                   g.p2m_sh, (const T *)lam, (T *)u, s);
    }
    for (size_t l = 0; l < forked; ++l) {
        const bool ok = hipEventRecord(b->lane_done[l], b->lanes[l]) == hipSuccess &&
                        hipStreamWaitEvent(b->stream, b->lane_done[l], 0) == hipSuccess;
        if (!ok && rc == RBF_OK) {
            set_error("batch: joining lane %zu failed", l);
            rc = RBF_EHIP;
        }
    }
    return rc;
}

int batch_launch(rbf_batch *b, const void *lam, void *u) {
    return b->dtype == RBF_F32 ? launch_all<float>(b, lam, u) : launch_all<double>(b, lam, u);
}

void batch_free(rbf_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (rbf_plan *p : b->plans) rbf_fmm_destroy(p);
    b->arena.release();
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    for (hipStream_t s : b->lanes) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (hipEvent_t e : b->lane_done) (void)hipEventDestroy(e);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace
}  // namespace rbf

using namespace rbf;

extern "C" int rbf_fmm_autotune(const void *points, int64_t n, int d, int dtype, int kernel, double shape, double tol,
                                const rbf_opts *base, int reps, void *stream, rbf_opts *best, double *best_ms) {
    if (kernel == RBF_GAUSSIAN_BANDLIMITED) {
        set_error("rbf_fmm_autotune: the band-limited Gaussian has one plan shape (an exact sum); nothing to tune");
        return RBF_EUNSUPPORTED;
    }
    if (!points || !best) { set_error("rbf_fmm_autotune: null argument"); return RBF_EINVAL; }
    if (n < 1) { set_error("rbf_fmm_autotune: n must be positive"); return RBF_EINVAL; }
    return autotune_impl(points, n, d, dtype, kernel, shape, tol, base, reps > 0 ? reps : 3, (hipStream_t)stream, false,
                         best, best_ms);
}

extern "C" int rbf_fmm_plan_batch(const void *points, const int64_t *offsets, int nprob, int d, int dtype, int kernel,
                                  const double *shapes, double tol, const rbf_opts *opts, int autotune, void *stream,
                                  rbf_batch **out) {
    if (!points || !offsets || !shapes || !out || nprob < 1) {
        set_error("rbf_fmm_plan_batch: bad arguments");
        return RBF_EINVAL;
    }
    for (int q = 0; q < nprob; ++q)
        if (offsets[q + 1] <= offsets[q] || offsets[q] < 0) {
            set_error("rbf_fmm_plan_batch: offsets must be strictly increasing from 0 (problem %d)", q);
            return RBF_EINVAL;
        }
    auto t0 = std::chrono::steady_clock::now();
    rbf_batch *b = new rbf_batch();
    b->nprob = nprob;
    b->d = d;
    b->dtype = dtype;
    b->kernel = kernel;
    b->user_stream = (hipStream_t)stream;
    b->offsets.assign(offsets, offsets + nprob + 1);
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        set_error("rbf_fmm_plan_batch: stream/event creation failed");
        batch_free(b);
        return RBF_EHIP;
    }
    // the caller's points must be ready before the batch stream reads them
    if (hipEventRecord(b->ev_in, b->user_stream) != hipSuccess ||
        hipStreamWaitEvent(b->stream, b->ev_in, 0) != hipSuccess) {
        set_error("rbf_fmm_plan_batch: stream ordering failed");
        batch_free(b);
        return RBF_EHIP;
    }
    const size_t tsz = dtype == RBF_F32 ? 4 : 8;
    int rc = RBF_OK;
    for (int q = 0; q < nprob && rc == RBF_OK; ++q) {
        const void *pq = (const char *)points + (size_t)offsets[q] * d * tsz;
        const int64_t nq = offsets[q + 1] - offsets[q];
        rbf_opts o;
        std::memset(&o, 0, sizeof(o));
        if (opts) o = *opts;
        else { o.coarse_level = -1; o.coarse_radius = -1; }
        // a batch runs the per-phase kernels of one frequency grid per problem: the banded far
        // field of the multiquadric kernels is not batched, they take the exact sum
        if (banded_kernel(kernel, d)) o.exact = 1;
        // the band-limited Gaussian has one plan shape (an exact sum over one leaf)
        if (autotune && kernel != RBF_GAUSSIAN_BANDLIMITED) {
            double ms = 0;
            rc = autotune_impl(pq, nq, d, dtype, kernel, shapes[q], tol, &o, 2, b->stream, true, &o, &ms);
            if (rc != RBF_OK) break;
        }
        rbf_plan *p = nullptr;
        rc = plan_create(pq, nq, d, dtype, kernel, shapes[q], tol, &o, b->stream, &p);
        if (rc != RBF_OK) {
            char msg[512];
            std::snprintf(msg, sizeof(msg), "batch problem %d: %s", q, rbf_last_error());
            set_error("%s", msg);
            break;
        }
        b->plans.push_back(p);
        b->n_max.push_back(p->n_max);
        b->nodes.push_back(p->far ? p->mn : 0);
        b->far.push_back(p->far);
    }
    if (rc == RBF_OK) rc = dtype == RBF_F32 ? build_groups<float>(b) : build_groups<double>(b);
    if (rc != RBF_OK) {
        batch_free(b);
        return rc;
    }
    b->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = b;
    return RBF_OK;
}

int rbf::batch_product(rbf_batch *b, const void *lambda, void *u) {
    RBF_HIP(hipEventRecord(b->ev_in, b->user_stream));
    RBF_HIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    if (b->use_graph) {
        if (!b->exec || b->g_lam != lambda || b->g_u != u) {
            if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
            if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
            RBF_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            int rc = batch_launch(b, lambda, u);   // joins its lanes even when it fails
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->stream, &g);
            if (rc != RBF_OK || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
                if (rc == RBF_OK) {
                    set_error("batch: graph capture failed: %s", hipGetErrorString(e));
                    rc = RBF_EHIP;
                }
                return rc;
            }
            b->graph = g;
            RBF_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            b->g_lam = lambda;
            b->g_u = u;
        }
        RBF_HIP(hipGraphLaunch(b->exec, b->stream));
    } else {
        RBF_TRY(batch_launch(b, lambda, u));
    }
    RBF_HIP(hipEventRecord(b->ev_out, b->stream));
    RBF_HIP(hipStreamWaitEvent(b->user_stream, b->ev_out, 0));
    return RBF_OK;
}

extern "C" int rbf_fmm_matvec_batch(rbf_batch *b, const void *lambda, void *u) {
    if (!b || !lambda || !u) { set_error("rbf_fmm_matvec_batch: null argument"); return RBF_EINVAL; }
    if (lambda == u) { set_error("rbf_fmm_matvec_batch: lambda and u must not alias"); return RBF_EINVAL; }
    return batch_product(b, lambda, u);
}

extern "C" int rbf_fmm_batch_set_graph(rbf_batch *b, int on) {
    if (!b) { set_error("rbf_fmm_batch_set_graph: null batch"); return RBF_EINVAL; }
    b->use_graph = on ? 1 : 0;
    return RBF_OK;
}

extern "C" int rbf_fmm_batch_info(const rbf_batch *b, rbf_batch_info *info, int32_t *n_max, int32_t *nodes) {
    if (!b || !info) { set_error("rbf_fmm_batch_info: null argument"); return RBF_EINVAL; }
    std::memset(info, 0, sizeof(*info));
    info->nprob = b->nprob;
    info->ngroups = (int)b->groups.size();
    info->use_graph = b->use_graph;
    info->total_n = b->offsets[b->nprob];
    int64_t bytes = b->arena.bytes, leaves = 0;
    int nfar = 0;
    for (rbf_plan *p : b->plans) {
        bytes += p->arena.bytes;
        leaves += p->nleaves;
        nfar += p->far;
    }
    info->nfar = nfar;
    info->total_leaves = leaves;
    info->device_bytes = bytes;
    info->plan_seconds = b->plan_seconds;
    for (int q = 0; q < b->nprob; ++q) {
        if (n_max) n_max[q] = b->n_max[q];
        if (nodes) nodes[q] = b->nodes[q];
    }
    return RBF_OK;
}

extern "C" int rbf_fmm_batch_destroy(rbf_batch *b) {
    batch_free(b);
    return RBF_OK;
}
