// The batch of independent problems shared by the batched product (batch.hip) and the
// batched solve (solve_batch.hip).
#pragma once
#include <vector>

#include "fmm_desc.h"
#include "internal.h"

struct rbf_batch {
    int nprob = 0, d = 0, dtype = 0, kernel = 0;
    hipStream_t user_stream = nullptr, stream = nullptr;
    std::vector<rbf_plan *> plans;
    std::vector<int64_t> offsets;
    std::vector<int> n_max, nodes, far;
    struct Group {
        int HP = 0, nprob = 0, lane = 0;
        int64_t points = 0;
        void *descs = nullptr;
        int *bstart[rbf::PH_COUNT] = {};
        int64_t nblocks[rbf::PH_COUNT] = {};
        size_t p2m_sh = 0;
    };
    std::vector<Group> groups;
    rbf::Arena arena;
    int use_graph = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *g_lam = nullptr;
    void *g_u = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // groups run concurrently on lanes: lane 0 is `stream`, lane k > 0 is lanes[k - 1], forked
    // from `stream` at ev_fork and joined back at lane_done[k - 1]
    std::vector<hipStream_t> lanes;
    std::vector<hipEvent_t> lane_done;
    hipEvent_t ev_fork = nullptr;
    double plan_seconds = 0;
};

namespace rbf {
int batch_product(rbf_batch *b, const void *lambda, void *u);   // rbf_fmm_matvec_batch without checks
}  // namespace rbf
