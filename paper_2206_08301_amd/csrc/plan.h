// plan.h -- launch plans for the MTTKRP / TTMc kernels.
#pragma once

#include <cstdint>
#include <string>

#include "deinsum.h"

namespace deinsum {

enum PlanFamily {
    PLAN_MTTKRP_KCONTIG = 1,  // free mode n < N-1
    PLAN_MTTKRP_MCONTIG = 2,  // free mode n = N-1
    PLAN_TTMC_FUSED = 3,      // TTMc, free mode n < N-1
};

struct MttkrpPlan {
    int family = 0;
    int prec = 0;
    int nt = 2;              // 16-column tiles per column block
    int kl = 16;             // K-contiguous: elements per lane per step (slice = 4 * kl)
    int mt = 2;              // M-contiguous: 16-row tiles per wave
    int wk = 4, wo = 1;      // K-contiguous: k-slices / outer sub-ranges per workgroup
    int waves = 4;
    int64_t n_tiles = 0, n_kgroups = 1, n_chunks = 1, n_igchunks = 1;
    int64_t o_per_chunk = 1, ig_per_chunk = 1;
    int64_t col_blocks = 1;
    int64_t groups = 0;      // workgroups per column block
    int64_t parts = 0;       // partial tiles per output tile
    size_t workspace = 0;    // bytes
    std::string name;
};

struct MttkrpProblem {
    int N = 0, n = 0;
    int64_t dims[DEINSUM_MAX_ORDER] = {0};
    int64_t R = 0;
    int prec = 0;
};

// Heuristic plan (plan_hint / split_hint override the choice of family and chunking).
deinsum_status plan_mttkrp(const MttkrpProblem &pb, int plan_hint, int split_hint, MttkrpPlan *out);

}  // namespace deinsum
