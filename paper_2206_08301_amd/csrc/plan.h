// plan.h -- launch plans for the MTTKRP streaming kernel.
#pragma once

#include <cstdint>
#include <string>

#include "deinsum.h"
#include "mttkrp.h"

namespace deinsum {

enum PlanFamily {
    PLAN_MTTKRP_KCONTIG = 1,  // free mode n < N-1
    PLAN_MTTKRP_MCONTIG = 2,  // free mode n = N-1
    PLAN_MTTKRP_KOUT = 3,     // order 3, free mode 0: mode-1 tiles walked per output row
};


struct MttkrpPlan {
    int family = 0;
    int prec = 0;
    const StreamKernelInfo *kernel = nullptr;
    int nt = 2, ni = 16, mt = 1;
    int slice = 64;           // positions of mode g per wave
    int wk = 4, waves = 4;
    int tile_rows = 16;
    int64_t n_tiles = 0, n_kgroups = 1, n_chunks = 1;
    int64_t o_per_chunk = 1;
    int order = 0;            // unit order (StreamArgs::order)
    int xcd = 0;              // XCD-aware unit remap (StreamArgs::xcd_remap)
    int64_t col_blocks = 1;
    int64_t groups = 0;       // workgroups per column block
    int64_t parts = 0;        // partial tiles per output tile
    int64_t O = 1;            // outer index count
    size_t w_offset = 0;      // byte offset of the outer-weight table in the workspace
    size_t workspace = 0;     // bytes
    std::string name;
};

struct MttkrpProblem {
    int N = 0, n = 0;
    int64_t dims[DEINSUM_MAX_ORDER] = {0};
    int64_t R = 0;
    int prec = 0;
};

// Order-3 mode 0 whose K-contiguous tiles would read rows far apart (at least 1 MiB
// between consecutive output rows): the mode-1-tiled walk streams one X slab per
// output row instead.  The FP64 form takes the fused TTMc pass for that (abi.cpp).
bool kout_default(const MttkrpProblem &pb);

// Launch geometry for a given kernel variant; split_hint > 0 forces the number of outer chunks.
deinsum_status plan_geometry(const MttkrpProblem &pb, const StreamKernelInfo *kernel, int split_hint, MttkrpPlan *out);

// Heuristic plan (kernel variant with the least padding of mode g, then plan_geometry).
deinsum_status plan_mttkrp(const MttkrpProblem &pb, int plan_hint, int split_hint, MttkrpPlan *out);

}  // namespace deinsum
