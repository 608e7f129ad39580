// ttmc.h -- TTMc host entry points and kernel arguments.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "kernels.h"

namespace deinsum {

// Fused two-mode TTM pass over X.
//   stage 1 (matrix cores): D[i_c, r_a] = sum_{i_a} X[slab, i_a, i_c] U^a[i_a, r_a]
//   stage 2 (if stage2):    Z[r_a, r_c] = sum_{i_c} D[i_c, r_a] U^c[i_c, r_c]
// where c = N-1 is the contiguous mode and `slab` enumerates the other modes.
struct TkArgs {
    const void *X;
    const void *Ua;          // U^a zero-padded to 16*NTA columns (FP64 or FP32, as X)
    const void *Uc;          // U^c zero-padded to 16*NTC columns, stage 2 only
    int64_t Ia, Ic, stride_a;
    OuterDesc od;            // slab modes (X strides only)
    int64_t n_slabs, slabs_per_group;
    int n_ctiles, nwaves, n_cgroups;
    int ra, rc;
    int vec_ok;
    int xcd_remap;           // 1: the workgroups of one XCD take one contiguous range of units
    int64_t n_groups;        // grid size
    double *P;               // stage2: [cgroup][slab][16*NTA][16*NTC]; else [slab][n_ctiles*16*MT][16*NTA]
};

deinsum_status ttmc_workspace_size(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks,
                                   const deinsum_opts &o, size_t *bytes);
// Plan-cache key of a TTMc problem (autotuned fused-kernel variant).
std::string ttmc_tune_key(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, int prec);

deinsum_status run_ttmc(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, const void *X,
                        const void *const *U, void *Y, const deinsum_opts &o, void *ws, size_t ws_bytes,
                        hipStream_t s);

}  // namespace deinsum
