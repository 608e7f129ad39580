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
    int64_t slab_stride;     // element distance of consecutive slabs when constant, else 0
    int n_ctiles, nwaves, n_cgroups;
    int ra, rc;
    int vec_ok;
    int xcd_remap;           // 1: the workgroups of one XCD take one contiguous range of units
    int64_t n_groups;        // grid size
    double *P;               // stage2: [cgroup][slab][ra][rc]; else [slab][n_ctiles*16*MT][16*NTA]
    // FX20 form only: X is the FP16 plane of the buffer, X2 its int8 plane, fx_hdr its
    // header (exponent e); Ua holds the packed FP16 hi parts of U^a scaled per column by
    // 2^-k, Ua2 the lo parts; ua_scale[col] = 2^k and ua_off[col] = 1152 * (sum of the hi
    // parts of the column) undo the scaling and the int8 operand's offset.
    const void *X2;
    const void *Ua2;
    const double *ua_scale;
    const double *ua_off;
    const void *fx_hdr;
};

deinsum_status ttmc_workspace_size(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks,
                                   const deinsum_opts &o, size_t *bytes);
// Plan-cache key of a TTMc problem (autotuned fused-kernel variant).
std::string ttmc_tune_key(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, int prec);

deinsum_status run_ttmc(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, const void *X,
                        const void *const *U, void *Y, const deinsum_opts &o, void *ws, size_t ws_bytes,
                        hipStream_t s);

// Mode-0 MTTKRP of an order-3 tensor through the fused TTMc pass, whose access
// pattern streams whole rows of X: Y[i, b, c] = sum_{j,k} X[i,j,k] U1[j,b] U2[k,c]
// with both ranks R (<= 64), then M[i, r] = Y[i, r, r] (with both as defined in
// Sec. III-B, the MTTKRP is this TTMc's diagonal).  variant: as the TTMc plan_hint (0 = tuned or default, k >= 1
// = compiled variant k-1).  prec: P_FP64 or P_FP32.
deinsum_status mttkrp_via_ttmc_workspace(const int64_t *dims, int64_t R, int prec, int variant, size_t *bytes);
deinsum_status run_mttkrp_via_ttmc(const int64_t *dims, int64_t R, const void *X, const void *U1, const void *U2,
                                   void *M, int prec, int out_dtype, int variant, void *ws, size_t ws_bytes,
                                   hipStream_t s);

}  // namespace deinsum
