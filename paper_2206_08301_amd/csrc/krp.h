// krp.h -- small dense helpers: the Khatri-Rao product of two factors (the merged
// factor of two adjacent contracted modes) and the matrix product that ends an
// MTTKRP-GEMM chain.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "deinsum.h"

namespace deinsum {

// K[p * Ib + q][r] = A[p][r] * B[q][r] for p < Ia, q < Ib, r < R (row-major, row
// stride R).  elem_bytes 4: FP32 factors, 8: FP64.  Device pointers; K must not
// overlap A or B.
deinsum_status launch_krp2(const void *A, const void *B, int64_t Ia, int64_t Ib, int64_t R, int elem_bytes,
                           void *K, hipStream_t s);

// Y[i][l] = sum_{r < R} M[i][r] * C[r][l] for i < I, l < L, summed in FP64 in
// increasing r.  M: FP64, row stride R; C: row-major R x L, elem_bytes 8 (f64) or
// 4 (f32); Y: row-major I x L in out_dtype (DEINSUM_F64 or DEINSUM_F32).
deinsum_status launch_chain_mm(const double *M, const void *C, int c_elem_bytes, int64_t I, int64_t R, int64_t L,
                               void *Y, int out_dtype, hipStream_t s);

}  // namespace deinsum
