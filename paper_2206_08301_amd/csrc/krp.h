// krp.h -- row-wise Khatri-Rao product of two factors (the merged factor of two
// adjacent contracted modes).
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

}  // namespace deinsum
