// als.h -- CP-ALS factor update used by the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "deinsum.h"

namespace deinsum {

constexpr int kAlsMaxRank = 64;
constexpr int kAlsRows = 64;  // rows of the factor handled by one solve workgroup

// One factor update U^n <- normalise(M V^{-1}), V = Hadamard of the Grams G^m, m != n.
// All buffers are device memory; sizes in doubles.
struct AlsJob {
    int32_t order, mode, R, prec;  // prec: P_FP64 or P_FP32 (factor storage)
    int64_t dims[DEINSUM_MAX_ORDER];
    const double *M;               // MTTKRP output, dims[mode] x R
    double *Xs;                    // unnormalised update, dims[mode] x R
    double *Gp;                    // partial Grams, als_blocks(dims[mode]) x R x R
    double *G;                     // Gram cache, order x R x R; G[m] = U^m^T U^m, G[mode] rewritten
    void *U[DEINSUM_MAX_ORDER];    // factors by mode; U[mode] is overwritten
    int64_t block_begin;           // first solve workgroup of this job in a batched launch
    int32_t *flag;                 // optional: set to 1 when V needed the pivot floor (never
                                   // cleared; device-visible host memory or device memory)
    double *lambda;                // optional: the R column norms of the unnormalised update
};

__host__ __device__ inline int64_t als_blocks(int64_t rows) { return (rows + kAlsRows - 1) / kAlsRows; }

// Batched update of njobs jobs (device table, block_begin set, total_blocks = sum of
// als_blocks(dims[mode])): one solve launch over all jobs' row blocks, one finish launch.
deinsum_status launch_als_batch(const AlsJob *d_jobs, int njobs, int64_t total_blocks, hipStream_t s);
// The same two kernels for a single job passed by value.
deinsum_status launch_als_one(const AlsJob &job, hipStream_t s);
// G[m] = U^m^T U^m for every mode of the job (set-up of the Gram cache).
deinsum_status launch_als_grams(const AlsJob &job, hipStream_t s);

}  // namespace deinsum
