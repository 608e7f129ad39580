// als.hip -- CP-ALS factor update that follows each MTTKRP in the serving loop:
//   U^n <- M (*_{m != n} G^m)^{-1},  G^m = U^m^T U^m,  then each column of U^n
//   scaled to unit 2-norm.
// This is the standard alternating-least-squares step of the CP decomposition
// (the paper names MTTKRP as the main kernel of CP; the update itself is not
// part of the paper).  The Gram matrices are cached per tensor: after an update
// only G^n changes, and it follows from the Gram of the unnormalised solution,
// G^n = D (Xs^T Xs) D with D = diag(1 / ||Xs[:, r]||).
//
// Two launches per update (or per batch of updates):
//   solve:  one workgroup per 64 rows of U^n.  Each workgroup forms V from the
//           cached Grams, inverts it in LDS (Gauss-Jordan; V is symmetric
//           positive definite, so no pivoting), multiplies its rows of M by
//           V^{-1} and writes them and their partial Gram.
//   finish: one workgroup per job.  Sums the partial Grams in a fixed order,
//           derives the column norms, writes G^n and the normalised U^n in its
//           storage precision.
// Every sum runs in a fixed order that depends only on the job's own shape, so
// an update is bitwise the same alone or in any batch.  FP64 throughout.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "als.h"
#include "internal.h"
#include "kernels.h"

namespace deinsum {

namespace {

constexpr int kAlsThreads = 256;
constexpr int kLd = kAlsMaxRank + 1;  // LDS row stride in doubles

__device__ __forceinline__ double ldf(const void *p, int64_t i, int prec)
{
    return prec == P_FP64 ? static_cast<const double *>(p)[i]
                          : static_cast<double>(static_cast<const float *>(p)[i]);
}

// Sum over `rows` LDS rows of B[row][r1] * B[row][r2] for a 4x4 tile of (r1, r2):
// thread (rg, cg) owns r1 = rg + 16a, r2 = cg + 16b.
__device__ __forceinline__ void gram_tile(const double *B, int rows, int rg, int cg, double acc[4][4])
{
    for (int row = 0; row < rows; ++row) {
        double x1[4], x2[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x1[a] = B[row * kLd + rg + 16 * a];
#pragma unroll
        for (int b = 0; b < 4; ++b) x2[b] = B[row * kLd + cg + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += x1[a] * x2[b];
    }
}

__device__ void als_solve_block(const AlsJob &j, int64_t blk)
{
    __shared__ double A[kAlsMaxRank * kLd];  // V, then V^{-1}
    __shared__ double B[kAlsRows * kLd];     // rows of M, then rows of the solution
    __shared__ double rowk[kAlsMaxRank], colk[kAlsMaxRank];
    __shared__ double diag_max;
    const int R = j.R;
    const int tid = threadIdx.x;
    const int64_t I = j.dims[j.mode];
    const int64_t i0 = blk * kAlsRows;
    const int rows = static_cast<int>(I - i0 < kAlsRows ? I - i0 : kAlsRows);
    // Unused LDS entries are zeroed so the fixed 4x4 tiles read defined values.
    for (int e = tid; e < kAlsMaxRank * kLd; e += kAlsThreads) A[e] = 0.0;
    for (int e = tid; e < kAlsRows * kLd; e += kAlsThreads) B[e] = 0.0;
    __syncthreads();
    for (int e = tid; e < R * R; e += kAlsThreads) {
        const int r1 = e / R, r2 = e % R;
        double v = 1.0;
        for (int m = 0; m < j.order; ++m)
            if (m != j.mode) v *= j.G[(static_cast<int64_t>(m) * R + r1) * R + r2];
        A[r1 * kLd + r2] = v;
    }
    for (int e = tid; e < rows * R; e += kAlsThreads) {
        const int r = e / R, c = e % R;
        B[r * kLd + c] = j.M[(i0 + r) * R + c];
    }
    __syncthreads();
    if (tid == 0) {
        double mx = 0.0;
        for (int k = 0; k < R; ++k) mx = fmax(mx, A[k * kLd + k]);
        diag_max = mx;
    }
    __syncthreads();
    // A pivot below this floor means V is (numerically) singular; the floor acts as a ridge
    // and the job's first workgroup reports it through j.flag.
    const double floor_p = diag_max > 0.0 ? 1e-14 * diag_max : 1e-300;
    bool floored = false;
    // In-place Gauss-Jordan inversion, one pivot per step.
    for (int k = 0; k < R; ++k) {
        if (tid < R) {
            rowk[tid] = A[k * kLd + tid];
            colk[tid] = A[tid * kLd + k];
        }
        __syncthreads();
        double p = rowk[k];
        if (!(p > floor_p)) {
            p = floor_p;
            floored = true;
        }
        const double inv = 1.0 / p;
        for (int e = tid; e < R * R; e += kAlsThreads) {
            const int i = e / R, c = e % R;
            double v;
            if (i == k) v = (c == k) ? inv : rowk[c] * inv;
            else if (c == k) v = -colk[i] * inv;
            else v = A[i * kLd + c] - colk[i] * (rowk[c] * inv);
            A[i * kLd + c] = v;
        }
        __syncthreads();
    }
    if (blk == 0 && tid == 0 && j.flag && floored) __atomic_store_n(j.flag, 1, __ATOMIC_RELAXED);
    // Rows of the solution: Xs = M V^{-1}, a 4x4 register tile per thread.
    const int rg = tid >> 4, cg = tid & 15;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int p = 0; p < R; ++p) {
        double mv[4], wv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) mv[a] = B[(rg + 16 * a) * kLd + p];
#pragma unroll
        for (int b = 0; b < 4; ++b) wv[b] = A[p * kLd + cg + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += mv[a] * wv[b];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int row = rg + 16 * a, col = cg + 16 * b;
            const bool live = row < rows && col < R;
            B[row * kLd + col] = live ? acc[a][b] : 0.0;
            if (live) j.Xs[(i0 + row) * R + col] = acc[a][b];
        }
    __syncthreads();
    // Partial Gram of this block's rows.
    double g[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) g[a][b] = 0.0;
    gram_tile(B, rows, rg, cg, g);
    double *gp = j.Gp + blk * R * R;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r1 = rg + 16 * a, r2 = cg + 16 * b;
            if (r1 < R && r2 < R) gp[r1 * R + r2] = g[a][b];
        }
}

__device__ void als_finish_job(const AlsJob &j)
{
    __shared__ double d[kAlsMaxRank];
    const int R = j.R;
    const int tid = threadIdx.x;
    const int64_t I = j.dims[j.mode];
    const int64_t nb = als_blocks(I);
    if (tid < R) {
        double s = 0.0;
        for (int64_t b = 0; b < nb; ++b) s += j.Gp[(b * R + tid) * R + tid];
        d[tid] = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
        if (j.lambda) j.lambda[tid] = sqrt(s);
    }
    __syncthreads();
    double *Gn = j.G + static_cast<int64_t>(j.mode) * R * R;
    for (int e = tid; e < R * R; e += kAlsThreads) {
        double s = 0.0;
        for (int64_t b = 0; b < nb; ++b) s += j.Gp[b * R * R + e];
        Gn[e] = d[e / R] * s * d[e % R];
    }
    const int64_t total = I * R;
    if (j.prec == P_FP64) {
        double *U = static_cast<double *>(j.U[j.mode]);
        for (int64_t e = tid; e < total; e += kAlsThreads) U[e] = j.Xs[e] * d[e % R];
    } else {
        float *U = static_cast<float *>(j.U[j.mode]);
        for (int64_t e = tid; e < total; e += kAlsThreads) U[e] = static_cast<float>(j.Xs[e] * d[e % R]);
    }
}

__device__ int find_als_job(const AlsJob *jobs, int njobs, int64_t blk)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block_begin <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kAlsThreads) als_solve_batch_kernel(const AlsJob *jobs, int njobs)
{
    const int64_t blk = blockIdx.x;
    const int q = find_als_job(jobs, njobs, blk);
    als_solve_block(jobs[q], blk - jobs[q].block_begin);
}

__global__ void __launch_bounds__(kAlsThreads) als_finish_batch_kernel(const AlsJob *jobs, int njobs)
{
    if (static_cast<int>(blockIdx.x) < njobs) als_finish_job(jobs[blockIdx.x]);
}

__global__ void __launch_bounds__(kAlsThreads) als_solve_one_kernel(const AlsJob job)
{
    als_solve_block(job, blockIdx.x);
}

__global__ void __launch_bounds__(kAlsThreads) als_finish_one_kernel(const AlsJob job) { als_finish_job(job); }

// G[m] = U^m^T U^m, one workgroup per mode, rows staged through LDS 64 at a time.
__global__ void __launch_bounds__(kAlsThreads) als_gram_kernel(const AlsJob job)
{
    __shared__ double B[kAlsRows * kLd];
    const int m = blockIdx.x;
    const int R = job.R;
    const int tid = threadIdx.x;
    const int rg = tid >> 4, cg = tid & 15;
    const int64_t I = job.dims[m];
    double g[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) g[a][b] = 0.0;
    for (int e = tid; e < kAlsRows * kLd; e += kAlsThreads) B[e] = 0.0;
    for (int64_t i0 = 0; i0 < I; i0 += kAlsRows) {
        const int rows = static_cast<int>(I - i0 < kAlsRows ? I - i0 : kAlsRows);
        __syncthreads();
        for (int e = tid; e < rows * R; e += kAlsThreads) {
            const int r = e / R, c = e % R;
            B[r * kLd + c] = ldf(job.U[m], (i0 + r) * R + c, job.prec);
        }
        __syncthreads();
        gram_tile(B, rows, rg, cg, g);
    }
    double *G = job.G + static_cast<int64_t>(m) * R * R;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r1 = rg + 16 * a, r2 = cg + 16 * b;
            if (r1 < R && r2 < R) G[r1 * R + r2] = g[a][b];
        }
}

bool job_ok(const AlsJob &j)
{
    return j.R >= 1 && j.R <= kAlsMaxRank && j.order >= 2 && j.order <= DEINSUM_MAX_ORDER && j.mode >= 0 &&
           j.mode < j.order && j.dims[j.mode] >= 1 && (j.prec == P_FP64 || j.prec == P_FP32);
}

}  // namespace

deinsum_status launch_als_batch(const AlsJob *d_jobs, int njobs, int64_t total_blocks, hipStream_t s)
{
    if (njobs <= 0) return DEINSUM_OK;
    if (total_blocks < njobs || total_blocks > (int64_t(1) << 31) - 1)
        return fail(DEINSUM_ERR_INVALID_ARG, "als_batch: bad block count");
    als_solve_batch_kernel<<<static_cast<unsigned>(total_blocks), kAlsThreads, 0, s>>>(d_jobs, njobs);
    if (deinsum_status st = check_launch("als_solve_batch")) return st;
    als_finish_batch_kernel<<<njobs, kAlsThreads, 0, s>>>(d_jobs, njobs);
    return check_launch("als_finish_batch");
}

deinsum_status launch_als_one(const AlsJob &job, hipStream_t s)
{
    if (!job_ok(job)) return fail(DEINSUM_ERR_INVALID_ARG, "als_one: bad job");
    als_solve_one_kernel<<<static_cast<unsigned>(als_blocks(job.dims[job.mode])), kAlsThreads, 0, s>>>(job);
    if (deinsum_status st = check_launch("als_solve_one")) return st;
    als_finish_one_kernel<<<1, kAlsThreads, 0, s>>>(job);
    return check_launch("als_finish_one");
}

deinsum_status launch_als_grams(const AlsJob &job, hipStream_t s)
{
    if (job.R < 1 || job.R > kAlsMaxRank || job.order < 2 || job.order > DEINSUM_MAX_ORDER)
        return fail(DEINSUM_ERR_INVALID_ARG, "als_grams: bad job");
    als_gram_kernel<<<job.order, kAlsThreads, 0, s>>>(job);
    return check_launch("als_grams");
}

}  // namespace deinsum
