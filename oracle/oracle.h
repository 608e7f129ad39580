/*
 * oracle.h -- plain, slow, obviously correct FP64 CPU reference for the two
 * multilinear kernels of Deinsum (Ziogas et al., "Deinsum: Practically I/O
 * Optimal Multilinear Algebra", arXiv 2206.08301).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or helper with the HIP
 * path.
 *
 * Conventions (all functions):
 *   - X is a dense order-N tensor, row-major (last index contiguous), with
 *     dims[0..N-1]; 1 <= N <= 8.
 *   - U is an array of N pointers indexed by MODE.  U[m] is the row-major
 *     I_m x R_m factor of mode m (R_m = R for MTTKRP).  U[n] (free mode) is
 *     ignored and may be NULL.
 *   - Outputs are overwritten (zero, then accumulate).
 *   - Return 0 on success, -1 on bad arguments, -2 on allocation failure.
 *   - OpenMP parallelism is over output rows only; every output element is
 *     summed by one thread in a fixed order, so results do not depend on the
 *     thread count.
 */
#ifndef DEINSUM_ORACLE_H
#define DEINSUM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Threads the oracle uses (OpenMP max threads). */
int oracle_num_threads(void);

/*
 * Mode-n MTTKRP, the multilinear map of Sec. III-B ("tensor operations"),
 * in the index form of the benchmark einsums of Tab. IV:
 *     M[i_n, r] = sum over all i_m (m != n) of X[i_0..i_{N-1}] * prod_{m != n} U^m[i_m, r]
 * The product is formed left to right in increasing mode order; the sum runs
 * over the other indices in row-major order.  M is I_n x R row-major.
 */
int oracle_mttkrp(int N, const int64_t *dims, int n, int64_t R,
                  const double *X, const double *const *U, double *M);

/* Same definition with 80-bit long double products and accumulators, used
 * only to bound the FP64 oracle's own rounding error. Output rounded to FP64. */
int oracle_mttkrp_ld(int N, const int64_t *dims, int n, int64_t R,
                     const double *X, const double *const *U, double *M);

/*
 * Mode-m tensor-times-matrix (TTM) of Sec. III-B, einsum
 *     i_0..i_{N-1}, i_m r -> i_0..i_{m-1} r i_{m+1}..i_{N-1}
 * i.e. Y[.., r, ..] = sum_{i_m} X[.., i_m, ..] * U[i_m, r]; U is I_m x Rm.
 * Y has the dims of X with dims[m] replaced by Rm.
 */
int oracle_ttm(int N, const int64_t *dims, int m, int64_t Rm,
               const double *X, const double *U, double *Y);

/*
 * Mode-n TTM chain (TTMc) of Sec. III-B: X x_0 U^0 ... x_{n-1} U^{n-1}
 * x_{n+1} U^{n+1} ... x_{N-1} U^{N-1}, evaluated as that chain of TTMs in
 * increasing mode order.  Output shape: R_0 x .. x R_{n-1} x I_n x R_{n+1}
 * x .. x R_{N-1} (row-major).  ranks[n] is ignored.
 */
int oracle_ttmc(int N, const int64_t *dims, int n, const int64_t *ranks,
                const double *X, const double *const *U, double *Y);

#ifdef __cplusplus
}
#endif
#endif
