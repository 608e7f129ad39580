/*
 * oracle.c -- plain FP64 CPU reference for MTTKRP and TTMc (Deinsum,
 * arXiv 2206.08301, Sec. III-B and Tab. IV).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the benchmark's CPU-baseline leg; never by the product library.  It is
 * written as the definitions read, with no blocking, fusion or reordering:
 *   - MTTKRP is the einsum of Tab. IV summed directly (every element of X
 *     times the product of the factor entries it meets);
 *   - TTMc is the chain of mode products the paper defines it as.
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no -ffast-math), so every
 * product and sum is a separately rounded IEEE FP64 operation.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_ORDER 8

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int check_dims(int N, const int64_t *dims)
{
    if (N < 1 || N > ORACLE_MAX_ORDER || dims == NULL) return -1;
    for (int m = 0; m < N; ++m)
        if (dims[m] < 1) return -1;
    return 0;
}

/* Row-major element strides of a tensor with the given dims. */
static void row_major_strides(int N, const int64_t *dims, int64_t *stride)
{
    int64_t s = 1;
    for (int m = N - 1; m >= 0; --m) {
        stride[m] = s;
        s *= dims[m];
    }
}

/*
 * MTTKRP by its definition (Sec. III-B; index form of Tab. IV):
 *   M[i_n, r] = sum_{i_m, m != n} X[i] * prod_{m != n} U^m[i_m, r].
 * For each output row i_n, walk every index tuple of the other modes in
 * row-major order (an odometer that skips mode n) and add the term for
 * each r.  The product is taken left to right in increasing mode order.
 */
#define MTTKRP_BODY(ACC_T)                                                     \
    if (check_dims(N, dims) || n < 0 || n >= N || R < 1 || !X || !U || !M)    \
        return -1;                                                             \
    for (int m = 0; m < N; ++m)                                                \
        if (m != n && U[m] == NULL) return -1;                                 \
    int64_t stride[ORACLE_MAX_ORDER];                                          \
    row_major_strides(N, dims, stride);                                        \
    int64_t other = 1; /* number of index tuples with i_n fixed */             \
    for (int m = 0; m < N; ++m)                                                \
        if (m != n) other *= dims[m];                                          \
    int bad = 0;                                                               \
    _Pragma("omp parallel for schedule(dynamic, 1)")                           \
    for (int64_t in = 0; in < dims[n]; ++in) {                                 \
        ACC_T *acc = (ACC_T *)calloc((size_t)R, sizeof(ACC_T));                \
        if (!acc) { bad = 1; continue; }                                       \
        int64_t idx[ORACLE_MAX_ORDER] = {0};                                   \
        idx[n] = in;                                                           \
        for (int64_t t = 0; t < other; ++t) {                                  \
            int64_t lin = 0;                                                   \
            for (int m = 0; m < N; ++m) lin += idx[m] * stride[m];             \
            for (int64_t r = 0; r < R; ++r) {                                  \
                ACC_T p = (ACC_T)X[lin];                                       \
                for (int m = 0; m < N; ++m)                                    \
                    if (m != n) p = p * (ACC_T)U[m][idx[m] * R + r];           \
                acc[r] = acc[r] + p;                                           \
            }                                                                  \
            /* advance the odometer over modes != n, last mode fastest */      \
            for (int m = N - 1; m >= 0; --m) {                                 \
                if (m == n) continue;                                          \
                if (++idx[m] < dims[m]) break;                                 \
                idx[m] = 0;                                                    \
            }                                                                  \
        }                                                                      \
        for (int64_t r = 0; r < R; ++r) M[in * R + r] = (double)acc[r];        \
        free(acc);                                                             \
    }                                                                          \
    return bad ? -2 : 0;

int oracle_mttkrp(int N, const int64_t *dims, int n, int64_t R,
                  const double *X, const double *const *U, double *M)
{
    MTTKRP_BODY(double)
}

int oracle_mttkrp_ld(int N, const int64_t *dims, int n, int64_t R,
                     const double *X, const double *const *U, double *M)
{
    MTTKRP_BODY(long double)
}

/*
 * Mode-m product (TTM, Sec. III-B): every mode-m fiber of X is multiplied
 * by U (I_m x Rm), contracting U's first index:
 *   Y[a, r, b] = sum_{c} X[a, c, b] * U[c, r],
 * where a runs over the modes before m, c over mode m, b over the modes
 * after m (all row-major).
 */
int oracle_ttm(int N, const int64_t *dims, int m, int64_t Rm,
               const double *X, const double *U, double *Y)
{
    if (check_dims(N, dims) || m < 0 || m >= N || Rm < 1 || !X || !U || !Y)
        return -1;
    int64_t left = 1, right = 1;
    for (int p = 0; p < m; ++p) left *= dims[p];
    for (int p = m + 1; p < N; ++p) right *= dims[p];
    const int64_t mid = dims[m];
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t a = 0; a < left; ++a) {
        for (int64_t r = 0; r < Rm; ++r) {
            for (int64_t b = 0; b < right; ++b) {
                double s = 0.0;
                for (int64_t c = 0; c < mid; ++c)
                    s = s + X[(a * mid + c) * right + b] * U[c * Rm + r];
                Y[(a * Rm + r) * right + b] = s;
            }
        }
    }
    return 0;
}

/*
 * TTMc (Sec. III-B): X x_0 U^0 ... (mode n skipped) ... x_{N-1} U^{N-1},
 * evaluated left to right, one TTM at a time, into fresh intermediates.
 */
int oracle_ttmc(int N, const int64_t *dims, int n, const int64_t *ranks,
                const double *X, const double *const *U, double *Y)
{
    if (check_dims(N, dims) || n < 0 || n >= N || !ranks || !X || !U || !Y)
        return -1;
    for (int m = 0; m < N; ++m)
        if (m != n && (U[m] == NULL || ranks[m] < 1)) return -1;

    int64_t cur_dims[ORACLE_MAX_ORDER];
    memcpy(cur_dims, dims, sizeof(int64_t) * (size_t)N);
    const double *cur = X;
    double *owned = NULL;
    int last = -1; /* last contracted mode */
    for (int m = N - 1; m >= 0; --m)
        if (m != n) { last = m; break; }
    if (last < 0) { /* N == 1: nothing to contract, Y = X */
        memcpy(Y, X, sizeof(double) * (size_t)dims[0]);
        return 0;
    }
    for (int m = 0; m < N; ++m) {
        if (m == n) continue;
        int64_t out_elems = 1;
        for (int p = 0; p < N; ++p) out_elems *= (p == m ? ranks[m] : cur_dims[p]);
        double *dst = (m == last) ? Y : (double *)malloc(sizeof(double) * (size_t)out_elems);
        if (!dst) { free(owned); return -2; }
        int rc = oracle_ttm(N, cur_dims, m, ranks[m], cur, U[m], dst);
        free(owned);
        owned = (m == last) ? NULL : dst;
        if (rc) { free(owned); return rc; }
        cur = dst;
        cur_dims[m] = ranks[m];
    }
    return 0;
}
