// decomp.hip -- the two decompositions that consume MTTKRP and TTMc (the paper's
// motivation, Sec. I), run on the device around the library's kernels:
//   * CP-ALS (Kolda & Bader 2009, Sec. 3.4): sweeps over the modes, each an MTTKRP
//     (deinsum_mttkrp) and the normal-equations factor update of the serving loop
//     (als.hip) with the column norms kept as lambda; after each sweep the fit
//     1 - ||X - [[lambda; U]]|| / ||X|| from the identity
//       ||X - [[lambda; U]]||^2 = ||X||^2 - 2 <X, [[lambda; U]]> + ||[[lambda; U]]||^2,
//       <X, [[lambda; U]]> = sum_r lambda_r sum_i M[i, r] U^n[i, r]   (M: the last
//       mode's MTTKRP, which used every other factor as it now stands),
//       ||[[lambda; U]]||^2 = lambda^T (*_m U^m^T U^m) lambda;
//   * Tucker by HOOI (Kolda & Bader 2009, Sec. 4.2): per mode n, Y = the TTM chain
//     over every other mode (deinsum_ttmc), then U^n = the R_n leading left singular
//     vectors of the mode-n unfolding Y_(n), found by subspace iteration
//     Q <- orth(Y_(n) orth(Y_(n)^T Q)) to convergence (each orth a CholeskyQR done
//     twice; orthonormalising both half steps keeps the Gram matrices' condition at
//     that of Y's leading singular values, not its square), then
//     Rayleigh-Ritz: the eigenvectors W of T = (Y^T Q)^T (Y^T Q) (cyclic Jacobi) give
//     U^n = Q W, columns by decreasing eigenvalue, each signed so that its entry of
//     largest magnitude is positive; after each sweep the core G = Y x_n U^n^T of the
//     last mode and the fit 1 - sqrt(||X||^2 - ||G||^2) / ||X|| (orthonormal factors).
// Every reduction runs in a fixed order (FP64), so results are run-to-run
// deterministic.  The drivers read one scalar per sweep (and per subspace
// iteration) to the host to test convergence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "als.h"
#include "internal.h"
#include "kernels.h"

namespace deinsum {

namespace {

constexpr int kT = 256;            // threads per workgroup of the small kernels
constexpr int kMaxR = 64;          // ranks handled by the one-workgroup kernels
constexpr int kSumBlocks = 1024;   // partial sums of the deterministic reductions

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ double ldx(const void *x, int dt, int64_t i)
{
    if (dt == DEINSUM_F64) return static_cast<const double *>(x)[i];
    if (dt == DEINSUM_F32) return static_cast<double>(static_cast<const float *>(x)[i]);
    return static_cast<double>(bf16_bits_to_f32(static_cast<const uint16_t *>(x)[i]));
}

// Fixed-order tree sum of one value per thread of a 256-thread workgroup.
__device__ double block_sum(double v, double *lds)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (t < s) lds[t] += lds[t + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- sums of squares
// sum (a - b)^2 over n elements (b may be null), in kSumBlocks fixed partials.
__global__ void __launch_bounds__(kT) sumsq_partials_kernel(const void *a, int adt, const double *b, int64_t n,
                                                            double *partials)
{
    __shared__ double lds[kT];
    double s = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kT) {
        const double v = ldx(a, adt, i) - (b ? b[i] : 0.0);
        s += v * v;
    }
    const double t = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kT) sum_partials_kernel(const double *partials, int n, double *out)
{
    __shared__ double lds[kT];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kT) s += partials[i];
    const double t = block_sum(s, lds);
    if (threadIdx.x == 0) *out = t;
}

deinsum_status sumsq(const void *a, int adt, const double *b, int64_t n, double *partials, double *out, hipStream_t s)
{
    sumsq_partials_kernel<<<kSumBlocks, kT, 0, s>>>(a, adt, b, n, partials);
    sum_partials_kernel<<<1, kT, 0, s>>>(partials, kSumBlocks, out);
    return check_launch("decomp_sumsq");
}

// ---------------------------------------------------------------- CP fit
struct CpFitArgs {
    const double *M;        // I_n x R, the last mode's MTTKRP
    const void *Un;         // I_n x R, its updated factor (storage udt)
    int udt;
    const double *lambda;   // R
    const double *G;        // order x R x R Gram cache (normalised factors)
    int order, R;
    int64_t In;
    const double *xnorm2;
    double *out;            // [0] fit, [1] <X, model>, [2] ||model||^2
};

__global__ void __launch_bounds__(kT) cp_fit_kernel(const CpFitArgs a)
{
    __shared__ double lds[kT];
    const int R = a.R;
    double ip = 0.0;
    for (int64_t e = threadIdx.x; e < a.In * R; e += kT)
        ip += a.lambda[e % R] * a.M[e] * ldx(a.Un, a.udt, e);
    ip = block_sum(ip, lds);
    double nm = 0.0;
    for (int e = threadIdx.x; e < R * R; e += kT) {
        double h = a.lambda[e / R] * a.lambda[e % R];
        for (int m = 0; m < a.order; ++m) h *= a.G[static_cast<int64_t>(m) * R * R + e];
        nm += h;
    }
    nm = block_sum(nm, lds);
    if (threadIdx.x == 0) {
        const double x2 = *a.xnorm2;
        const double res2 = fmax(0.0, x2 - 2.0 * ip + nm);
        a.out[0] = x2 > 0.0 ? 1.0 - sqrt(res2) / sqrt(x2) : 0.0;
        a.out[1] = ip;
        a.out[2] = nm;
    }
}

// ---------------------------------------------------------------- HOOI building blocks
// Y viewed as [pre][In][post] (the mode-n unfolding's row index i, column (p, q)).
struct YView {
    const double *Y;
    int64_t pre, In, post;
};

// out[p*sp + q*sq + r*sr] = sum_i Y[p, i, q] Q[i, r]   (Y_(n)^T Q, or the core).
__global__ void __launch_bounds__(kT) ytq_kernel(const YView y, const double *Q, int R, double *out, int64_t sp,
                                                 int64_t sq, int64_t sr)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    const int64_t P = y.pre * y.post;
    if (e >= P * R) return;
    const int r = static_cast<int>(e % R);
    const int64_t pq = e / R, p = pq / y.post, q = pq % y.post;
    const double *col = y.Y + p * y.In * y.post + q;
    double s = 0.0;
    for (int64_t i = 0; i < y.In; ++i) s += col[i * y.post] * Q[i * R + r];
    out[p * sp + q * sq + r * sr] = s;
}

// Z[i, r] = sum_{p,q} Y[p, i, q] B[p*post + q, r]: one workgroup per row i, lane r of
// each of the four waves, waves over (p, q) in a fixed stride, then summed in wave order.
__global__ void __launch_bounds__(kT) yb_kernel(const YView y, const double *B, int R, double *Z)
{
    __shared__ double part[4][kMaxR];
    const int64_t i = blockIdx.x;
    const int w = threadIdx.x >> 6, r = threadIdx.x & 63;
    const int64_t P = y.pre * y.post;
    double s = 0.0;
    if (r < R)
        for (int64_t pq = w; pq < P; pq += 4) {
            const int64_t p = pq / y.post, q = pq % y.post;
            s += y.Y[(p * y.In + i) * y.post + q] * B[pq * R + r];
        }
    part[w][r] = s;
    __syncthreads();
    if (w == 0 && r < R) Z[i * R + r] = ((part[0][r] + part[1][r]) + part[2][r]) + part[3][r];
}

// out[r1, r2] = sum_i A[i, r1] B[i, r2] (A, B: rows x R): one workgroup per (r1, r2).
__global__ void __launch_bounds__(kT) crossprod_kernel(const double *A, const double *B, int64_t rows, int R,
                                                       double *out)
{
    __shared__ double lds[kT];
    const int r1 = blockIdx.x / R, r2 = blockIdx.x % R;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += kT) s += A[i * R + r1] * B[i * R + r2];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[r1 * R + r2] = s;
}

// out[i, c] = sum_k A[i, k] W[k, c] (A rows x R, W R x R).
__global__ void __launch_bounds__(kT) rowmat_kernel(const double *A, const double *W, int64_t rows, int R,
                                                    double *out)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (e >= rows * R) return;
    const int64_t i = e / R;
    const int c = static_cast<int>(e % R);
    double s = 0.0;
    for (int k = 0; k < R; ++k) s += A[i * R + k] * W[k * R + c];
    out[e] = s;
}

// G (R x R, symmetric positive definite) = L L^T; W = L^{-T} (upper triangular), so
// that Z W has orthonormal columns when G = Z^T Z.  *bad = 1 on a pivot that is not
// positive relative to the largest diagonal entry (rank-deficient Z).
__global__ void __launch_bounds__(kT) chol_inv_kernel(const double *G, int R, double *W, int *bad)
{
    __shared__ double L[kMaxR][kMaxR + 1];
    __shared__ double Li[kMaxR][kMaxR + 1];
    __shared__ double dmax;
    const int t = threadIdx.x;
    for (int e = t; e < R * R; e += kT) {
        L[e / R][e % R] = G[e];
        Li[e / R][e % R] = 0.0;
    }
    __syncthreads();
    if (t == 0) {
        double m = 0.0;
        for (int k = 0; k < R; ++k) m = fmax(m, L[k][k]);
        dmax = m;
    }
    __syncthreads();
    // Right-looking Cholesky, one column per step (lower triangle of L).
    for (int k = 0; k < R; ++k) {
        if (t == 0) {
            const double d = L[k][k];
            if (!(d > 1e-28 * dmax)) *bad = 1;
            L[k][k] = sqrt(fmax(d, 1e-300));
        }
        __syncthreads();
        for (int i = k + 1 + t; i < R; i += kT) L[i][k] /= L[k][k];
        __syncthreads();
        for (int e = t; e < R * R; e += kT) {
            const int i = e / R, j = e % R;
            if (i > k && j > k && j <= i) L[i][j] -= L[i][k] * L[j][k];
        }
        __syncthreads();
    }
    // Li = L^{-1} by forward substitution, one column of the identity per thread.
    if (t < R) {
        const int c = t;
        for (int i = 0; i < R; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= L[i][k] * Li[k][c];
            Li[i][c] = (i >= c) ? s / L[i][i] : 0.0;
        }
    }
    __syncthreads();
    for (int e = t; e < R * R; e += kT) W[e] = Li[e % R][e / R];  // W = Li^T
}

// Eigenvectors of the symmetric R x R matrix T by cyclic Jacobi rotations, columns of
// V ordered by decreasing eigenvalue (one workgroup).
__global__ void __launch_bounds__(kT) jacobi_eig_kernel(const double *T, int R, double *V, double *evals)
{
    __shared__ double A[kMaxR][kMaxR + 1];
    __shared__ double E[kMaxR][kMaxR + 1];
    __shared__ double cs[2];
    __shared__ double off;
    __shared__ int order[kMaxR];
    const int t = threadIdx.x;
    for (int e = t; e < R * R; e += kT) {
        A[e / R][e % R] = T[e];
        E[e / R][e % R] = (e / R == e % R) ? 1.0 : 0.0;
    }
    __syncthreads();
    double total = 0.0;
    if (t == 0) {
        for (int e = 0; e < R * R; ++e) total += A[e / R][e % R] * A[e / R][e % R];
        off = total;
    }
    __syncthreads();
    const double tiny = 1e-30 * off;
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (t == 0) {
            double o = 0.0;
            for (int i = 0; i < R; ++i)
                for (int j = 0; j < R; ++j)
                    if (i != j) o += A[i][j] * A[i][j];
            off = o;
        }
        __syncthreads();
        const bool done = !(off > tiny);
        __syncthreads();  // every thread has read `off` before thread 0 writes it again
        if (done) break;
        for (int p = 0; p < R - 1; ++p)
            for (int q = p + 1; q < R; ++q) {
                if (t == 0) {
                    const double apq = A[p][q];
                    double c = 1.0, s = 0.0;
                    if (apq != 0.0) {
                        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                        const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(tt * tt + 1.0);
                        s = tt * c;
                    }
                    cs[0] = c;
                    cs[1] = s;
                }
                __syncthreads();
                const double c = cs[0], s = cs[1];
                if (s != 0.0) {
                    // A <- J^T A J on rows/columns p, q; E <- E J.
                    if (t < R) {
                        const double akp = A[t][p], akq = A[t][q];
                        A[t][p] = c * akp - s * akq;
                        A[t][q] = s * akp + c * akq;
                    }
                    __syncthreads();
                    if (t < R) {
                        const double apk = A[p][t], aqk = A[q][t];
                        A[p][t] = c * apk - s * aqk;
                        A[q][t] = s * apk + c * aqk;
                        const double ekp = E[t][p], ekq = E[t][q];
                        E[t][p] = c * ekp - s * ekq;
                        E[t][q] = s * ekp + c * ekq;
                    }
                }
                __syncthreads();
            }
    }
    if (t == 0) {
        for (int k = 0; k < R; ++k) order[k] = k;
        for (int a = 0; a < R; ++a)  // selection sort, decreasing eigenvalue (stable)
            for (int b = a + 1; b < R; ++b)
                if (A[order[b]][order[b]] > A[order[a]][order[a]]) {
                    const int tmp = order[a];
                    order[a] = order[b];
                    order[b] = tmp;
                }
    }
    __syncthreads();
    for (int e = t; e < R * R; e += kT) V[e] = E[e / R][order[e % R]];
    if (t < R) evals[t] = A[order[t]][order[t]];
}

// Each column of U (rows x R) times -1 when its entry of largest magnitude (the first
// on ties) is negative; written in the factor's storage precision.
__global__ void __launch_bounds__(kT) signfix_store_kernel(const double *U, int64_t rows, int R, void *out, int odt)
{
    __shared__ double bv[kT];
    __shared__ int64_t bi[kT];
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    double best = -1.0;
    int64_t arg = rows;
    for (int64_t i = t; i < rows; i += kT) {
        const double v = fabs(U[i * R + c]);
        if (v > best) {
            best = v;
            arg = i;
        }
    }
    bv[t] = best;
    bi[t] = arg;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (t < s && (bv[t + s] > bv[t] || (bv[t + s] == bv[t] && bi[t + s] < bi[t]))) {
            bv[t] = bv[t + s];
            bi[t] = bi[t + s];
        }
        __syncthreads();
    }
    const double sg = (bi[0] < rows && U[bi[0] * R + c] < 0.0) ? -1.0 : 1.0;
    for (int64_t i = t; i < rows; i += kT) {
        const double v = sg * U[i * R + c];
        if (odt == DEINSUM_F64) static_cast<double *>(out)[i * R + c] = v;
        else static_cast<float *>(out)[i * R + c] = static_cast<float>(v);
    }
}

__global__ void zero_i32_kernel(int *p)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

__global__ void __launch_bounds__(kT) to_f64_kernel(const void *src, int dt, int64_t n, double *dst)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kT + threadIdx.x;
    if (e < n) dst[e] = ldx(src, dt, e);
}

unsigned grid(int64_t n) { return static_cast<unsigned>(cdiv(n, kT)); }

deinsum_spec spec_for(int kind, int order, int n)
{
    deinsum_spec sp;
    std::memset(&sp, 0, sizeof(sp));
    sp.kind = kind;
    sp.order = order;
    sp.free_mode = n;
    sp.n_factors = order - 1;
    int k = 0;
    for (int m = 0; m < order; ++m) {
        sp.tensor_idx[m] = static_cast<char>('a' + m);
        sp.rank_idx[m] = m == n ? '-' : static_cast<char>(kind == DEINSUM_TTMC ? 'A' + m : 'z');
        sp.out_idx[m] = m == n ? sp.tensor_idx[m] : sp.rank_idx[m];
        sp.operand_of_mode[m] = -1;
        if (m == n) continue;
        sp.factor_mode[k] = m;
        sp.operand_of_mode[m] = k;
        ++k;
    }
    if (kind == DEINSUM_MTTKRP) {
        sp.out_idx[0] = sp.tensor_idx[n];
        sp.out_idx[1] = 'z';
        sp.out_idx[2] = 0;
    }
    return sp;
}

// Device state of a driver: one allocation, released on every exit path.
struct DevBuf {
    char *p = nullptr;
    ~DevBuf()
    {
        if (p) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
        }
    }
};

deinsum_status read_scalars(const double *d, double *h, int n, hipStream_t s)
{
    if (hipMemcpyAsync(h, d, sizeof(double) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(DEINSUM_ERR_DEVICE, "decomposition: copy of a convergence scalar failed");
    return DEINSUM_OK;
}

deinsum_status check_common(int32_t order, const int64_t *dims, const void *X, void *const *U,
                            const deinsum_decomp_opts &o)
{
    if (order < 2 || order > DEINSUM_MAX_ORDER) return fail(DEINSUM_ERR_SHAPE, "order must be 2..8");
    if (!dims || !X || !U) return fail(DEINSUM_ERR_INVALID_ARG, "null dims, X or factor table");
    for (int m = 0; m < order; ++m) {
        if (dims[m] < 1) return fail(DEINSUM_ERR_SHAPE, "dims must be >= 1");
        if (!U[m]) return fail(DEINSUM_ERR_INVALID_ARG, "null factor");
    }
    if (o.max_sweeps < 1) return fail(DEINSUM_ERR_INVALID_ARG, "max_sweeps must be >= 1");
    if (!(o.tol >= 0)) return fail(DEINSUM_ERR_INVALID_ARG, "tol must be >= 0");
    return DEINSUM_OK;
}

}  // namespace
}  // namespace deinsum

using namespace deinsum;

extern "C" {

void deinsum_decomp_opts_init(deinsum_decomp_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = DEINSUM_PREC_FP64;
    o->max_sweeps = 25;
    o->tol = 1e-10;
    o->max_iters = 200;
    o->iter_tol = 1e-11;
}

deinsum_status deinsum_cp_als(int32_t order, const int64_t *dims, int64_t R, const void *X, void *const *U,
                              double *lambda, const deinsum_decomp_opts *opts, deinsum_decomp_result *result,
                              void *stream)
{
    deinsum_decomp_opts o;
    deinsum_decomp_opts_init(&o);
    if (opts) o = *opts;
    if (deinsum_status st = check_common(order, dims, X, U, o)) return st;
    if (R < 1 || R > kAlsMaxRank) return fail(DEINSUM_ERR_SHAPE, "CP rank must be 1..64");
    if (!lambda) return fail(DEINSUM_ERR_INVALID_ARG, "null lambda");
    if (o.precision != DEINSUM_PREC_FP64 && o.precision != DEINSUM_PREC_FP32 && o.precision != DEINSUM_PREC_BF16X3)
        return fail(DEINSUM_ERR_UNSUPPORTED, "CP-ALS runs the FP64, FP32 and BF16X3 MTTKRP forms");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int xdt = o.precision == DEINSUM_PREC_FP64 ? DEINSUM_F64 : DEINSUM_F32;
    int64_t maxd = 0, nx = 1;
    for (int m = 0; m < order; ++m) {
        maxd = std::max(maxd, dims[m]);
        nx *= dims[m];
    }
    // State: M, Xs (maxd x R), partial Grams, Gram cache, sum partials, scalars, flag.
    const size_t rows = static_cast<size_t>(maxd * R) * 8;
    const size_t gp = static_cast<size_t>(als_blocks(maxd) * R * R) * 8;
    const size_t g = static_cast<size_t>(order * R * R) * 8;
    const size_t part = kSumBlocks * 8;
    const size_t total = 2 * rows + gp + g + part + 64;
    DevBuf buf;
    if (hipMalloc(reinterpret_cast<void **>(&buf.p), total) != hipSuccess) {
        (void)hipGetLastError();
        buf.p = nullptr;
        return fail(DEINSUM_ERR_NO_MEMORY, "cp_als: state allocation failed");
    }
    double *M = reinterpret_cast<double *>(buf.p);
    double *Xs = reinterpret_cast<double *>(buf.p + rows);
    double *Gp = reinterpret_cast<double *>(buf.p + 2 * rows);
    double *G = reinterpret_cast<double *>(buf.p + 2 * rows + gp);
    double *partials = reinterpret_cast<double *>(buf.p + 2 * rows + gp + g);
    double *scal = reinterpret_cast<double *>(buf.p + 2 * rows + gp + g + part);  // xnorm2, fit, ip, nrm2
    int32_t *flag = reinterpret_cast<int32_t *>(scal + 4);
    zero_i32_kernel<<<1, 64, 0, s>>>(flag);
    AlsJob job;
    std::memset(&job, 0, sizeof(job));
    job.order = order;
    job.R = static_cast<int32_t>(R);
    job.prec = xdt == DEINSUM_F64 ? P_FP64 : P_FP32;
    for (int m = 0; m < order; ++m) {
        job.dims[m] = dims[m];
        job.U[m] = U[m];
    }
    job.M = M;
    job.Xs = Xs;
    job.Gp = Gp;
    job.G = G;
    job.flag = flag;
    job.lambda = lambda;
    if (deinsum_status st = launch_als_grams(job, s)) return st;
    if (deinsum_status st = sumsq(X, xdt, nullptr, nx, partials, scal, s)) return st;
    double prev = NAN, fit = NAN;
    int sweep = 0;
    for (; sweep < o.max_sweeps; ++sweep) {
        for (int n = 0; n < order; ++n) {
            const deinsum_spec sp = spec_for(DEINSUM_MTTKRP, order, n);
            const void *ops[DEINSUM_MAX_ORDER];
            for (int k = 0; k < order - 1; ++k) ops[k] = U[sp.factor_mode[k]];
            deinsum_opts mo;
            deinsum_opts_init(&mo);
            mo.precision = o.precision;
            mo.out_dtype = DEINSUM_F64;
            if (deinsum_status st = deinsum_mttkrp(&sp, dims, R, X, ops, M, &mo, s)) return st;
            job.mode = n;
            if (deinsum_status st = launch_als_one(job, s)) return st;
        }
        CpFitArgs fa;
        fa.M = M;
        fa.Un = U[order - 1];
        fa.udt = xdt;
        fa.lambda = lambda;
        fa.G = G;
        fa.order = order;
        fa.R = static_cast<int>(R);
        fa.In = dims[order - 1];
        fa.xnorm2 = scal;
        fa.out = scal + 1;
        cp_fit_kernel<<<1, kT, 0, s>>>(fa);
        if (deinsum_status st = check_launch("cp_fit")) return st;
        double h[1];
        if (deinsum_status st = read_scalars(scal + 1, h, 1, s)) return st;
        fit = h[0];
        if (o.fit_trace) o.fit_trace[sweep] = fit;
        if (sweep > 0 && std::fabs(fit - prev) < o.tol) {
            ++sweep;
            break;
        }
        prev = fit;
    }
    int32_t hflag = 0;
    if (hipMemcpyAsync(&hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(DEINSUM_ERR_DEVICE, "cp_als: final synchronisation failed");
    if (result) {
        std::memset(result, 0, sizeof(*result));
        result->sweeps = std::min(sweep, o.max_sweeps);
        result->fit = fit;
        result->flags = hflag ? DEINSUM_DECOMP_REGULARISED : 0;
    }
    clear_error();
    return DEINSUM_OK;
}

deinsum_status deinsum_tucker_hooi(int32_t order, const int64_t *dims, const int64_t *ranks, const void *X,
                                   void *const *U, double *core, const deinsum_decomp_opts *opts,
                                   deinsum_decomp_result *result, void *stream)
{
    deinsum_decomp_opts o;
    deinsum_decomp_opts_init(&o);
    if (opts) o = *opts;
    if (deinsum_status st = check_common(order, dims, X, U, o)) return st;
    if (!ranks || !core) return fail(DEINSUM_ERR_INVALID_ARG, "null ranks or core");
    if (o.precision != DEINSUM_PREC_FP64 && o.precision != DEINSUM_PREC_FP32)
        return fail(DEINSUM_ERR_UNSUPPORTED, "HOOI runs the FP64 and FP32 TTMc forms");
    if (o.max_iters < 1 || !(o.iter_tol > 0)) return fail(DEINSUM_ERR_INVALID_ARG, "max_iters >= 1, iter_tol > 0");
    double prodr = 1;
    for (int m = 0; m < order; ++m) {
        if (ranks[m] < 1 || ranks[m] > 64 || ranks[m] > dims[m])
            return fail(DEINSUM_ERR_SHAPE, "Tucker ranks must be 1..min(64, dims[m])");
        prodr *= static_cast<double>(ranks[m]);
    }
    for (int m = 0; m < order; ++m)
        if (static_cast<double>(ranks[m]) > prodr / static_cast<double>(ranks[m]))
            return fail(DEINSUM_ERR_SHAPE, "each Tucker rank must be at most the product of the others");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int xdt = o.precision == DEINSUM_PREC_FP64 ? DEINSUM_F64 : DEINSUM_F32;
    int64_t nx = 1, maxd = 0, ymax = 0, pmax = 0;
    for (int m = 0; m < order; ++m) {
        nx *= dims[m];
        maxd = std::max(maxd, dims[m]);
    }
    for (int n = 0; n < order; ++n) {
        int64_t P = 1;
        for (int m = 0; m < order; ++m)
            if (m != n) P *= ranks[m];
        ymax = std::max(ymax, P * dims[n]);
        pmax = std::max(pmax, P);
    }
    const size_t yb = static_cast<size_t>(ymax) * 8, bb = static_cast<size_t>(pmax * kMaxR) * 8;
    const size_t qb = static_cast<size_t>(maxd * kMaxR) * 8, rr = static_cast<size_t>(kMaxR * kMaxR) * 8;
    const size_t total = yb + 2 * bb + 4 * qb + 4 * rr + kSumBlocks * 8 + 64;
    DevBuf buf;
    if (hipMalloc(reinterpret_cast<void **>(&buf.p), total) != hipSuccess) {
        (void)hipGetLastError();
        buf.p = nullptr;
        return fail(DEINSUM_ERR_NO_MEMORY, "tucker_hooi: state allocation failed");
    }
    char *c = buf.p;
    double *Y = reinterpret_cast<double *>(c); c += yb;
    double *B = reinterpret_cast<double *>(c); c += bb;
    double *B2 = reinterpret_cast<double *>(c); c += bb;
    double *Q = reinterpret_cast<double *>(c); c += qb;
    double *Z = reinterpret_cast<double *>(c); c += qb;
    double *Q1 = reinterpret_cast<double *>(c); c += qb;
    double *E = reinterpret_cast<double *>(c); c += qb;
    double *Gm = reinterpret_cast<double *>(c); c += rr;
    double *W = reinterpret_cast<double *>(c); c += rr;
    double *V = reinterpret_cast<double *>(c); c += rr;
    double *ev = reinterpret_cast<double *>(c); c += rr;
    double *partials = reinterpret_cast<double *>(c); c += kSumBlocks * 8;
    double *scal = reinterpret_cast<double *>(c);  // xnorm2, gnorm2, delta2
    int *bad = reinterpret_cast<int *>(scal + 3);
    zero_i32_kernel<<<1, 64, 0, s>>>(bad);
    // out = A with orthonormal columns (rows x R), by CholeskyQR twice through tmp.
    auto cholqr2 = [&](const double *A, int64_t rows, int R, double *tmp, double *out) {
        crossprod_kernel<<<R * R, kT, 0, s>>>(A, A, rows, R, Gm);
        chol_inv_kernel<<<1, kT, 0, s>>>(Gm, R, W, bad);
        rowmat_kernel<<<grid(rows * R), kT, 0, s>>>(A, W, rows, R, tmp);
        crossprod_kernel<<<R * R, kT, 0, s>>>(tmp, tmp, rows, R, Gm);
        chol_inv_kernel<<<1, kT, 0, s>>>(Gm, R, W, bad);
        rowmat_kernel<<<grid(rows * R), kT, 0, s>>>(tmp, W, rows, R, out);
    };
    if (deinsum_status st = sumsq(X, xdt, nullptr, nx, partials, scal, s)) return st;
    double xnorm2 = 0;
    if (deinsum_status st = read_scalars(scal, &xnorm2, 1, s)) return st;
    double prev = NAN, fit = NAN;
    int64_t iters_total = 0;
    int32_t flags = 0;
    int sweep = 0;
    for (; sweep < o.max_sweeps; ++sweep) {
        YView yv{Y, 1, 1, 1};
        for (int n = 0; n < order; ++n) {
            // Y = X x_m U^m^T for every m != n, i_n in place, FP64.
            const deinsum_spec sp = spec_for(DEINSUM_TTMC, order, n);
            const void *ops[DEINSUM_MAX_ORDER];
            int64_t rk[DEINSUM_MAX_ORDER];
            for (int k = 0; k < order - 1; ++k) {
                ops[k] = U[sp.factor_mode[k]];
                rk[k] = ranks[sp.factor_mode[k]];
            }
            deinsum_opts to;
            deinsum_opts_init(&to);
            to.precision = o.precision;
            to.out_dtype = DEINSUM_F64;
            if (deinsum_status st = deinsum_ttmc(&sp, dims, rk, X, ops, Y, &to, s)) return st;
            yv.pre = yv.post = 1;
            for (int m = 0; m < order; ++m) {
                if (m < n) yv.pre *= ranks[m];
                if (m > n) yv.post *= ranks[m];
            }
            yv.In = dims[n];
            const int Rn = static_cast<int>(ranks[n]);
            const int64_t In = dims[n], P = yv.pre * yv.post;
            to_f64_kernel<<<grid(In * Rn), kT, 0, s>>>(U[n], xdt, In * Rn, Q);
            int it = 0;
            for (; it < o.max_iters; ++it) {
                // Q_new = orth(Y_(n) orth(Y_(n)^T Q)).
                ytq_kernel<<<grid(P * Rn), kT, 0, s>>>(yv, Q, Rn, B, static_cast<int64_t>(yv.post) * Rn, Rn, 1);
                cholqr2(B, P, Rn, B2, B);
                yb_kernel<<<static_cast<unsigned>(In), kT, 0, s>>>(yv, B, Rn, Z);
                cholqr2(Z, In, Rn, Q1, Z);  // Z: the new Q
                // Subspace change ||Q_new - Q Q^T Q_new||_F.
                crossprod_kernel<<<Rn * Rn, kT, 0, s>>>(Q, Z, In, Rn, Gm);
                rowmat_kernel<<<grid(In * Rn), kT, 0, s>>>(Q, Gm, In, Rn, E);
                if (deinsum_status st = sumsq(Z, DEINSUM_F64, E, In * Rn, partials, scal + 2, s)) return st;
                std::swap(Q, Z);
                double h[1];
                if (deinsum_status st = read_scalars(scal + 2, h, 1, s)) return st;
                if (std::sqrt(h[0]) < o.iter_tol) {
                    ++it;
                    break;
                }
            }
            if (it >= o.max_iters) flags |= DEINSUM_DECOMP_MAX_ITERS;
            iters_total += it;
            // Rayleigh-Ritz: T = (Y^T Q)^T (Y^T Q), U^n = Q W by decreasing eigenvalue.
            ytq_kernel<<<grid(P * Rn), kT, 0, s>>>(yv, Q, Rn, B, static_cast<int64_t>(yv.post) * Rn, Rn, 1);
            crossprod_kernel<<<Rn * Rn, kT, 0, s>>>(B, B, P, Rn, Gm);
            jacobi_eig_kernel<<<1, kT, 0, s>>>(Gm, Rn, V, ev);
            rowmat_kernel<<<grid(In * Rn), kT, 0, s>>>(Q, V, In, Rn, Q1);
            signfix_store_kernel<<<Rn, kT, 0, s>>>(Q1, In, Rn, U[n], xdt);
            if (deinsum_status st = check_launch("tucker_hooi_mode")) return st;
        }
        // Core G = Y x_{N-1} U^{N-1}^T (Y: the last mode's chain), layout [r_0 .. r_{N-1}].
        const int Rl = static_cast<int>(ranks[order - 1]);
        to_f64_kernel<<<grid(dims[order - 1] * Rl), kT, 0, s>>>(U[order - 1], xdt, dims[order - 1] * Rl, Q);
        ytq_kernel<<<grid(yv.pre * Rl), kT, 0, s>>>(yv, Q, Rl, core, Rl, 0, 1);
        if (deinsum_status st = check_launch("tucker_hooi_core")) return st;
        if (deinsum_status st = sumsq(core, DEINSUM_F64, nullptr, static_cast<int64_t>(prodr), partials, scal + 1, s))
            return st;
        double g2 = 0;
        if (deinsum_status st = read_scalars(scal + 1, &g2, 1, s)) return st;
        fit = xnorm2 > 0 ? 1.0 - std::sqrt(std::max(0.0, xnorm2 - g2)) / std::sqrt(xnorm2) : 0.0;
        if (o.fit_trace) o.fit_trace[sweep] = fit;
        if (sweep > 0 && std::fabs(fit - prev) < o.tol) {
            ++sweep;
            break;
        }
        prev = fit;
    }
    int hbad = 0;
    if (hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(DEINSUM_ERR_DEVICE, "tucker_hooi: final synchronisation failed");
    if (hbad) flags |= DEINSUM_DECOMP_RANK_DEFICIENT;
    if (result) {
        std::memset(result, 0, sizeof(*result));
        result->sweeps = std::min(sweep, o.max_sweeps);
        result->fit = fit;
        result->flags = flags;
        result->iters = iters_total;
    }
    clear_error();
    return DEINSUM_OK;
}

}  // extern "C"
