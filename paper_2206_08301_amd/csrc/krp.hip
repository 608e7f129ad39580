// krp.hip -- Khatri-Rao product of two factor matrices, the column-wise Kronecker
// product of Sec. III-B.  For two adjacent contracted modes a, b of X it is the
// factor of the merged mode with index i_a * I_b + i_b.
#include "krp.h"

#include "internal.h"

namespace deinsum {
namespace {

template <typename T>
__global__ void __launch_bounds__(256) krp2_kernel(const T *__restrict__ A, const T *__restrict__ B, int64_t Ib,
                                                   int64_t R, int64_t total, T *__restrict__ K)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t r = e % R;
    const int64_t row = e / R;
    K[e] = A[(row / Ib) * R + r] * B[(row % Ib) * R + r];
}

template <typename T>
__global__ void __launch_bounds__(256) chain_mm_kernel(const double *__restrict__ M, const T *__restrict__ C,
                                                       int64_t I, int64_t R, int64_t L, void *Y, int out_dtype)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= I * L) return;
    const int64_t i = e / L, l = e % L;
    double acc = 0.0;
    for (int64_t r = 0; r < R; ++r) acc += M[i * R + r] * static_cast<double>(C[r * L + l]);
    if (out_dtype == DEINSUM_F64) static_cast<double *>(Y)[e] = acc;
    else static_cast<float *>(Y)[e] = static_cast<float>(acc);
}

}  // namespace

deinsum_status launch_chain_mm(const double *M, const void *C, int c_elem_bytes, int64_t I, int64_t R, int64_t L,
                               void *Y, int out_dtype, hipStream_t s)
{
    const int64_t total = I * L;
    if (total == 0) return DEINSUM_OK;
    const unsigned grid = static_cast<unsigned>((total + 255) / 256);
    if (c_elem_bytes == 8)
        chain_mm_kernel<double><<<grid, 256, 0, s>>>(M, static_cast<const double *>(C), I, R, L, Y, out_dtype);
    else
        chain_mm_kernel<float><<<grid, 256, 0, s>>>(M, static_cast<const float *>(C), I, R, L, Y, out_dtype);
    if (hipGetLastError() != hipSuccess) return fail(DEINSUM_ERR_DEVICE, "chain product launch failed");
    return DEINSUM_OK;
}

deinsum_status launch_krp2(const void *A, const void *B, int64_t Ia, int64_t Ib, int64_t R, int elem_bytes,
                           void *K, hipStream_t s)
{
    const int64_t total = Ia * Ib * R;
    if (total == 0) return DEINSUM_OK;
    const unsigned grid = static_cast<unsigned>((total + 255) / 256);
    if (elem_bytes == 8)
        krp2_kernel<double><<<grid, 256, 0, s>>>(static_cast<const double *>(A), static_cast<const double *>(B), Ib, R,
                                                 total, static_cast<double *>(K));
    else
        krp2_kernel<float><<<grid, 256, 0, s>>>(static_cast<const float *>(A), static_cast<const float *>(B), Ib, R,
                                                total, static_cast<float *>(K));
    if (hipGetLastError() != hipSuccess) return fail(DEINSUM_ERR_DEVICE, "krp2 launch failed");
    return DEINSUM_OK;
}

}  // namespace deinsum
