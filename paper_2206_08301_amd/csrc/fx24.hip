// fx24.hip -- encoder of the FX24 storage of X (24-bit fixed point, one
// power-of-two scale, two planes; layout in include/deinsum.h).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace deinsum {


namespace {

__global__ void fx24_init_kernel(Fx24Header *h, int64_t count)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        h->magic = 0;
        h->exp2 = 0;
        h->count = count;
        h->max_abs = 0.0;
    }
}

// max |x| into the header; the bit patterns of non-negative doubles order like
// the values, so an integer atomic max gives the exact maximum in any order.
template <typename T>
__global__ void __launch_bounds__(256) fx24_maxabs_kernel(const T *__restrict__ x, int64_t n, Fx24Header *h)
{
    double m = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        m = fmax(m, fabs(static_cast<double>(x[i])));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(&h->max_abs),
                  static_cast<unsigned long long>(__double_as_longlong(m)));
}

__global__ void fx24_exponent_kernel(Fx24Header *h)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int e = 0;
        if (h->max_abs > 0.0) {
            (void)frexp(h->max_abs, &e);  // max|X| < 2^e
            e -= 23;
        }
        h->exp2 = e;
        h->magic = kFx24Magic;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) fx24_encode_kernel(const T *__restrict__ x, int64_t n,
                                                          const Fx24Header *__restrict__ h,
                                                          uint16_t *__restrict__ hi, uint8_t *__restrict__ lo)
{
    const int e = h->exp2;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double v = rint(ldexp(static_cast<double>(x[i]), -e));
        v = fmin(fmax(v, -8388608.0), 8388607.0);
        const int32_t m = static_cast<int32_t>(v);
        hi[i] = static_cast<uint16_t>(static_cast<uint32_t>(m >> 8) & 0xffffu);
        lo[i] = static_cast<uint8_t>(m & 255);
    }
}

unsigned grid_for(int64_t n) { return static_cast<unsigned>(n / 256 + 1 < 8192 ? n / 256 + 1 : 8192); }

}  // namespace
}  // namespace deinsum

using namespace deinsum;

extern "C" {

deinsum_status deinsum_fx24_size(int64_t count, size_t *bytes)
{
    if (!bytes || count < 0) return fail(DEINSUM_ERR_INVALID_ARG, "fx24_size: bad argument");
    *bytes = static_cast<size_t>(fx24_bytes(count));
    return DEINSUM_OK;
}

deinsum_status deinsum_fx24_encode(const void *src, int32_t src_dtype, int64_t count, void *dst, size_t dst_bytes,
                                   void *stream)
{
    if (count < 0 || !dst || (count > 0 && !src)) return fail(DEINSUM_ERR_INVALID_ARG, "fx24_encode: bad argument");
    if (src_dtype != DEINSUM_F64 && src_dtype != DEINSUM_F32)
        return fail(DEINSUM_ERR_INVALID_ARG, "fx24_encode: source must be F64 or F32");
    if (dst_bytes < static_cast<size_t>(fx24_bytes(count)))
        return fail(DEINSUM_ERR_NO_MEMORY, "fx24_encode: destination smaller than deinsum_fx24_size(count)");
    if (reinterpret_cast<uintptr_t>(dst) % 256 != 0)
        return fail(DEINSUM_ERR_INVALID_ARG, "fx24_encode: destination must be 256-byte aligned");
    const size_t sb = src_dtype == DEINSUM_F64 ? 8 : 4;
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
    if (count > 0 && s0 < d0 + static_cast<uintptr_t>(fx24_bytes(count)) && d0 < s0 + count * sb)
        return fail(DEINSUM_ERR_INVALID_ARG, "fx24_encode: source and destination overlap");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Fx24Header *h = static_cast<Fx24Header *>(dst);
    uint16_t *hi = reinterpret_cast<uint16_t *>(static_cast<char *>(dst) + kFx24Header);
    uint8_t *lo = reinterpret_cast<uint8_t *>(static_cast<char *>(dst) + fx24_lo_offset(count));
    fx24_init_kernel<<<1, 64, 0, s>>>(h, count);
    if (deinsum_status st = check_launch("fx24_init")) return st;
    if (count > 0) {
        if (src_dtype == DEINSUM_F64)
            fx24_maxabs_kernel<double><<<grid_for(count), 256, 0, s>>>(static_cast<const double *>(src), count, h);
        else
            fx24_maxabs_kernel<float><<<grid_for(count), 256, 0, s>>>(static_cast<const float *>(src), count, h);
        if (deinsum_status st = check_launch("fx24_maxabs")) return st;
    }
    fx24_exponent_kernel<<<1, 64, 0, s>>>(h);
    if (deinsum_status st = check_launch("fx24_exponent")) return st;
    if (count > 0) {
        if (src_dtype == DEINSUM_F64)
            fx24_encode_kernel<double><<<grid_for(count), 256, 0, s>>>(static_cast<const double *>(src), count, h, hi, lo);
        else
            fx24_encode_kernel<float><<<grid_for(count), 256, 0, s>>>(static_cast<const float *>(src), count, h, hi, lo);
        if (deinsum_status st = check_launch("fx24_encode")) return st;
    }
    clear_error();
    return DEINSUM_OK;
}

}  // extern "C"
