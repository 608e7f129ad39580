// fx20.hip -- encoder of the FX20 storage of X (20-bit fixed point, one
// power-of-two scale, an FP16 plane and an int8 plane; layout in include/deinsum.h).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace deinsum {


namespace {

__global__ void fx20_init_kernel(Fx20Header *h, int64_t count)
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
__global__ void __launch_bounds__(256) fx20_maxabs_kernel(const T *__restrict__ x, int64_t n, Fx20Header *h)
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

__global__ void fx20_exponent_kernel(Fx20Header *h)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int e = 0;
        if (h->max_abs > 0.0) {
            (void)frexp(h->max_abs, &e);  // max|X| < 2^e
            e -= 19;
        }
        h->exp2 = e;
        h->magic = kFx20Magic;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) fx20_encode_kernel(const T *__restrict__ x, int64_t n,
                                                          const Fx20Header *__restrict__ h,
                                                          uint16_t *__restrict__ hi, uint8_t *__restrict__ lo)
{
    const int e = h->exp2;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double v = rint(ldexp(static_cast<double>(x[i]), -e));
        v = fmin(fmax(v, -524288.0), 524288.0);
        const int32_t m = static_cast<int32_t>(v);
        const int32_t hq = (m + 128) >> 8;  // floor division: m = 256 hq + l, l in [-128, 127]
        const int32_t l = m - 256 * hq;
        const _Float16 hf = static_cast<_Float16>(static_cast<float>(hq));  // |hq| <= 2048: exact
        hi[i] = __builtin_bit_cast(uint16_t, hf);
        lo[i] = static_cast<uint8_t>(static_cast<int8_t>(l));
    }
}

unsigned grid_for(int64_t n) { return static_cast<unsigned>(n / 256 + 1 < 8192 ? n / 256 + 1 : 8192); }

}  // namespace
}  // namespace deinsum

using namespace deinsum;

extern "C" {

deinsum_status deinsum_fx20_size(int64_t count, size_t *bytes)
{
    if (!bytes || count < 0) return fail(DEINSUM_ERR_INVALID_ARG, "fx20_size: bad argument");
    *bytes = static_cast<size_t>(fx20_bytes(count));
    return DEINSUM_OK;
}

deinsum_status deinsum_fx20_encode(const void *src, int32_t src_dtype, int64_t count, void *dst, size_t dst_bytes,
                                   void *stream)
{
    if (count < 0 || !dst || (count > 0 && !src)) return fail(DEINSUM_ERR_INVALID_ARG, "fx20_encode: bad argument");
    if (src_dtype != DEINSUM_F64 && src_dtype != DEINSUM_F32)
        return fail(DEINSUM_ERR_INVALID_ARG, "fx20_encode: source must be F64 or F32");
    if (dst_bytes < static_cast<size_t>(fx20_bytes(count)))
        return fail(DEINSUM_ERR_NO_MEMORY, "fx20_encode: destination smaller than deinsum_fx20_size(count)");
    if (reinterpret_cast<uintptr_t>(dst) % 256 != 0)
        return fail(DEINSUM_ERR_INVALID_ARG, "fx20_encode: destination must be 256-byte aligned");
    const size_t sb = src_dtype == DEINSUM_F64 ? 8 : 4;
    const uintptr_t s0 = reinterpret_cast<uintptr_t>(src), d0 = reinterpret_cast<uintptr_t>(dst);
    if (count > 0 && s0 < d0 + static_cast<uintptr_t>(fx20_bytes(count)) && d0 < s0 + count * sb)
        return fail(DEINSUM_ERR_INVALID_ARG, "fx20_encode: source and destination overlap");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Fx20Header *h = static_cast<Fx20Header *>(dst);
    uint16_t *hi = reinterpret_cast<uint16_t *>(static_cast<char *>(dst) + kFx20Header);
    uint8_t *lo = reinterpret_cast<uint8_t *>(static_cast<char *>(dst) + fx20_lo_offset(count));
    fx20_init_kernel<<<1, 64, 0, s>>>(h, count);
    if (deinsum_status st = check_launch("fx20_init")) return st;
    if (count > 0) {
        if (src_dtype == DEINSUM_F64)
            fx20_maxabs_kernel<double><<<grid_for(count), 256, 0, s>>>(static_cast<const double *>(src), count, h);
        else
            fx20_maxabs_kernel<float><<<grid_for(count), 256, 0, s>>>(static_cast<const float *>(src), count, h);
        if (deinsum_status st = check_launch("fx20_maxabs")) return st;
    }
    fx20_exponent_kernel<<<1, 64, 0, s>>>(h);
    if (deinsum_status st = check_launch("fx20_exponent")) return st;
    if (count > 0) {
        if (src_dtype == DEINSUM_F64)
            fx20_encode_kernel<double><<<grid_for(count), 256, 0, s>>>(static_cast<const double *>(src), count, h, hi, lo);
        else
            fx20_encode_kernel<float><<<grid_for(count), 256, 0, s>>>(static_cast<const float *>(src), count, h, hi, lo);
        if (deinsum_status st = check_launch("fx20_encode")) return st;
    }
    clear_error();
    return DEINSUM_OK;
}

}  // extern "C"
