// fx20.hip -- encoder of the FX20 storage of X (20-bit fixed point, one
// power-of-two scale, an FP16 plane and an int8 plane; layout in include/deinsum.h).
#include <hip/hip_runtime.h>

#include <cmath>
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
        h->sumsq_q = 0;
        h->errsq_q = 0;
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

// Encodes, and records the storage error: each wave sums (x 2^-(e+19))^2 and the
// squared rounding error (x 2^-e - m)^2 in FP64 in a fixed order (the grid depends
// only on n), rounds the two sums to fixed point and adds them with integer
// atomics, so the header's totals do not depend on the order the waves finish in.
template <typename T>
__global__ void __launch_bounds__(256) fx20_encode_kernel(const T *__restrict__ x, int64_t n,
                                                          Fx20Header *__restrict__ h,
                                                          uint16_t *__restrict__ hi, uint8_t *__restrict__ lo)
{
    const int e = h->exp2;
    double ss = 0.0, es = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double xs = ldexp(static_cast<double>(x[i]), -e);
        double v = rint(xs);
        v = fmin(fmax(v, -524288.0), 524288.0);
        const int32_t m = static_cast<int32_t>(v);
        const int32_t hq = (m + 128) >> 8;  // floor division: m = 256 hq + l, l in [-128, 127]
        const int32_t l = m - 256 * hq;
        const _Float16 hf = static_cast<_Float16>(static_cast<float>(hq));  // |hq| <= 2048: exact
        hi[i] = __builtin_bit_cast(uint16_t, hf);
        lo[i] = static_cast<uint8_t>(static_cast<int8_t>(l));
        const double xu = xs * 0x1p-19;  // |xu| < 1
        ss += xu * xu;
        es += (xs - v) * (xs - v);        // |xs - v| <= 1/2
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ss += __shfl_xor(ss, off);
        es += __shfl_xor(es, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&h->sumsq_q),
                  static_cast<unsigned long long>(rint(ss * 0x1p24)));
        atomicAdd(reinterpret_cast<unsigned long long *>(&h->errsq_q),
                  static_cast<unsigned long long>(rint(es * 0x1p28)));
    }
}

unsigned grid_for(int64_t n) { return static_cast<unsigned>(n / 256 + 1 < 8192 ? n / 256 + 1 : 8192); }

// deinsum_tensor_stats: max |x| (exact, integer atomic max on the bit patterns), then
// the sum of (x 2^-e)^2 with max |x| < 2^e, per wave in FP64 in a fixed order and
// added in fixed point (units of 2^-24) with integer atomics.
struct StatsAcc {
    double max_abs;
    uint64_t sumsq_q;
};

__device__ __forceinline__ double elem_f64(const void *x, int dt, int64_t i)
{
    if (dt == DEINSUM_F64) return static_cast<const double *>(x)[i];
    if (dt == DEINSUM_F32) return static_cast<double>(static_cast<const float *>(x)[i]);
    return static_cast<double>(bf16_bits_to_f32(static_cast<const uint16_t *>(x)[i]));
}

__global__ void stats_init_kernel(StatsAcc *a)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        a->max_abs = 0.0;
        a->sumsq_q = 0;
    }
}

__global__ void __launch_bounds__(256) stats_max_kernel(const void *__restrict__ x, int dt, int64_t n,
                                                        StatsAcc *a)
{
    double m = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        m = fmax(m, fabs(elem_f64(x, dt, i)));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(&a->max_abs),
                  static_cast<unsigned long long>(__double_as_longlong(m)));
}

__global__ void __launch_bounds__(256) stats_sumsq_kernel(const void *__restrict__ x, int dt, int64_t n,
                                                          StatsAcc *a)
{
    int e = 0;
    (void)frexp(a->max_abs, &e);
    double ss = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double v = ldexp(elem_f64(x, dt, i), -e);
        ss += v * v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    if ((threadIdx.x & 63) == 0)
        atomicAdd(reinterpret_cast<unsigned long long *>(&a->sumsq_q),
                  static_cast<unsigned long long>(rint(ss * 0x1p24)));
}

}  // namespace

deinsum_status fx20_storage_error(const void *X, int64_t count, void *stream, double *err)
{
    if (!X || !err) return fail(DEINSUM_ERR_INVALID_ARG, "fx20 header: null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Fx20Header h{};
    if (hipMemcpyAsync(&h, X, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return fail(DEINSUM_ERR_DEVICE, "fx20 header: copy to the host failed");
    if (h.magic != kFx20Magic || h.count != count)
        return fail(DEINSUM_ERR_INVALID_ARG, "X is not an FX20 buffer of this tensor's element count");
    // ||X - X_stored|| / ||X|| = sqrt(errsq 2^-28 2^2e / (sumsq 2^-24 2^(2e+38))).
    *err = h.sumsq_q ? std::sqrt(static_cast<double>(h.errsq_q) / static_cast<double>(h.sumsq_q)) * 0x1p-21 : 0.0;
    return DEINSUM_OK;
}

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

deinsum_status deinsum_tensor_stats(const void *X, int32_t dtype, int64_t count, double *max_abs, double *rms,
                                    void *stream)
{
    if (!max_abs || !rms || count < 0 || (count > 0 && !X))
        return fail(DEINSUM_ERR_INVALID_ARG, "tensor_stats: bad argument");
    if (dtype != DEINSUM_F64 && dtype != DEINSUM_F32 && dtype != DEINSUM_BF16)
        return fail(DEINSUM_ERR_INVALID_ARG, "tensor_stats: dtype must be F64, F32 or BF16");
    *max_abs = 0.0;
    *rms = 0.0;
    if (count == 0) return DEINSUM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *buf = nullptr;
    if (deinsum_status st = pool_get(sizeof(StatsAcc), stream, &buf)) return st;
    StatsAcc *acc = static_cast<StatsAcc *>(buf);
    stats_init_kernel<<<1, 64, 0, s>>>(acc);
    stats_max_kernel<<<grid_for(count), 256, 0, s>>>(X, dtype, count, acc);
    stats_sumsq_kernel<<<grid_for(count), 256, 0, s>>>(X, dtype, count, acc);
    if (deinsum_status st = check_launch("tensor_stats")) return st;
    StatsAcc host{};
    if (hipMemcpyAsync(&host, acc, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(DEINSUM_ERR_DEVICE, "tensor_stats: copy of the result failed");
    int e = 0;
    (void)std::frexp(host.max_abs, &e);
    *max_abs = host.max_abs;
    *rms = std::ldexp(std::sqrt(static_cast<double>(host.sumsq_q) * 0x1p-24 / static_cast<double>(count)), e);
    clear_error();
    return DEINSUM_OK;
}

}  // extern "C"
