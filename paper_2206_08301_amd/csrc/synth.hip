// synth.hip -- synthetic input generation and dtype conversion on the device
// (setup for the benchmarks and tests; not part of the method).
//
// Counter-based SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): element e of
// a stream seeded with s is mix64(s + (e + 1) * golden_gamma).  Each thread
// produces one element from its index, so any sub-range can be generated
// independently and the device values equal the host generator's bit for bit.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace deinsum {

namespace {

__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double synth_value(uint64_t seed, uint64_t index, int dist)
{
    const uint64_t z = splitmix64_mix(seed + (index + 1ull) * 0x9E3779B97F4A7C15ull);
    if (dist == 1) return static_cast<double>(static_cast<int64_t>((z >> 32) % 5ull)) - 2.0;
    if (dist == 2) return static_cast<double>(static_cast<int64_t>((z >> 32) % 3ull)) - 1.0;
    return 2.0 * (static_cast<double>(z >> 11) * 0x1.0p-53) - 1.0;
}

template <typename T>
__global__ void __launch_bounds__(256) synth_fill_kernel(T *__restrict__ x, int64_t count,
                                                         uint64_t seed, int64_t offset, int dist)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += stride)
        x[e] = from_f64<T>(synth_value(seed, static_cast<uint64_t>(offset + e), dist));
}

template <typename S, typename D>
__global__ void __launch_bounds__(256) convert_kernel(const S *__restrict__ src, D *__restrict__ dst,
                                                      int64_t count)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += stride)
        dst[e] = from_f64<D>(to_f64(src[e]));
}

int grid_for(int64_t count)
{
    int64_t g = (count + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

}  // namespace

deinsum_status launch_synth_fill(void *x, int dtype, int64_t count, uint64_t seed, int64_t offset,
                                 int dist, hipStream_t stream)
{
    const int g = grid_for(count);
    switch (dtype) {
    case DEINSUM_F64:
        synth_fill_kernel<double><<<g, 256, 0, stream>>>(static_cast<double *>(x), count, seed, offset, dist);
        break;
    case DEINSUM_F32:
        synth_fill_kernel<float><<<g, 256, 0, stream>>>(static_cast<float *>(x), count, seed, offset, dist);
        break;
    case DEINSUM_BF16:
        synth_fill_kernel<bf16_t><<<g, 256, 0, stream>>>(static_cast<bf16_t *>(x), count, seed, offset, dist);
        break;
    default:
        return fail(DEINSUM_ERR_INVALID_ARG, "synth_fill: bad dtype");
    }
    return check_launch("synth_fill");
}

deinsum_status launch_convert(const void *src, int sdt, void *dst, int ddt, int64_t count,
                              hipStream_t stream)
{
    const int g = grid_for(count);
    if (sdt == DEINSUM_F64 && ddt == DEINSUM_F32)
        convert_kernel<double, float><<<g, 256, 0, stream>>>(static_cast<const double *>(src), static_cast<float *>(dst), count);
    else if (sdt == DEINSUM_F64 && ddt == DEINSUM_BF16)
        convert_kernel<double, bf16_t><<<g, 256, 0, stream>>>(static_cast<const double *>(src), static_cast<bf16_t *>(dst), count);
    else if (sdt == DEINSUM_F32 && ddt == DEINSUM_BF16)
        convert_kernel<float, bf16_t><<<g, 256, 0, stream>>>(static_cast<const float *>(src), static_cast<bf16_t *>(dst), count);
    else
        return fail(DEINSUM_ERR_UNSUPPORTED, "convert: supported pairs are f64->f32, f64->bf16, f32->bf16");
    return check_launch("convert");
}

}  // namespace deinsum
