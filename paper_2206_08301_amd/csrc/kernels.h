// kernels.h -- device-side building blocks shared by the gfx950 kernels, and
// the host launch interface of each kernel family.
//
// Matrix-core operand layouts on gfx950 (wave64, 16x16 output tiles; lane l,
// g = l / 16, c = l % 16), established on the device:
//   v_mfma_f64_16x16x4_f64 : A[c][g], B[g][c];           D reg v = D[4v + g][c]
//   v_mfma_f32_16x16x4_f32 : A[c][g], B[g][c];           D reg v = D[4g + v][c]
//   v_mfma_f32_16x16x32_bf16: A[c][8g+e], B[8g+e][c] (e=0..7); D reg v = D[4g + v][c]
// The pairing of A and B along k only requires both operands to use the same
// (g, e) slot for the same k, so kernels assign k to slots freely.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "deinsum.h"
#include "internal.h"

namespace deinsum {

// ----------------------------------------------------------------- types
struct __align__(2) bf16_t {
    uint16_t u;
};

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// Streaming loads of X.  NTL marks them non-temporal: each element is read
// once, and the hint keeps the re-read factor rows in the caches (a kernel
// variant property; it pays for some layouts and costs for others).
template <bool NTL, typename V>
__device__ __forceinline__ V ld_stream(const V *p)
{
    if constexpr (NTL) return __builtin_nontemporal_load(p);
    else return *p;
}

enum PrecisionId { P_FP64 = 0, P_FP32 = 1, P_BF16 = 2, P_BF16X3 = 3, P_FX20 = 4 };

// FX20 storage of X: X ~ (256 h + l) * 2^e with one exponent e per tensor,
// h in [-2048, 2048] kept as FP16 bit patterns (exact) and l in [-128, 127] as
// int8, in two planes behind a header; see include/deinsum.h.
constexpr int kFx20Header = 256;
__host__ __device__ inline int64_t fx20_align(int64_t b) { return (b + 255) / 256 * 256; }
__host__ __device__ inline int64_t fx20_lo_offset(int64_t count) { return kFx20Header + fx20_align(2 * count); }
__host__ __device__ inline int64_t fx20_bytes(int64_t count) { return fx20_lo_offset(count) + fx20_align(count); }
struct Fx20Header {
    uint32_t magic;   // kFx20Magic
    int32_t exp2;     // X ~ (256 h + l) * 2^exp2
    int64_t count;
    double max_abs;   // max |X| before encoding
    // Integer sums, exact and independent of summation order:
    uint64_t sumsq_q; // sum of (x 2^-(exp2+19))^2, in units of 2^-24 (per-wave sums rounded)
    uint64_t errsq_q; // sum of ((x - stored x) 2^-exp2)^2, in units of 2^-28 (per-wave sums rounded)
};
constexpr uint32_t kFx20Magic = 0x30325846u;  // "FX20"

// Round-to-nearest-even FP32 -> BF16 (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h)
{
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// Two FP32 values rounded to BF16 (nearest even, as f32_to_bf16_bits for every finite
// value) by one packed conversion instruction; v[0] in the low half.
__device__ __forceinline__ uint32_t f32x2_to_bf16x2_bits(f32x2 v)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
// Split of two FP32 values into BF16 hi = RNE(x) and lo = RNE(x - hi) (x - hi is exact
// in FP32), packed two per word: three conversions and two subtractions per pair.
__device__ __forceinline__ void split_bf16x2(f32x2 v, uint32_t &hi, uint32_t &lo)
{
    hi = f32x2_to_bf16x2_bits(v);
    const f32x2 hf = {__uint_as_float(hi << 16), __uint_as_float(hi & 0xffff0000u)};
    lo = f32x2_to_bf16x2_bits(v - hf);
}

__device__ __forceinline__ double to_f64(double x) { return x; }
__device__ __forceinline__ double to_f64(float x) { return static_cast<double>(x); }
__device__ __forceinline__ double to_f64(bf16_t x) { return static_cast<double>(bf16_bits_to_f32(x.u)); }

template <typename T> __device__ __forceinline__ T from_f64(double x);
template <> __device__ __forceinline__ double from_f64<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_f64<float>(double x) { return static_cast<float>(x); }
// f64 -> bf16 goes through f32 (RNE at each step), the convention of the host generator.
template <> __device__ __forceinline__ bf16_t from_f64<bf16_t>(double x)
{
    bf16_t r;
    r.u = f32_to_bf16_bits(static_cast<float>(x));
    return r;
}

// ----------------------------------------------------------------- matrix-core wrappers
__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f32x4 mfma_f16(u16x8 a, u16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0,
                                                  0);
}
__device__ __forceinline__ f32x4 mfma_bf16(u16x8 a, u16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Row of the 16x16 output tile held in register v of lane l.
template <int P> __device__ __forceinline__ int tile_row(int lane, int v);
template <> __device__ __forceinline__ int tile_row<P_FP64>(int lane, int v) { return 4 * v + (lane >> 4); }
template <> __device__ __forceinline__ int tile_row<P_FP32>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int tile_row<P_BF16>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int tile_row<P_BF16X3>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int tile_row<P_FX20>(int lane, int v) { return 4 * (lane >> 4) + v; }

// ----------------------------------------------------------------- launch interface
// Modes other than the free mode and the matrix-core mode ("outer" modes), in
// increasing mode order; the last one varies fastest in the walk.
constexpr int kMaxOuter = DEINSUM_MAX_ORDER - 2;
struct OuterDesc {
    int n_outer;
    int64_t dim[kMaxOuter];
    int64_t xstride[kMaxOuter];  // element stride of that mode in X
    const void *U[kMaxOuter];    // factor of that mode, column block applied
};

deinsum_status check_launch(const char *what);

deinsum_status launch_synth_fill(void *x, int dtype, int64_t count, uint64_t seed, int64_t offset,
                                 int dist, hipStream_t stream);
deinsum_status launch_convert(const void *src, int sdt, void *dst, int ddt, int64_t count,
                              hipStream_t stream);

}  // namespace deinsum
