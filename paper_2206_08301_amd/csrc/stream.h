// stream.h -- device building blocks of the streaming MTTKRP unit (shared by
// the per-call kernels and the persistent batch kernel).  See mttkrp.hip for
// the method; this header holds the tile geometry, the loaders, the outer
// odometer and stream_unit(), which processes one workgroup unit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.h"
#include "mttkrp.h"

namespace deinsum {
namespace dev {

template <int P> struct PrecTypes;
template <> struct PrecTypes<P_FP64> { using XT = double; using DT = f64x4; static constexpr int KE = 1; };
template <> struct PrecTypes<P_FP32> { using XT = float;  using DT = f32x4; static constexpr int KE = 1; };
template <> struct PrecTypes<P_BF16> { using XT = bf16_t; using DT = f32x4; static constexpr int KE = 8; };
template <> struct PrecTypes<P_BF16X3> { using XT = float; using DT = f32x4; static constexpr int KE = 8; };
// FX20: the ring holds raw words of the two planes; values are decoded per step.
template <> struct PrecTypes<P_FX20> { using XT = uint32_t; using DT = f32x4; static constexpr int KE = 8; };

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t imax64(int64_t a, int64_t b) { return a > b ? a : b; }

__device__ __forceinline__ double ld_u(const void *p, int64_t i, int prec)
{
    return prec == P_FP64 ? static_cast<const double *>(p)[i]
                          : static_cast<double>(static_cast<const float *>(p)[i]);
}

// Load `n` contiguous elements; `vec` = whole 16-byte (or 8-byte) words allowed.
template <typename T, int n, bool NTL = false>
__device__ __forceinline__ void load_contig(T *dst, const T *__restrict__ src, bool vec, int64_t valid)
{
    if constexpr ((n * sizeof(T)) % 16 == 0) {
        if (vec && valid >= n) {
            constexpr int NV = n * sizeof(T) / 16;
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                const u32x4 v = ld_stream<NTL>(reinterpret_cast<const u32x4 *>(src) + i);
                __builtin_memcpy(dst + i * (16 / sizeof(T)), &v, 16);
            }
            return;
        }
    } else if constexpr (n * sizeof(T) == 8) {
        if (vec && valid >= n) {
            const uint64_t v = ld_stream<NTL>(reinterpret_cast<const uint64_t *>(src));
            __builtin_memcpy(dst, &v, 8);
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < n; ++i) dst[i] = (i < valid) ? src[i] : T{};
}

// Outer-index odometer over the X offset only (no loads): the per-mode loop is
// unrolled over the maximum number of outer modes so the indices stay in
// registers and the walk adds no memory waits to the streaming loop.
struct Odometer {
    int64_t idx[kMaxOuter];
    int64_t off;
    __device__ __forceinline__ void init(const OuterDesc &od, int64_t o)
    {
        off = 0;
#pragma unroll
        for (int m = kMaxOuter - 1; m >= 0; --m) {
            idx[m] = 0;
            if (m < od.n_outer) {
                idx[m] = o % od.dim[m];
                o /= od.dim[m];
                off += idx[m] * od.xstride[m];
            }
        }
    }
    __device__ __forceinline__ void next(const OuterDesc &od)
    {
        bool carry = true;
#pragma unroll
        for (int m = kMaxOuter - 1; m >= 0; --m) {
            if (m < od.n_outer && carry) {
                off += od.xstride[m];
                if (++idx[m] < od.dim[m]) {
                    carry = false;
                } else {
                    off -= idx[m] * od.xstride[m];
                    idx[m] = 0;
                }
            }
        }
    }
};

// Geometry of one wave's tile.
//   NI : matrix-core K-instructions per column tile per step; KE k-values each.
//   SLICE = 4 * NI * KE positions of mode g per wave.
//   K-contiguous: the lane's run of NI*KE elements is cut into chunks of VE
//     contiguous elements; chunk j of lane group g starts at slice position
//     j*4*VE + g*VE, so the four lanes of a row read 4*VE contiguous elements
//     per load instruction.  Run element t sits at
//         pos(t, g) = (t / VE) * 4 * VE + g * VE + t % VE.
//   M-contiguous: instruction q, lane group g, element e reads row
//         pos(q, g, e) = q * 4 * KE + g * KE + e
//     of the slice, MT contiguous output indices per lane.
template <int P, int L, int NI, int MT>
struct Tile {
    using XT = typename PrecTypes<P>::XT;
    static constexpr int KE = PrecTypes<P>::KE;
    static constexpr int SLICE = 4 * NI * KE;
    static constexpr int VE = (P == P_BF16X3) ? 8 : (P == P_FX20 ? 16 : static_cast<int>(16 / sizeof(XT)));
    static constexpr int XN = (L == L_KCONTIG) ? NI * KE : NI * KE * MT;  // X elements per lane per step
    // FX20 ring words per step.  K-contiguous: XN/2 words of the FP16 plane, then XN/4
    // of the int8 plane.  M-contiguous: per slice row (q, g, e), FHW words holding its
    // MT FP16 values, then one word per row holding its MT int8 values.
    static constexpr int FHW = (MT + 1) / 2;
    static constexpr int FROWS = NI * KE;  // slice rows of one lane per step (M-contiguous)
    static constexpr int XW = (P != P_FX20) ? XN : (L == L_KCONTIG ? XN / 2 + XN / 4 : FROWS * (FHW + 1));
    static_assert(L == L_MCONTIG || (NI * KE) % VE == 0, "K-contiguous runs must be whole chunks");
    static_assert(P != P_FX20 || L == L_KCONTIG || MT == 1 || MT == 2 || MT == 4,
                  "FX20 M-contiguous tiles hold 1, 2 or 4 indices per lane");

    __device__ static int pos_k(int t, int g) { return (t / VE) * 4 * VE + g * VE + t % VE; }
    __device__ static int pos_m(int q, int g, int e) { return q * 4 * KE + g * KE + e; }
    // slice position of the K slot (g, e) of instruction q
    __device__ static int slot_pos(int q, int g, int e)
    {
        return (L == L_KCONTIG) ? pos_k(q * KE + e, g) : pos_m(q, g, e);
    }
};

template <typename T, int n, bool NTL = false>
__device__ __forceinline__ void load_vec(T *dst, const T *__restrict__ src)
{
    static_assert((n * sizeof(T)) % 8 == 0, "vector runs are whole 8-byte words");
    if constexpr ((n * sizeof(T)) % 16 == 0) {
#pragma unroll
        for (int i = 0; i < static_cast<int>(n * sizeof(T) / 16); ++i) {
            const u32x4 v = ld_stream<NTL>(reinterpret_cast<const u32x4 *>(src) + i);
            __builtin_memcpy(dst + i * (16 / sizeof(T)), &v, 16);
        }
    } else {
#pragma unroll
        for (int i = 0; i < static_cast<int>(n * sizeof(T) / 8); ++i) {
            const uint64_t v = ld_stream<NTL>(reinterpret_cast<const uint64_t *>(src) + i);
            __builtin_memcpy(dst + i * (8 / sizeof(T)), &v, 8);
        }
    }
}

// One step's X tile of a lane.  FULL: every element in range and aligned, so
// the tile is a fixed sequence of vector loads (a static load count lets the
// compiler wait for exactly the oldest tile); otherwise masked element loads.
template <int P, int L, int NI, int MT, bool FULL, bool NTL>
__device__ __forceinline__ void load_tile(typename Tile<P, L, NI, MT>::XT *x,
                                          const typename Tile<P, L, NI, MT>::XT *__restrict__ base,
                                          const StreamArgs &a, int g, int64_t lim, int ivalid)
{
    using TL = Tile<P, L, NI, MT>;
    using XT = typename TL::XT;
    if constexpr (L == L_KCONTIG) {
        // base = row start + slice start + g*VE; lim = slice elements available from there
        constexpr int NCH = (NI * TL::KE) / TL::VE;
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            if constexpr (FULL) load_vec<XT, TL::VE, NTL>(x + j * TL::VE, base + j * 4 * TL::VE);
            else  // whole chunks in range still take vector loads
                load_contig<XT, TL::VE>(x + j * TL::VE, base + j * 4 * TL::VE, a.vec_ok != 0, lim - j * 4 * TL::VE);
        }
    } else {
        // base = slice row 0 + first output index of the lane; lim = slice rows available
#pragma unroll
        for (int q = 0; q < NI; ++q)
#pragma unroll
            for (int e = 0; e < TL::KE; ++e) {
                const int r = TL::pos_m(q, g, e);
                const XT *src = base + static_cast<int64_t>(r) * a.stride_g;
                XT *dst = x + (q * TL::KE + e) * MT;
                if constexpr (FULL && (MT * sizeof(XT)) % 8 == 0) {
                    load_vec<XT, MT, NTL>(dst, src);
                } else if constexpr (FULL) {
#pragma unroll
                    for (int i = 0; i < MT; ++i) dst[i] = src[i];
                } else {
                    load_contig<XT, MT>(dst, src, a.vec_ok != 0, r < lim ? ivalid : 0);  // whole runs: one load
                }
            }
    }
}

// FX20 tile of a lane: element offset `off` of its first element in both
// planes (same layout as load_tile).  Element t of the run lands in 16-bit
// word t/2 (half t%2) and in 8-bit word XN/2 + t/4 (byte t%4).
template <int L, int NI, int MT, bool FULL, bool NTL>
__device__ __forceinline__ void load_tile_fx20(uint32_t *x, int64_t off, const StreamArgs &a, int64_t lim,
                                               int ivalid, int g)
{
    using TL = Tile<P_FX20, L, NI, MT>;
    constexpr int XN = TL::XN;
    const uint16_t *__restrict__ H = static_cast<const uint16_t *>(a.X) + off;
    const uint8_t *__restrict__ B = static_cast<const uint8_t *>(a.X2) + off;
    uint32_t *xh = x, *xl = x + XN / 2;
    if constexpr (L == L_KCONTIG) {
        constexpr int NCH = (NI * TL::KE) / TL::VE;  // chunks of 16 elements, 4*16 apart in the slice
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const int64_t e0 = static_cast<int64_t>(j) * 4 * TL::VE;
            if constexpr (FULL) {
                const u32x4 h0 = ld_stream<NTL>(reinterpret_cast<const u32x4 *>(H + e0));
                const u32x4 h1 = ld_stream<NTL>(reinterpret_cast<const u32x4 *>(H + e0) + 1);
                const u32x4 l0 = ld_stream<NTL>(reinterpret_cast<const u32x4 *>(B + e0));
                __builtin_memcpy(xh + j * 8, &h0, 16);
                __builtin_memcpy(xh + j * 8 + 4, &h1, 16);
                __builtin_memcpy(xl + j * 4, &l0, 16);
            } else {
                const int64_t valid = lim - e0;
                if (a.vec_ok && valid >= TL::VE) {  // a whole chunk in range: vector loads
                    const u32x4 h0 = reinterpret_cast<const u32x4 *>(H + e0)[0];
                    const u32x4 h1 = reinterpret_cast<const u32x4 *>(H + e0)[1];
                    const u32x4 l0 = reinterpret_cast<const u32x4 *>(B + e0)[0];
                    __builtin_memcpy(xh + j * 8, &h0, 16);
                    __builtin_memcpy(xh + j * 8 + 4, &h1, 16);
                    __builtin_memcpy(xl + j * 4, &l0, 16);
                } else {
#pragma unroll
                    for (int w = 0; w < 8; ++w) xh[j * 8 + w] = 0;
#pragma unroll
                    for (int w = 0; w < 4; ++w) xl[j * 4 + w] = 0;
#pragma unroll
                    for (int i = 0; i < TL::VE; ++i)
                        if (i < valid) {
                            xh[j * 8 + i / 2] |= static_cast<uint32_t>(H[e0 + i]) << (16 * (i % 2));
                            xl[j * 4 + i / 4] |= static_cast<uint32_t>(B[e0 + i]) << (8 * (i % 4));
                        }
                }
            }
        }
    } else {
        // Row (q, g, e) of the slice: MT FP16 values and MT int8 values of the lane's indices.
        constexpr int FHW = TL::FHW, HW = TL::FROWS * FHW;
#pragma unroll
        for (int q = 0; q < NI; ++q)
#pragma unroll
            for (int e = 0; e < TL::KE; ++e) {
                const int rr = q * TL::KE + e;  // ring row
                const int r = TL::pos_m(q, g, e);
                const int64_t e0 = static_cast<int64_t>(r) * a.stride_g;
                uint32_t *wh = xh + rr * FHW;
                uint32_t &wl = x[HW + rr];
                // A whole run in range (every tile of an aligned full tensor; in a
                // ragged tile the lanes whose MT indices all exist): vector loads.
                if (FULL || (MT >= 2 && a.vec_ok && r < lim && ivalid >= MT)) {
                    if constexpr (MT == 4) {
                        const uint64_t h = ld_stream<NTL>(reinterpret_cast<const uint64_t *>(H + e0));
                        wh[0] = static_cast<uint32_t>(h);
                        wh[1] = static_cast<uint32_t>(h >> 32);
                        wl = ld_stream<NTL>(reinterpret_cast<const uint32_t *>(B + e0));
                    } else if constexpr (MT == 2) {
                        wh[0] = ld_stream<NTL>(reinterpret_cast<const uint32_t *>(H + e0));
                        wl = ld_stream<NTL>(reinterpret_cast<const uint16_t *>(B + e0));
                    } else {
                        wh[0] = H[e0];
                        wl = B[e0];
                    }
                } else {
#pragma unroll
                    for (int w = 0; w < FHW; ++w) wh[w] = 0;
                    wl = 0;
                    if (r < lim) {
#pragma unroll
                        for (int i = 0; i < MT; ++i)
                            if (i < ivalid) {
                                wh[i / 2] |= static_cast<uint32_t>(H[e0 + i]) << (16 * (i % 2));
                                wl |= static_cast<uint32_t>(B[e0 + i]) << (8 * i);
                            }
                    }
                }
            }
    }
}

// FP16 operands of an FX20 K-contiguous instruction q (elements 8q .. 8q+7 of the
// run): h is the FP16 plane itself; l enters as the FP16 value (1152 + l) / 256,
// exact, built from the int8 byte b as the bit pattern 0x4400 | (b ^ 0x80)
// (4 + (l + 128) / 256), so h*u and the l part accumulate in one register set;
// the 1152/256 offset is removed with the factor column sum.
template <int XN>
__device__ __forceinline__ void fx20_operands(const uint32_t *x, int q, u16x8 &ah, u16x8 &al)
{
    __builtin_memcpy(&ah, x + 4 * q, 16);
    uint32_t o[4];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const uint32_t b = x[XN / 2 + 2 * q + w] ^ 0x80808080u;
        o[2 * w] = __builtin_amdgcn_perm(0u, b, 0x0C010C00u) | 0x44004400u;
        o[2 * w + 1] = __builtin_amdgcn_perm(0u, b, 0x0C030C02u) | 0x44004400u;
    }
    __builtin_memcpy(&al, o, 16);
}

// FP16 operands of an FX20 M-contiguous instruction q for output index mt of the
// lane: K slot e is slice row (q, g, e); the same int8 offset encoding as above.
template <int NI, int MT>
__device__ __forceinline__ void fx20_operands_m(const uint32_t *x, int q, int mt, u16x8 &ah, u16x8 &al)
{
    constexpr int KE = 8, FHW = (MT + 1) / 2, HW = NI * KE * FHW;
    const int hs = 2 * (mt & 1);
    const uint32_t selh = static_cast<uint32_t>(hs) | (static_cast<uint32_t>(hs + 1) << 8) |
                          (static_cast<uint32_t>(hs + 4) << 16) | (static_cast<uint32_t>(hs + 5) << 24);
    const uint32_t sell = static_cast<uint32_t>(mt) | (0x0Cu << 8) | (static_cast<uint32_t>(mt + 4) << 16) | (0x0Cu << 24);
    uint32_t oh[4], ol[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r0 = q * KE + 2 * j, r1 = r0 + 1;
        oh[j] = __builtin_amdgcn_perm(x[r1 * FHW + mt / 2], x[r0 * FHW + mt / 2], selh);
        ol[j] = __builtin_amdgcn_perm(x[HW + r1] ^ 0x80808080u, x[HW + r0] ^ 0x80808080u, sell) | 0x44004400u;
    }
    __builtin_memcpy(&ah, oh, 16);
    __builtin_memcpy(&al, ol, 16);
}

template <int L, int NT, int MT>
constexpr int unit_lds_elems() { return L == L_KOUT ? 1 : ((L == L_KCONTIG) ? 16 : 16 * MT) * 16 * NT; }

// One workgroup unit: block index b of the launch geometry in `a` (see
// StreamArgs).  `lds` holds unit_lds_elems() doubles.  Called by the
// per-call kernel below and by the persistent batch kernel.  XNT: X loads
// are non-temporal.
template <int P, int L0, int NT, int NI, int MT, int NBUF, bool XNT = false>
__device__ __forceinline__ void stream_unit(const StreamArgs &a, int64_t b, double *lds)
{
    // L_KOUT streams tiles exactly as the K-contiguous layout does (rows of 16 along
    // mode 1 instead of the free mode); only the unit walk and the fold differ.
    constexpr bool KOUT = (L0 == L_KOUT);
    constexpr int L = KOUT ? L_KCONTIG : L0;
    static_assert(!KOUT || MT == 1, "L_KOUT tiles are K-contiguous tiles");
    static_assert(!KOUT || P != P_FP64, "L_KOUT weights are packed for the FP32 accumulator layout (row 4g + v)");
    using TL = Tile<P, L, NI, MT>;
    using XT = typename TL::XT;
    using DT = typename PrecTypes<P>::DT;
    constexpr int KE = TL::KE;
    constexpr int XN = TL::XN;
    constexpr int TROWS = (L == L_KCONTIG) ? 16 : 16 * MT;
    constexpr int TCOLS = 16 * NT;

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index: uniform in the wave
    const int nwaves = blockDim.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    int64_t u = b;
    if (a.xcd_remap) {
        const int64_t q = a.n_groups >> 3, r = a.n_groups & 7, x = b & 7;
        u = x * q + (x < r ? x : r) + (b >> 3);
    }
    const int kgroup = static_cast<int>(u % a.n_kgroups);
    int tile;
    int64_t chunk;
    if (KOUT) {
        tile = 0;
        chunk = u / a.n_kgroups;
    } else if (a.order == 0) {
        tile = static_cast<int>((u / a.n_kgroups) % a.n_tiles);
        chunk = u / (static_cast<int64_t>(a.n_kgroups) * a.n_tiles);
    } else {
        chunk = (u / a.n_kgroups) % a.n_chunks;
        tile = static_cast<int>(u / (a.n_kgroups * a.n_chunks));
    }
    const int ks = kgroup * a.wk + (w % a.wk);
    const int osub = w / a.wk;
    const int64_t s0 = static_cast<int64_t>(ks) * TL::SLICE;  // slice start in mode g
    const int64_t slice_avail = a.Ig - s0;                     // <= 0: empty slice

    // Lane geometry.  `full` (wave-uniform): the wave's whole tile is in range
    // and X allows aligned vector loads.
    int64_t xlane;  // offset of this lane's first element (excluding the outer offset)
    int64_t lim;    // K-contig: run elements available; M-contig: slice rows available
    int ivalid = 0;
    bool full;
    if constexpr (KOUT) {
        // row c of every mode-1 tile; per-step offsets and limits come from the walk
        xlane = s0 + g * TL::VE;
        lim = slice_avail - g * TL::VE;
        full = a.vec_ok && a.od.dim[0] % 16 == 0 && slice_avail >= TL::SLICE;
    } else if constexpr (L == L_KCONTIG) {
        const int64_t row = static_cast<int64_t>(tile) * 16 + c;
        xlane = row * a.stride_n + s0 + g * TL::VE;
        lim = (row < a.In) ? slice_avail - g * TL::VE : 0;
        full = a.vec_ok && (static_cast<int64_t>(tile) + 1) * 16 <= a.In && slice_avail >= TL::SLICE;
    } else {
        const int64_t ibase = static_cast<int64_t>(tile) * 16 * MT + MT * c;
        ivalid = static_cast<int>(imin64(MT, imax64(0, a.In - ibase)));
        xlane = s0 * a.stride_g + ibase;
        lim = slice_avail;
        full = a.vec_ok && (static_cast<int64_t>(tile) + 1) * 16 * MT <= a.In && slice_avail >= TL::SLICE;
    }

    // Register-resident slice of U^g for every K slot of every instruction.
    constexpr bool FX16 = (P == P_FX20);  // FX20 runs on FP16 matrix cores
    double fr64[(P == P_FP64) ? NI * NT : 1];
    float fr32[(P == P_FP32) ? NI * NT : 1];
    u16x8 frh[(P == P_BF16 || P == P_BF16X3 || FX16) ? NI * NT : 1];
    u16x8 frl[(P == P_BF16X3 || FX16) ? NI * NT : 1];
    // FX16: each factor column of the slice is scaled by 2^-k (|u| < 1) before
    // the FP16 split; cs = 2^k, and sh = the column sum of the FP16 hi parts
    // (removes the 1152 offset of the int8 operand).
    double cs[FX16 ? NT : 1], sh[FX16 ? NT : 1];
    if constexpr (FX16) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int col = nt * 16 + c;
            float mx = 0.0f;
#pragma unroll
            for (int q = 0; q < NI; ++q)
#pragma unroll
                for (int e = 0; e < KE; ++e) {
                    const int pos = TL::slot_pos(q, g, e);
                    if (pos < slice_avail && col < a.ncols)
                        mx = fmaxf(mx, fabsf(static_cast<const float *>(a.Ug)[(s0 + pos) * a.ldu + col]));
                }
            mx = fmaxf(mx, __shfl_xor(mx, 16));
            mx = fmaxf(mx, __shfl_xor(mx, 32));
            int k = 0;
            if (mx > 0.0f) (void)frexpf(mx, &k);  // mx < 2^k
            double psum = 0.0;
#pragma unroll
            for (int q = 0; q < NI; ++q) {
                u16x8 hi, lo;
#pragma unroll
                for (int e = 0; e < KE; ++e) {
                    const int pos = TL::slot_pos(q, g, e);
                    const float v = (pos < slice_avail && col < a.ncols)
                                        ? ldexpf(static_cast<const float *>(a.Ug)[(s0 + pos) * a.ldu + col], -k)
                                        : 0.0f;
                    const _Float16 h = static_cast<_Float16>(v);
                    const _Float16 l = static_cast<_Float16>(v - static_cast<float>(h));
                    hi[e] = __builtin_bit_cast(uint16_t, h);
                    lo[e] = __builtin_bit_cast(uint16_t, l);
                    psum += static_cast<double>(static_cast<float>(h));
                }
                frh[q * NT + nt] = hi;
                frl[q * NT + nt] = lo;
            }
            psum += __shfl_xor(psum, 16);
            psum += __shfl_xor(psum, 32);
            cs[nt] = ldexp(1.0, k);
            sh[nt] = psum;
        }
    }
#pragma unroll
    for (int q = 0; q < NI; ++q)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int col = nt * 16 + c;
            if constexpr (FX16) {
                // built above
            } else if constexpr (KE == 1) {
                const int pos = TL::slot_pos(q, g, 0);
                const double v = (pos < slice_avail && col < a.ncols) ? ld_u(a.Ug, (s0 + pos) * a.ldu + col, P) : 0.0;
                if constexpr (P == P_FP64) fr64[q * NT + nt] = v;
                else fr32[q * NT + nt] = static_cast<float>(v);
            } else {
                u16x8 hi, lo;
#pragma unroll
                for (int e = 0; e < KE; ++e) {
                    const int pos = TL::slot_pos(q, g, e);
                    const float v = (pos < slice_avail && col < a.ncols)
                                        ? static_cast<const float *>(a.Ug)[(s0 + pos) * a.ldu + col] : 0.0f;
                    const uint16_t h = f32_to_bf16_bits(v);
                    hi[e] = h;
                    lo[e] = f32_to_bf16_bits(v - bf16_bits_to_f32(h));
                }
                frh[q * NT + nt] = hi;
                if constexpr (P == P_BF16X3) frl[q * NT + nt] = lo;
            }
        }

    double acc[MT][NT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[mt][nt][v] = 0.0;
    // FP64 with 64-index tiles: the step's Hadamard weights scale the factor operand
    // (one multiply per operand register) and the matrix cores accumulate straight into
    // acc across steps, so no per-step product tile is held (it does not fit beside the
    // accumulators and the ring).
    constexpr bool WB = (P == P_FP64 && MT >= 4);
    // L_KOUT: each column's weighted sum over the tile rows and the mode-1 tiles of
    // the current output row (the step's weights are 4 * NT values: the lane's four
    // tile rows of U^1 per column tile).
    double tacc[KOUT ? NT : 1];
#pragma unroll
    for (int nt = 0; nt < (KOUT ? NT : 1); ++nt) tacc[nt] = 0.0;

    // One step: stage 1 on the matrix cores, then the Hadamard fold (stage 2).
    auto step = [&](const XT *x, const auto *wv) {  // wv: double, or float (L_KOUT)
        if constexpr (WB) {
#pragma unroll
            for (int q = 0; q < NI; ++q)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const double b = fr64[q * NT + nt] * wv[nt];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const double xa = (L == L_KCONTIG) ? x[q] : x[q * MT + mt];
                        f64x4 t = {acc[mt][nt][0], acc[mt][nt][1], acc[mt][nt][2], acc[mt][nt][3]};
                        t = mfma_f64(xa, b, t);
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[mt][nt][v] = t[v];
                    }
                }
        } else if constexpr (FX16) {
            // sum_k (256 h + l) u' = 256 (h.uh + h.ul + ((1152 + l)/256).uh) - 1152 sum uh
            DT dh[MT][NT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) dh[mt][nt] = DT{0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < NI; ++q)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    u16x8 ah, al;
                    if constexpr (L == L_KCONTIG) fx20_operands<XN>(x, q, ah, al);
                    else fx20_operands_m<NI, MT>(x, q, mt, ah, al);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        dh[mt][nt] = mfma_f16(ah, frh[q * NT + nt], dh[mt][nt]);
                        dh[mt][nt] = mfma_f16(ah, frl[q * NT + nt], dh[mt][nt]);
                        dh[mt][nt] = mfma_f16(al, frh[q * NT + nt], dh[mt][nt]);
                    }
                }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const double off = 1152.0 * sh[nt];
                if constexpr (KOUT) {
                    double sum = 0.0;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        sum += (256.0 * static_cast<double>(dh[0][nt][v]) - off) * static_cast<double>(wv[v * NT + nt]);
                    tacc[nt] += sum * cs[nt];
                } else {
                    const double wc = wv[nt] * cs[nt];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            acc[mt][nt][v] += (256.0 * static_cast<double>(dh[mt][nt][v]) - off) * wc;
                }
            }
        } else {
        DT d[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) d[mt][nt] = DT{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < NI; ++q)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                // A operand of instruction q for M tile mt: element e of the K slot.
                auto xe = [&](int e) -> XT {
                    return (L == L_KCONTIG) ? x[q * KE + e] : x[(q * KE + e) * MT + mt];
                };
                if constexpr (P == P_FP64 || P == P_FP32) {
                    const XT xa = xe(0);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        if constexpr (P == P_FP64) d[mt][nt] = mfma_f64(xa, fr64[q * NT + nt], d[mt][nt]);
                        else d[mt][nt] = mfma_f32(xa, fr32[q * NT + nt], d[mt][nt]);
                    }
                } else if constexpr (P == P_BF16) {
                    u16x8 xa;
#pragma unroll
                    for (int e = 0; e < 8; ++e) xa[e] = xe(e).u;
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) d[mt][nt] = mfma_bf16(xa, frh[q * NT + nt], d[mt][nt]);
                } else {
                    u16x8 xh, xl;
                    uint32_t wh[4], wl[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) split_bf16x2(f32x2{xe(2 * j), xe(2 * j + 1)}, wh[j], wl[j]);
                    __builtin_memcpy(&xh, wh, 16);
                    __builtin_memcpy(&xl, wl, 16);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        d[mt][nt] = mfma_bf16(xh, frh[q * NT + nt], d[mt][nt]);
                        d[mt][nt] = mfma_bf16(xh, frl[q * NT + nt], d[mt][nt]);
                        d[mt][nt] = mfma_bf16(xl, frh[q * NT + nt], d[mt][nt]);
                    }
                }
            }
        if constexpr (KOUT) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    tacc[nt] += static_cast<double>(d[0][nt][v]) * static_cast<double>(wv[v * NT + nt]);
        } else {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[mt][nt][v] += static_cast<double>(d[mt][nt][v]) * wv[nt];
        }
        }
    };

    // Outer range of this wave.
    const int64_t c0 = chunk * a.o_per_chunk;
    const int64_t c1 = imin64(a.O, c0 + a.o_per_chunk);
    const int wo = nwaves / a.wk;
    const int64_t per = (c1 - c0 + wo - 1) / wo;
    const int64_t o0 = imin64(c1, c0 + osub * per);
    const int64_t o1 = imin64(c1, o0 + per);
    const XT *__restrict__ X = static_cast<const XT *>(a.X);

    if constexpr (KOUT) {
        // Output rows [o0, o1) of this wave; per row, the n_tiles mode-1 tiles in order.
        const int64_t I1 = a.od.dim[0], rs = a.od.xstride[0];
        const int njt = a.n_tiles;
        double *__restrict__ Pout = a.P + static_cast<int64_t>(ks) * a.O * a.ldw;
        if (slice_avail <= 0) {  // a slice past mode 2: its partial rows are zero
            if (g == 0)
                for (int64_t i = o0; i < o1; ++i)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) Pout[i * a.ldw + nt * 16 + c] = 0.0;
            return;
        }
        // Fixed-order sum over the four lane groups, then lane group 0 writes the row.
        auto flush = [&](int64_t i) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                double v = tacc[nt];
                v += __shfl_xor(v, 16);
                v += __shfl_xor(v, 32);
                if (g == 0) Pout[i * a.ldw + nt * 16 + c] = v;
                tacc[nt] = 0.0;
            }
        };
        auto walk_kout = [&](auto full_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            XT xb[NBUF][TL::XW];
            float wb[NBUF][4 * NT];
            int64_t li = o0;  // output row and mode-1 tile of the next load
            int ljt = 0;
            int64_t ci = o0;  // output row and tile of the next step
            int cjt = 0;
            // The lane's 4 * NT weights of a tile, packed contiguously by the weight kernel.
            const float *__restrict__ Wk = reinterpret_cast<const float *>(a.W) + static_cast<int64_t>(lane) * 4 * NT;
            auto issue = [&](int slot) {
                const int64_t j0 = static_cast<int64_t>(ljt) * 16;
                load_vec<float, 4 * NT>(wb[slot], Wk + static_cast<int64_t>(ljt) * 64 * 4 * NT);
                const int64_t row = j0 + c;
                const int64_t off = li * a.stride_n + row * rs + xlane;
                const int64_t lim_t = (row < I1) ? lim : 0;
                if constexpr (P == P_FX20)
                    load_tile_fx20<L, NI, MT, FULL, XNT>(xb[slot], off, a, lim_t, 0, g);
                else
                    load_tile<P, L, NI, MT, FULL, XNT>(xb[slot], X + off, a, g, lim_t, 0);
                if (++ljt == njt) {
                    ljt = 0;
                    ++li;
                }
            };
            auto consume = [&](int slot) {
                step(xb[slot], wb[slot]);
                if (++cjt == njt) {
                    flush(ci);
                    cjt = 0;
                    ++ci;
                }
            };
            const int64_t nsteps = (o1 - o0) * njt;
#pragma unroll
            for (int u = 0; u < NBUF - 1; ++u)
                if (u < nsteps) issue(u);
            int64_t t = 0;
            for (; t + 2 * NBUF - 2 < nsteps; t += NBUF) {
#pragma unroll
                for (int u = 0; u < NBUF; ++u) {
                    issue((u + NBUF - 1) % NBUF);
                    consume(u);
                }
            }
            for (; t < nsteps; t += NBUF) {
#pragma unroll
                for (int u = 0; u < NBUF; ++u) {
                    if (t + u < nsteps) {
                        if (t + u + NBUF - 1 < nsteps) issue((u + NBUF - 1) % NBUF);
                        consume(u);
                    }
                }
            }
        };
        if (o0 < o1) {
            if (full) walk_kout(std::true_type{});
            else walk_kout(std::false_type{});
        }
        return;
    }

    // Walk of the outer range with an NBUF-deep register ring: the tile and the
    // Hadamard weights of step t+NBUF-1 are loaded while step t computes.
    auto walk = [&](auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        XT xb[NBUF][TL::XW];
        double wb[NBUF][NT];
        Odometer od;
        od.init(a.od, o0);
        int64_t lo = o0;  // outer index of the next load
        auto issue = [&](int slot) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) wb[slot][nt] = a.W[lo * a.ldw + nt * 16 + c];
            if constexpr (P == P_FX20)
                load_tile_fx20<L, NI, MT, FULL, XNT>(xb[slot], od.off + xlane, a, lim, ivalid, g);
            else
                load_tile<P, L, NI, MT, FULL, XNT>(xb[slot], X + od.off + xlane, a, g, lim, ivalid);
            od.next(a.od);
            ++lo;
        };
        const int64_t nsteps = o1 - o0;
#pragma unroll
        for (int u = 0; u < NBUF - 1; ++u)
            if (u < nsteps) issue(u);
        // Steady state: every load of the iteration is in range, so the loop
        // body issues a fixed sequence of loads and the compiler can wait for
        // exactly the oldest slot.
        int64_t t = 0;
        for (; t + 2 * NBUF - 2 < nsteps; t += NBUF) {
#pragma unroll
            for (int u = 0; u < NBUF; ++u) {
                issue((u + NBUF - 1) % NBUF);
                step(xb[u], wb[u]);
            }
        }
        // Tail: the last < 2*NBUF-1 steps with guarded prefetch.
        for (; t < nsteps; t += NBUF) {
#pragma unroll
            for (int u = 0; u < NBUF; ++u) {
                if (t + u < nsteps) {
                    if (t + u + NBUF - 1 < nsteps) issue((u + NBUF - 1) % NBUF);
                    step(xb[u], wb[u]);
                }
            }
        }
    };
    if (o0 < o1 && slice_avail > 0) {
        if (full) walk(std::true_type{});
        else walk(std::false_type{});
    }

    // Workgroup reduction in wave order through LDS, then one partial tile.
    for (int ww = 0; ww < nwaves; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = (L == L_KCONTIG) ? tile_row<P>(lane, v) : MT * tile_row<P>(lane, v) + mt;
                        const int i = r * TCOLS + nt * 16 + c;
                        lds[i] = (ww == 0) ? acc[mt][nt][v] : lds[i] + acc[mt][nt][v];
                    }
        }
        __syncthreads();
    }
    const int64_t part = chunk * a.n_kgroups + kgroup;
    double *out = a.P + (part * a.n_tiles + tile) * (TROWS * TCOLS);
    for (int i = threadIdx.x; i < TROWS * TCOLS; i += blockDim.x) out[i] = lds[i];
}

}  // namespace dev
}  // namespace deinsum
