// ttmc.hip -- mode-n TTM chain (paper Sec. III-B; TTMc-O5-M0 of Tab. IV):
//   Y[r_0..i_n..r_{N-1}] = sum_{i_m, m != n} X[i] prod_{m != n} U^m[i_m, r_m].
//
// The chain is evaluated with X streamed from HBM once.  One fused pass
// contracts two modes per X slab (all indices but i_a, i_c fixed):
//   stage 1, matrix cores, K = i_a:  D[i_c, r_a] = sum_{i_a} X[slab, i_a, i_c] U^a[i_a, r_a]
//       (the contiguous mode c = N-1 is the matrix-core M dimension, so each
//       lane streams a contiguous run of X; U^a rows are read per K-step);
//   stage 2, matrix cores, K = i_c:  Z[r_a, r_c] = sum_{i_c} D[i_c, r_a] U^c[i_c, r_c]
//       with D taken straight from the accumulator registers as the B operand.
// If the free mode is the contiguous one, stage 2 is skipped (i_c = i_n stays).
// Partial Z tiles of the workgroups are summed in a fixed order; the modes
// left after the fused pass are contracted one at a time on the (much
// smaller) intermediate, the last product writing Y in its output order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "mttkrp.h"
#include "ttmc.h"
#include "tune.h"

namespace deinsum {

namespace {

constexpr int kMaxTtmcRank = 64;

// Per form: X element, stage-1 factor element (UT), stage-2 factor element (CT),
// accumulator tile, rows of the contracted mode a per matrix-core K step (KR) and
// per lane (LR).  The factor copies the kernel reads are zero-padded to whole
// column tiles: FP64 and FP32 in the form's type, row-major; BF16 stage-1 packed
// per K block and lane (eight rows of one column per lane, one 16-byte load),
// stage 2 in FP32.
template <int P> struct TkTypes;
template <> struct TkTypes<P_FP64> {
    using XT = double; using UT = double; using CT = double; using DT = f64x4;
    static constexpr int KR = 4, LR = 1;
};
template <> struct TkTypes<P_FP32> {
    using XT = float; using UT = float; using CT = float; using DT = f32x4;
    static constexpr int KR = 4, LR = 1;
};
template <> struct TkTypes<P_BF16> {
    using XT = uint16_t; using UT = u16x8; using CT = float; using DT = f32x4;
    static constexpr int KR = 32, LR = 8;
};
// FX20: the FP16 plane as the BF16 form's X (2-byte values, 32 rows per K step), the
// int8 plane beside it; stage 1 on the FP16 matrix cores, stage 2 as the FP32 form.
template <> struct TkTypes<P_FX20> {
    using XT = uint16_t; using UT = u16x8; using CT = float; using DT = f32x4;
    static constexpr int KR = 32, LR = 8;
};

__device__ __forceinline__ int64_t tmin(int64_t a, int64_t b) { return a < b ? a : b; }

__device__ __forceinline__ double ldu_p(const void *p, int64_t i, int prec)
{
    return prec == P_FP64 ? static_cast<const double *>(p)[i]
                          : static_cast<double>(static_cast<const float *>(p)[i]);
}

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

template <typename T, int n, bool NTL = false>
__device__ __forceinline__ void load_vec_n(T *dst, const T *__restrict__ src)
{
    static_assert((n * sizeof(T)) % 8 == 0, "whole 8-byte words");
    if constexpr ((n * sizeof(T)) % 16 == 0) {
#pragma unroll
        for (int i = 0; i < static_cast<int>(n * sizeof(T) / 16); ++i) {
            const v4u v = ld_stream<NTL>(reinterpret_cast<const v4u *>(src) + i);
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

// Element offset in X of slab s (the slab modes in row-major order).  With a constant
// slab stride (the slab modes are the leading modes of X) it is s * stride; otherwise
// the index is decomposed, once per slab, which keeps no odometer state in scalar
// registers across the K loop.
__device__ __forceinline__ int64_t slab_offset(const OuterDesc &od, int64_t stride, int64_t s)
{
    if (stride) return s * stride;
    int64_t off = 0;
#pragma unroll
    for (int m = kMaxOuter - 1; m >= 0; --m)
        if (m < od.n_outer) {
            const int64_t d = od.dim[m];
            off += (s % d) * od.xstride[m];
            s /= d;
        }
    return off;
}

// Fused two-mode pass.  Per slab, the K loop over i_a runs in ring steps of
// LDS of the fused kernel.  Stage-2 factor rows of the workgroup are held in LDS
// when a four-wave workgroup's rows fit in 32 KB (they are the same for every
// slab); per-wave Z tiles are summed after one barrier when four of them and those
// rows stay within 64 KB for FP32 rows (two workgroups per CU still fit in its
// 160 KB) or 40 KB for FP64 rows, else accumulated wave by wave in one tile, one
// barrier per wave.  Sized at launch for the workgroup's actual wave count
// (dynamic shared memory).
template <int P, int NTA, int NTC, int MT, bool STAGE2>
struct TkLds {
    using CT = typename TkTypes<P>::CT;
    static constexpr int TA = 16 * NTA, TC = 16 * NTC;
    static constexpr size_t UC_BYTES = static_cast<size_t>(4 * 16 * MT) * TC * sizeof(CT);
    static constexpr bool UC_LDS = STAGE2 && UC_BYTES <= 32768;
    // FP64 factor rows keep the 40 KB limit: the 60^5 R=24 FP64 pass (two-wave
    // workgroups, 32 KB of rows) ran 2.5 -> 3.5 ms with the extra LDS per workgroup.
    static constexpr size_t Z_PAR_LDS = sizeof(CT) == 4 ? 65536 : 40960;
    static constexpr bool Z_PAR = STAGE2 && 4 * TA * TC * sizeof(double) + (UC_LDS ? UC_BYTES : 0) <= Z_PAR_LDS;
    __host__ __device__ static size_t z_elems(int nwaves) { return STAGE2 ? static_cast<size_t>(Z_PAR ? nwaves : 1) * TA * TC : 0; }
    __host__ __device__ static size_t bytes(int nwaves)
    {
        return z_elems(nwaves) * sizeof(double) + (UC_LDS ? static_cast<size_t>(nwaves) * 16 * MT * TC * sizeof(CT) : 0);
    }
};

// UB K-steps (4*UB rows), prefetched NBUF-1 steps ahead; complete steps issue
// a fixed sequence of unmasked loads (the factors are zero-padded to whole
// column tiles), so the compiler waits for exactly the oldest step.
template <int P, int NTA, int NTC, int MT, bool STAGE2, int UB, int NBUF, bool XNT>
__global__ void __launch_bounds__(256, 2) ttmc_fused_kernel(const TkArgs a)
{
    // UB: K-steps (of KR rows) per ring step; NBUF: ring depth.
    using XT = typename TkTypes<P>::XT;
    using UT = typename TkTypes<P>::UT;
    using CT = typename TkTypes<P>::CT;
    using DT = typename TkTypes<P>::DT;
    constexpr int KR = TkTypes<P>::KR, LR = TkTypes<P>::LR;
    constexpr int TA = 16 * NTA, TC = 16 * NTC;
    using L = TkLds<P, NTA, NTC, MT, STAGE2>;
    constexpr bool UC_LDS = L::UC_LDS, Z_PAR = L::Z_PAR;
    extern __shared__ double tk_lds[];
    double *lds = tk_lds;                                                     // Z tiles
    CT *lds_uc = reinterpret_cast<CT *>(tk_lds + L::z_elems(a.nwaves));       // stage-2 factor rows

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, c = lane & 15;
    int64_t b = blockIdx.x;
    if (a.xcd_remap) {  // workgroups are dispatched round-robin over the 8 XCDs
        const int64_t q = a.n_groups >> 3, r = a.n_groups & 7, x = b & 7;
        b = x * q + (x < r ? x : r) + (b >> 3);
    }
    const int cgroup = static_cast<int>(b % a.n_cgroups);
    const int64_t sg = b / a.n_cgroups;
    const int ctile = cgroup * a.nwaves + w;
    // A lane's MT indices of the contiguous mode come in chunks of V (at most 16
    // bytes); chunk j of lane c starts at j*16*V + c*V of the wave's tile, so one
    // load instruction reads 16*V contiguous elements of a row.
    constexpr int V = (MT * static_cast<int>(sizeof(XT)) <= 16) ? MT : 16 / static_cast<int>(sizeof(XT));
    constexpr int NCH = MT / V;
    static_assert(NCH * V == MT, "MT must be whole chunks");
    const int64_t cbase = static_cast<int64_t>(ctile) * 16 * MT;
    const int64_t ibase = cbase + V * c;
    const bool full = a.vec_ok && ctile < a.n_ctiles && cbase + 16 * MT <= a.Ic && (V * sizeof(XT)) % 8 == 0;
    const int64_t s0 = sg * a.slabs_per_group;
    const int64_t s1 = tmin(a.n_slabs, s0 + a.slabs_per_group);
    const XT *__restrict__ X = static_cast<const XT *>(a.X);
    const XT *__restrict__ Ua = static_cast<const XT *>(a.Ua);  // zero-padded copy (row stride TA, or packed)
    const CT *__restrict__ Uc = static_cast<const CT *>(a.Uc);  // zero-padded copy, row stride TC
    const int64_t nsteps = (a.Ia + KR * UB - 1) / (KR * UB);
    const int64_t nfull = a.Ia / (KR * UB);           // ring steps whose rows are all in range
    const int64_t nkb = (a.Ia + KR - 1) / KR;         // K steps with any row in range
    const int64_t nsp = (nsteps + NBUF - 1) / NBUF * NBUF;  // whole ring turns per slab

    const int64_t crow0 = static_cast<int64_t>(cgroup) * a.nwaves * 16 * MT;
    if constexpr (UC_LDS) {
        const int n = a.nwaves * 16 * MT * TC;
        for (int i = threadIdx.x; i < n; i += 64 * a.nwaves) {
            const int64_t row = crow0 + i / TC;
            lds_uc[i] = row < a.Ic ? Uc[row * TC + i % TC] : CT{};
        }
        __syncthreads();
    }

    // FX20: the tensor's scale exponent e (the column scales and offsets are read per slab).
    int fx_e = 0;
    if constexpr (P == P_FX20) fx_e = static_cast<const Fx20Header *>(a.fx_hdr)->exp2;

    auto run = [&](auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        // The lane's LR rows of X per K step, MT indices each (BF16 and FX20's FP16 plane:
        // two per 32-bit word; FX20's int8 plane: the MT = 4 bytes of a row in one word).
        constexpr bool H16 = (P == P_BF16 || P == P_FX20);
        constexpr bool FX = (P == P_FX20);
        static_assert(!H16 || MT % 2 == 0, "16-bit tiles hold whole words");
        static_assert(!FX || MT == 4 || MT == 2, "FX20 tiles take the int8 values of a row in one word");
        constexpr int XWN = H16 ? MT / 2 : MT;
        using XWT = std::conditional_t<H16, uint32_t, XT>;
        XWT xb[NBUF][UB][LR][XWN];
        UT ub[NBUF][UB][NTA];
        uint32_t xl[FX ? NBUF : 1][FX ? UB : 1][FX ? LR : 1];
        UT ub2[FX ? NBUF : 1][FX ? UB : 1][FX ? NTA : 1];
        // Ring step st of the slab at xsrc into ring slot `slot`.  FULL and unguarded:
        // a fixed sequence of unmasked vector loads, so the compiler waits for exactly
        // the oldest step; otherwise rows past I_a (and dead steps) read as zero.
        auto issue = [&](int slot, const XT *xsrc, int64_t st, bool guard, bool live) {
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int64_t kb = st * UB + u;  // K step
                if constexpr (H16) {
                    // B operand: eight rows of one column, packed per lane by the pad kernel.
                    const bool bv = live && kb < nkb;
#pragma unroll
                    for (int nt = 0; nt < NTA; ++nt) {
                        const int64_t pk = ((kb * NTA + nt) * 64 + lane) * 8;
                        ub[slot][u][nt] = bv ? *reinterpret_cast<const u16x8 *>(Ua + pk) : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                        if constexpr (FX)
                            ub2[slot][u][nt] = bv ? *reinterpret_cast<const u16x8 *>(static_cast<const XT *>(a.Ua2) + pk)
                                                  : u16x8{0, 0, 0, 0, 0, 0, 0, 0};
                    }
                }
#pragma unroll
                for (int q = 0; q < LR; ++q) {
                    // lane group g holds K slots LR*g .. LR*g + LR-1 of the step (KR = 4 * LR rows)
                    const int64_t r = kb * KR + LR * g + q;
                    const bool rv = live && (!guard || r < a.Ia);
                    if constexpr (FX) {
                        // int8 plane: the lane's MT = 4 bytes of the row (zero out of range).
                        const uint8_t *lsrc = static_cast<const uint8_t *>(a.X2) + (xsrc - X) + r * a.stride_a;
                        uint32_t wv = 0;
                        if (rv) {
                            if (FULL || (a.vec_ok && ibase + MT <= a.Ic)) {
                                if constexpr (MT == 4) wv = ld_stream<XNT>(reinterpret_cast<const uint32_t *>(lsrc));
                                else wv = ld_stream<XNT>(reinterpret_cast<const uint16_t *>(lsrc));
                            } else {
#pragma unroll
                                for (int i = 0; i < MT; ++i)
                                    if (ibase + i < a.Ic) wv |= static_cast<uint32_t>(lsrc[i]) << (8 * i);
                            }
                        }
                        xl[slot][u][q] = wv;
                    }
                    if constexpr (!H16) {
#pragma unroll
                        for (int nt = 0; nt < NTA; ++nt) ub[slot][u][nt] = rv ? Ua[r * TA + nt * 16 + c] : UT{};
                    }
                    if constexpr (FULL && (V * sizeof(XT)) % 8 == 0) {
                        if (rv) {
#pragma unroll
                            for (int j = 0; j < NCH; ++j)
                                load_vec_n<XWT, V * sizeof(XT) / sizeof(XWT), XNT>(
                                    xb[slot][u][q] + j * V * sizeof(XT) / sizeof(XWT),
                                    reinterpret_cast<const XWT *>(xsrc + r * a.stride_a + j * 16 * V));
                        } else {
#pragma unroll
                            for (int i = 0; i < XWN; ++i) xb[slot][u][q][i] = XWT{};
                        }
                    } else {
                        // Ragged tile: chunks wholly in range still take one vector load.
                        constexpr int VW = V * static_cast<int>(sizeof(XT)) / static_cast<int>(sizeof(XWT));
                        auto elem = [&](int i) {
                            const int64_t e = (i / V) * 16 * V + i % V;
                            return (rv && ibase + e < a.Ic) ? xsrc[r * a.stride_a + e] : XT{};
                        };
#pragma unroll
                        for (int j = 0; j < NCH; ++j) {
                            const int64_t e0 = static_cast<int64_t>(j) * 16 * V;
                            bool done = false;
                            if constexpr ((V * sizeof(XT)) % 8 == 0) {
                                if (a.vec_ok && rv && ibase + e0 + V <= a.Ic) {
                                    load_vec_n<XWT, VW, XNT>(xb[slot][u][q] + j * VW,
                                                             reinterpret_cast<const XWT *>(xsrc + r * a.stride_a + e0));
                                    done = true;
                                }
                            }
                            if (!done) {
#pragma unroll
                                for (int k = 0; k < VW; ++k) {
                                    if constexpr (H16)
                                        xb[slot][u][q][j * VW + k] =
                                            static_cast<uint32_t>(elem(j * V + 2 * k)) |
                                            (static_cast<uint32_t>(elem(j * V + 2 * k + 1)) << 16);
                                    else
                                        xb[slot][u][q][j * VW + k] = elem(j * V + k);
                                }
                            }
                        }
                    }
                }
            }
        };
        DT d[MT][NTA];
        auto mac = [&](int slot) {
#pragma unroll
            for (int u = 0; u < UB; ++u)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    if constexpr (H16) {
                        // A operand: index mt of the lane's eight rows, two 16-bit values per word
                        uint32_t w4[4];
                        constexpr uint32_t kLo = 0x05040100u, kHi = 0x07060302u;  // low / high halves
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            w4[k] = __builtin_amdgcn_perm(xb[slot][u][2 * k + 1][mt / 2], xb[slot][u][2 * k][mt / 2],
                                                          (mt & 1) ? kHi : kLo);
                        u16x8 av;
                        __builtin_memcpy(&av, w4, 16);
                        if constexpr (FX) {
                            // int8 operand: byte mt of each row as the FP16 value (1152 + l) / 256,
                            // bit pattern 0x4400 | (b ^ 0x80); sum_k (256 h + l) u' =
                            // 256 (h.uh + h.ul + ((1152 + l)/256).uh) - 1152 sum uh.
                            const uint32_t sel = static_cast<uint32_t>(mt) | (0x0Cu << 8) |
                                                 (static_cast<uint32_t>(mt + 4) << 16) | (0x0Cu << 24);
                            uint32_t o4[4];
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                o4[k] = __builtin_amdgcn_perm(xl[slot][u][2 * k + 1] ^ 0x80808080u,
                                                              xl[slot][u][2 * k] ^ 0x80808080u, sel) | 0x44004400u;
                            u16x8 al;
                            __builtin_memcpy(&al, o4, 16);
#pragma unroll
                            for (int nt = 0; nt < NTA; ++nt) {
                                d[mt][nt] = mfma_f16(av, ub[slot][u][nt], d[mt][nt]);
                                d[mt][nt] = mfma_f16(av, ub2[slot][u][nt], d[mt][nt]);
                                d[mt][nt] = mfma_f16(al, ub[slot][u][nt], d[mt][nt]);
                            }
                        } else {
#pragma unroll
                            for (int nt = 0; nt < NTA; ++nt) d[mt][nt] = mfma_bf16(av, ub[slot][u][nt], d[mt][nt]);
                        }
                    } else {
#pragma unroll
                        for (int nt = 0; nt < NTA; ++nt) {
                            if constexpr (P == P_FP64)
                                d[mt][nt] = mfma_f64(xb[slot][u][0][mt], ub[slot][u][nt], d[mt][nt]);
                            else
                                d[mt][nt] = mfma_f32(xb[slot][u][0][mt], ub[slot][u][nt], d[mt][nt]);
                        }
                    }
                }
        };

        const XT *xs = X + slab_offset(a.od, a.slab_stride, s0) + ibase;
        // The ring runs on across slab boundaries: the first NBUF-1 steps of a slab are
        // issued during the last ring turn of the previous one, so the loads stay in
        // flight through stage 2 and the workgroup reduction.
#pragma unroll
        for (int u = 0; u < NBUF - 1; ++u) issue(u, xs, u, u >= nfull, s0 < s1);
        for (int64_t slab = s0; slab < s1; ++slab) {
            const bool has_next = slab + 1 < s1;
            const XT *xn = has_next ? X + slab_offset(a.od, a.slab_stride, slab + 1) + ibase : xs;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NTA; ++nt) d[mt][nt] = DT{0, 0, 0, 0};
            int64_t t = 0;
            for (; t + 2 * NBUF - 2 < nfull; t += NBUF) {
#pragma unroll
                for (int u = 0; u < NBUF; ++u) {
                    issue((u + NBUF - 1) % NBUF, xs, t + u + NBUF - 1, false, true);
                    mac(u);
                }
            }
            for (; t < nsp; t += NBUF) {
#pragma unroll
                for (int u = 0; u < NBUF; ++u) {
                    const int64_t tn = t + u + NBUF - 1;
                    const bool cur = tn < nsp;
                    issue((u + NBUF - 1) % NBUF, cur ? xs : xn, cur ? tn : tn - nsp, true, cur || has_next);
                    if (t + u < nsteps) mac(u);
                }
            }

            if constexpr (FX) {
                // D = 2^(e + k_col) (256 D' - 1152 sum uh): back to the values of X and U^a.
#pragma unroll
                for (int ta = 0; ta < NTA; ++ta) {
                    const double sc = ldexp(a.ua_scale[ta * 16 + c], fx_e), off = a.ua_off[ta * 16 + c];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            d[mt][ta][v] = static_cast<float>((256.0 * static_cast<double>(d[mt][ta][v]) - off) * sc);
                }
            }
            if constexpr (STAGE2) {
                // Z[r_c, r_a] = sum_{i_c} U^c[i_c, r_c] D[i_c, r_a]: K-step v pairs slot g
                // with the D row that lanes of group g hold in register v.
                DT z[NTC][NTA];
#pragma unroll
                for (int tc = 0; tc < NTC; ++tc)
#pragma unroll
                    for (int ta = 0; ta < NTA; ++ta) z[tc][ta] = DT{0, 0, 0, 0};
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int tr = tile_row<P>(lane, v);
                        const int64_t rowc = cbase + (mt / V) * 16 * V + tr * V + mt % V;
                        const bool rv = ctile < a.n_ctiles && rowc < a.Ic;
#pragma unroll
                        for (int tc = 0; tc < NTC; ++tc) {
                            CT u;
                            if constexpr (UC_LDS) u = lds_uc[(rowc - crow0) * TC + tc * 16 + c];  // zero past I_c
                            else u = rv ? Uc[rowc * TC + tc * 16 + c] : CT{};
#pragma unroll
                            for (int ta = 0; ta < NTA; ++ta) {
                                if constexpr (P == P_FP64)
                                    z[tc][ta] = mfma_f64(u, d[mt][ta][v], z[tc][ta]);
                                else
                                    z[tc][ta] = mfma_f32(u, d[mt][ta][v], z[tc][ta]);
                            }
                        }
                    }
                // Fixed-order reduction over the workgroup's c-tiles (wave order); the
                // partial tile is stored unpadded, r_a x r_c.
                const int zn = a.ra * a.rc;
                double *out = a.P + (static_cast<int64_t>(cgroup) * a.n_slabs + slab) * zn;
                if constexpr (Z_PAR) {
#pragma unroll
                    for (int tc = 0; tc < NTC; ++tc)
#pragma unroll
                        for (int ta = 0; ta < NTA; ++ta)
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                lds[w * TA * TC + (ta * 16 + c) * TC + tc * 16 + tile_row<P>(lane, v)] =
                                    static_cast<double>(z[tc][ta][v]);
                    __syncthreads();
                    // Thread t sums column t % TC of rows t / TC, + 4 nwaves / NTC, ...: no
                    // runtime divisions (TC is a compile-time power of two).
                    for (int ra = static_cast<int>(threadIdx.x) / TC; ra < a.ra; ra += 64 * a.nwaves / TC) {
                        const int col = static_cast<int>(threadIdx.x) % TC;
                        if (col < a.rc) {
                            const int j = ra * TC + col;
                            double acc = lds[j];
                            for (int ww = 1; ww < a.nwaves; ++ww) acc += lds[ww * TA * TC + j];
                            out[ra * a.rc + col] = acc;
                        }
                    }
                } else {
                    for (int ww = 0; ww < a.nwaves; ++ww) {
                        if (w == ww) {
#pragma unroll
                            for (int tc = 0; tc < NTC; ++tc)
#pragma unroll
                                for (int ta = 0; ta < NTA; ++ta)
#pragma unroll
                                    for (int v = 0; v < 4; ++v) {
                                        const int i = (ta * 16 + c) * TC + tc * 16 + tile_row<P>(lane, v);
                                        const double zv = static_cast<double>(z[tc][ta][v]);
                                        lds[i] = (ww == 0) ? zv : lds[i] + zv;
                                    }
                        }
                        __syncthreads();
                    }
                    for (int ra = static_cast<int>(threadIdx.x) / TC; ra < a.ra; ra += 64 * a.nwaves / TC) {
                        const int col = static_cast<int>(threadIdx.x) % TC;
                        if (col < a.rc) out[ra * a.rc + col] = lds[ra * TC + col];
                    }
                }
                __syncthreads();
            } else {
                const int64_t rows = static_cast<int64_t>(a.n_ctiles) * 16 * MT;
                double *out = a.P + slab * rows * TA;
                if (ctile < a.n_ctiles) {
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int ta = 0; ta < NTA; ++ta)
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                out[(cbase + (mt / V) * 16 * V + tile_row<P>(lane, v) * V + mt % V) * TA + ta * 16 + c] =
                                    static_cast<double>(d[mt][ta][v]);
                }
            }
            xs = xn;
        }
    };
    if (full) run(std::true_type{});
    else run(std::false_type{});
}

// Zero-padded copy of a factor in the fused kernel's element type T (the form's
// own: FP64 or FP32, so the copy is exact): dst[i][j] = src[i][j] for j < r, 0 up to ldd.
template <typename T>
__global__ void __launch_bounds__(256) pad_factor_kernel(const T *src, int64_t rows, int r, int ldd, T *dst)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= rows * ldd) return;
    const int64_t i = e / ldd;
    const int j = static_cast<int>(e % ldd);
    dst[e] = (j < r) ? src[i * r + j] : T{};
}

// Stage-1 factor of the FX20 form, one workgroup per (padded) column: the column's
// power-of-two scale 2^-k with |u| 2^-k < 1 (tree maximum; scale = 2^k, zero columns
// past r take k = 0), then its values scaled, split into FP16 hi + lo and written
// into the per-K-step, per-lane packing of the BF16 form (eight rows of one column
// per lane; zero past the rows), and off = 1152 * the sum of the hi parts (removes the
// int8 operand's offset).  Rows are strided over the threads and both reductions are
// fixed-order trees, so the results do not depend on timing.
__global__ void __launch_bounds__(256) fx20_factor_cols_kernel(const float *src, int64_t rows, int r, int nta,
                                                               int64_t nkb, int *kexp, double *scale, double *off,
                                                               uint16_t *hi, uint16_t *lo)
{
    __shared__ float smx[256];
    __shared__ double ssum[256];
    const int col = static_cast<int>(blockIdx.x);
    const int t = static_cast<int>(threadIdx.x);
    float mx = 0.0f;
    if (col < r)
        for (int64_t i = t; i < rows; i += 256) mx = fmaxf(mx, fabsf(src[i * r + col]));
    smx[t] = mx;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) smx[t] = fmaxf(smx[t], smx[t + h]);
        __syncthreads();
    }
    int k = 0;
    if (smx[0] > 0.0f) (void)frexpf(smx[0], &k);
    const int nt = col / 16, c = col % 16;
    double sh = 0.0;
    for (int64_t i = t; i < nkb * 32; i += 256) {
        const float v = (col < r && i < rows) ? ldexpf(src[i * r + col], -k) : 0.0f;
        const _Float16 h = static_cast<_Float16>(v);
        const _Float16 l = static_cast<_Float16>(v - static_cast<float>(h));
        sh += static_cast<double>(static_cast<float>(h));
        const int64_t kb = i / 32;
        const int w = static_cast<int>(i % 32);
        const int64_t e = ((kb * nta + nt) * 64 + 16 * (w / 8) + c) * 8 + w % 8;
        hi[e] = __builtin_bit_cast(uint16_t, h);
        lo[e] = __builtin_bit_cast(uint16_t, l);
    }
    ssum[t] = sh;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) ssum[t] += ssum[t + h];
        __syncthreads();
    }
    if (t == 0) {
        kexp[col] = k;
        scale[col] = ldexp(1.0, k);
        off[col] = 1152.0 * ssum[0];
    }
}

// BF16 stage-1 factor: for K step kb (rows 32 kb ..), column tile nt and lane
// (g, c), the eight BF16 values of rows 32 kb + 8 g .. + 7 in column 16 nt + c,
// contiguous (one 16-byte load per lane); zero past the factor's rows and columns.
__global__ void __launch_bounds__(256) pack_factor_bf16_kernel(const float *src, int64_t rows, int r, int nta,
                                                              int64_t nkb, uint16_t *dst)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nkb * nta * 512) return;
    const int q = static_cast<int>(e % 8);
    const int lane = static_cast<int>((e / 8) % 64);
    const int nt = static_cast<int>((e / 512) % nta);
    const int64_t kb = e / (512 * static_cast<int64_t>(nta));
    const int64_t row = kb * 32 + 8 * (lane >> 4) + q;
    const int col = nt * 16 + (lane & 15);
    dst[e] = (row < rows && col < r) ? f32_to_bf16_bits(src[row * r + col]) : uint16_t{0};
}

// Bytes of the padded stage-1 factor copy of a rows x (16 nta) tile set.
size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Stage-1 factor copy.  FX20: hi pack, lo pack, then per column 2^k (double),
// 1152 * sum of hi (double) and k (int), each 256-byte aligned.
size_t stage1_factor_bytes(int prec, int64_t rows, int nta)
{
    const size_t pack = static_cast<size_t>((rows + 31) / 32) * nta * 512 * sizeof(uint16_t);
    if (prec == P_BF16) return pack;
    if (prec == P_FX20)
        return 2 * align256(pack) + 2 * align256(static_cast<size_t>(16 * nta) * 8) + align256(16 * nta * 4);
    return static_cast<size_t>(rows) * 16 * nta * (prec == P_FP64 ? 8 : 4);
}

// Sum `parts` padded partial tensors and scatter into a strided destination.
// Element (s, x, y): s over the slab modes (dims sdim), x < X1 (padded PX), y < Y1 (padded PY).
struct ReduceArgs {
    const double *P;
    int64_t parts, part_stride;
    int nd;
    int64_t sdim[DEINSUM_MAX_ORDER];
    int64_t sstr[DEINSUM_MAX_ORDER];  // destination strides of the slab modes
    int64_t X1, PX, xstr, Y1, PY, ystr;
    int64_t total;
    void *out;
    int out_dtype;
};

__global__ void __launch_bounds__(256) reduce_strided_kernel(const ReduceArgs a)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= a.total) return;
    const int64_t y = e % a.Y1;
    const int64_t x = (e / a.Y1) % a.X1;
    int64_t s = e / (a.Y1 * a.X1);
    int64_t off = x * a.xstr + y * a.ystr;
    const int64_t slab = s;
    for (int m = a.nd - 1; m >= 0; --m) {
        off += (s % a.sdim[m]) * a.sstr[m];
        s /= a.sdim[m];
    }
    const double *p = a.P + (slab * a.PX + x) * a.PY + y;
    double acc = 0.0;
    for (int64_t q = 0; q < a.parts; ++q) acc += p[q * a.part_stride];
    if (a.out_dtype == DEINSUM_F64) static_cast<double *>(a.out)[off] = acc;
    else static_cast<float *>(a.out)[off] = static_cast<float>(acc);
}

// One mode product on an FP64 intermediate with a strided destination.  A thread
// computes RB consecutive ranks of one output fibre, reading each input value once;
// RB is the rank rounded up to 8, 16, 24 or 32 (8 beyond that), so for ranks up to 32
// every input fibre is read by one thread only.
constexpr int kTtmRB = 8;  // granularity of RB
int ttm_rb(int64_t r) { return r <= 32 ? static_cast<int>((r + 7) / 8 * 8) : 8; }
struct SmallTtmArgs {
    const double *T;
    int nd;
    int64_t odim[DEINSUM_MAX_ORDER];  // output extents (dim m is Rm)
    int64_t tstr[DEINSUM_MAX_ORDER];  // input strides
    int64_t ostr[DEINSUM_MAX_ORDER];  // output strides
    int m;
    int64_t Im;
    const void *U;
    int64_t ldu;
    int uprec;
    int64_t total;                    // threads: product of odim with dim m counted in blocks of RB
    void *out;
    int out_dtype;
    int lds;                          // 1: U staged in LDS (dynamic shared memory)
};

// Largest factor (rows x ranks rounded up to RB, FP64) staged in LDS per workgroup.
constexpr size_t kTtmLdsBytes = 48 * 1024;
// Below this many output fibres (four waves' worth on each of the 1024 SIMDs) a small
// TTM takes the pipelined row walk, when the staged factor and the waves' partial sums
// fit in this much LDS.
constexpr int64_t kTtmPipeThreads = int64_t{1024} * 4 * 64;
constexpr size_t kTtmPipeLdsBytes = 64 * 1024;

// Where a thread's factor weights come from: global memory per lane (ranks in
// blocks of RB), LDS (the factor staged per workgroup), or, when one block holds
// every rank, global memory at wave-uniform addresses (scalar loads into SGPRs, the
// products' scalar operand; no LDS traffic, which bounds the LDS form: every row
// returns RB broadcast weights to all 64 lanes for RB products per lane).
enum { kTtmWGlobal = 0, kTtmWLds = 1, kTtmWUniform = 2 };
using const_f64_k = const __attribute__((address_space(4))) double;
using const_f32_k = const __attribute__((address_space(4))) float;

template <int RB, int WM, bool PIPE>
__global__ void __launch_bounds__(256) small_ttm_kernel(const SmallTtmArgs a)
{
    constexpr bool LDS = (WM == kTtmWLds);
    extern __shared__ double su[];  // LDS: U as FP64, row stride ldl = ranks rounded up to RB
    const int64_t ldl = (a.odim[a.m] + RB - 1) / RB * RB;
    if constexpr (LDS) {
        for (int64_t i = threadIdx.x; i < a.Im * ldl; i += blockDim.x) {
            const int64_t row = i / ldl, r = i % ldl;
            su[i] = r < a.odim[a.m] ? ldu_p(a.U, row * a.ldu + r, a.uprec) : 0.0;
        }
        __syncthreads();
    }
    // PIPE: a workgroup's four waves share its 64 fibres, wave w summing rows
    // [w Im / 4, (w + 1) Im / 4); otherwise one thread per fibre over every row.
    const int wv = PIPE ? static_cast<int>(threadIdx.x >> 6) : 0;
    const int64_t e = PIPE ? static_cast<int64_t>(blockIdx.x) * 64 + (threadIdx.x & 63)
                           : static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool valid = e < a.total;
    if (!PIPE && !valid) return;
    int64_t rem = valid ? e : 0, ioff = 0, ooff = 0, r0 = 0;
    for (int d = a.nd - 1; d >= 0; --d) {
        const int64_t ext = (d == a.m) ? (a.odim[d] + RB - 1) / RB : a.odim[d];
        const int64_t i = rem % ext;
        rem /= ext;
        if (d == a.m) {
            r0 = i * RB;
        } else {
            ooff += i * a.ostr[d];
            ioff += i * a.tstr[d];
        }
    }
    const int nr = static_cast<int>(tmin(RB, a.odim[a.m] - r0));
    double acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = 0.0;
    const int64_t sm = a.tstr[a.m];
    // Rows of the input fibre summed in ascending order, in batches of eight loads.
    // PIPE (launches with few fibres, e.g. 192^4 R=16: 768 fibre waves) splits the rows
    // over four waves, and each takes batches of sixteen, issuing the next batch's
    // loads before the current batch's products and reading each row's weights
    // together, so that up to 32 loads per thread are in flight: such a launch is
    // otherwise bound by one memory latency per batch.  Without PIPE the kernel keeps
    // its lower register count, and the occupancy that hides latency in launches with
    // many fibres.
    auto walk = [&](auto wt) {  // wt(i, q): factor entry of row i, rank r0 + q
        if constexpr (!PIPE) {
            int64_t i = 0;
            for (; i + 8 <= a.Im; i += 8) {
                double t[8];  // eight loads in flight per thread
#pragma unroll
                for (int k = 0; k < 8; ++k) t[k] = a.T[ioff + (i + k) * sm];
#pragma unroll
                for (int k = 0; k < 8; ++k)
#pragma unroll
                    for (int q = 0; q < RB; ++q) acc[q] += t[k] * wt(i + k, q);
            }
            for (; i < a.Im; ++i) {
                const double t = a.T[ioff + i * sm];
#pragma unroll
                for (int q = 0; q < RB; ++q) acc[q] += t * wt(i, q);
            }
            return;
        }
        constexpr int KB = 16;  // rows per batch
        const int64_t r_lo = wv * a.Im / 4, r_hi = (wv + 1) * a.Im / 4;
        if (!valid) return;
        const int64_t nb = r_lo + (r_hi - r_lo) / KB * KB;
        double ta[KB], tb[KB];
        auto load = [&](double(&t)[KB], int64_t i) {
#pragma unroll
            for (int k = 0; k < KB; ++k) t[k] = a.T[ioff + (i + k) * sm];
        };
        auto use = [&](const double(&t)[KB], int64_t i) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                double w[RB];
#pragma unroll
                for (int q = 0; q < RB; ++q) w[q] = wt(i + k, q);
#pragma unroll
                for (int q = 0; q < RB; ++q) acc[q] += t[k] * w[q];
            }
        };
        int64_t i = r_lo;
        if (nb > r_lo) load(ta, r_lo);
        for (; i < nb; i += 2 * KB) {
            const bool more = i + KB < nb;
            if (more) load(tb, i + KB);
            use(ta, i);
            if (!more) {
                i += KB;
                break;
            }
            if (i + 2 * KB < nb) load(ta, i + 2 * KB);
            use(tb, i + KB);
        }
        for (; i < r_hi; ++i) {
            const double t = a.T[ioff + i * sm];
#pragma unroll
            for (int q = 0; q < RB; ++q) acc[q] += t * wt(i, q);
        }
    };
    if constexpr (WM == kTtmWUniform) {
        // launched only when the factor has exactly RB columns: r0 = 0 in every thread
        if (a.uprec == P_FP64) {
            const_f64_k *U = (const_f64_k *)(a.U);
            walk([&](int64_t i, int q) { return U[i * a.ldu + q]; });
        } else {
            const_f32_k *U = (const_f32_k *)(a.U);
            walk([&](int64_t i, int q) { return static_cast<double>(U[i * a.ldu + q]); });
        }
    } else if constexpr (LDS) {
        // every rank of the block is staged (zero past the last): no clamping needed
        walk([&](int64_t i, int q) { return su[i * ldl + r0 + q]; });
    } else {
        // Factor read from global memory; ranks past the last are clamped (their sums dropped),
        // so the loads of an unrolled step are unconditional.
        if (a.uprec == P_FP64) {
            const double *U = static_cast<const double *>(a.U);
            walk([&](int64_t i, int q) { return U[i * a.ldu + r0 + (q < nr ? q : 0)]; });
        } else {
            const float *U = static_cast<const float *>(a.U);
            walk([&](int64_t i, int q) { return static_cast<double>(U[i * a.ldu + r0 + (q < nr ? q : 0)]); });
        }
    }
    if constexpr (PIPE) {
        // Waves 1-3 hand their partial sums to wave 0 through LDS (after the staged
        // factor); wave 0 adds them in wave order and stores.
        double *red = su + (LDS ? a.Im * ldl : 0);
        if (wv > 0)
#pragma unroll
            for (int q = 0; q < RB; ++q) red[((wv - 1) * RB + q) * 64 + (threadIdx.x & 63)] = acc[q];
        __syncthreads();
        if (wv > 0 || !valid) return;
#pragma unroll
        for (int w = 0; w < 3; ++w)
#pragma unroll
            for (int q = 0; q < RB; ++q) acc[q] += red[(w * RB + q) * 64 + threadIdx.x];
    }
    // Predicated stores, not an early exit: a loop that leaves early is not unrolled,
    // and indexing acc in it would place acc in scratch memory.
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        if (q < nr) {
            const int64_t o = ooff + (r0 + q) * a.ostr[a.m];
            if (a.out_dtype == DEINSUM_F64) static_cast<double *>(a.out)[o] = acc[q];
            else static_cast<float *>(a.out)[o] = static_cast<float>(acc[q]);
        }
    }
}

template <int P, int NTA, int NTC, int MT, bool S2, int UB, int NB, bool XNT>
void launch_tk(const TkArgs &a, int64_t grid, hipStream_t s)
{
    const size_t lds = TkLds<P, NTA, NTC, MT, S2>::bytes(a.nwaves);
    ttmc_fused_kernel<P, NTA, NTC, MT, S2, UB, NB, XNT><<<static_cast<unsigned>(grid), 64 * a.nwaves, lds, s>>>(a);
}

using TkLaunch = void (*)(const TkArgs &, int64_t, hipStream_t);
struct TkEntry {
    int p, nta, ntc, mt, ub, nbuf;
    bool s2;
    TkLaunch fn;
};
// M tiles per wave and ring depth are chosen per rank tile to stay within
// 2 waves per SIMD without spills.  Wider M tiles read each factor row for
// more X (the factor rows come from L2: a 16*NTA-wide row per 16*MT X values).
// For each (precision, NTA, NTC) the first entry is the default; later ones
// are alternatives selectable by plan_hint.
#define TK(P, A, C, MT, UB, NB) {P, A, C, MT, UB, NB, true, &launch_tk<P, A, C, MT, true, UB, NB, false>}
#define TKN(P, A, C, MT, UB, NB) {P, A, C, MT, UB, NB, true, &launch_tk<P, A, C, MT, true, UB, NB, true>}
#define TK1(P, A, MT, UB, NB) {P, A, 0, MT, UB, NB, false, &launch_tk<P, A, 1, MT, false, UB, NB, false>}
const TkEntry kTkTable[] = {
    TKN(P_FP64, 1, 1, 4, 2, 4), TK(P_FP64, 1, 2, 4, 2, 4), TK(P_FP64, 1, 4, 4, 2, 4),
    TK(P_FP64, 2, 1, 4, 2, 3), TKN(P_FP64, 2, 2, 4, 2, 3), TK(P_FP64, 2, 4, 2, 2, 4),
    TK(P_FP64, 4, 1, 2, 2, 3), TK(P_FP64, 4, 2, 2, 2, 3), TK(P_FP64, 4, 4, 1, 2, 3),
    // alternatives (plan_hint 1, 2, ...)
    TK(P_FP64, 1, 1, 4, 3, 2), TKN(P_FP64, 1, 1, 4, 3, 2), TK(P_FP64, 1, 1, 4, 2, 4), TK(P_FP64, 1, 2, 4, 3, 2),
    TKN(P_FP64, 1, 2, 4, 3, 2), TK(P_FP64, 2, 1, 4, 3, 2), TKN(P_FP64, 2, 1, 4, 3, 2), TK(P_FP64, 2, 2, 4, 2, 3),
    TK(P_FP64, 2, 2, 4, 3, 2), TKN(P_FP64, 2, 2, 4, 3, 2), TK(P_FP64, 2, 2, 2, 2, 4), TKN(P_FP64, 2, 2, 4, 2, 2),
    TK(P_FP64, 2, 1, 2, 2, 4),
    TK(P_FP64, 4, 1, 1, 2, 4), TK(P_FP64, 4, 2, 1, 2, 4),
    TKN(P_FP32, 1, 1, 4, 2, 4), TK(P_FP32, 1, 2, 4, 2, 4), TK(P_FP32, 1, 4, 4, 2, 4), TK(P_FP32, 2, 1, 4, 2, 4),
    TKN(P_FP32, 2, 2, 4, 4, 2), TK(P_FP32, 2, 4, 4, 2, 4), TK(P_FP32, 4, 1, 2, 2, 4), TK(P_FP32, 4, 2, 2, 2, 4),
    TK(P_FP32, 4, 4, 2, 2, 3),
    TK(P_FP32, 1, 1, 4, 2, 4), TK(P_FP32, 1, 1, 4, 4, 2), TK(P_FP32, 2, 2, 4, 2, 4), TKN(P_FP32, 2, 2, 4, 2, 4),
    TK(P_FP32, 2, 2, 4, 4, 2), TK(P_FP32, 2, 2, 8, 2, 2), TKN(P_FP32, 2, 2, 8, 2, 2),
    TK(P_FP32, 1, 1, 8, 2, 3), TKN(P_FP32, 1, 1, 8, 2, 3),
    TKN(P_BF16, 1, 1, 4, 1, 3), TK(P_BF16, 1, 2, 4, 1, 3), TK(P_BF16, 1, 4, 4, 1, 3), TK(P_BF16, 2, 1, 4, 1, 3),
    TK(P_BF16, 2, 2, 4, 1, 3), TK(P_BF16, 2, 4, 4, 1, 2), TK(P_BF16, 4, 1, 4, 1, 2), TK(P_BF16, 4, 2, 4, 1, 2),
    TK(P_BF16, 4, 4, 2, 1, 2),
    TK(P_BF16, 1, 1, 4, 1, 3), TK(P_BF16, 1, 1, 8, 1, 2), TKN(P_BF16, 2, 2, 4, 1, 3), TK(P_BF16, 2, 2, 4, 1, 2),
    TKN(P_BF16, 2, 2, 4, 1, 2),
    TK(P_FX20, 1, 1, 4, 2, 2), TK(P_FX20, 1, 2, 4, 1, 2), TK(P_FX20, 1, 4, 4, 1, 2), TK(P_FX20, 2, 1, 4, 1, 2),
    TK(P_FX20, 2, 2, 4, 1, 3), TK(P_FX20, 2, 4, 4, 1, 2), TK(P_FX20, 4, 1, 4, 1, 2), TK(P_FX20, 4, 2, 4, 1, 2),
    TK(P_FX20, 4, 4, 4, 1, 2),
    TK(P_FX20, 1, 1, 4, 1, 2), TKN(P_FX20, 1, 1, 4, 1, 2), TK(P_FX20, 1, 1, 4, 1, 3), TKN(P_FX20, 1, 1, 4, 2, 2),
    TKN(P_FX20, 2, 2, 4, 1, 2), TK(P_FX20, 2, 2, 4, 1, 2),
    TKN(P_FX20, 2, 2, 4, 1, 3), TK(P_FX20, 2, 2, 4, 1, 4), TK(P_FX20, 2, 2, 4, 2, 2),
    TK1(P_FP64, 1, 4, 2, 4), TK1(P_FP64, 2, 2, 2, 4), TK1(P_FP64, 4, 1, 2, 4),
    TK1(P_FP32, 1, 4, 2, 4), TK1(P_FP32, 2, 4, 2, 4), TK1(P_FP32, 4, 2, 2, 4),
    TK1(P_BF16, 1, 4, 1, 3), TK1(P_BF16, 2, 4, 1, 2), TK1(P_BF16, 4, 4, 1, 2),
    TK1(P_FX20, 1, 4, 1, 2), TK1(P_FX20, 2, 4, 1, 2), TK1(P_FX20, 4, 4, 1, 2),
};
#undef TK
#undef TKN
#undef TK1

// The variant-th compiled kernel (0 = default) for this precision and rank tiles.
const TkEntry *find_tk(int prec, int nta, int ntc, bool s2, int variant)
{
    for (const auto &e : kTkTable)
        if (e.p == prec && e.nta == nta && e.s2 == s2 && (!s2 || e.ntc == ntc) && variant-- == 0) return &e;
    return nullptr;
}

int64_t cdivl(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Untuned pick: the table's first entry, unless the contiguous mode is too short
// to give that entry's workgroup its four waves (one wave per 16*MT-wide c-tile);
// then the first entry with the most waves.  A 60-wide mode with MT = 4 leaves one
// wave per workgroup and nothing to hide the slab loads behind.
int default_variant(int prec, int nta, int ntc, bool s2, int64_t Ic)
{
    int best = 0, best_w = -1;
    for (int v = 0;; ++v) {
        const TkEntry *e = find_tk(prec, nta, ntc, s2, v);
        if (!e) break;
        const int w = static_cast<int>(std::min<int64_t>(4, cdivl(Ic, 16 * e->mt)));
        if (w > best_w) {
            best = v;
            best_w = w;
        }
        if (w == 4) break;
    }
    return best;
}

}  // namespace

std::string ttmc_tune_key(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, int prec)
{
    std::string k = "t:N" + std::to_string(spec->order) + ":n" + std::to_string(spec->free_mode) + ":p" +
                    std::to_string(prec) + ":R";
    for (int m = 0, first = 1; m < spec->order; ++m) {
        if (m == spec->free_mode) continue;
        k += (first ? "" : "x") + std::to_string(ranks[spec->operand_of_mode[m]]);
        first = 0;
    }
    k += ":";
    for (int m = 0; m < spec->order; ++m) k += (m ? "x" : "") + std::to_string(dims[m]);
    return k;
}

namespace {
int ntiles_for(int64_t r) { return r <= 16 ? 1 : (r <= 32 ? 2 : 4); }

// ------------------------------------------------------------------ host plan
struct DimInfo {
    int mode;
    int64_t extent;
};

struct TtmcPlan {
    int N = 0, n = 0, a = -1, c = -1;
    bool stage2 = true, via_mttkrp = false;
    int64_t I[DEINSUM_MAX_ORDER] = {0}, Rm[DEINSUM_MAX_ORDER] = {0};
    int nta = 1, ntc = 1, mt = 4;
    const TkEntry *kernel = nullptr;
    std::vector<int> slab_modes;
    int64_t n_slabs = 1;
    int n_ctiles = 1, nwaves = 1, n_cgroups = 1;
    int64_t spg = 1, groups = 0;
    size_t p_bytes = 0, z_bytes = 0, t_bytes = 0, pad_bytes = 0, total = 0;
};

deinsum_status make_plan(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, int prec,
                         int variant, TtmcPlan *out)
{
    TtmcPlan p;
    p.N = spec->order;
    p.n = spec->free_mode;
    for (int m = 0; m < p.N; ++m) {
        p.I[m] = dims[m];
        if (m == p.n) continue;
        const int64_t r = ranks[spec->operand_of_mode[m]];
        if (r < 1 || r > kMaxTtmcRank)
            return fail(DEINSUM_ERR_SHAPE, "TTMc ranks must be 1.." + std::to_string(kMaxTtmcRank));
        p.Rm[m] = r;
    }
    if (prec != P_FP64 && prec != P_FP32 && prec != P_BF16 && prec != P_FX20)
        return fail(DEINSUM_ERR_UNSUPPORTED, "TTMc supports the FP64, FP32, BF16 and FX20 forms");
    const int N = p.N, n = p.n;
    if (N == 2 && n == 0) {  // a single product over the contiguous mode: the MTTKRP kernel computes it
        p.via_mttkrp = true;
        *out = p;
        return DEINSUM_OK;
    }
    p.c = N - 1;
    if (n == N - 1) {
        p.stage2 = false;
        p.a = N - 2;
    } else {
        p.stage2 = true;
        p.a = (N - 2 != n) ? N - 2 : N - 3;
    }
    p.nta = ntiles_for(p.Rm[p.a]);
    p.ntc = p.stage2 ? ntiles_for(p.Rm[p.c]) : 1;
    for (int m = 0; m < N; ++m)
        if (m != p.a && m != p.c) {
            p.slab_modes.push_back(m);
            p.n_slabs *= p.I[m];
        }
    // plan_hint 0: the autotuned variant for this problem if cached, else the default;
    // plan_hint k >= 1: compiled variant k - 1.
    int v = variant > 0 ? variant - 1 : 0;
    if (variant == 0) {
        TuneChoice tc;
        if (tune_lookup(ttmc_tune_key(spec, dims, ranks, prec), &tc) && find_tk(prec, p.nta, p.ntc, p.stage2, tc.split))
            v = tc.split;
        else
            v = default_variant(prec, p.nta, p.ntc, p.stage2, dims[p.c]);
    }
    p.kernel = find_tk(prec, p.nta, p.ntc, p.stage2, v);
    if (!p.kernel)
        return fail(variant ? DEINSUM_ERR_INVALID_ARG : DEINSUM_ERR_UNSUPPORTED,
                    variant ? "plan_hint names no compiled TTMc kernel variant"
                            : "no fused TTMc kernel for this precision and ranks");
    p.mt = p.kernel->mt;
    p.n_ctiles = static_cast<int>(cdivl(p.I[p.c], 16 * p.mt));
    p.nwaves = std::min(4, p.n_ctiles);
    p.n_cgroups = static_cast<int>(cdivl(p.n_ctiles, p.nwaves));
    if (!p.stage2) p.n_cgroups = static_cast<int>(cdivl(p.n_ctiles, p.nwaves));
    p.spg = std::max<int64_t>(1, (p.n_slabs * p.n_cgroups) / 4096);
    p.groups = p.n_cgroups * cdivl(p.n_slabs, p.spg);
    const int64_t TA = 16 * p.nta, TC = 16 * p.ntc;
    if (p.stage2) p.p_bytes = static_cast<size_t>(p.n_cgroups * p.n_slabs * p.Rm[p.a] * p.Rm[p.c]) * 8;
    else p.p_bytes = static_cast<size_t>(p.n_slabs * p.n_ctiles * 16 * p.mt * TA) * 8;
    // Intermediate after the fused pass, then ping-pong buffers for the remaining products.
    int64_t zel = p.n_slabs * p.Rm[p.a] * (p.stage2 ? p.Rm[p.c] : p.I[n]);
    const bool remaining = p.slab_modes.size() > (p.stage2 ? 1u : 0u);
    if (remaining) {
        p.z_bytes = static_cast<size_t>(zel) * 8;
        p.t_bytes = p.z_bytes;  // every later intermediate is no larger (ranks <= extents not assumed)
        // Same order as run_ttmc: the remaining modes are contracted last mode first.
        int64_t cur = zel, mx = 0;
        for (auto it = p.slab_modes.rbegin(); it != p.slab_modes.rend(); ++it) {
            const int m = *it;
            if (m == n) continue;
            cur = cur / p.I[m] * p.Rm[m];
            mx = std::max(mx, cur);
        }
        p.t_bytes = static_cast<size_t>(mx) * 8;
    }
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    p.pad_bytes = align(stage1_factor_bytes(prec, p.I[p.a], p.nta)) +
                  (p.stage2 ? align(static_cast<size_t>(p.I[p.c]) * TC * 8) : 0);
    p.total = align(p.p_bytes) + align(p.z_bytes) + 2 * align(p.t_bytes) + p.pad_bytes;
    *out = p;
    return DEINSUM_OK;
}

}  // namespace

deinsum_status ttmc_workspace_size(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks,
                                   const deinsum_opts &o, size_t *bytes)
{
    if (!spec || !dims || !ranks || !bytes) return fail(DEINSUM_ERR_INVALID_ARG, "null argument");
    if (spec->kind != DEINSUM_TTMC) return fail(DEINSUM_ERR_INVALID_ARG, "spec is not a TTMc");
    for (int m = 0; m < spec->order; ++m)
        if (dims[m] < 1) return fail(DEINSUM_ERR_SHAPE, "TTMc dims must be >= 1");
    TtmcPlan p;
    if (o.plan_hint < 0) return fail(DEINSUM_ERR_INVALID_ARG, "TTMc plan_hint must be >= 0");
    if (deinsum_status st = make_plan(spec, dims, ranks, o.precision, o.plan_hint, &p)) return st;
    if (p.via_mttkrp) {
        const int64_t R = ranks[0];
        deinsum_spec ms = *spec;
        ms.kind = DEINSUM_MTTKRP;
        deinsum_opts o2 = o;
        o2.plan_hint = 0;  // the TTMc variant index means nothing to the MTTKRP planner
        return deinsum_workspace_size(&ms, dims, &R, &o2, bytes);
    }
    *bytes = p.total;
    return DEINSUM_OK;
}

deinsum_status run_ttmc(const deinsum_spec *spec, const int64_t *dims, const int64_t *ranks, const void *X,
                        const void *const *U, void *Y, const deinsum_opts &o, void *ws, size_t ws_bytes,
                        hipStream_t s)
{
    if (!ranks || !U || !Y || !X) return fail(DEINSUM_ERR_INVALID_ARG, "null argument");
    for (int m = 0; m < spec->order; ++m)
        if (dims[m] < 1) return fail(DEINSUM_ERR_SHAPE, "TTMc dims must be >= 1");
    TtmcPlan p;
    if (o.plan_hint < 0) return fail(DEINSUM_ERR_INVALID_ARG, "TTMc plan_hint must be >= 0");
    if (deinsum_status st = make_plan(spec, dims, ranks, o.precision, o.plan_hint, &p)) return st;
    const int N = p.N, n = p.n;
    const bool fx20 = o.precision == P_FX20;
    const size_t xb = o.precision == P_FP64 ? 8 : (o.precision == P_FP32 ? 4 : 2);  // FX20: the FP16 plane
    const size_t ub = o.precision == P_FP64 ? 8 : 4;  // factors: FP64, else FP32
    const size_t ob = o.out_dtype == DEINSUM_F64 ? 8 : 4;
    const void *Um[DEINSUM_MAX_ORDER] = {nullptr};
    int64_t nx = 1, ny = 1;
    for (int m = 0; m < N; ++m) {
        nx *= p.I[m];
        ny *= (m == n) ? p.I[m] : p.Rm[m];
        if (m != n) {
            Um[m] = U[spec->operand_of_mode[m]];
            if (!Um[m]) return fail(DEINSUM_ERR_INVALID_ARG, "null factor");
        }
    }
    {
        auto ov = [](const void *a0, size_t na, const void *b0, size_t nb) {
            const uintptr_t pa = reinterpret_cast<uintptr_t>(a0), pb = reinterpret_cast<uintptr_t>(b0);
            return pa < pb + nb && pb < pa + na;
        };
        if (ov(Y, ny * ob, X, fx20 ? static_cast<size_t>(fx20_bytes(nx)) : nx * xb))
            return fail(DEINSUM_ERR_INVALID_ARG, "output overlaps X");
        if (fx20 && reinterpret_cast<uintptr_t>(X) % 256 != 0)
            return fail(DEINSUM_ERR_INVALID_ARG, "an FX20 X buffer must be 256-byte aligned");
        for (int m = 0; m < N; ++m)
            if (m != n && ov(Y, ny * ob, Um[m], p.I[m] * p.Rm[m] * ub))
                return fail(DEINSUM_ERR_INVALID_ARG, "output overlaps a factor");
    }
    if (p.via_mttkrp) {
        const int64_t R = p.Rm[1];
        deinsum_spec ms = *spec;
        ms.kind = DEINSUM_MTTKRP;
        deinsum_opts o2 = o;
        o2.workspace = ws;
        o2.workspace_bytes = ws_bytes;
        o2.plan_hint = 0;
        return deinsum_mttkrp(&ms, dims, R, X, U, Y, &o2, s);
    }
    int64_t stride[DEINSUM_MAX_ORDER], ystr[DEINSUM_MAX_ORDER];
    {
        int64_t st = 1, sy = 1;
        for (int m = N - 1; m >= 0; --m) {
            stride[m] = st;
            st *= p.I[m];
            ystr[m] = sy;
            sy *= (m == n) ? p.I[m] : p.Rm[m];
        }
    }
    auto align = [](size_t x) { return (x + 255) / 256 * 256; };
    char *base = static_cast<char *>(ws);
    double *P = reinterpret_cast<double *>(base);
    double *Z = reinterpret_cast<double *>(base + align(p.p_bytes));
    double *T0 = reinterpret_cast<double *>(base + align(p.p_bytes) + align(p.z_bytes));
    double *T1 = reinterpret_cast<double *>(base + align(p.p_bytes) + align(p.z_bytes) + align(p.t_bytes));
    char *Ua_pad = base + align(p.p_bytes) + align(p.z_bytes) + 2 * align(p.t_bytes);
    char *Uc_pad = Ua_pad + align(stage1_factor_bytes(o.precision, p.I[p.a], p.nta));
    {
        auto pad = [&](int m, int ld, char *dst) {
            const int64_t n = p.I[m] * ld;
            const unsigned grid = static_cast<unsigned>(cdivl(n, 256));
            if (o.precision == P_FP64)
                pad_factor_kernel<double><<<grid, 256, 0, s>>>(static_cast<const double *>(Um[m]), p.I[m],
                                                               static_cast<int>(p.Rm[m]), ld, reinterpret_cast<double *>(dst));
            else
                pad_factor_kernel<float><<<grid, 256, 0, s>>>(static_cast<const float *>(Um[m]), p.I[m],
                                                              static_cast<int>(p.Rm[m]), ld, reinterpret_cast<float *>(dst));
        };
        if (o.precision == P_BF16) {
            const int64_t nkb = cdivl(p.I[p.a], 32), n = nkb * p.nta * 512;
            pack_factor_bf16_kernel<<<static_cast<unsigned>(cdivl(n, 256)), 256, 0, s>>>(
                static_cast<const float *>(Um[p.a]), p.I[p.a], static_cast<int>(p.Rm[p.a]), p.nta, nkb,
                reinterpret_cast<uint16_t *>(Ua_pad));
        } else if (fx20) {
            const int64_t nkb = cdivl(p.I[p.a], 32), n = nkb * p.nta * 512;
            const size_t pk = align256(static_cast<size_t>(n) * sizeof(uint16_t)), ta = 16 * p.nta;
            char *lo = Ua_pad + pk;
            double *scale = reinterpret_cast<double *>(lo + pk);
            double *off = reinterpret_cast<double *>(lo + pk + align256(ta * 8));
            int *kexp = reinterpret_cast<int *>(lo + pk + 2 * align256(ta * 8));
            fx20_factor_cols_kernel<<<static_cast<unsigned>(ta), 256, 0, s>>>(
                static_cast<const float *>(Um[p.a]), p.I[p.a], static_cast<int>(p.Rm[p.a]), p.nta, nkb, kexp, scale,
                off, reinterpret_cast<uint16_t *>(Ua_pad), reinterpret_cast<uint16_t *>(lo));
        } else {
            pad(p.a, 16 * p.nta, Ua_pad);
        }
        if (p.stage2) pad(p.c, 16 * p.ntc, Uc_pad);
        if (deinsum_status st = check_launch("ttmc_pad_factor")) return st;
    }

    // ---- fused pass
    TkArgs a{};
    a.X = fx20 ? static_cast<const void *>(static_cast<const char *>(X) + kFx20Header) : X;
    a.Ua = Ua_pad;
    if (fx20) {
        const int64_t nkb = cdivl(p.I[p.a], 32);
        const size_t pk = align256(static_cast<size_t>(nkb * p.nta * 512) * sizeof(uint16_t)), ta = 16 * p.nta;
        a.X2 = static_cast<const char *>(X) + fx20_lo_offset(nx);
        a.fx_hdr = X;
        a.Ua2 = Ua_pad + pk;
        a.ua_scale = reinterpret_cast<const double *>(Ua_pad + 2 * pk);
        a.ua_off = reinterpret_cast<const double *>(Ua_pad + 2 * pk + align256(ta * 8));
    }
    a.Uc = p.stage2 ? Uc_pad : nullptr;
    a.Ia = p.I[p.a];
    a.Ic = p.I[p.c];
    a.stride_a = stride[p.a];
    a.od.n_outer = static_cast<int>(p.slab_modes.size());
    for (size_t k = 0; k < p.slab_modes.size(); ++k) {
        a.od.dim[k] = p.I[p.slab_modes[k]];
        a.od.xstride[k] = stride[p.slab_modes[k]];
        a.od.U[k] = nullptr;
    }
    a.n_slabs = p.n_slabs;
    // Slab modes 0 .. N-3 ahead of (a, c) = (N-2, N-1): slabs are equally spaced.
    {
        bool lead = p.a == N - 2 && p.c == N - 1;
        for (size_t k = 0; k < p.slab_modes.size(); ++k) lead &= p.slab_modes[k] == static_cast<int>(k);
        a.slab_stride = lead ? p.I[p.a] * p.I[p.c] : 0;
    }
    a.slabs_per_group = p.spg;
    a.n_ctiles = p.n_ctiles;
    a.nwaves = p.nwaves;
    a.n_cgroups = p.n_cgroups;
    a.ra = static_cast<int>(p.Rm[p.a]);
    a.rc = p.stage2 ? static_cast<int>(p.Rm[p.c]) : 0;
    a.vec_ok = fx20 ? (p.I[p.c] % 4 == 0)  // planes are 256-byte aligned; rows of whole 4-element groups
                    : ((p.I[p.c] * xb) % 8 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
    a.xcd_remap = 1;
    a.n_groups = p.groups;
    a.P = P;
    const int kt = ktimer_begin(s, KK_TTMC_FUSED);
    p.kernel->fn(a, p.groups, s);
    ktimer_end(kt, s);
    if (deinsum_status st = check_launch("ttmc_fused")) return st;

    // ---- logical dims of the intermediate: slab modes, then (a, c) or (n, a)
    std::vector<DimInfo> zd;
    for (int m : p.slab_modes) zd.push_back({m, p.I[m]});
    std::vector<int> remaining;
    for (int m : p.slab_modes)
        if (m != n) remaining.push_back(m);
    const int64_t TA = 16 * p.nta, TC = 16 * p.ntc;
    ReduceArgs r{};
    r.P = P;
    r.nd = static_cast<int>(p.slab_modes.size());
    for (int k = 0; k < r.nd; ++k) r.sdim[k] = p.I[p.slab_modes[k]];
    if (p.stage2) {
        r.parts = p.n_cgroups;
        r.part_stride = p.n_slabs * p.Rm[p.a] * p.Rm[p.c];
        r.X1 = p.Rm[p.a];
        r.PX = p.Rm[p.a];  // stage-2 tiles are stored unpadded
        r.Y1 = p.Rm[p.c];
        r.PY = p.Rm[p.c];
    } else {
        r.parts = 1;
        r.part_stride = 0;
        r.X1 = p.I[p.c];
        r.PX = static_cast<int64_t>(p.n_ctiles) * 16 * p.mt;
        r.Y1 = p.Rm[p.a];
        r.PY = TA;
    }
    r.total = p.n_slabs * r.X1 * r.Y1;
    const int xmode = p.stage2 ? p.a : p.c, ymode = p.stage2 ? p.c : p.a;
    if (remaining.empty()) {
        // Straight into Y.
        for (int k = 0; k < r.nd; ++k) r.sstr[k] = ystr[p.slab_modes[k]];
        r.xstr = ystr[xmode];
        r.ystr = ystr[ymode];
        r.out = Y;
        r.out_dtype = o.out_dtype;
    } else {
        // Contiguous FP64 intermediate [slab modes..., x, y].
        int64_t st = r.X1 * r.Y1;
        for (int k = r.nd - 1; k >= 0; --k) {
            r.sstr[k] = st;
            st *= r.sdim[k];
        }
        r.xstr = r.Y1;
        r.ystr = 1;
        r.out = Z;
        r.out_dtype = DEINSUM_F64;
    }
    // ---- remaining mode products on the intermediate; with a single partial the first
    // product reads the fused pass's padded tiles directly
    std::vector<DimInfo> cur = zd;
    cur.push_back({xmode, r.X1});
    cur.push_back({ymode, r.Y1});
    std::vector<int64_t> sext;  // extents of the source layout (padded for the tiles)
    for (const auto &d : cur) sext.push_back(d.extent);
    const double *src = Z;
    if (remaining.empty() || r.parts > 1) {
        reduce_strided_kernel<<<static_cast<unsigned>(cdivl(r.total, 256)), 256, 0, s>>>(r);
        if (deinsum_status st = check_launch("ttmc_reduce")) return st;
        if (remaining.empty()) return DEINSUM_OK;
    } else {
        src = P;
        sext[sext.size() - 2] = r.PX;
        sext[sext.size() - 1] = r.PY;
    }
    for (size_t k = 0; k < remaining.size(); ++k) {
        const int m = remaining[remaining.size() - 1 - k];  // last mode first
        const bool last = (k + 1 == remaining.size());
        SmallTtmArgs t{};
        t.T = src;
        t.nd = static_cast<int>(cur.size());
        int pos = -1;
        for (int d = 0; d < t.nd; ++d)
            if (cur[d].mode == m) pos = d;
        t.m = pos;
        t.Im = p.I[m];
        int64_t st = 1;
        for (int d = t.nd - 1; d >= 0; --d) {
            t.tstr[d] = st;
            st *= sext[d];
        }
        cur[pos].extent = p.Rm[m];
        // Whole rank range per thread when its factor fits in LDS; else blocks of 8.
        int rb = ttm_rb(p.Rm[m]);
        if (static_cast<size_t>(p.I[m] * cdivl(p.Rm[m], rb) * rb) * 8 > kTtmLdsBytes) rb = kTtmRB;
        int64_t nout = 1;
        t.total = 1;
        for (int d = 0; d < t.nd; ++d) {
            t.odim[d] = cur[d].extent;
            nout *= cur[d].extent;
            t.total *= (d == pos) ? cdivl(cur[d].extent, rb) : cur[d].extent;
            sext[d] = cur[d].extent;
        }
        if (!last && static_cast<size_t>(nout) * 8 > p.t_bytes)
            return fail(DEINSUM_ERR_NO_MEMORY, "ttmc: intermediate larger than its workspace slot");
        void *dst = last ? Y : static_cast<void *>((k % 2 == 0) ? T0 : T1);
        if (last) {
            for (int d = 0; d < t.nd; ++d) t.ostr[d] = ystr[cur[d].mode];
        } else {
            int64_t so = 1;
            for (int d = t.nd - 1; d >= 0; --d) {
                t.ostr[d] = so;
                so *= cur[d].extent;
            }
        }
        t.U = Um[m];
        t.ldu = p.Rm[m];
        t.uprec = o.precision == P_FP64 ? P_FP64 : P_FP32;  // factor storage
        t.out = dst;
        t.out_dtype = last ? o.out_dtype : DEINSUM_F64;
        const size_t ubytes = static_cast<size_t>(t.Im * cdivl(p.Rm[m], rb) * rb) * 8;
        t.lds = ubytes <= kTtmLdsBytes;
        const unsigned tg = static_cast<unsigned>(cdivl(t.total, 256));
        // Few fibres (fewer than four waves' worth per SIMD of the chip): the pipelined
        // row walk, four waves per 64 fibres, factor in LDS when it fits beside the
        // waves' partial sums.  Many fibres and one block of exactly every rank: the
        // weights as scalar operands.
        const size_t red_bytes = static_cast<size_t>(3 * 64) * rb * 8;
        const bool pipe = t.total < kTtmPipeThreads && (t.lds ? ubytes : 0) + red_bytes <= kTtmPipeLdsBytes;
        auto go = [&](auto pipe_tag) {
            constexpr bool PP = decltype(pipe_tag)::value;
            if constexpr (!PP) {
                if (p.Rm[m] == rb) {
                    if (rb == 8) small_ttm_kernel<8, kTtmWUniform, false><<<tg, 256, 0, s>>>(t);
                    else if (rb == 16) small_ttm_kernel<16, kTtmWUniform, false><<<tg, 256, 0, s>>>(t);
                    else if (rb == 24) small_ttm_kernel<24, kTtmWUniform, false><<<tg, 256, 0, s>>>(t);
                    else small_ttm_kernel<32, kTtmWUniform, false><<<tg, 256, 0, s>>>(t);
                    return;
                }
            }
            const unsigned g = PP ? static_cast<unsigned>(cdivl(t.total, 64)) : tg;
            const size_t lb = (t.lds ? ubytes : 0) + (PP ? red_bytes : 0);
            if (!t.lds) small_ttm_kernel<8, kTtmWGlobal, PP><<<g, 256, lb, s>>>(t);
            else if (rb == 8) small_ttm_kernel<8, kTtmWLds, PP><<<g, 256, lb, s>>>(t);
            else if (rb == 16) small_ttm_kernel<16, kTtmWLds, PP><<<g, 256, lb, s>>>(t);
            else if (rb == 24) small_ttm_kernel<24, kTtmWLds, PP><<<g, 256, lb, s>>>(t);
            else small_ttm_kernel<32, kTtmWLds, PP><<<g, 256, lb, s>>>(t);
        };
        if (pipe) go(std::true_type{});
        else go(std::false_type{});
        if (deinsum_status st2 = check_launch("ttmc_small_ttm")) return st2;
        src = static_cast<const double *>(dst);
    }
    return DEINSUM_OK;
}

namespace {

__global__ void __launch_bounds__(256) diag_kernel(const double *Y, int64_t I, int64_t R, void *M, int out_dtype)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= I * R) return;
    const int64_t i = e / R, r = e % R;
    const double v = Y[(i * R + r) * R + r];
    if (out_dtype == DEINSUM_F64) static_cast<double *>(M)[e] = v;
    else static_cast<float *>(M)[e] = static_cast<float>(v);
}

deinsum_status m0_ttmc_setup(const int64_t *dims, int64_t R, int prec, int variant, deinsum_spec *sp,
                             deinsum_opts *o, size_t *ttmc_bytes)
{
    if (deinsum_status st = parse_spec("ijk,jb,kc->ibc", sp)) return st;
    const int64_t ranks[2] = {R, R};
    deinsum_opts_init(o);
    o->precision = prec;
    o->out_dtype = DEINSUM_F64;
    o->plan_hint = variant;
    return ttmc_workspace_size(sp, dims, ranks, *o, ttmc_bytes);
}

}  // namespace

deinsum_status mttkrp_via_ttmc_workspace(const int64_t *dims, int64_t R, int prec, int variant, size_t *bytes)
{
    deinsum_spec sp;
    deinsum_opts o;
    size_t need = 0;
    if (deinsum_status st = m0_ttmc_setup(dims, R, prec, variant, &sp, &o, &need)) return st;
    *bytes = (need + 255) / 256 * 256 + static_cast<size_t>(dims[0] * R * R) * sizeof(double);
    return DEINSUM_OK;
}

deinsum_status run_mttkrp_via_ttmc(const int64_t *dims, int64_t R, const void *X, const void *U1, const void *U2,
                                   void *M, int prec, int out_dtype, int variant, void *ws, size_t ws_bytes,
                                   hipStream_t s)
{
    deinsum_spec sp;
    deinsum_opts o;
    size_t need = 0;
    if (deinsum_status st = m0_ttmc_setup(dims, R, prec, variant, &sp, &o, &need)) return st;
    const size_t ybytes = static_cast<size_t>(dims[0] * R * R) * sizeof(double);
    const size_t yoff = (need + 255) / 256 * 256;
    if (ws_bytes < yoff + ybytes) return fail(DEINSUM_ERR_NO_MEMORY, "mttkrp via ttmc: workspace too small");
    double *Y = reinterpret_cast<double *>(static_cast<char *>(ws) + yoff);
    const int64_t ranks[2] = {R, R};
    const void *U[2] = {U1, U2};
    if (deinsum_status st = run_ttmc(&sp, dims, ranks, X, U, Y, o, ws, need, s)) return st;
    const int64_t total = dims[0] * R;
    diag_kernel<<<static_cast<unsigned>(cdivl(total, 256)), 256, 0, s>>>(Y, dims[0], R, M, out_dtype);
    return check_launch("mttkrp_via_ttmc_diag");
}

}  // namespace deinsum
