// mttkrp.hip -- gfx950 kernels for mode-n MTTKRP (paper Sec. III-B, Tab. IV):
//   M[i_n, r] = sum_{i_m, m != n} X[i] * prod_{m != n} U^m[i_m, r].
//
// The Khatri-Rao product is never formed in memory.  Following the fused
// schedule that Sec. IV-D shows to move the least data (partition P2: every
// partial product is consumed as soon as it is made), each wave computes
//   stage 1 (matrix cores): T[i_n, r] = sum_{i_g} X[.., i_n, .., i_g] U^g[i_g, r]
//       over a slice of one contracted mode g, with the other ("outer") indices
//       fixed, and immediately
//   stage 2 (Hadamard-and-reduce): acc[i_n, r] += T[i_n, r] * prod_outer U^m[i_m, r]
// so X is streamed from HBM exactly once and each element meets the factor
// entries in registers.  Two layouts cover every mode:
//   * K-contiguous (free mode n < N-1): g = N-1 is the contiguous mode.  Each
//     lane streams a contiguous run of one X row (i_n fixed) along i_g; the
//     U^g slice lives in registers for the whole walk over the outer indices.
//   * M-contiguous (free mode n = N-1): g = N-2.  The output index i_n is the
//     contiguous one, so each lane streams a contiguous run along i_n; rows
//     i_g are walked four at a time and U^g rows are read per step.
// Partial outputs of the workgroups are summed in a fixed order by
// reduce_partials, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

#include "kernels.h"
#include "mttkrp.h"

namespace deinsum {

namespace {

template <int P> struct PrecTypes;
template <> struct PrecTypes<P_FP64> { using XT = double; using UT = double; using DT = f64x4; static constexpr int KE = 1; };
template <> struct PrecTypes<P_FP32> { using XT = float;  using UT = float;  using DT = f32x4; static constexpr int KE = 1; };
template <> struct PrecTypes<P_BF16> { using XT = bf16_t; using UT = float;  using DT = f32x4; static constexpr int KE = 8; };
template <> struct PrecTypes<P_BF16X3> { using XT = float; using UT = float; using DT = f32x4; static constexpr int KE = 8; };

__device__ __forceinline__ double ld_u(const void *p, int64_t i, int prec)
{
    return prec == P_FP64 ? static_cast<const double *>(p)[i]
                          : static_cast<double>(static_cast<const float *>(p)[i]);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t imax64(int64_t a, int64_t b) { return a > b ? a : b; }

// Contiguous load of KL elements (16-byte non-temporal vector loads when `vec`
// and the run is whole 16-byte words), zero where masked.
template <typename T, int KL>
__device__ __forceinline__ void load_run(T (&dst)[KL], const T *__restrict__ src, bool vec, int valid)
{
    if constexpr ((KL * sizeof(T)) % 16 == 0) {
        if (vec && valid >= KL) {
            constexpr int NV = KL * sizeof(T) / 16;
            const u32x4 *s = reinterpret_cast<const u32x4 *>(src);
            u32x4 tmp[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) tmp[i] = __builtin_nontemporal_load(s + i);
            __builtin_memcpy(dst, tmp, sizeof(dst));
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < KL; ++i) dst[i] = (i < valid) ? src[i] : T{};
}

// Outer-index walk: decomposes a linear outer index into per-mode indices and
// yields the X offset and the Hadamard weight of the current column.
struct OuterWalk {
    int64_t idx[kMaxOuter];
    int64_t off;
    __device__ void init(const OuterDesc &od, int64_t o)
    {
        off = 0;
        for (int m = od.n_outer - 1; m >= 0; --m) {
            idx[m] = o % od.dim[m];
            o /= od.dim[m];
            off += idx[m] * od.xstride[m];
        }
    }
    __device__ void next(const OuterDesc &od)
    {
        for (int m = od.n_outer - 1; m >= 0; --m) {
            off += od.xstride[m];
            if (++idx[m] < od.dim[m]) return;
            off -= idx[m] * od.xstride[m];
            idx[m] = 0;
        }
    }
    __device__ double weight(const OuterDesc &od, int64_t ldu, int col, int prec) const
    {
        double w = 1.0;
        for (int m = 0; m < od.n_outer; ++m) w *= ld_u(od.U[m], idx[m] * ldu + col, prec);
        return w;
    }
};

// Workgroup reduction of per-wave FP64 tiles through LDS, in wave order.
template <int ELEMS, int WAVES>
__device__ __forceinline__ void wg_reduce_store(double *lds, const double (&vals)[ELEMS],
                                                const int (&pos)[ELEMS], double *__restrict__ out,
                                                int tile_elems)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < ELEMS; ++e) lds[w * tile_elems + pos[e]] = vals[e];
    __syncthreads();
    for (int i = threadIdx.x; i < tile_elems; i += 64 * WAVES) {
        double s = lds[i];
        for (int ww = 1; ww < WAVES; ++ww) s += lds[ww * tile_elems + i];
        out[i] = s;
    }
    (void)lane;
}

// ------------------------------------------------------------------------------------
// K-contiguous kernel (free mode n < N-1).
// Block b: kgroup = b % n_kgroups, tile = (b / n_kgroups) % n_tiles, chunk = rest.
// Wave w: k-slice kgroup*WK + w % WK, outer sub-range w / WK of the chunk.
template <int P, int NT, int KL, int WAVES>
__global__ void __launch_bounds__(64 * WAVES)
mttkrp_kcontig_kernel(const Mk1Args a)
{
    using PT = PrecTypes<P>;
    using XT = typename PT::XT;
    using DT = typename PT::DT;
    constexpr int KE = PT::KE;
    constexpr int NI = KL / KE;  // matrix-core instructions per column tile per step
    static_assert(KL % KE == 0, "slice per lane must be whole instructions");
    __shared__ double lds[WAVES * 16 * NT * 16];

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t b = blockIdx.x;
    const int kgroup = static_cast<int>(b % a.n_kgroups);
    const int tile = static_cast<int>((b / a.n_kgroups) % a.n_tiles);
    const int64_t chunk = b / (static_cast<int64_t>(a.n_kgroups) * a.n_tiles);
    const int ks = kgroup * a.wk + (w % a.wk);
    const int osub = w / a.wk;
    const int64_t kbase = static_cast<int64_t>(ks) * (4 * KL) + g * KL;
    // k-run of this lane: the U^g slice (B operand) depends on k only; the X run
    // (A operand, row tile*16 + c) is also masked by the row.
    const int kvalid_u = static_cast<int>(imin64(KL, imax64(0, a.Ig - kbase)));
    const int64_t row = static_cast<int64_t>(tile) * 16 + c;
    const int kvalid = (row < a.In) ? kvalid_u : 0;

    // Outer range of this wave.
    const int64_t c0 = chunk * a.o_per_chunk;
    const int64_t c1 = imin64(a.O, c0 + a.o_per_chunk);
    const int64_t per = (c1 - c0 + a.wo - 1) / a.wo;
    const int64_t o0 = imin64(c1, c0 + osub * per);
    const int64_t o1 = imin64(c1, o0 + per);

    // Register-resident U^g slice: slot (g, e) of instruction q holds k = kbase + q*KE + e.
    // FP64/FP32: one value per (q, column tile); BF16: 8 packed; BF16X3: hi and lo parts.
    double fr64[(P == P_FP64) ? NI * NT : 1];
    float fr32[(P == P_FP32) ? NI * NT : 1];
    u16x8 frh[(P >= P_BF16) ? NI * NT : 1];
    u16x8 frl[(P == P_BF16X3) ? NI * NT : 1];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int col = nt * 16 + c;
            if constexpr (P == P_FP64 || P == P_FP32) {
                const int64_t k = kbase + q;
                double v = (q < kvalid_u && col < a.ncols) ? ld_u(a.Ug, k * a.ldu + col, P) : 0.0;
                if constexpr (P == P_FP64) fr64[q * NT + nt] = v;
                else fr32[q * NT + nt] = static_cast<float>(v);
            } else {
                u16x8 hi, lo;
#pragma unroll
                for (int e = 0; e < KE; ++e) {
                    const int64_t k = kbase + q * KE + e;
                    float v = (q * KE + e < kvalid_u && col < a.ncols)
                                  ? static_cast<const float *>(a.Ug)[k * a.ldu + col] : 0.0f;
                    const uint16_t h = f32_to_bf16_bits(v);
                    hi[e] = h;
                    lo[e] = f32_to_bf16_bits(v - bf16_bits_to_f32(h));
                }
                frh[q * NT + nt] = hi;
                if constexpr (P == P_BF16X3) frl[q * NT + nt] = lo;
            }
        }
    }

    double acc[NT][4];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[nt][v] = 0.0;

    const XT *__restrict__ X = static_cast<const XT *>(a.X);
    const int64_t lane_off = row * a.stride_n + kbase;
    const bool vec = a.vec_ok != 0;

    auto step = [&](const XT (&xv)[KL], const double (&wv)[NT]) {
        DT d[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) d[nt] = DT{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < NI; ++q) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                if constexpr (P == P_FP64) {
                    d[nt] = mfma_f64(xv[q], fr64[q * NT + nt], d[nt]);
                } else if constexpr (P == P_FP32) {
                    d[nt] = mfma_f32(xv[q], fr32[q * NT + nt], d[nt]);
                } else if constexpr (P == P_BF16) {
                    u16x8 xa;
#pragma unroll
                    for (int e = 0; e < 8; ++e) xa[e] = xv[q * 8 + e].u;
                    d[nt] = mfma_bf16(xa, frh[q * NT + nt], d[nt]);
                } else {
                    u16x8 xh, xl;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const float x = xv[q * 8 + e];
                        const uint16_t h = f32_to_bf16_bits(x);
                        xh[e] = h;
                        xl[e] = f32_to_bf16_bits(x - bf16_bits_to_f32(h));
                    }
                    d[nt] = mfma_bf16(xh, frh[q * NT + nt], d[nt]);
                    d[nt] = mfma_bf16(xh, frl[q * NT + nt], d[nt]);
                    d[nt] = mfma_bf16(xl, frh[q * NT + nt], d[nt]);
                }
            }
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[nt][v] += static_cast<double>(d[nt][v]) * wv[nt];
    };

    if (o0 < o1) {
        OuterWalk walk;
        walk.init(a.od, o0);
        XT xa[KL], xb[KL];
        double wa[NT], wb[NT];
        load_run<XT, KL>(xa, X + walk.off + lane_off, vec, kvalid);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) wa[nt] = (nt * 16 + c < a.ncols) ? walk.weight(a.od, a.ldu, nt * 16 + c, P) : 0.0;
        for (int64_t o = o0; o < o1; o += 2) {
            const bool has_b = o + 1 < o1;
            if (has_b) {
                walk.next(a.od);
                load_run<XT, KL>(xb, X + walk.off + lane_off, vec, kvalid);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) wb[nt] = (nt * 16 + c < a.ncols) ? walk.weight(a.od, a.ldu, nt * 16 + c, P) : 0.0;
            }
            step(xa, wa);
            if (!has_b) break;
            if (o + 2 < o1) {
                walk.next(a.od);
                load_run<XT, KL>(xa, X + walk.off + lane_off, vec, kvalid);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) wa[nt] = (nt * 16 + c < a.ncols) ? walk.weight(a.od, a.ldu, nt * 16 + c, P) : 0.0;
            }
            step(xb, wb);
        }
    }

    // Workgroup reduction over its waves, then one partial tile per block.
    double vals[NT * 4];
    int pos[NT * 4];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            vals[nt * 4 + v] = acc[nt][v];
            pos[nt * 4 + v] = tile_row<P>(lane, v) * (NT * 16) + nt * 16 + c;
        }
    const int64_t part = chunk * a.n_kgroups + kgroup;
    double *out = a.P + (part * a.n_tiles + tile) * (16 * NT * 16);
    wg_reduce_store<NT * 4, WAVES>(lds, vals, pos, out, 16 * NT * 16);
}

// ------------------------------------------------------------------------------------
// M-contiguous kernel (free mode n = N-1): M[i_n, r] = sum_rows X[row, i_n] W[row, r].
// Block b: tile = b % n_tiles (16*MT output indices), chunk = b / n_tiles.
// Wave w: i_g slice w of the WAVES slices.  Lane (g, c): i_n = tile0 + MT*c + mt.
template <int P, int NT, int MT, int WAVES>
__global__ void __launch_bounds__(64 * WAVES)
mttkrp_mcontig_kernel(const Mk2Args a)
{
    using PT = PrecTypes<P>;
    using XT = typename PT::XT;
    using DT = typename PT::DT;
    static_assert(P == P_FP64 || P == P_FP32, "M-contiguous form: FP64 and FP32 products");
    constexpr int UB = 4;  // K-steps loaded ahead
    __shared__ double lds[WAVES * 16 * MT * NT * 16];

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t b = blockIdx.x;
    const int tile = static_cast<int>(b % a.n_tiles);
    const int64_t chunk = b / a.n_tiles;  // = ochunk * n_igchunks + igchunk
    const int64_t igc = chunk % a.n_igchunks, oc = chunk / a.n_igchunks;
    const int64_t ibase = static_cast<int64_t>(tile) * 16 * MT + MT * c;
    const int ivalid = static_cast<int>(imin64(MT, imax64(0, a.In - ibase)));
    // i_g range of the workgroup, split into WAVES slices of whole K-steps.
    const int64_t wg0 = igc * a.ig_per_chunk;
    const int64_t wg1 = imin64(a.Ig, wg0 + a.ig_per_chunk);
    const int64_t slice = ((wg1 - wg0 + WAVES - 1) / WAVES + 3) / 4 * 4;
    const int64_t g0 = imin64(wg1, wg0 + w * slice);
    const int64_t g1 = imin64(wg1, g0 + slice);
    const int64_t c0 = oc * a.o_per_chunk;
    const int64_t c1 = imin64(a.O, c0 + a.o_per_chunk);

    const XT *__restrict__ X = static_cast<const XT *>(a.X);
    const bool vec = a.vec_ok != 0;

    DT d[MT][NT];
    double acc[MT][NT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            d[mt][nt] = DT{0, 0, 0, 0};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[mt][nt][v] = 0.0;
        }

    if (g0 < g1 && c0 < c1) {
        OuterWalk walk;
        walk.init(a.od, c0);
        for (int64_t o = c0; o < c1; ++o) {
            double wo[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                wo[nt] = (nt * 16 + c < a.ncols) ? walk.weight(a.od, a.ldu, nt * 16 + c, P) : 0.0;
            const XT *xo = X + walk.off + ibase;
            const int64_t nsteps = (g1 - g0 + 3) / 4;
            // Blocks of UB K-steps, the next block's loads issued before this block's products.
            XT xbuf[2][UB][MT];
            double ubuf[2][UB][NT];
            auto load_block = [&](int s, int64_t st0) {
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int64_t r = g0 + (st0 + u) * 4 + g;
                    const bool rv = (st0 + u) < nsteps && r < g1;
                    load_run<XT, MT>(xbuf[s][u], xo + r * a.stride_g, vec, rv ? ivalid : 0);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const int col = nt * 16 + c;
                        ubuf[s][u][nt] = (rv && col < a.ncols) ? ld_u(a.Ug, r * a.ldu + col, P) : 0.0;
                    }
                }
            };
            auto mac_block = [&](int s) {
#pragma unroll
                for (int u = 0; u < UB; ++u)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
                            if constexpr (P == P_FP64)
                                d[mt][nt] = mfma_f64(xbuf[s][u][mt], ubuf[s][u][nt] * wo[nt], d[mt][nt]);
                            else
                                d[mt][nt] = mfma_f32(xbuf[s][u][mt], static_cast<float>(ubuf[s][u][nt]), d[mt][nt]);
                        }
            };
            load_block(0, 0);
            for (int64_t st = 0; st < nsteps; st += 2 * UB) {
                if (st + UB < nsteps) load_block(1, st + UB);
                mac_block(0);
                if (st + UB >= nsteps) break;
                if (st + 2 * UB < nsteps) load_block(0, st + 2 * UB);
                mac_block(1);
            }
            if constexpr (P != P_FP64) {
                // Close the FP32 chain for this outer index: FP64 Hadamard accumulation.
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[mt][nt][v] += static_cast<double>(d[mt][nt][v]) * wo[nt];
                        d[mt][nt] = DT{0, 0, 0, 0};
                    }
            }
            walk.next(a.od);
        }
    }
    if constexpr (P == P_FP64) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[mt][nt][v] = d[mt][nt][v];
    }

    double vals[MT * NT * 4];
    int pos[MT * NT * 4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e = (mt * NT + nt) * 4 + v;
                vals[e] = acc[mt][nt][v];
                pos[e] = (MT * tile_row<P>(lane, v) + mt) * (NT * 16) + nt * 16 + c;
            }
    double *out = a.P + (chunk * a.n_tiles + tile) * (16 * MT * NT * 16);
    wg_reduce_store<MT * NT * 4, WAVES>(lds, vals, pos, out, 16 * MT * NT * 16);
}

// ------------------------------------------------------------------------------------
// Fixed-order FP64 sum of the partial tiles into the output column block.
// P layout: [part][tile][tile_rows][cols]; output row i lives in tile i / tile_rows.
template <typename OT>
__global__ void __launch_bounds__(256)
reduce_partials_kernel(const double *__restrict__ P, int64_t nparts, int64_t n_tiles, int tile_rows,
                       int cols_pad, int64_t rows, int ncols, OT *__restrict__ out, int64_t ldo)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= rows * ncols) return;
    const int64_t i = e / ncols;
    const int col = static_cast<int>(e % ncols);
    const int64_t t = i / tile_rows, ir = i % tile_rows;
    const int64_t tile_elems = static_cast<int64_t>(tile_rows) * cols_pad;
    const double *p = P + t * tile_elems + ir * cols_pad + col;
    const int64_t part_stride = n_tiles * tile_elems;
    double s = 0.0;
    for (int64_t q = 0; q < nparts; ++q) s += p[q * part_stride];
    out[i * ldo + col] = from_f64<OT>(s);
}

template <int P, int NT, int KL, int WAVES>
void launch_k(const Mk1Args &a, int64_t grid, hipStream_t s)
{
    mttkrp_kcontig_kernel<P, NT, KL, WAVES><<<static_cast<unsigned>(grid), 64 * WAVES, 0, s>>>(a);
}
template <int P, int NT, int MT, int WAVES>
void launch_m(const Mk2Args &a, int64_t grid, hipStream_t s)
{
    mttkrp_mcontig_kernel<P, NT, MT, WAVES><<<static_cast<unsigned>(grid), 64 * WAVES, 0, s>>>(a);
}

}  // namespace

// ------------------------------------------------------------------------------------
// Kernel tables: (precision, column tiles, per-lane run) -> launcher.
using KLaunch = void (*)(const Mk1Args &, int64_t, hipStream_t);
using MLaunch = void (*)(const Mk2Args &, int64_t, hipStream_t);

#define K_ENTRY(P, NT, KL) {P, NT, KL, &launch_k<P, NT, KL, 4>}
static const struct { int p, nt, kl; KLaunch fn; } kKTable[] = {
    K_ENTRY(P_FP64, 1, 16), K_ENTRY(P_FP64, 2, 16), K_ENTRY(P_FP64, 4, 8),
    K_ENTRY(P_FP64, 1, 20), K_ENTRY(P_FP64, 2, 20), K_ENTRY(P_FP64, 4, 20),
    K_ENTRY(P_FP64, 1, 8),  K_ENTRY(P_FP64, 2, 8),
    K_ENTRY(P_FP32, 1, 32), K_ENTRY(P_FP32, 2, 32), K_ENTRY(P_FP32, 4, 16),
    K_ENTRY(P_FP32, 1, 20), K_ENTRY(P_FP32, 2, 20), K_ENTRY(P_FP32, 4, 20),
    K_ENTRY(P_FP32, 1, 8),  K_ENTRY(P_FP32, 2, 8),
    K_ENTRY(P_BF16, 1, 64), K_ENTRY(P_BF16, 2, 64), K_ENTRY(P_BF16, 4, 32),
    K_ENTRY(P_BF16, 1, 24), K_ENTRY(P_BF16, 2, 24), K_ENTRY(P_BF16, 4, 24),
    K_ENTRY(P_BF16, 1, 8),  K_ENTRY(P_BF16, 2, 8),
    K_ENTRY(P_BF16X3, 1, 32), K_ENTRY(P_BF16X3, 2, 32), K_ENTRY(P_BF16X3, 4, 16),
    K_ENTRY(P_BF16X3, 1, 24), K_ENTRY(P_BF16X3, 2, 24), K_ENTRY(P_BF16X3, 4, 24),
    K_ENTRY(P_BF16X3, 1, 8),  K_ENTRY(P_BF16X3, 2, 8),
};
#undef K_ENTRY

#define M_ENTRY(P, NT, MT) {P, NT, MT, &launch_m<P, NT, MT, 4>}
static const struct { int p, nt, mt; MLaunch fn; } kMTable[] = {
    M_ENTRY(P_FP64, 1, 4), M_ENTRY(P_FP64, 2, 4), M_ENTRY(P_FP64, 4, 2),
    M_ENTRY(P_FP64, 1, 2), M_ENTRY(P_FP64, 2, 2),
    M_ENTRY(P_FP32, 1, 4), M_ENTRY(P_FP32, 2, 4), M_ENTRY(P_FP32, 4, 4),
};
#undef M_ENTRY

bool kcontig_available(int prec, int nt, int kl)
{
    for (const auto &e : kKTable)
        if (e.p == prec && e.nt == nt && e.kl == kl) return true;
    return false;
}
bool mcontig_available(int prec, int nt, int mt)
{
    for (const auto &e : kMTable)
        if (e.p == prec && e.nt == nt && e.mt == mt) return true;
    return false;
}

deinsum_status launch_mttkrp_kcontig(int prec, int nt, int kl, const Mk1Args &a, int64_t grid,
                                     hipStream_t s)
{
    for (const auto &e : kKTable)
        if (e.p == prec && e.nt == nt && e.kl == kl) {
            e.fn(a, grid, s);
            return check_launch("mttkrp_kcontig");
        }
    return fail(DEINSUM_ERR_UNSUPPORTED, "no K-contiguous kernel for this precision/tile");
}

deinsum_status launch_mttkrp_mcontig(int prec, int nt, int mt, const Mk2Args &a, int64_t grid,
                                     hipStream_t s)
{
    for (const auto &e : kMTable)
        if (e.p == prec && e.nt == nt && e.mt == mt) {
            e.fn(a, grid, s);
            return check_launch("mttkrp_mcontig");
        }
    return fail(DEINSUM_ERR_UNSUPPORTED, "no M-contiguous kernel for this precision/tile");
}

deinsum_status launch_reduce_partials(const double *P, int64_t nparts, int64_t n_tiles, int tile_rows,
                                      int cols_pad, int64_t rows, int ncols, void *out, int out_dtype,
                                      int64_t ldo, hipStream_t s)
{
    const int64_t total = rows * ncols;
    const unsigned grid = static_cast<unsigned>((total + 255) / 256);
    if (out_dtype == DEINSUM_F64)
        reduce_partials_kernel<double><<<grid, 256, 0, s>>>(P, nparts, n_tiles, tile_rows, cols_pad, rows,
                                                            ncols, static_cast<double *>(out), ldo);
    else if (out_dtype == DEINSUM_F32)
        reduce_partials_kernel<float><<<grid, 256, 0, s>>>(P, nparts, n_tiles, tile_rows, cols_pad, rows,
                                                           ncols, static_cast<float *>(out), ldo);
    else
        return fail(DEINSUM_ERR_INVALID_ARG, "output dtype must be f64 or f32");
    return check_launch("reduce_partials");
}

}  // namespace deinsum
