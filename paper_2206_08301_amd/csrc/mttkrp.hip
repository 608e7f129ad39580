// mttkrp.hip -- gfx950 kernels for mode-n MTTKRP (paper Sec. III-B, Tab. IV):
//   M[i_n, r] = sum_{i_m, m != n} X[i] * prod_{m != n} U^m[i_m, r].
//
// The Khatri-Rao product is never formed in memory.  Following the fused
// schedule that Sec. IV-E shows to move the least data (partition P2: every
// partial product is consumed as soon as it is made), each wave computes
//   stage 1 (matrix cores): T[i_n, r] = sum_{i_g in slice} X[.., i_n, .., i_g] U^g[i_g, r]
//       for one slice of a contracted mode g with the other ("outer")
//       indices fixed, then immediately
//   stage 2 (Hadamard-and-reduce): acc[i_n, r] += T[i_n, r] * prod_outer U^m[i_m, r]
// so X is streamed from HBM exactly once and meets the factors in registers.
// The slice of U^g lives in registers for the wave's whole walk over the
// outer indices; X tiles are prefetched NBUF-1 steps ahead in a register ring.
// Two layouts cover every mode:
//   * K-contiguous (free mode n < N-1): g = N-1 is the contiguous mode; a
//     lane streams runs of one X row (i_n fixed) along i_g.
//   * M-contiguous (free mode n = N-1): g = N-2; the output index i_n is the
//     contiguous one, so a lane streams a run along i_n from each row i_g.
// Partial outputs are summed per workgroup through LDS in wave order and then
// across workgroups by reduce_partials in index order: deterministic results.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "kernels.h"
#include "mttkrp.h"
#include "stream.h"

namespace deinsum {

namespace {

using namespace dev;

template <int P, int L, int NT, int NI, int MT, int NBUF, bool XNT>
__global__ void __launch_bounds__(256, 2) mttkrp_stream_kernel(const StreamArgs a)
{
    __shared__ double lds[unit_lds_elems<L, NT, MT>()];
    stream_unit<P, L, NT, NI, MT, NBUF, XNT>(a, blockIdx.x, lds);
}

// Hadamard weights of the outer modes: W[o, col] = prod_outer U^m[i_m, col]
// (FP64, zero in padded columns), i.e. the Khatri-Rao product of the outer
// factors only -- O x R values, a small fraction of X for every shape here.
__global__ void __launch_bounds__(256) outer_weights_kernel(const OuterDesc od, int64_t O, int64_t ldu, int ncols,
                                                            int ldw, int prec, double *__restrict__ W)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= O * ldw) return;
    int64_t o = e / ldw;
    const int col = static_cast<int>(e % ldw);
    double w = 0.0;
    if (col < ncols) {
        w = 1.0;
        for (int m = od.n_outer - 1; m >= 0; --m) {
            const int64_t i = o % od.dim[m];
            o /= od.dim[m];
            w *= ld_u(od.U[m], i * ldu + col, prec);
        }
    }
    W[e] = w;
}

__global__ void __launch_bounds__(256) kout_weights_kernel(const void *U1, int64_t I1, int64_t ldu, int ncols,
                                                           int nt, int prec, float *__restrict__ W, int64_t total)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int ntt = static_cast<int>(e % nt);
    const int v = static_cast<int>((e / nt) % 4);
    const int lane = static_cast<int>((e / (4 * nt)) % 64);
    const int64_t tile = e / (256 * nt);
    const int64_t row = tile * 16 + 4 * (lane >> 4) + v;
    const int col = ntt * 16 + (lane & 15);
    W[e] = (row < I1 && col < ncols) ? static_cast<float>(ld_u(U1, row * ldu + col, prec)) : 0.0f;
}

// Fixed-order FP64 sum of the partial tiles into the output column block.
// P layout: [part][tile][tile_rows][cols_pad]; output row i lives in tile i / tile_rows.
template <typename OT>
__global__ void __launch_bounds__(256)
reduce_partials_kernel(const double *__restrict__ P, int64_t nparts, int64_t n_tiles, int tile_rows,
                       int cols_pad, int64_t rows, int ncols, OT *__restrict__ out, int64_t ldo,
                       const Fx20Header *__restrict__ hx, int64_t nx)
{
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= rows * ncols) return;
    const int64_t i = e / ncols;
    const int col = static_cast<int>(e % ncols);
    const int64_t t = i / tile_rows, ir = i % tile_rows;
    const int64_t tile_elems = static_cast<int64_t>(tile_rows) * cols_pad;
    const double *p = P + t * tile_elems + ir * cols_pad + col;
    const int64_t part_stride = n_tiles * tile_elems;
    // Index order; eight loads in flight per step.
    double s = 0.0;
    int64_t q = 0;
    for (; q + 8 <= nparts; q += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(q + u) * part_stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; q < nparts; ++q) s += p[q * part_stride];
    if (hx) s = (hx->magic == kFx20Magic && hx->count == nx) ? ldexp(s, hx->exp2) : __builtin_nan("");
    out[i * ldo + col] = from_f64<OT>(s);
}

template <int P, int L, int NT, int NI, int MT, int NBUF, bool XNT>
void launch_stream(const StreamArgs &a, int64_t grid, int waves, hipStream_t s)
{
    mttkrp_stream_kernel<P, L, NT, NI, MT, NBUF, XNT><<<static_cast<unsigned>(grid), 64 * waves, 0, s>>>(a);
}

}  // namespace

// ------------------------------------------------------------------------------------
// Kernel table: (precision, layout, column tiles, instructions per step, M tiles) -> launcher.
#define SK(P, L, NT, NI, MT, NB) {P, L, NT, NI, MT, NB, 0, &launch_stream<P, L, NT, NI, MT, NB, false>}
#define SKN(P, L, NT, NI, MT, NB) {P, L, NT, NI, MT, NB, 1, &launch_stream<P, L, NT, NI, MT, NB, true>}
static const StreamKernelInfo kStreamTable[] = {
    // K-contiguous: per-lane run NI*KE elements (128 bytes by default; 80-element slices for dims of 80)
    SK(P_FP64, L_KCONTIG, 1, 16, 1, 3), SK(P_FP64, L_KCONTIG, 2, 16, 1, 3), SK(P_FP64, L_KCONTIG, 4, 8, 1, 2),
    SK(P_FP64, L_KCONTIG, 1, 20, 1, 3), SK(P_FP64, L_KCONTIG, 2, 20, 1, 2), SK(P_FP64, L_KCONTIG, 4, 10, 1, 2),
    SK(P_FP64, L_KCONTIG, 1, 8, 1, 3),  SK(P_FP64, L_KCONTIG, 2, 8, 1, 3),
    SK(P_FP32, L_KCONTIG, 1, 32, 1, 3), SK(P_FP32, L_KCONTIG, 2, 32, 1, 3), SK(P_FP32, L_KCONTIG, 4, 16, 1, 2),
    SK(P_FP32, L_KCONTIG, 1, 20, 1, 3), SK(P_FP32, L_KCONTIG, 2, 20, 1, 3), SK(P_FP32, L_KCONTIG, 4, 20, 1, 2),
    SK(P_FP32, L_KCONTIG, 1, 8, 1, 3),  SK(P_FP32, L_KCONTIG, 2, 8, 1, 3),
    SK(P_BF16, L_KCONTIG, 1, 8, 1, 2),  SK(P_BF16, L_KCONTIG, 2, 8, 1, 2),  SK(P_BF16, L_KCONTIG, 4, 4, 1, 2),
    SK(P_BF16, L_KCONTIG, 1, 3, 1, 3),  SK(P_BF16, L_KCONTIG, 2, 3, 1, 3),  SK(P_BF16, L_KCONTIG, 4, 3, 1, 2),
    SK(P_BF16, L_KCONTIG, 1, 1, 1, 3),  SK(P_BF16, L_KCONTIG, 2, 1, 1, 3),
    SK(P_BF16X3, L_KCONTIG, 1, 4, 1, 3), SK(P_BF16X3, L_KCONTIG, 2, 4, 1, 2), SK(P_BF16X3, L_KCONTIG, 4, 2, 1, 2),
    SK(P_BF16X3, L_KCONTIG, 1, 3, 1, 3), SK(P_BF16X3, L_KCONTIG, 2, 3, 1, 2), SK(P_BF16X3, L_KCONTIG, 4, 3, 1, 2),
    SK(P_BF16X3, L_KCONTIG, 1, 1, 1, 3), SK(P_BF16X3, L_KCONTIG, 2, 1, 1, 3), SK(P_BF16X3, L_KCONTIG, 2, 2, 1, 4),
    // FX20: FP16 matrix cores; runs of 16 elements per chunk (32 bytes of the FP16 plane, 16 of the int8 plane)
    SK(P_FX20, L_KCONTIG, 1, 4, 1, 3), SK(P_FX20, L_KCONTIG, 2, 4, 1, 3), SK(P_FX20, L_KCONTIG, 4, 2, 1, 2),
    SK(P_FX20, L_KCONTIG, 1, 2, 1, 3), SK(P_FX20, L_KCONTIG, 2, 2, 1, 3),
    // Order-3 mode 0, mode-1 tiles walked per output row (the K-contiguous tile and loads)
    SK(P_FP32, L_KOUT, 1, 32, 1, 3), SK(P_FP32, L_KOUT, 2, 32, 1, 3),
    SK(P_BF16, L_KOUT, 1, 8, 1, 2), SK(P_BF16, L_KOUT, 2, 8, 1, 2), SK(P_BF16, L_KOUT, 4, 4, 1, 2),
    SK(P_BF16X3, L_KOUT, 1, 4, 1, 3), SK(P_BF16X3, L_KOUT, 2, 4, 1, 3),
    SK(P_FX20, L_KOUT, 1, 4, 1, 3), SK(P_FX20, L_KOUT, 2, 4, 1, 3),
    // M-contiguous: NI K-steps of 4*KE rows; MT output indices per lane
    // (FP64: non-temporal X loads first -- they keep the per-K-step factor rows cached, 1.50 -> 1.37 ms
    //  for the 1024^3 R=24 last mode; the K-contiguous kernels lose with them and keep plain loads.)
    SKN(P_FP64, L_MCONTIG, 1, 8, 2, 3), SKN(P_FP64, L_MCONTIG, 2, 8, 2, 2), SKN(P_FP64, L_MCONTIG, 4, 8, 1, 2),
    SK(P_FP64, L_MCONTIG, 1, 8, 2, 3), SK(P_FP64, L_MCONTIG, 2, 8, 2, 2), SK(P_FP64, L_MCONTIG, 4, 8, 1, 2),
    SK(P_FP32, L_MCONTIG, 1, 8, 4, 3), SK(P_FP32, L_MCONTIG, 2, 8, 2, 3), SK(P_FP32, L_MCONTIG, 4, 8, 2, 2),
    SKN(P_FP32, L_MCONTIG, 1, 8, 4, 3), SKN(P_FP32, L_MCONTIG, 2, 8, 2, 3), SKN(P_FP32, L_MCONTIG, 4, 8, 2, 2),
    // 64-index tiles: a contiguous mode of at most 64 is one tile, so no row of X is split
    // between workgroups (60^5 last mode: 480-byte rows)
    SKN(P_FP64, L_MCONTIG, 2, 4, 4, 3), SK(P_FP64, L_MCONTIG, 2, 4, 4, 3), SKN(P_FP64, L_MCONTIG, 2, 2, 4, 3),
    SKN(P_FP32, L_MCONTIG, 2, 4, 4, 3), SK(P_FP32, L_MCONTIG, 2, 4, 4, 3),
    SK(P_BF16, L_MCONTIG, 1, 2, 4, 2), SK(P_BF16, L_MCONTIG, 2, 2, 2, 2), SK(P_BF16, L_MCONTIG, 4, 2, 1, 2),
    SK(P_BF16X3, L_MCONTIG, 1, 2, 2, 3), SK(P_BF16X3, L_MCONTIG, 2, 2, 2, 2), SK(P_BF16X3, L_MCONTIG, 4, 2, 1, 2),
    SKN(P_BF16X3, L_MCONTIG, 1, 2, 2, 3), SKN(P_BF16X3, L_MCONTIG, 2, 2, 2, 2), SKN(P_BF16X3, L_MCONTIG, 4, 2, 1, 2),
    SK(P_BF16X3, L_MCONTIG, 2, 1, 4, 2), SKN(P_BF16X3, L_MCONTIG, 2, 1, 4, 2),
    // FX20: 8 slice rows per instruction, MT output indices per lane (2*MT bytes of the FP16 plane and
    // MT of the int8 plane per row)
    SK(P_FX20, L_MCONTIG, 2, 1, 4, 2), SKN(P_FX20, L_MCONTIG, 2, 1, 4, 2), SK(P_FX20, L_MCONTIG, 2, 1, 2, 3),
    SKN(P_FX20, L_MCONTIG, 2, 1, 2, 3), SK(P_FX20, L_MCONTIG, 2, 2, 2, 2), SK(P_FX20, L_MCONTIG, 1, 1, 4, 3),
    SK(P_FX20, L_MCONTIG, 1, 2, 2, 3), SKN(P_FX20, L_MCONTIG, 1, 2, 2, 3), SK(P_FX20, L_MCONTIG, 4, 1, 1, 2),
};
#undef SK
#undef SKN

const StreamKernelInfo *stream_kernels(int *count)
{
    *count = static_cast<int>(sizeof(kStreamTable) / sizeof(kStreamTable[0]));
    return kStreamTable;
}

deinsum_status launch_mttkrp_stream(const StreamKernelInfo &k, const StreamArgs &a, int64_t grid, int waves,
                                    hipStream_t s)
{
    k.fn(a, grid, waves, s);
    return check_launch("mttkrp_stream");
}

deinsum_status launch_outer_weights(const OuterDesc &od, int64_t O, int64_t ldu, int ncols, int ldw, int prec,
                                    double *W, hipStream_t s)
{
    const int64_t total = O * ldw;
    outer_weights_kernel<<<static_cast<unsigned>((total + 255) / 256), 256, 0, s>>>(od, O, ldu, ncols, ldw, prec, W);
    return check_launch("outer_weights");
}

deinsum_status launch_kout_weights(const void *U1, int64_t I1, int64_t ldu, int ncols, int nt, int prec, float *W,
                                   hipStream_t s)
{
    const int64_t total = (I1 + 15) / 16 * 256 * nt;
    kout_weights_kernel<<<static_cast<unsigned>((total + 255) / 256), 256, 0, s>>>(U1, I1, ldu, ncols, nt, prec, W, total);
    return check_launch("kout_weights");
}

deinsum_status launch_reduce_partials(const double *P, int64_t nparts, int64_t n_tiles, int tile_rows,
                                      int cols_pad, int64_t rows, int ncols, void *out, int out_dtype,
                                      int64_t ldo, const Fx20Header *hx, int64_t nx, hipStream_t s)
{
    const int64_t total = rows * ncols;
    const unsigned grid = static_cast<unsigned>((total + 255) / 256);
    if (out_dtype == DEINSUM_F64)
        reduce_partials_kernel<double><<<grid, 256, 0, s>>>(P, nparts, n_tiles, tile_rows, cols_pad, rows,
                                                            ncols, static_cast<double *>(out), ldo, hx, nx);
    else if (out_dtype == DEINSUM_F32)
        reduce_partials_kernel<float><<<grid, 256, 0, s>>>(P, nparts, n_tiles, tile_rows, cols_pad, rows,
                                                           ncols, static_cast<float *>(out), ldo, hx, nx);
    else
        return fail(DEINSUM_ERR_INVALID_ARG, "output dtype must be f64 or f32");
    return check_launch("reduce_partials");
}

}  // namespace deinsum
