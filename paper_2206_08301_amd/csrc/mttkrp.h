// mttkrp.h -- launch interface of the MTTKRP streaming kernel (host <-> device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace deinsum {

enum StreamLayout {
    L_KCONTIG = 0,  // free mode n < N-1, matrix-core K over the contiguous mode N-1
    L_MCONTIG = 1,  // free mode n = N-1 (the contiguous one), K over mode N-2
    L_KOUT = 2,     // order 3, free mode 0: matrix-core rows over mode 1, K over mode 2;
                    // the walk takes output rows outside and mode-1 tiles inside
};

// One launch processes one column block of the output.
//   grid  = n_chunks * n_tiles * n_kgroups workgroups of `waves` waves;
//   block b -> unit u: b itself, or with xcd_remap the b-th workgroup dispatched
//     to XCD b % 8 takes the next unit of that XCD's contiguous range of units
//     (workgroups are handed to the 8 XCDs round-robin), so each XCD's L2 and
//     TLB see one region of X;
//   unit u: kgroup = u % n_kgroups, then (order 0) tile = (u / n_kgroups) % n_tiles,
//     chunk = rest, or (order 1) chunk = (u / n_kgroups) % n_chunks, tile = rest;
//   wave w: slice kgroup*wk + w % wk of mode g, outer sub-range w / wk of the chunk.
// L_KOUT (order 3, n = 0): unit u -> kgroup = u % n_kgroups, chunk = u / n_kgroups of
//   the output rows i (O = I_0 of them, o_per_chunk per chunk); a wave walks its rows
//   i and, for each, the n_tiles 16-row tiles of mode 1 (od.dim[0] = I_1 rows of
//   stride od.xstride[0]; W = U^1 in FP32 packed per tile and lane,
//   [n_tiles][64 lanes][4 tile rows][NT] (kout_weights_kernel)); each row's sum over mode 1
//   is written to P[slice][i][ldw] (n_kgroups * wk partials, no tile structure).
struct StreamArgs {
    const void *X;       // FX20: the 16-bit plane
    const void *X2;      // FX20: the 8-bit plane (unused otherwise)
    const void *Ug;      // factor of mode g, column block applied; row stride ldu
    int64_t ldu;
    OuterDesc od;        // modes other than n and g
    int64_t In, Ig;      // sizes of the free mode and of mode g
    int64_t stride_n;    // X stride of the free mode (K-contiguous layout)
    int64_t stride_g;    // X stride of mode g (M-contiguous layout)
    int ncols;           // valid columns in this block (<= 16 * NT)
    int n_tiles;         // free-mode tiles (16 or 16*MT indices)
    int order;           // unit order: 0 tile-major within a chunk, 1 chunk-major within a tile
    int xcd_remap;       // 1: contiguous unit range per XCD (needs n_groups)
    int64_t n_chunks;    // outer chunks
    int64_t n_groups;    // workgroups of this launch
    int n_kgroups;       // groups of wk slices of mode g
    int wk;              // slices per workgroup
    int64_t O, o_per_chunk;
    int vec_ok;          // X allows 16-byte aligned vector loads
    const double *W;     // outer weights [O][ldw] (outer_weights_kernel)
    int64_t ldw;         // = 16 * NT
    double *P;           // partials [n_chunks * n_kgroups][n_tiles][tile_rows][16 * NT]
};

struct StreamKernelInfo {
    int prec, layout, nt, ni, mt, nbuf;
    int xnt;  // X loads non-temporal
    void (*fn)(const StreamArgs &, int64_t grid, int waves, hipStream_t s);
};

// Every compiled kernel variant.
const StreamKernelInfo *stream_kernels(int *count);
deinsum_status launch_mttkrp_stream(const StreamKernelInfo &k, const StreamArgs &a, int64_t grid, int waves,
                                    hipStream_t s);
// L_KOUT weights: U^1's column block in FP32 as [tile][lane][v][nt] =
// U^1[16 tile + 4 (lane / 16) + v][16 nt + lane % 16] (zero past I_1 or ncols), the
// FP32 matrix-core output rows each lane holds.
deinsum_status launch_kout_weights(const void *U1, int64_t I1, int64_t ldu, int ncols, int nt, int prec, float *W,
                                   hipStream_t s);
deinsum_status launch_outer_weights(const OuterDesc &od, int64_t O, int64_t ldu, int ncols, int ldw, int prec,
                                    double *W, hipStream_t s);
// hx (FX20 only, else null): the header of X; the sums are scaled by 2^exp2, and
// a header that is not an FX20 header of nx elements turns the output into NaN.
deinsum_status launch_reduce_partials(const double *P, int64_t nparts, int64_t n_tiles, int tile_rows,
                                      int cols_pad, int64_t rows, int ncols, void *out, int out_dtype,
                                      int64_t ldo, const Fx20Header *hx, int64_t nx, hipStream_t s);

}  // namespace deinsum
