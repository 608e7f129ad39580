// mttkrp.h -- launch arguments of the MTTKRP kernels (host <-> device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace deinsum {

// K-contiguous form (free mode n < N-1); g = N-1.
struct Mk1Args {
    const void *X;
    const void *Ug;      // U^{N-1}, column block applied; row stride ldu
    int64_t ldu;
    OuterDesc od;        // modes other than n and N-1
    int64_t In, stride_n, Ig;
    int ncols;           // valid columns in this block (<= 16 * NT)
    int n_tiles;         // ceil(In / 16)
    int n_kgroups;       // ceil(Ig / (4 * KL * wk))
    int wk, wo;          // per workgroup: k-slices and outer sub-ranges (wk * wo = waves)
    int64_t O, o_per_chunk;
    int vec_ok;          // X rows allow 16-byte aligned vector loads
    double *P;           // partials [chunks * n_kgroups][n_tiles][16][16 * NT]
};

// M-contiguous form (free mode n = N-1); g = N-2.
struct Mk2Args {
    const void *X;
    const void *Ug;      // U^{N-2}, column block applied
    int64_t ldu;
    OuterDesc od;        // modes 0..N-3
    int64_t In, Ig, stride_g;
    int ncols;
    int n_tiles;         // ceil(In / (16 * MT))
    int64_t O, o_per_chunk;
    int64_t n_igchunks, ig_per_chunk;  // i_g split across workgroups
    int vec_ok;
    double *P;           // partials [ochunks * n_igchunks][n_tiles][16 * MT][16 * NT]
};

bool kcontig_available(int prec, int nt, int kl);
bool mcontig_available(int prec, int nt, int mt);
deinsum_status launch_mttkrp_kcontig(int prec, int nt, int kl, const Mk1Args &a, int64_t grid,
                                     hipStream_t s);
deinsum_status launch_mttkrp_mcontig(int prec, int nt, int mt, const Mk2Args &a, int64_t grid,
                                     hipStream_t s);
deinsum_status launch_reduce_partials(const double *P, int64_t nparts, int64_t n_tiles, int tile_rows,
                                      int cols_pad, int64_t rows, int ncols, void *out, int out_dtype,
                                      int64_t ldo, hipStream_t s);

}  // namespace deinsum
