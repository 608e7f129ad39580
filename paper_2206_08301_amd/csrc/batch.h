// batch.h -- descriptors of the persistent batched MTTKRP launch (host <-> device).
#pragma once

#include <cstdint>

#include "mttkrp.h"

namespace deinsum {

// One column block of one MTTKRP job, as the device sees it.
struct BatchJob {
    StreamArgs a;            // geometry of the streaming units (P, W point into the batch arena)
    int32_t variant;         // index into the persistent kernel's variant list
    int32_t prec;            // factor dtype for the weights (P_FP64: f64, else f32)
    int64_t unit_begin;      // first queue unit of this job
    int64_t n_units;
    int64_t w_begin;         // first weight-table entry (global numbering)
    int64_t ldu;             // factor row stride (= R)
    int64_t out_begin;       // first output element (global numbering), rows * ncols elements
    int64_t rows;            // I_n
    int64_t parts, n_tiles;
    int32_t tile_rows, cols_pad;
    void *out;               // output column block (row stride ldo)
    int64_t ldo;
    int32_t out_dtype;
    int32_t pad_;
};

struct BatchHeader {
    int32_t njobs;
    int32_t pad_;
    int64_t total_units, total_w, total_out;
};

// Variants compiled into the persistent kernel (slices of 32 along mode g,
// two-deep prefetch: sized for the small and uneven tensors of batched work).
struct BatchVariant {
    int prec, layout, nt, ni, mt;
};
const BatchVariant *batch_variants(int *count);

}  // namespace deinsum
