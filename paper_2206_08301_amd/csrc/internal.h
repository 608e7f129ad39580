// internal.h -- shared host-side declarations of the library (not installed).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "deinsum.h"

namespace deinsum {

// Thread-local error message plumbing (deinsum_last_error).
void set_error(const std::string &msg);
void clear_error();
deinsum_status fail(deinsum_status st, const std::string &msg);

// The library's grow-only device workspace of the current device for `stream` (a
// hipStream_t; abi.cpp): work on one stream reuses its buffer in stream order, work
// on different streams gets different buffers.
deinsum_status pool_get(size_t bytes, void *stream, void **out);

// Argument checks shared by the entry points (abi.cpp): a spec as deinsum_parse
// writes it (order, free mode, one factor operand per other mode) and dims >= 0
// with a representable element count; whether two byte ranges overlap.
deinsum_status check_dims(const deinsum_spec *spec, const int64_t *dims);
bool overlaps(const void *a, size_t na, const void *b, size_t nb);

// Normwise relative storage error ||X - X_stored|| / ||X|| recorded in the header of
// an FX20 buffer of `count` elements (fx20.hip).  Copies the header to the host and
// synchronises `stream`.
deinsum_status fx20_storage_error(const void *X, int64_t count, void *stream, double *err);

// Live kernel timing (ktimer.cpp, deinsum_kernel_timing): ktimer_begin records the
// start event of the next main-kernel launch on `stream` (a hipStream_t) and
// returns its slot (-1 when timing is off or full); ktimer_end records the stop.
enum KernelKind { KK_MTTKRP_STREAM = 1, KK_TTMC_FUSED = 2 };
int ktimer_begin(void *stream, int kind);
void ktimer_end(int slot, void *stream);

// Einsum parser (parse.cpp).
deinsum_status parse_spec(const char *text, deinsum_spec *out);

}  // namespace deinsum
