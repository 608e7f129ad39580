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

// Einsum parser (parse.cpp).
deinsum_status parse_spec(const char *text, deinsum_spec *out);

}  // namespace deinsum
