// errors.cpp -- thread-local error message for deinsum_last_error().
#include <string>

#include "internal.h"

namespace deinsum {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

deinsum_status fail(deinsum_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

}  // namespace deinsum

extern "C" const char *deinsum_last_error(void) { return deinsum::g_last_error.c_str(); }
