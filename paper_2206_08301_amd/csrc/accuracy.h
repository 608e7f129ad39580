// accuracy.h -- a-priori error estimate of each arithmetic form (host only),
// the rule behind DEINSUM_PREC_AUTO and deinsum_report.est_err.
#pragma once

#include <cstdint>

namespace deinsum {

struct ErrInputs {
    int prec = 0;            // PrecisionId of the form
    int order = 3;           // N
    double L = 1;            // contraction length: product of the contracted extents
    double k32 = 0;          // terms summed in FP32 before a fold into FP64 (0: FP64 form)
    double x_storage = -1;   // FX20: ||X - X_stored|| / ||X|| (from the header); < 0: the model
};

// Estimated normwise relative error of the form's result against the exact result
// for the FP64 operands the caller's storage was rounded from (the rule is stated
// with deinsum_estimate_error in deinsum.h).
double estimate_error(const ErrInputs &in);

// Normwise relative storage error of FX20 for a tensor with these max |x| and rms,
// taking the rounding error of each element as uniform in +-2^(e-1).
double fx20_storage_model(double max_abs, double rms);

}  // namespace deinsum
