// accuracy.cpp -- a-priori error estimate of the arithmetic forms.
//
// Root-sum-square model of independent rounding errors, valid for data whose sums
// do not cancel much more than sums of random-sign terms, doubled as a margin:
//   est = 2 sqrt(dx^2 + d_op^2 + (N-2) d_store^2 + d_drop^2 + d_acc^2)
//   dx      : normwise relative error of X as the form reads it;
//   d_op    : the factor (or factor product) that is the other matrix-core operand,
//             as the form reads it;
//   d_store : each remaining factor, applied in FP64 from its storage;
//   d_drop  : product terms the form leaves out;
//   d_acc   : accumulation, u64 sqrt(L/3) for FP64 sums over L terms plus
//             u32 sqrt(k/3) for the k terms summed in FP32 before each fold into FP64
//             (n rounding errors of rms u/sqrt(3), each relative to a partial sum
//             taken as large as the result).
// A value rounded to nearest with unit roundoff u carries a relative error that is
// close to uniform in +-u, rms u / sqrt(3); a hi + lo split of one format leaves the
// product of two such errors, rms u^2 / 3.
#include "accuracy.h"

#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace deinsum {

namespace {

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53
constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24
constexpr double kUbf = 3.90625e-03;             // 2^-8  (BF16: 8-bit significand)
constexpr double kUh = 4.8828125e-04;            // 2^-11 (FP16: 11-bit significand)

double rnd(double u) { return u / std::sqrt(3.0); }
double split(double u) { return u * u / 3.0; }
double rss(double a, double b) { return std::sqrt(a * a + b * b); }

}  // namespace

double estimate_error(const ErrInputs &in)
{
    const double stores = std::max(0, in.order - 2);
    double dx = 0, dop = 0, dst = 0, ddrop = 0;
    double dacc = kU64 * std::sqrt(std::max(1.0, in.L) / 3.0);
    const double acc32 = kU32 * std::sqrt(std::max(1.0, in.k32) / 3.0);
    switch (in.prec) {
    case P_FP64:
        break;
    case P_FP32:
        dx = dop = dst = rnd(kU32);
        dacc += acc32;
        break;
    case P_BF16:
        dx = rnd(kUbf);
        dop = rss(rnd(kU32), rnd(kUbf));
        dst = rnd(kU32);
        dacc += acc32;
        break;
    case P_BF16X3:
        dx = dop = rss(rnd(kU32), split(kUbf));
        dst = rnd(kU32);
        ddrop = split(kUbf);  // lo * lo
        dacc += acc32;
        break;
    case P_FX20:
        // X's 20-bit storage error is data dependent: exact from the header when known.
        dx = in.x_storage >= 0 ? in.x_storage : rnd(std::ldexp(1.0, -19));
        dop = rss(rnd(kU32), split(kUh));
        dst = rnd(kU32);
        ddrop = split(kUh);  // l * u_lo
        // The FP32 tile holds the fixed-point offset that is removed after the fold,
        // about doubling the magnitude its rounding errors are relative to.
        dacc += 2.0 * acc32;
        break;
    default:
        return NAN;
    }
    return 2.0 * std::sqrt(dx * dx + dop * dop + stores * dst * dst + ddrop * ddrop + dacc * dacc);
}

double fx20_storage_model(double max_abs, double rms)
{
    if (!(max_abs > 0) || !(rms > 0)) return NAN;
    int e = 0;
    (void)std::frexp(max_abs, &e);  // max |x| < 2^e; the FX20 exponent is e - 19
    return rnd(std::ldexp(1.0, e - 20)) / rms;
}

}  // namespace deinsum
