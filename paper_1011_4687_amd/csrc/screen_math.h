// Arithmetic of the pair-list decisions, shared by the host packer and the
// device build so that both take every decision from the same bits.
//
// Every function here is a fixed sequence of IEEE-754 operations (add,
// multiply, divide, square root, round-to-integer, scale by a power of two),
// each correctly rounded on the host and on gfx950, with contraction into
// fused multiply-adds switched off.  The screening bound therefore uses its
// own exponential (Cody-Waite reduction by ln 2 split into a 32-bit head and
// a tail, then the Taylor series of e^r on |r| <= ln2/2), not the C library's
// or the device library's, whose last bits differ; and the far-field radius
// bands are found by comparing r2far with band edges computed once, not by a
// logarithm per pair.  A .hip file includes this header between
// "#pragma clang force_cuda_host_device begin" and "... end".
#pragma once

#include <cstdint>

namespace envpot {
namespace sm {

constexpr double kPi = 3.14159265358979323846;

// e^x for x <= 0 (the screening exponent); 0 below -708, where e^x is
// below the smallest normal double and no screening threshold is that small.
inline double exp_neg(double x) {
#pragma clang fp contract(off)
    if (!(x > -708.0)) return 0.0;
    if (x > 0.0) x = 0.0;
    const double inv_ln2 = 1.4426950408889634;
    const double ln2_hi = 6.93147180369123816490e-01;  // 32 trailing zero bits: k * ln2_hi is exact
    const double ln2_lo = 1.90821492927058770002e-10;
    const double k = __builtin_rint(x * inv_ln2);
    const double r = (x - k * ln2_hi) - k * ln2_lo;
    // e^r = sum_{n <= 13} r^n / n!, truncation < 1e-17 relative for |r| <= 0.347
    double s = 1.0 / 6227020800.0;
    s = s * r + 1.0 / 479001600.0;
    s = s * r + 1.0 / 39916800.0;
    s = s * r + 1.0 / 3628800.0;
    s = s * r + 1.0 / 362880.0;
    s = s * r + 1.0 / 40320.0;
    s = s * r + 1.0 / 5040.0;
    s = s * r + 1.0 / 720.0;
    s = s * r + 1.0 / 120.0;
    s = s * r + 1.0 / 24.0;
    s = s * r + 1.0 / 6.0;
    s = s * r + 0.5;
    s = s * r + 1.0;
    s = s * r + 1.0;
    return __builtin_ldexp(s, int(k));
}

// |A - B|^2 in the order x, y, z.
inline double dist2(const double* A, const double* B) {
#pragma clang fp contract(off)
    const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
    return dx * dx + dy * dy + dz * dz;
}

// Screening bound of the primitive pair (a on A, b on B, rab2 = |A - B|^2):
// the largest value of its normalised s-type overlap charge,
//   |c_a c_b| N_a N_b (pi/p)^{3/2} exp(-a b |A - B|^2 / p),
// with N = (2 alpha / pi)^{3/4} passed in as n0a, n0b.
inline double screen_bound(double ca, double cb, double n0a, double n0b, double a, double b, double rab2) {
#pragma clang fp contract(off)
    const double p = a + b, mu = a * b / p;
    const double pp = kPi / p, pp32 = pp * __builtin_sqrt(pp);
    return __builtin_fabs(ca * cb) * n0a * n0b * pp32 * exp_neg(-mu * rab2);
}

// Gaussian product centre (a A + b B) / p of one coordinate.
inline double prod_centre(double a, double A, double b, double B, double p) {
#pragma clang fp contract(off)
    return (a * A + b * B) / p;
}

// c1 = 2 sqrt(p / pi) of a record.
inline double rec_c1(double p) {
#pragma clang fp contract(off)
    return 2.0 * __builtin_sqrt(p / kPi);
}

// r2far of a pair as its record stores it: tfar64[L] / p (FP64), or that
// quotient with tfar32[L] rounded to float (FP32C).
inline double rec_r2far(double tfar, double p, bool fp64) {
#pragma clang fp contract(off)
    return fp64 ? tfar / p : double(float(tfar / p));
}

// Radius band of a one-centre pair: the number of edges E[1..bands-1] that
// r2far reaches (edges from band_edges, ascending).
inline int band_of(double r2far, const double* E, int bands) {
    int b = 0;
    while (b < bands - 1 && r2far >= E[b + 1]) ++b;
    return b;
}

// Cost term of one cluster in its segment's cost: the merged evaluation plus
// the share of waves that evaluate the members.
inline double cluster_term(double w_merged, double near_share, double member_cost) {
#pragma clang fp contract(off)
    return w_merged + near_share * member_cost;
}

}  // namespace sm
}  // namespace envpot
