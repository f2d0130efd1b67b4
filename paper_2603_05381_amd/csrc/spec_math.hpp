// FP64 exp, log1p and Jacobian logarithm with a fixed evaluation order, for
// the bit-reproducible decoding mode.
//
// The paper's soft maximum is folded pairwise with the Jacobian logarithm
// max*(x, y) = max(x, y) + ln(1 + exp(-|x - y|)) (Sec. II.B).  Its two
// transcendental parts are evaluated here by textbook methods, every fused
// step written as an explicit fma, so a result depends on nothing but its
// inputs:
//   exp(x), x <= 709: x = n ln2 + r with n = floor(x / ln2 + 1/2) and
//     r = (x - n LN2_HI) - n LN2_LO (Cody-Waite, two fmas), then the Taylor
//     polynomial sum_{k<=13} r^k / k! by Horner's rule in fmas, scaled by 2^n;
//     x < -708 gives 0.
//   log1p(y), 0 <= y <= 1: 2 atanh(z), z = y / (2 + y), with
//     atanh(z) = z sum_{k<=17} z^(2k) / (2k+1) by Horner's rule in z^2.
// Files that include this header must not let the compiler contract a*b+c.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace bpm {
namespace specmath {

constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;    // nearest double to ln 2
constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;   // ln 2 - kLn2Hi
constexpr double kInvLn2 = 0x1.71547652b82fep0;

constexpr double inv_factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= (double)i;
    return 1.0 / f;
}

__device__ __forceinline__ double exp_fixed(double x) {
    if (x < -708.0) return 0.0;
    if (x > 709.0) return __builtin_huge_val();
    double t = x * kInvLn2;
    double n = floor(t + 0.5);
    double r = fma(-n, kLn2Hi, x);
    r = fma(-n, kLn2Lo, r);
    double p = inv_factorial(13);
    p = fma(p, r, inv_factorial(12));
    p = fma(p, r, inv_factorial(11));
    p = fma(p, r, inv_factorial(10));
    p = fma(p, r, inv_factorial(9));
    p = fma(p, r, inv_factorial(8));
    p = fma(p, r, inv_factorial(7));
    p = fma(p, r, inv_factorial(6));
    p = fma(p, r, inv_factorial(5));
    p = fma(p, r, inv_factorial(4));
    p = fma(p, r, inv_factorial(3));
    p = fma(p, r, inv_factorial(2));
    p = fma(p, r, inv_factorial(1));
    p = fma(p, r, inv_factorial(0));
    return ldexp(p, (int)n);
}

__device__ __forceinline__ double log1p_fixed(double y) {
    double z = y / (2.0 + y);
    double w = z * z;
    double p = 1.0 / 35.0;
#pragma unroll
    for (int k = 16; k >= 0; --k) p = fma(p, w, 1.0 / (double)(2 * k + 1));
    double two_z = 2.0 * z;
    return two_z * p;
}

// Natural log of x > 0: x = m 2^k with m in [1, 2), then
// k ln2_hi + (k ln2_lo + log1p(m - 1)), both products fused.
__device__ __forceinline__ double log_fixed(double x) {
    int k;
    double m = frexp(x, &k);            // x = m 2^k, m in [1/2, 1)
    m *= 2.0;
    k -= 1;
    const double kd = (double)k;
    return fma(kd, kLn2Hi, fma(kd, kLn2Lo, log1p_fixed(m - 1.0)));
}

__device__ __forceinline__ double maxstar(double a, double b) {
    double d = a - b;
    double m, z;
    if (d >= 0.0) { m = a; z = -d; }
    else          { m = b; z = d; }
    return m + log1p_fixed(exp_fixed(z));
}

}  // namespace specmath
}  // namespace bpm
