/*
 * FP64 exp, log1p and the Jacobian logarithm for the oracle's belief
 * propagation -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper evaluates the soft maximum max*(x1..xn) = ln sum exp(xi) by
 * folding its two-argument form max*(x,y) = max(x,y) + ln(1 + exp(-|x-y|))
 * (Sec. II.B, "Belief Propagation").  The two transcendental functions are
 * written here from textbook methods so that their results are fixed by this
 * file and not by the platform's libm:
 *
 *   exp(x):   Cody-Waite argument reduction x = n ln2 + r, |r| <= ln2/2, with
 *             ln2 split into a head and a tail, then the Taylor polynomial of
 *             degree 13 in r by Horner's rule with fused multiply-adds, then
 *             scaling by 2^n.  Inputs below -708 return 0 (the result would
 *             be subnormal); the only use here is exp(-|x-y|).
 *   log1p(y): for y in [0, 1], log1p(y) = 2 atanh(z) with z = y / (2 + y),
 *             z in [0, 1/3], and atanh(z) = z * sum_k z^(2k) / (2k+1) summed
 *             to k = 17 by Horner's rule in z^2 with fused multiply-adds.
 *
 * Compile with -ffp-contract=off: every fused operation is an explicit fma().
 * The oracle's tests check exp to 1 ulp and log1p to 3 ulp of the exact value.
 */
#include <math.h>
#include "oracle.h"

#define EXP_DEG 13
#define ATANH_TERMS 18

static double exp_coef[EXP_DEG + 1];     /* 1/k!       */
static double atanh_coef[ATANH_TERMS];   /* 1/(2k + 1) */

__attribute__((constructor)) static void or_spec_math_init(void)
{
    double f = 1.0;
    exp_coef[0] = 1.0;
    for (int k = 1; k <= EXP_DEG; ++k) {
        f *= (double)k;                 /* k! is exact in double for k <= 18 */
        exp_coef[k] = 1.0 / f;
    }
    for (int k = 0; k < ATANH_TERMS; ++k)
        atanh_coef[k] = 1.0 / (double)(2 * k + 1);
}

/* ln 2 = LN2_HI + LN2_LO: the nearest double to ln 2 and the remainder. */
static const double LN2_HI  = 0x1.62e42fefa39efp-1;
static const double LN2_LO  = 0x1.abc9e3b39803fp-56;
static const double INV_LN2 = 0x1.71547652b82fep0;

double or_exp(double x)
{
    if (x < -708.0) return 0.0;
    if (x > 709.0) return INFINITY;
    double t = x * INV_LN2;
    double n = floor(t + 0.5);
    double r = fma(-n, LN2_HI, x);
    r = fma(-n, LN2_LO, r);
    double p = exp_coef[EXP_DEG];
    for (int k = EXP_DEG - 1; k >= 0; --k)
        p = fma(p, r, exp_coef[k]);
    return ldexp(p, (int)n);
}

double or_log1p(double y)
{
    double z = y / (2.0 + y);
    double w = z * z;
    double p = atanh_coef[ATANH_TERMS - 1];
    for (int k = ATANH_TERMS - 2; k >= 0; --k)
        p = fma(p, w, atanh_coef[k]);
    double two_z = 2.0 * z;
    return two_z * p;
}

/* max*(a, b) = max(a, b) + ln(1 + exp(-|a - b|))  (Sec. II.B). */
double or_maxstar(double a, double b)
{
    double d = a - b;
    double m, z;
    if (d >= 0.0) { m = a; z = -d; }
    else          { m = b; z = d; }
    return m + or_log1p(or_exp(z));
}
