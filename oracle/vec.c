/*
 * Array helpers so that the oracle's tests can call its scalar routines on
 * many inputs at once -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include "oracle.h"

void or_exp_v(const double *x, double *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = or_exp(x[i]);
}

void or_log1p_v(const double *x, double *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = or_log1p(x[i]);
}

void or_maxstar_v(const double *a, const double *b, double *y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = or_maxstar(a[i], b[i]);
}

void or_philox_v(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) or_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

void or_threshold_v(const double *q, uint32_t *thr, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) thr[i] = or_threshold(q[i]);
}

void or_prior_llr_v(const int64_t *dist, double *llr, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) llr[i] = or_prior_llr(dist[i]);
}

void or_fixed_weight_v(const double *q, int64_t *w, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) w[i] = or_fixed_weight(q[i]);
}
