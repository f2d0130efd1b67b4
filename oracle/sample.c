/*
 * Syndrome sampler -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Every mechanism m of shot sigma fires independently with probability q_m
 * (the detector error model of Sec. III.E).  The draw is a keyed hash:
 *   key     = (seed mod 2^32, seed div 2^32)
 *   counter = (m div 4, sigma mod 2^32, sigma div 2^32, 0)
 *   u       = word (m mod 4) of Philox4x32-10(counter, key)
 * and m fires iff u < thr_m with thr_m = round(q_m * 2^32) clamped to
 * [0, 2^32 - 1], so the decision is made in integers.
 *
 * Output layout (bit planes): syn[k * W + w] bit b is detector k of batch
 * shot 64 w + b, W = ceil(n / 64); obs[w] likewise; err[m * W + w] (if not
 * NULL) bit b: mechanism m fired in that shot.  Trailing bits are 0.
 */
#include <string.h>
#include <math.h>
#include "oracle.h"

uint32_t or_threshold(double q)
{
    double t = floor(q * 4294967296.0 + 0.5);
    if (t < 0.0) t = 0.0;
    if (t > 4294967295.0) t = 4294967295.0;
    return (uint32_t)t;
}

void or_sample(const or_dem *g, uint64_t seed, uint64_t shot0, uint64_t n_shots,
               uint64_t *syn, uint64_t *obs, uint64_t *err)
{
    uint64_t W = (n_shots + 63) / 64;
    memset(syn, 0, sizeof(uint64_t) * W * (uint64_t)g->n_det);
    memset(obs, 0, sizeof(uint64_t) * W);
    if (err) memset(err, 0, sizeof(uint64_t) * W * (uint64_t)g->n_mech);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint64_t b = 0; b < n_shots; ++b) {
        uint64_t sigma = shot0 + b;
        uint64_t bit = (uint64_t)1 << (b & 63);
        uint32_t r[4] = {0, 0, 0, 0};
        for (int m = 0; m < g->n_mech; ++m) {
            if ((m & 3) == 0) {
                uint32_t ctr[4] = {(uint32_t)(m >> 2), (uint32_t)sigma, (uint32_t)(sigma >> 32), 0};
                or_philox4x32_10(ctr, key, r);
            }
            if (r[m & 3] < or_threshold(g->q[m])) {
                if (err) err[(uint64_t)m * W + (b >> 6)] ^= bit;
                for (int e = g->off[m]; e < g->off[m + 1]; ++e)
                    syn[(uint64_t)g->dets[e] * W + (b >> 6)] ^= bit;
                if (g->obs[m]) obs[b >> 6] ^= bit;
            }
        }
    }
}
