/*
 * Quaternary BP and B-BP4MF for code-capacity depolarizing noise -- TEST
 * INFRASTRUCTURE ONLY (see oracle.h).
 *
 * B-BP4MF (Sec. III.D, "Belief-BP4MF"; Sec. II.E, correlated decoding):
 *  1. quaternary BP on the code's Tanner graph (both check types) with the
 *     depolarizing prior; if an iteration's hard decision reproduces both
 *     syndromes, that decision is the output;
 *  2. otherwise each qubit's posterior probability of a Z component,
 *     P(Z) + P(Y), re-weights its edge of the decoding graph, the shortest
 *     paths between the shot's defects (boundary as a sink) are recomputed,
 *     and
 *  3. BP4MF runs on the priors of those paths.
 *
 * Quaternary BP, flooding, in the scalar form for binary-syndrome checks:
 * messages are log-ratios ln P(commute)/P(anticommute) with the check's Pauli
 * on the qubit (X for X checks, Z for Z checks); init check->qubit mu = 0.
 * Iteration t:
 *   qubit->check:  L(E) = prior(E) - sum_{c' != c, E anticommutes with c'} mu_c'
 *                  nu = max*(L over E commuting with c) - max*(L over the rest)
 *   check->qubit:  mu = (-1)^z * 2 atanh( prod_{q' != q} tanh(nu_q' / 2) )
 *   posterior:     L(E) = prior(E) - sum_{c, E anticommutes} mu_c, hard = argmax
 * E in the order I, X, Y, Z; X commutes with X checks' X and anticommutes
 * with Z checks' Z, and so on.  Stop at the first t whose hard decision has
 * both syndromes.
 *
 * Fixed operation order (shared by any implementation that is to agree bit
 * for bit; the exp and log1p are the ones of spec_math.c):
 *   - a qubit's checks are its X checks, then its Z checks, each ascending;
 *     sums over them run in that order, skipping the excluded one;
 *   - nu for an X check = max*(L_I, L_X) - max*(L_Y, L_Z); for a Z check
 *     max*(L_I, L_Z) - max*(L_X, L_Y);
 *   - a check's qubits ascend; t starts at 1.0 and multiplies th(nu) of the
 *     others in that order, th(x) = s (1 - e) / (1 + e), e = exp(-|x|),
 *     s = sign of x (+ for 0);
 *   - a = min(|t|, 1 - 2^-40); r = log((1 + a) / (1 - a)); mu = -r if
 *     (t < 0) xor (syndrome bit) else r;
 *   - log(x) = k ln2_hi + (k ln2_lo + log1p(m - 1)) (fused) with x = m 2^k,
 *     m in [1, 2);
 *   - posterior P of a Z component: mx = max over L_I, L_X, L_Y, L_Z in that
 *     order, e_E = exp(L_E - mx), P = (e_Y + e_Z) / (((e_I + e_X) + e_Y) + e_Z);
 *   - edge weight (2^-32 units): 1 if P >= 1/2, else
 *     floor(log((1 - P) / P) 2^32 + 1/2) clamped to [1, 2^40];
 *   - prior of a path of weight D: -D - log(1 - exp(-D)).
 * The priors are ln(p/3) (X, Y, Z) and log1p(-p) (I) from the C library.
 *
 * Joint sampler: per qubit v and shot sigma, u = word 0 of
 * Philox4x32-10(counter (v, sigma mod 2^32, sigma div 2^32, 0x44455031),
 * key (seed mod 2^32, seed div 2^32)); the error is X if u < t1, Y if
 * u < t2, Z if u < t3, else I, with t_k = round(k p/3 2^32) (k = 1, 2) and
 * t3 = round(p 2^32).
 */
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>
#include "oracle.h"

static const double LN2_HI = 0x1.62e42fefa39efp-1;
static const double LN2_LO = 0x1.abc9e3b39803fp-56;

double or_spec_log(double x)
{
    int k;
    double m = frexp(x, &k);           /* x = m 2^k, m in [1/2, 1) */
    m *= 2.0;                          /* exact: m in [1, 2)       */
    k -= 1;
    double kd = (double)k;
    return fma(kd, LN2_HI, fma(kd, LN2_LO, or_log1p(m - 1.0)));
}

double or_spec_prior(int64_t dist_fixed)
{
    double D = ldexp((double)dist_fixed, -32);
    double e = or_exp(-D);
    return (-D) - or_spec_log(1.0 - e);
}

int64_t or_qbp_weight(double P)
{
    if (P >= 0.5) return 1;
    double f = floor(or_spec_log((1.0 - P) / P) * 4294967296.0 + 0.5);
    if (f < 1.0) return 1;
    if (f > 1099511627776.0) return (int64_t)1 << 40;
    return (int64_t)f;
}

static double th(double x)
{
    double e = or_exp(-fabs(x));
    double r = (1.0 - e) / (1.0 + e);
    return x < 0.0 ? -r : r;
}

static int anti(int E, int xcheck) { return xcheck ? (E >= 2) : (E == 1 || E == 2); }

void or_sample_depolarizing(const or_tanner *T, double p, uint64_t seed, uint64_t shot0, uint64_t n,
                            uint64_t *synx, uint64_t *synz, uint64_t *obs)
{
    uint64_t W = (n + 63) / 64;
    memset(synx, 0, sizeof(uint64_t) * W * (uint64_t)T->n_xc);
    memset(synz, 0, sizeof(uint64_t) * W * (uint64_t)T->n_zc);
    memset(obs, 0, sizeof(uint64_t) * W);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t t1 = or_threshold(1.0 * p / 3.0), t2 = or_threshold(2.0 * p / 3.0), t3 = or_threshold(p);
    for (uint64_t b = 0; b < n; ++b) {
        uint64_t sigma = shot0 + b, bit = (uint64_t)1 << (b & 63);
        for (int v = 0; v < T->n_q; ++v) {
            uint32_t ctr[4] = {(uint32_t)v, (uint32_t)sigma, (uint32_t)(sigma >> 32), 0x44455031u}, r[4];
            or_philox4x32_10(ctr, key, r);
            uint32_t u = r[0];
            int E = u < t1 ? 1 : u < t2 ? 2 : u < t3 ? 3 : 0;
            if (E == 1 || E == 2)                       /* X component: Z checks */
                for (int k = 0; k < 2; ++k)
                    if (T->qz[2 * v + k] >= 0) synz[(uint64_t)T->qz[2 * v + k] * W + (b >> 6)] ^= bit;
            if (E >= 2) {                               /* Z component: X checks */
                for (int k = 0; k < 2; ++k)
                    if (T->qx[2 * v + k] >= 0) synx[(uint64_t)T->qx[2 * v + k] * W + (b >> 6)] ^= bit;
                if (T->qobs[v]) obs[b >> 6] ^= bit;
            }
        }
    }
}

/* Incident checks of qubit v in the fixed order: X checks, then Z checks. */
typedef struct { int n; int id[4]; int isx[4]; } qchecks;

static qchecks checks_of(const or_tanner *T, int v)
{
    qchecks q = {0, {0}, {0}};
    for (int k = 0; k < 2; ++k) if (T->qx[2 * v + k] >= 0) { q.id[q.n] = T->qx[2 * v + k]; q.isx[q.n++] = 1; }
    for (int k = 0; k < 2; ++k) if (T->qz[2 * v + k] >= 0) { q.id[q.n] = T->n_xc + T->qz[2 * v + k]; q.isx[q.n++] = 0; }
    return q;
}

int or_qbp(const or_tanner *T, double p, const uint8_t *zx, const uint8_t *zz, int max_iters,
           int stop, int *iters_out, uint8_t *hard, double *post)
{
    const int nq = T->n_q, nc = T->n_xc + T->n_zc;
    const double pri[4] = {log1p(-p), log(p / 3.0), log(p / 3.0), log(p / 3.0)};
    double *mu = calloc((size_t)nq * 4, sizeof(double));    /* [v][slot] check -> qubit */
    double *nu = calloc((size_t)nq * 4, sizeof(double));    /* [v][slot] qubit -> check */
    qchecks *QC = malloc(sizeof(qchecks) * nq);
    for (int v = 0; v < nq; ++v) QC[v] = checks_of(T, v);
    int conv = 0, t = 0;
    for (t = 1; t <= max_iters && !(conv && stop); ++t) {
        /* qubit -> check */
        for (int v = 0; v < nq; ++v) {
            const qchecks *q = &QC[v];
            for (int k = 0; k < q->n; ++k) {
                double L[4];
                for (int E = 0; E < 4; ++E) {
                    L[E] = pri[E];
                    for (int k2 = 0; k2 < q->n; ++k2)
                        if (k2 != k && anti(E, q->isx[k2])) L[E] = L[E] - mu[4 * v + k2];
                }
                double cm, an;
                if (q->isx[k]) { cm = or_maxstar(L[0], L[1]); an = or_maxstar(L[2], L[3]); }
                else           { cm = or_maxstar(L[0], L[3]); an = or_maxstar(L[1], L[2]); }
                nu[4 * v + k] = cm - an;
            }
        }
        /* check -> qubit */
        for (int c = 0; c < nc; ++c) {
            int z = c < T->n_xc ? zx[c] : zz[c - T->n_xc];
            int qs[4], sl[4], m = 0;
            for (int i = 0; i < 4; ++i) {
                int v = T->cq[4 * c + i];
                if (v < 0) continue;
                int s = 0;
                while (QC[v].id[s] != c) ++s;
                qs[m] = v; sl[m++] = s;
            }
            for (int i = 0; i < m; ++i) {
                double tt = 1.0;
                for (int i2 = 0; i2 < m; ++i2)
                    if (i2 != i) tt = tt * th(nu[4 * qs[i2] + sl[i2]]);
                double a = fabs(tt);
                if (a > 1.0 - 0x1p-40) a = 1.0 - 0x1p-40;
                double r = or_spec_log((1.0 + a) / (1.0 - a));
                mu[4 * qs[i] + sl[i]] = ((tt < 0.0) != (z != 0)) ? -r : r;
            }
        }
        /* posteriors and hard decision */
        for (int v = 0; v < nq; ++v) {
            const qchecks *q = &QC[v];
            double L[4];
            for (int E = 0; E < 4; ++E) {
                L[E] = pri[E];
                for (int k = 0; k < q->n; ++k)
                    if (anti(E, q->isx[k])) L[E] = L[E] - mu[4 * v + k];
            }
            int h = 0;
            for (int E = 1; E < 4; ++E) if (L[E] > L[h]) h = E;
            hard[v] = (uint8_t)h;
            if (post) for (int E = 0; E < 4; ++E) post[4 * v + E] = L[E];
        }
        /* both syndromes reproduced? */
        conv = 1;
        for (int c = 0; c < nc && conv; ++c) {
            int isx = c < T->n_xc, par = 0;
            for (int i = 0; i < 4; ++i) {
                int v = T->cq[4 * c + i];
                if (v >= 0) par ^= anti(hard[v], isx);
            }
            conv = par == (isx ? zx[c] : zz[c - T->n_xc]);
        }
    }
    if (iters_out) *iters_out = t - 1;
    free(mu); free(nu); free(QC);
    return conv;
}

double or_qbp_zprob(const double *L)
{
    double mx = L[0];
    for (int E = 1; E < 4; ++E) mx = fmax(mx, L[E]);
    double e[4];
    for (int E = 0; E < 4; ++E) e[E] = or_exp(L[E] - mx);
    return (e[2] + e[3]) / (((e[0] + e[1]) + e[2]) + e[3]);
}

int or_bbp4mf_shot(const or_dem *g, const or_tanner *T, double p, const uint8_t *zx, const uint8_t *zz,
                   int ob, const or_opts *o, int32_t *s_out, int32_t *partner, int32_t s_cap)
{
    const int nq = T->n_q, N = g->n_det;
    uint8_t *hard = malloc(nq);
    double *post = malloc(sizeof(double) * 4 * (size_t)nq);
    int iters = 0, flags = 0, pred = 0;
    int conv = or_qbp(T, p, zx, zz, o->max_iters, 1, &iters, hard, post);
    int s = 0;
    for (int k = 0; k < N; ++k) s += zx[k];
    *s_out = s;
    if (conv) {
        flags |= OR_F_QBP | OR_F_CONVERGED_ANY;
        for (int v = 0; v < nq; ++v) if (hard[v] >= 2 && T->qobs[v]) pred ^= 1;
    } else if (s > s_cap) {
        free(hard); free(post);
        return OR_F_OVERFLOW;
    } else {
        int64_t *w = malloc(sizeof(int64_t) * g->n_mech);
        for (int v = 0; v < nq; ++v) w[T->qmech[v]] = or_qbp_weight(or_qbp_zprob(post + 4 * v));
        or_tables tab;
        int rc = or_build_tables_w(g, w, &tab);
        free(w);
        if (rc) { free(hard); free(post); return -1; }
        int *def = malloc(sizeof(int) * (s + 1));
        int m = 0;
        for (int k = 0; k < N; ++k) if (zx[k]) def[m++] = k;
        if (s == 0) {
            flags |= OR_F_CONVERGED_ANY;
        } else if (s == 1) {
            partner[0] = 0;
            pred = tab.par[(size_t)def[0] * N + def[0]];
            flags |= OR_F_CONVERGED_ANY;
        } else if (s >= 2) {
            double *L = malloc(sizeof(double) * s * s);
            int64_t *Wt = malloc(sizeof(int64_t) * s * s);
            for (int i = 0; i < s; ++i)
                for (int j = 0; j < s; ++j) {
                    int a = i <= j ? def[i] : def[j], b = i <= j ? def[j] : def[i];
                    int64_t D = tab.dist[(size_t)a * N + b];
                    L[i * s + j] = or_spec_prior(D);
                    Wt[i * s + j] = D;
                }
            int64_t wbest = 0;
            flags |= or_bp4m_instance(L, Wt, s, o, partner, &wbest, NULL, NULL);
            for (int i = 0; i < s; ++i) {
                int q = partner[i];
                if (q < i) continue;
                pred ^= tab.par[(size_t)def[i] * N + def[q]];
            }
            free(L); free(Wt);
        }
        free(def);
        or_tables_free(&tab);
    }
    if (pred) flags |= OR_F_PRED;
    if (pred != ob) flags |= OR_F_FAIL;
    free(hard); free(post);
    return flags;
}

typedef struct {
    const or_dem *g; const or_tanner *T; double p;
    const uint64_t *synx, *synz, *obs; uint64_t n, b0, b1; const or_opts *o;
    uint8_t *flags; int32_t *s_out; int32_t *partner; int32_t s_cap;
} bjob;

static void *bbp4mf_range(void *arg)
{
    bjob *j = arg;
    const or_tanner *T = j->T;
    uint64_t W = (j->n + 63) / 64;
    uint8_t *zx = malloc(T->n_xc + 1), *zz = malloc(T->n_zc + 1);
    for (uint64_t b = j->b0; b < j->b1; ++b) {
        uint64_t w = b >> 6, bit = (uint64_t)1 << (b & 63);
        for (int c = 0; c < T->n_xc; ++c) zx[c] = (j->synx[(uint64_t)c * W + w] & bit) != 0;
        for (int c = 0; c < T->n_zc; ++c) zz[c] = (j->synz[(uint64_t)c * W + w] & bit) != 0;
        int ob = j->obs ? (j->obs[w] & bit) != 0 : 0;
        int32_t *pt = j->partner + b * (uint64_t)j->s_cap;
        for (int i = 0; i < j->s_cap; ++i) pt[i] = -1;
        int f = or_bbp4mf_shot(j->g, T, j->p, zx, zz, ob, j->o, &j->s_out[b], pt, j->s_cap);
        j->flags[b] = (uint8_t)(f < 0 ? 0xFF : f);
    }
    free(zx); free(zz);
    return NULL;
}

int or_bbp4mf_decode(const or_dem *g, const or_tanner *T, double p, const uint64_t *synx,
                     const uint64_t *synz, const uint64_t *obs, uint64_t n, const or_opts *o,
                     int n_threads, uint8_t *flags, int32_t *s_out, int32_t *partner, int32_t s_cap)
{
    if (n_threads < 1) n_threads = 1;
    if ((uint64_t)n_threads > n) n_threads = (int)(n ? n : 1);
    pthread_t *th = malloc(sizeof(pthread_t) * n_threads);
    bjob *jobs = malloc(sizeof(bjob) * n_threads);
    for (int i = 0; i < n_threads; ++i) {
        bjob j = {g, T, p, synx, synz, obs, n, n * i / n_threads, n * (i + 1) / n_threads, o,
                  flags, s_out, partner, s_cap};
        jobs[i] = j;
        pthread_create(&th[i], NULL, bbp4mf_range, &jobs[i]);
    }
    for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    free(th); free(jobs);
    return 0;
}
