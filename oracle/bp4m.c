/*
 * BP4M / BP4MF decoding of one syndrome at a time -- TEST INFRASTRUCTURE
 * ONLY (see oracle.h).
 *
 * Factor graph (Sec. II.A): for s defects, variables v_ij (i <= j) are the
 * decoding-graph edges (v_ii: defect i to the boundary); factor c_i is the
 * exactly-one constraint over v_i1..v_is (syndrome-factor equation); v_ij
 * carries the prior LLR l_ij.  Messages are kept as an s x s matrix
 * M[i][j] = m_{c_i -> v_ij}; the diagonal M[i][i] goes to v_ii.
 *
 * Sum-product in the log domain (Sec. II.B), flooding schedule: every
 * iteration t first forms all variable-to-factor messages from the factor
 * messages of iteration t-1 and then all factor-to-variable messages:
 *   m_{v_ik -> c_i} = l_ik + (1/alpha) m_{c_k -> v_ik}   (k != i; v_ik has one
 *                                                       other factor, c_k)
 *   m_{v_ii -> c_i} = l_ii                               (no other factor)
 *   m_{c_i -> v_ij} = - max*_{k != j} m_{v_ik -> c_i}
 * with m_{c -> v} = 0 before the first iteration; alpha = 1 is plain
 * sum-product and alpha != 1 is the memory variant of Sec. III.E ("BP Improvements").  The
 * leave-one-out soft maximum is the pairwise Jacobian fold of prefixes and
 * suffixes:  A_k = max*(A_{k-1}, x_k),  B_k = max*(x_k, B_{k+1}),
 * LOO_j = max*(A_{j-1}, B_{j+1}) (one side alone at the ends).
 * Posterior (marginalization equation):
 *   lambda_ij = l_ij + (M[i][j] + M[j][i]),   lambda_ii = l_ii + M[i][i].
 *
 * Marginalization (Sec. II.D): v is chosen iff lambda_v > 0; the candidate
 * has converged iff every factor has exactly one chosen variable (Sec. II.C).
 * Forced convergence (Sec. II.D): take the variables in order of decreasing
 * lambda and accept each one whose factors are both still unmatched.  When a
 * block maximum conflicts with an earlier choice the paper's text leaves the
 * next step open; this is the reading that matches its Fig. 2 example and its
 * "recursively pick the most probable variable" description.  Equal lambda
 * is broken by the smaller (i, j).
 *
 * BP4M (Sec. III.A): run T iterations, marginalize at each, keep the
 * lowest-weight converged candidate (the earliest on ties); if iteration T
 * did not converge, run forced convergence on its posteriors and output it
 * iff its weight is strictly lower than the best converged one (or there is
 * none).  BP4MF (Sec. III.B): run forced convergence at every iteration whose
 * marginalization did not converge and keep the lowest-weight candidate.
 * The weight of a candidate is the sum of its matched path weights.
 *
 * Diagnostic switches (or_opts) evaluate other readings of the text: the
 * printed update indices taken literally (both message types of iteration
 * t+1 from those of iteration t, which repeats every factor message once:
 * iterations 2k-1 and 2k of it equal flooding iteration k), the block-maxima
 * forced convergence with conflicts matched to the boundary, and the weight
 * of the XOR of the matched paths.
 */
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include "oracle.h"

void or_factor_update(const double *x, int s, double *out)
{
    double *A = malloc(sizeof(double) * s), *B = malloc(sizeof(double) * s);
    A[0] = x[0];
    for (int k = 1; k < s; ++k) A[k] = or_maxstar(A[k - 1], x[k]);
    B[s - 1] = x[s - 1];
    for (int k = s - 2; k >= 0; --k) B[k] = or_maxstar(x[k], B[k + 1]);
    for (int j = 0; j < s; ++j) {
        double v;
        if (j == 0) v = B[1];
        else if (j == s - 1) v = A[s - 2];
        else v = or_maxstar(A[j - 1], B[j + 1]);
        out[j] = -v;
    }
    free(A); free(B);
}

int or_marginal_decision(const double *lam, int s, int32_t *partner)
{
    int conv = 1;
    for (int i = 0; i < s; ++i) {
        int cnt = 0, p = -1;
        for (int j = 0; j < s; ++j)
            if (lam[(size_t)i * s + j] > 0.0) { cnt++; p = j; }
        if (cnt != 1) conv = 0;
        partner[i] = p;
    }
    return conv;
}

typedef struct { double lam; int32_t i, j; } fc_item;

static int fc_cmp(const void *pa, const void *pb)
{
    const fc_item *a = pa, *b = pb;
    if (a->lam != b->lam) return a->lam > b->lam ? -1 : 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    return (a->j > b->j) - (a->j < b->j);
}

void or_forced_convergence(const double *lam, int s, int32_t *partner)
{
    size_t n = (size_t)s * (s + 1) / 2, k = 0;
    fc_item *it = malloc(sizeof(fc_item) * n);
    for (int i = 0; i < s; ++i)
        for (int j = i; j < s; ++j) {
            it[k].lam = lam[(size_t)i * s + j]; it[k].i = i; it[k].j = j; k++;
        }
    qsort(it, n, sizeof(fc_item), fc_cmp);
    char *used = calloc(s, 1);
    for (int i = 0; i < s; ++i) partner[i] = -1;
    for (size_t a = 0; a < n; ++a) {
        int i = it[a].i, j = it[a].j;
        if (used[i] || used[j]) continue;
        used[i] = used[j] = 1;
        partner[i] = j; partner[j] = i;
    }
    free(used); free(it);
}

/* Block maxima (Sec. II.D) over the partition v_ij -> c_i (i <= j): each
 * check's representative is its block's largest posterior (ties: smaller
 * j); representatives are taken by decreasing posterior (ties: smaller i);
 * a representative v_ii, or one whose partner check is already matched,
 * matches its check to the boundary; otherwise it matches both checks. */
void or_forced_convergence_blocks(const double *lam, int s, int32_t *partner)
{
    fc_item *it = malloc(sizeof(fc_item) * (s > 0 ? s : 1));
    for (int i = 0; i < s; ++i) {
        int best = i;
        for (int j = i + 1; j < s; ++j)
            if (lam[(size_t)i * s + j] > lam[(size_t)i * s + best]) best = j;
        it[i].lam = lam[(size_t)i * s + best]; it[i].i = i; it[i].j = best;
    }
    qsort(it, s, sizeof(fc_item), fc_cmp);
    for (int i = 0; i < s; ++i) partner[i] = -1;
    for (int a = 0; a < s; ++a) {
        int i = it[a].i, j = it[a].j;
        if (partner[i] >= 0) continue;
        if (j == i || partner[j] >= 0) { partner[i] = i; continue; }
        partner[i] = j; partner[j] = i;
    }
    free(it);
}

static int64_t cand_weight(const int64_t *W, int s, const int32_t *partner)
{
    int64_t w = 0;
    for (int i = 0; i < s; ++i)
        if (partner[i] >= i) w += W[(size_t)i * s + partner[i]];
    return w;
}

/*
 * Candidate bookkeeping of BP4M (Sec. III.A) and BP4MF (Sec. III.B), fed
 * with the posteriors of one iteration at a time:
 *  - marginalize; a converged candidate is offered with its weight;
 *  - BP4MF: an iteration that did not converge offers its forced-convergence
 *    candidate instead;
 *  - a candidate replaces the kept one only if its weight is strictly lower,
 *    so among equal weights the earliest stays;
 *  - BP4M, at the end: if the last iteration did not converge, its forced-
 *    convergence candidate is offered the same way (a converged candidate
 *    of equal weight stays).
 */
void or_selector_init(or_selector *S, int s, int variant)
{
    memset(S, 0, sizeof(*S));
    S->s = s;
    S->variant = variant;
    S->cand = malloc(sizeof(int32_t) * (s > 0 ? s : 1));
    S->best = malloc(sizeof(int32_t) * (s > 0 ? s : 1));
}

static void selector_offer(or_selector *S, const int64_t *W, int fc)
{
    int64_t w = S->wfn ? S->wfn(S->wctx, S->cand, S->s) : cand_weight(W, S->s, S->cand);
    if (!S->have_best || w < S->best_w) {
        memcpy(S->best, S->cand, sizeof(int32_t) * S->s);
        S->best_w = w; S->have_best = 1; S->best_fc = fc;
    }
}

void or_selector_step(or_selector *S, const double *lam, const int64_t *W)
{
    S->conv_last = or_marginal_decision(lam, S->s, S->cand);
    if (S->conv_last) {
        S->flags |= OR_F_CONVERGED_ANY;
        selector_offer(S, W, 0);
    } else if (S->variant == 1) {
        S->flags |= OR_F_FC_RAN;
        if (S->fc_rule == 1) or_forced_convergence_blocks(lam, S->s, S->cand);
        else or_forced_convergence(lam, S->s, S->cand);
        selector_offer(S, W, 1);
    }
}

int or_selector_finish(or_selector *S, const double *lam_last, const int64_t *W,
                       int32_t *partner, int64_t *weight)
{
    if (S->variant == 0 && !S->conv_last) {
        S->flags |= OR_F_FC_RAN;
        if (S->fc_rule == 1) or_forced_convergence_blocks(lam_last, S->s, S->cand);
        else or_forced_convergence(lam_last, S->s, S->cand);
        selector_offer(S, W, 1);
    }
    if (S->best_fc) S->flags |= OR_F_FC_CHOSEN;
    memcpy(partner, S->best, sizeof(int32_t) * S->s);
    *weight = S->best_w;
    int fl = S->flags;
    free(S->cand); free(S->best);
    S->cand = S->best = NULL;
    return fl;
}

int or_bp4m_instance(const double *L, const int64_t *W, int s, const or_opts *o,
                     int32_t *partner, int64_t *weight, double *Mout, double *lamout)
{
    return or_bp4m_instance_ex(L, W, s, o, NULL, NULL, partner, weight, Mout, lamout);
}

int or_bp4m_instance_ex(const double *L, const int64_t *W, int s, const or_opts *o,
                        or_weight_fn wfn, void *wctx,
                        int32_t *partner, int64_t *weight, double *Mout, double *lamout)
{
    if (s == 0) { *weight = 0; return OR_F_CONVERGED_ANY; }
    if (s == 1) { partner[0] = 0; *weight = wfn ? wfn(wctx, partner, 1) : W[0]; return OR_F_CONVERGED_ANY; }
    size_t ss = (size_t)s * s;
    double *M = calloc(ss, sizeof(double)), *Mn = malloc(sizeof(double) * ss);
    double *lam = malloc(sizeof(double) * ss), *X = malloc(sizeof(double) * s);
    /* literal schedule: variable-to-factor messages V[i][k] (from v_ik to
     * c_i) kept from the previous iteration, starting at the priors */
    double *V = NULL, *Vn = NULL;
    if (o->schedule == 1) {
        V = malloc(sizeof(double) * ss); Vn = malloc(sizeof(double) * ss);
        memcpy(V, L, sizeof(double) * ss);
    }
    double inv_alpha = 1.0 / o->alpha;
    or_selector S;
    or_selector_init(&S, s, o->variant);
    S.fc_rule = o->fc_rule;
    S.wfn = wfn;
    S.wctx = wctx;

    for (int t = 1; t <= o->max_iters; ++t) {
        for (int i = 0; i < s; ++i) {
            if (o->schedule == 1) {
                for (int k = 0; k < s; ++k)
                    Vn[(size_t)i * s + k] = (k == i) ? L[(size_t)i * s + i]
                                                     : L[(size_t)i * s + k] + M[(size_t)k * s + i] * inv_alpha;
                or_factor_update(V + (size_t)i * s, s, Mn + (size_t)i * s);
                continue;
            }
            for (int k = 0; k < s; ++k)
                X[k] = (k == i) ? L[(size_t)i * s + i]
                                : L[(size_t)i * s + k] + M[(size_t)k * s + i] * inv_alpha;
            or_factor_update(X, s, Mn + (size_t)i * s);
        }
        double *sw = M; M = Mn; Mn = sw;
        if (o->schedule == 1) { sw = V; V = Vn; Vn = sw; }
        for (int i = 0; i < s; ++i) {
            lam[(size_t)i * s + i] = L[(size_t)i * s + i] + M[(size_t)i * s + i];
            for (int j = i + 1; j < s; ++j) {
                double v = L[(size_t)i * s + j] + (M[(size_t)i * s + j] + M[(size_t)j * s + i]);
                lam[(size_t)i * s + j] = v;
                lam[(size_t)j * s + i] = v;
            }
        }
        or_selector_step(&S, lam, W);
    }
    int flags = or_selector_finish(&S, lam, W, partner, weight);
    if (Mout) memcpy(Mout, M, sizeof(double) * ss);
    if (lamout) memcpy(lamout, lam, sizeof(double) * ss);
    free(M); free(Mn); free(lam); free(X); free(V); free(Vn);
    return flags;
}

/* Candidate selection over a whole sequence of posteriors lam[T][s][s]
 * (the posteriors of iterations 1..T, e.g. another implementation's). */
int or_select_sequence(const double *lam_seq, int T, int s, const int64_t *W, int variant,
                       int32_t *partner, int64_t *weight)
{
    if (s == 0) { *weight = 0; return OR_F_CONVERGED_ANY; }
    if (s == 1) { partner[0] = 0; *weight = W[0]; return OR_F_CONVERGED_ANY; }
    or_selector S;
    or_selector_init(&S, s, variant);
    size_t ss = (size_t)s * s;
    for (int t = 0; t < T; ++t) or_selector_step(&S, lam_seq + (size_t)t * ss, W);
    return or_selector_finish(&S, lam_seq + (size_t)(T - 1) * ss, W, partner, weight);
}

/* ------------------------------------------------------------------------- */

typedef struct {
    const or_dem *g; const or_tables *t; const uint64_t *syn, *obs;
    uint64_t n_shots, w0, w1; const or_opts *o;
    uint8_t *flags; int32_t *s_out, *partner; int32_t s_cap; uint64_t *corr;
} job_t;

static void toggle(uint64_t *corr, uint64_t W, int e, uint64_t b)
{
    corr[(uint64_t)e * W + (b >> 6)] ^= (uint64_t)1 << (b & 63);
}

/* Weight of the XOR of a candidate's matched paths (or_opts.weight_rule 1):
 * every matched pair's shortest path (boundary paths for v_ii) toggles its
 * edges; the weight is the sum of the fixed-point weights of the edges
 * toggled an odd number of times. */
typedef struct {
    const or_dem *g; const or_tables *t; const int32_t *def;
    uint8_t *par; int32_t *touched; int64_t *wfix;
} xor_ctx;

static void xor_toggle(xor_ctx *X, int e, int *nt)
{
    if (!X->par[e]) X->touched[(*nt)++] = e;
    X->par[e] ^= 1;
}

static int64_t xor_weight(void *ctx, const int32_t *partner, int s)
{
    xor_ctx *X = ctx;
    int N = X->g->n_det, nt = 0;
    for (int i = 0; i < s; ++i) {
        int p = partner[i];
        if (p < i) continue;
        int u = X->def[i], v = X->def[p], y;
        if (p == i) {
            int e = X->t->pred[(size_t)u * N + u];
            xor_toggle(X, e, &nt);
            y = X->g->dets[X->g->off[e]];
        } else {
            y = v;
        }
        while (y != u) {
            int e = X->t->pred[(size_t)u * N + y];
            xor_toggle(X, e, &nt);
            int a0 = X->g->dets[X->g->off[e]], a1 = X->g->dets[X->g->off[e] + 1];
            y = (a0 == y) ? a1 : a0;
        }
    }
    int64_t w = 0;
    for (int k = 0; k < nt; ++k) {
        int e = X->touched[k];
        if (X->par[e]) w += X->wfix[e];
        X->par[e] = 0;
    }
    return w;
}

static void *decode_range(void *arg)
{
    job_t *J = arg;
    const or_tables *t = J->t;
    int N = J->g->n_det;
    uint64_t W = (J->n_shots + 63) / 64;
    int32_t *def = malloc(sizeof(int32_t) * (N + 1));
    int32_t *part = malloc(sizeof(int32_t) * (N + 1));
    uint8_t *xpar = NULL; int32_t *xtouched = NULL; int64_t *xw = NULL;
    if (J->o->weight_rule == 1) {
        int M = J->g->n_mech;
        xpar = calloc(M, 1);
        xtouched = malloc(sizeof(int32_t) * M);
        xw = malloc(sizeof(int64_t) * M);
        for (int e = 0; e < M; ++e) xw[e] = or_fixed_weight(J->g->q[e]);
    }
    for (uint64_t b = J->w0 * 64; b < J->w1 * 64 && b < J->n_shots; ++b) {
        int s = 0;
        for (int k = 0; k < N; ++k)
            if ((J->syn[(uint64_t)k * W + (b >> 6)] >> (b & 63)) & 1) def[s++] = k;
        size_t ss = (size_t)s * s;
        double *L = malloc(sizeof(double) * (ss ? ss : 1));
        int64_t *Wt = malloc(sizeof(int64_t) * (ss ? ss : 1));
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) {
                size_t k = (size_t)def[i] * N + def[j];
                L[(size_t)i * s + j] = t->llr[k];
                Wt[(size_t)i * s + j] = t->dist[k];
            }
        int64_t w;
        int fl;
        if (J->o->weight_rule == 1) {
            xor_ctx X = {J->g, t, def, xpar, xtouched, xw};
            fl = or_bp4m_instance_ex(L, Wt, s, J->o, xor_weight, &X, part, &w, NULL, NULL);
        } else {
            fl = or_bp4m_instance(L, Wt, s, J->o, part, &w, NULL, NULL);
        }
        int pred = 0;
        for (int i = 0; i < s; ++i) {
            int p = part[i];
            if (p < i) continue;
            int u = def[i], v = def[p];           /* u <= v */
            pred ^= t->par[(size_t)u * N + v];
            if (J->corr) {
                int y;
                if (p == i) {
                    int e = t->pred[(size_t)u * N + u];
                    toggle(J->corr, W, e, b);
                    y = J->g->dets[J->g->off[e]];
                } else {
                    y = v;
                }
                while (y != u) {
                    int e = t->pred[(size_t)u * N + y];
                    toggle(J->corr, W, e, b);
                    int a0 = J->g->dets[J->g->off[e]];
                    int a1 = J->g->dets[J->g->off[e] + 1];
                    y = (a0 == y) ? a1 : a0;
                }
            }
        }
        int ob = (J->obs[b >> 6] >> (b & 63)) & 1;
        if (pred) fl |= OR_F_PRED;
        if (pred != ob) fl |= OR_F_FAIL;
        J->flags[b] = (uint8_t)fl;
        if (J->s_out) J->s_out[b] = s;
        if (J->partner && s <= J->s_cap)
            for (int i = 0; i < s; ++i) J->partner[b * J->s_cap + i] = part[i];
        free(L); free(Wt);
    }
    free(def); free(part); free(xpar); free(xtouched); free(xw);
    return NULL;
}

int or_decode(const or_dem *g, const or_tables *t, const uint64_t *syn,
              const uint64_t *obs, uint64_t n_shots, const or_opts *o,
              int n_threads, uint8_t *flags, int32_t *s_out, int32_t *partner,
              int32_t s_cap, uint64_t *corr)
{
    if (o->max_iters < 1 || !(o->alpha > 0.0)) return -1;
    uint64_t W = (n_shots + 63) / 64;
    if (corr) memset(corr, 0, sizeof(uint64_t) * W * (uint64_t)g->n_mech);
    if (n_threads < 1) n_threads = 1;
    if ((uint64_t)n_threads > W) n_threads = (int)(W ? W : 1);
    pthread_t *th = malloc(sizeof(pthread_t) * n_threads);
    job_t *jobs = malloc(sizeof(job_t) * n_threads);
    for (int i = 0; i < n_threads; ++i) {
        job_t j = {g, t, syn, obs, n_shots, W * i / n_threads, W * (i + 1) / n_threads,
                   o, flags, s_out, partner, s_cap, corr};
        jobs[i] = j;
        pthread_create(&th[i], NULL, decode_range, &jobs[i]);
    }
    for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    free(th); free(jobs);
    return 0;
}
