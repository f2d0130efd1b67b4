/*
 * Oracle for the BP4M decoding pipeline -- TEST INFRASTRUCTURE ONLY.
 *
 * This is a plain, slow FP64 CPU implementation of what the GPU library
 * computes.  Only tests/, the package smoke check and bench.py's CPU baseline
 * may load it.  It shares no code with the library under
 * paper_2603_05381_amd/ and includes none of its headers.
 *
 * Paper: "Achieving Thresholds via Standalone Belief Propagation on Surface
 * Codes" (arXiv 2603.05381).  Each function cites the passage it follows.
 */
#ifndef BPM_ORACLE_H
#define BPM_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- spec_math.c : FP64 exp / log1p written from textbook methods ---------- */
double or_exp(double x);      /* Cody-Waite reduction + degree-13 Taylor (x <= 709) */
double or_log1p(double y);    /* 2*atanh(y/(2+y)) series, domain y in [0, 1]        */
double or_maxstar(double a, double b); /* Jacobian logarithm, Sec. II.B            */

/* ---- philox.c : Philox4x32-10 (Salmon et al., SC'11) ----------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* ---- codes.c : detector graphs ---------------------------------------------- */
/* A mechanism list in CSR form: mechanism m flips detectors
 * dets[off[m] .. off[m+1]) and the observable iff obs[m]; probability q[m]. */
typedef struct {
    int32_t n_det;
    int32_t n_mech;
    int32_t *off;     /* n_mech + 1 */
    int32_t *dets;    /* off[n_mech] */
    uint8_t *obs;     /* n_mech */
    double  *q;       /* n_mech */
} or_dem;

void or_dem_free(or_dem *g);
/* Code capacity, rotated surface code, Z errors decoded on X checks.        */
int  or_build_code_capacity(int d, double p, or_dem *out);
/* Unrotated surface code, code capacity (d >= 2). */
int  or_build_code_capacity_unrotated(int d, double p, or_dem *out);
/* Circuit-level memory-Z, rotated surface code, R rounds (Sec. III.E).      */
int  or_build_memory_z(int d, int rounds, double p, or_dem *out,
                       int32_t *n_hyper_out, int32_t *n_gauge_bad_out);
/* Circuit-level memory-Z, unrotated surface code (d >= 2), R rounds.        */
int  or_build_memory_z_unrotated(int d, int rounds, double p, or_dem *out,
                                 int32_t *n_hyper_out, int32_t *n_gauge_bad_out);

/* Tanner graph of a code-capacity code with both check types (B-BP4MF,
 * Sec. II.E, III.D): qubit v has X checks qx[2v..2v+1] and Z checks qz[2v..2v+1]
 * (ascending, -1 = none); check c (X checks 0..n_xc-1, then Z checks) has
 * qubits cq[4c..4c+3] (ascending, -1 = none); qobs[v] = a Z error on v flips
 * the observable; qmech[v] = the mechanism of the code-capacity DEM that is
 * v's Z error (same X checks and observable). */
typedef struct {
    int32_t n_q, n_xc, n_zc;
    int32_t *qx, *qz;
    uint8_t *qobs;
    int32_t *qmech;
    int32_t *cq;
} or_tanner;
int  or_build_tanner_code_capacity(int d, int unrotated, const or_dem *dem, or_tanner *t);
void or_tanner_free(or_tanner *t);

/* ---- paths.c : shortest paths and priors ------------------------------------ */
/* Full N x N tables; the diagonal entry [u][u] holds the boundary path of u. */
typedef struct {
    int32_t  n;
    int64_t *dist;     /* fixed-point path weight, 2^-32 units */
    int32_t *hops;
    uint8_t *par;      /* observable parity of the path */
    int32_t *pred;     /* edge id of the last edge of the path */
    double  *llr;      /* prior log-likelihood ratio */
} or_tables;

int  or_build_tables(const or_dem *g, or_tables *t);
/* The same with given fixed-point mechanism weights w[n_mech] instead of
 * round(ln((1-q)/q) 2^32) (llr is still the libm prior of each path). */
int  or_build_tables_w(const or_dem *g, const int64_t *w, or_tables *t);
void or_tables_free(or_tables *t);
int64_t or_fixed_weight(double q);
double  or_prior_llr(int64_t dist_fixed);

/* ---- sample.c ----------------------------------------------------------------- */
uint32_t or_threshold(double q);
void or_sample(const or_dem *g, uint64_t seed, uint64_t shot0, uint64_t n_shots,
               uint64_t *syn, uint64_t *obs, uint64_t *err /* NULL or [n_mech][W] */);

/* ---- bp4m.c ------------------------------------------------------------------- */
typedef struct {
    int32_t max_iters;
    int32_t variant;      /* 0 = BP4M, 1 = BP4MF */
    double  alpha;        /* memory factor; 1 = plain sum-product */
    /* Diagnostic switches for readings of the paper (0 = the reading used
     * everywhere else):
     *  schedule    1: the update indices as printed in Sec. II.B, both message
     *                 types of iteration t+1 formed from those of iteration t
     *  fc_rule     1: forced convergence by the block-maxima procedure of
     *                 Sec. II.D over the partition v_ij -> c_min(i,j); a
     *                 representative whose partner check is already matched
     *                 matches its own check to the boundary
     *  weight_rule 1: a candidate's weight is that of the XOR of its matched
     *                 paths' edge sets (or_decode only) instead of the sum of
     *                 the path weights */
    int32_t schedule;
    int32_t fc_rule;
    int32_t weight_rule;
} or_opts;

/* Per-shot result flags. */
enum {
    OR_F_CONVERGED_ANY = 1,  /* marginalization converged at some iteration */
    OR_F_FC_RAN        = 2,  /* forced convergence was evaluated            */
    OR_F_FC_CHOSEN     = 4,  /* the output is a forced-convergence candidate */
    OR_F_PRED          = 8,  /* predicted observable flip                   */
    OR_F_FAIL          = 16, /* prediction != sampled observable            */
    OR_F_OVERFLOW      = 32, /* more defects than s_cap: not decoded        */
    OR_F_QBP           = 64  /* B-BP4MF: quaternary BP reproduced both syndromes */
};

/* Factor update of one exactly-one factor over s incoming LLRs x[0..s). */
void or_factor_update(const double *x, int s, double *out);
/* Forced convergence on symmetric posteriors lam[s*s] -> partner[s]. */
void or_forced_convergence(const double *lam, int s, int32_t *partner);
/* The block-maxima procedure with conflicts matched to the boundary
 * (or_opts.fc_rule = 1; a diagnostic reading). */
void or_forced_convergence_blocks(const double *lam, int s, int32_t *partner);
/* Marginal hard decision; returns 1 iff every factor has exactly one chosen
 * variable (then partner[] is filled). */
int  or_marginal_decision(const double *lam, int s, int32_t *partner);

/* Candidate bookkeeping of BP4M / BP4MF (Sec. III.A-B), one iteration's
 * posteriors at a time: init, step per iteration, finish (which runs BP4M's
 * final forced convergence when the last iteration did not converge, frees
 * the selector and returns the OR_F_* flags). */
typedef int64_t (*or_weight_fn)(void *ctx, const int32_t *partner, int s);
typedef struct {
    int s, variant, have_best, best_fc, conv_last, flags;
    int fc_rule;                  /* or_opts.fc_rule (0 after init)          */
    or_weight_fn wfn;             /* NULL: sum of W over matched pairs       */
    void *wctx;
    int64_t best_w;
    int32_t *cand, *best;
} or_selector;
void or_selector_init(or_selector *S, int s, int variant);
void or_selector_step(or_selector *S, const double *lam, const int64_t *W);
int  or_selector_finish(or_selector *S, const double *lam_last, const int64_t *W,
                        int32_t *partner, int64_t *weight);
/* The same over a sequence of posteriors lam_seq[T][s][s], T >= 1. */
int  or_select_sequence(const double *lam_seq, int T, int s, const int64_t *W, int variant,
                        int32_t *partner, int64_t *weight);

/* Run BP4M on one instance given its prior matrix L[s*s] (diag = boundary)
 * and integer weights W[s*s].  Outputs: partner[s], flags, best weight,
 * and the final messages M[s*s] and posteriors lam[s*s] (may be NULL). */
int  or_bp4m_instance(const double *L, const int64_t *W, int s, const or_opts *o,
                      int32_t *partner, int64_t *weight, double *M, double *lam);
/* The same with a candidate weight function (NULL: sum of W). */
int  or_bp4m_instance_ex(const double *L, const int64_t *W, int s, const or_opts *o,
                         or_weight_fn wfn, void *wctx,
                         int32_t *partner, int64_t *weight, double *M, double *lam);

/* Decode n_shots shots of syndrome planes with tables t.  Writes per-shot
 * flags, defect counts s, partner lists (s_cap per shot, partner = own index
 * for a boundary match), and optional correction planes corr[n_edges][W]. */
int  or_decode(const or_dem *g, const or_tables *t, const uint64_t *syn,
               const uint64_t *obs, uint64_t n_shots, const or_opts *o,
               int n_threads, uint8_t *flags, int32_t *s_out, int32_t *partner,
               int32_t s_cap, uint64_t *corr);

/* ---- qbp.c : quaternary BP and B-BP4MF, code-capacity depolarizing noise ---- */
double  or_spec_log(double x);           /* fixed-order natural log, x > 0       */
double  or_spec_prior(int64_t dist_fixed); /* -D - log(1 - exp(-D)), own exp/log */
int64_t or_qbp_weight(double P);         /* edge weight from P(Z component)      */
double  or_qbp_zprob(const double *L);   /* P(Z component) from 4 log-posteriors */
void or_sample_depolarizing(const or_tanner *T, double p, uint64_t seed, uint64_t shot0, uint64_t n,
                            uint64_t *synx, uint64_t *synz, uint64_t *obs);
/* Quaternary BP on one shot (syndrome bytes zx[n_xc], zz[n_zc]); returns 1
 * iff the last iteration's hard decision (hard[v] in 0..3 = I, X, Y, Z)
 * reproduced both syndromes; post[4v..4v+3] = its log-posteriors.  stop: end
 * at the first such iteration (B-BP4MF), else run all max_iters. */
int  or_qbp(const or_tanner *T, double p, const uint8_t *zx, const uint8_t *zz, int max_iters,
            int stop, int *iters_out, uint8_t *hard, double *post);
/* B-BP4MF on one shot; returns its OR_F_* flags (partner[] for stage-3
 * shots); stage 3 runs o->variant (1 = BP4MF as in the paper). */
int  or_bbp4mf_shot(const or_dem *g, const or_tanner *T, double p, const uint8_t *zx, const uint8_t *zz,
                    int ob, const or_opts *o, int32_t *s_out, int32_t *partner, int32_t s_cap);
int  or_bbp4mf_decode(const or_dem *g, const or_tanner *T, double p, const uint64_t *synx,
                      const uint64_t *synz, const uint64_t *obs, uint64_t n, const or_opts *o,
                      int n_threads, uint8_t *flags, int32_t *s_out, int32_t *partner, int32_t s_cap);

#ifdef __cplusplus
}
#endif
#endif
