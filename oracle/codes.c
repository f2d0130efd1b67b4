/*
 * Detector error models of the rotated surface code -- TEST INFRASTRUCTURE
 * ONLY (see oracle.h).
 *
 * Layout.  Data qubit (r, c), 0 <= r, c < d, has index r*d + c.  Plaquette
 * (r, c), -1 <= r, c <= d-1, covers the data corners (r,c) (r,c+1) (r+1,c)
 * (r+1,c+1) that exist; it is X-type when r + c is even, Z-type otherwise.
 * All (d-1)^2 interior plaquettes are stabilizers; the weight-2 X plaquettes
 * sit on the top and bottom rows, the weight-2 Z plaquettes on the left and
 * right columns.  Stabilizers of each type are numbered in row-major order of
 * (r, c).
 *
 * Code capacity (Sec. I.B; Sec. III.E): Z errors on the data qubits are seen
 * by the X checks.  A depolarizing channel of strength p flips the Z part of
 * a qubit with probability q = 2p/3.  One mechanism per data qubit, in qubit
 * order; it flips the observable (overlap with the X logical on column 0)
 * when the qubit is in column 0.
 *
 * Unrotated code, code capacity: the X checks form a (d-1) x d grid of
 * vertices (i, j) (index i*d + j).  Data qubits are its edges: d "vertical"
 * edges per column j joining (i-1, j) and (i, j) for i = 0..d-1, where row
 * -1 (top) and row d-1 (bottom) stand for the boundary, and (d-1)^2
 * "horizontal" edges joining (i, j) and (i, j+1).  The X logical crosses
 * every column once, through the top boundary edges, which therefore flip
 * the observable.  Mechanisms are sorted by (detector tuple, observable).
 *
 * Circuit level (Sec. III.E): a memory-Z experiment of R rounds with
 * depolarizing noise after every Clifford gate and on the data before each
 * round, and flips after resets and before measurements, all of strength p.
 * The detectors are the Z stabilizers of every round plus the final data
 * readout; the observable is the Z logical on data row 0.  The unrotated
 * code runs the same round on its own grid (or_build_memory_z_unrotated):
 * CNOT layers N, W, E, S for X stabilizers and N, E, W, S for Z
 * stabilizers, observable on data column 0.  The oracle finds
 * each fault's detectors by propagating Pauli frames FORWARD through the
 * circuit, all fault generators at once as bit columns.  A channel becomes
 * independent mechanisms that reproduce its outcome distribution exactly:
 * each of the 3 (1-qubit) or 15 (2-qubit) non-identity Paulis fires
 * independently with q where (1-2q) = sqrt(1 - 4p/3), resp.
 * (1-2q)^8 = 1 - 16p/15; an X flip fires with p.  Outcomes with the same
 * detectors and observable are merged by XOR of independent events:
 * 1 - 2q_merged = product of (1 - 2q_i), multiplied class by class
 * (X flips, then 1-qubit, then 2-qubit terms).  Mechanisms are sorted by
 * (detector tuple, observable) in lexicographic order.
 */
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include "oracle.h"

/* (detector tuple, observable) order of mechanisms a and b, given each one's
 * detectors as a sorted pair (second = -1 if only one). */
static int mech_cmp(const int32_t *a, int oa, const int32_t *b, int ob)
{
    for (int k = 0; k < 2; ++k) {
        if (a[k] == b[k]) continue;
        if (a[k] < 0) return -1;              /* a shorter tuple first */
        if (b[k] < 0) return 1;
        return a[k] < b[k] ? -1 : 1;
    }
    return oa - ob;
}

int or_build_code_capacity_unrotated(int d, double p, or_dem *out)
{
    if (d < 2 || !(p > 0.0) || p >= 0.75) return -1;
    memset(out, 0, sizeof(*out));
    const int nq = d * d + (d - 1) * (d - 1);
    int32_t (*pair)[2] = malloc(sizeof(int32_t) * 2 * nq);
    int *ob = malloc(sizeof(int) * nq);
    int m = 0;
    for (int j = 0; j < d; ++j)                   /* vertical edges */
        for (int i = 0; i < d; ++i) {
            int a = i - 1, b = i;                 /* vertex rows joined */
            int u = (a >= 0) ? a * d + j : -1, v = (b <= d - 2) ? b * d + j : -1;
            if (u < 0) { u = v; v = -1; }
            pair[m][0] = u; pair[m][1] = v;
            ob[m] = (i == 0);                     /* top boundary edge */
            ++m;
        }
    for (int i = 0; i < d - 1; ++i)               /* horizontal edges */
        for (int j = 0; j + 1 < d; ++j) {
            pair[m][0] = i * d + j; pair[m][1] = i * d + j + 1;
            ob[m] = 0;
            ++m;
        }
    /* insertion sort into canonical order */
    for (int x = 1; x < nq; ++x) {
        int32_t t0 = pair[x][0], t1 = pair[x][1];
        int to = ob[x], y = x - 1;
        int32_t key[2] = {t0, t1};
        while (y >= 0 && mech_cmp(pair[y], ob[y], key, to) > 0) {
            pair[y + 1][0] = pair[y][0]; pair[y + 1][1] = pair[y][1]; ob[y + 1] = ob[y];
            --y;
        }
        pair[y + 1][0] = t0; pair[y + 1][1] = t1; ob[y + 1] = to;
    }
    out->n_det = d * (d - 1);
    out->n_mech = nq;
    out->off = malloc(sizeof(int32_t) * (nq + 1));
    out->dets = malloc(sizeof(int32_t) * 2 * nq);
    out->obs = malloc(nq);
    out->q = malloc(sizeof(double) * nq);
    int n = 0;
    for (int k = 0; k < nq; ++k) {
        out->off[k] = n;
        out->dets[n++] = pair[k][0];
        if (pair[k][1] >= 0) out->dets[n++] = pair[k][1];
        out->obs[k] = (uint8_t)ob[k];
        out->q[k] = (2.0 * p) / 3.0;
    }
    out->off[nq] = n;
    free(pair);
    free(ob);
    return 0;
}

void or_dem_free(or_dem *g)
{
    free(g->off); free(g->dets); free(g->obs); free(g->q);
    memset(g, 0, sizeof(*g));
}

static int is_x_type(int r, int c) { return ((r + c) & 1) == 0; }

/* Is plaquette (r, c) a stabilizer of the given type (1 = X, 0 = Z)? */
static int plaquette_valid(int d, int r, int c, int want_x)
{
    if (r < -1 || r > d - 1 || c < -1 || c > d - 1) return 0;
    int x = is_x_type(r, c);
    if (x != want_x) return 0;
    int rb = (r == -1 || r == d - 1), cb = (c == -1 || c == d - 1);
    if (rb && cb) return 0;                 /* corners are never stabilizers   */
    if (!rb && !cb) return 1;               /* interior                         */
    if (rb) return want_x;                  /* top/bottom rows hold X checks    */
    return !want_x;                         /* left/right columns hold Z checks */
}

/* Index of plaquette (r, c) among the stabilizers of its type, or -1. */
static int plaquette_index(int d, int r, int c, int want_x)
{
    if (!plaquette_valid(d, r, c, want_x)) return -1;
    int idx = 0;
    for (int rr = -1; rr <= d - 1; ++rr)
        for (int cc = -1; cc <= d - 1; ++cc) {
            if (rr == r && cc == c) return idx;
            if (plaquette_valid(d, rr, cc, want_x)) ++idx;
        }
    return -1;
}

int or_build_code_capacity(int d, double p, or_dem *out)
{
    if (d < 3 || (d & 1) == 0 || !(p > 0.0) || p >= 0.75) return -1;
    memset(out, 0, sizeof(*out));
    int nq = d * d;
    out->n_det = (d * d - 1) / 2;
    out->n_mech = nq;
    out->off = malloc(sizeof(int32_t) * (nq + 1));
    out->dets = malloc(sizeof(int32_t) * 2 * nq);
    out->obs = malloc(nq);
    out->q = malloc(sizeof(double) * nq);
    double q = (2.0 * p) / 3.0;
    int n = 0;
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c) {
            int m = r * d + c;
            out->off[m] = n;
            int cand[4][2] = {{r - 1, c - 1}, {r - 1, c}, {r, c - 1}, {r, c}};
            int found[4], nf = 0;
            for (int k = 0; k < 4; ++k) {
                int id = plaquette_index(d, cand[k][0], cand[k][1], 1);
                if (id >= 0) found[nf++] = id;
            }
            /* ascending order */
            for (int a = 0; a < nf; ++a)
                for (int b = a + 1; b < nf; ++b)
                    if (found[b] < found[a]) { int t = found[a]; found[a] = found[b]; found[b] = t; }
            for (int k = 0; k < nf; ++k) out->dets[n++] = found[k];
            out->obs[m] = (c == 0);
            out->q[m] = q;
        }
    out->off[nq] = n;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Circuit-level memory-Z                                                     */
/* ------------------------------------------------------------------------- */

enum { OP_R, OP_H, OP_CX, OP_M, OP_DEP1, OP_DEP2, OP_XERR };
typedef struct { int kind, a, b; } op_t;

typedef struct { op_t *v; int n, cap; } oplist;
static void push(oplist *L, int kind, int a, int b)
{
    if (L->n == L->cap) { L->cap = L->cap ? 2 * L->cap : 1024; L->v = realloc(L->v, sizeof(op_t) * L->cap); }
    L->v[L->n].kind = kind; L->v[L->n].a = a; L->v[L->n].b = b; L->n++;
}

/* bitset rows */
typedef uint64_t word;

typedef struct { int32_t *d; int n; uint8_t obs; uint8_t cls; } contrib;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Lexicographic comparison of (detector tuple, observable). */
static int cmp_sym(const int32_t *a, int na, int oa, const int32_t *b, int nb, int ob)
{
    int n = na < nb ? na : nb;
    for (int i = 0; i < n; ++i)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    if (na != nb) return na < nb ? -1 : 1;
    return (oa > ob) - (oa < ob);
}

static int cmp_contrib(const void *pa, const void *pb)
{
    const contrib *a = pa, *b = pb;
    return cmp_sym(a->d, a->n, a->obs, b->d, b->n, b->obs);
}

/* Qubits and CNOT schedule of one memory-Z round: data 0..nd-1, then the X
 * ancillas, then the Z ancillas.  In CNOT layer k, X stabilizer i is the
 * control of a CNOT onto data xc[4*i+k] and Z stabilizer i the target of one
 * from data zc[4*i+k] (-1: none).  zsup[4*i..] (zsup_n[i] entries) is Z
 * stabilizer i's support; obsq[0..nobs) the data read into the observable. */
typedef struct {
    int nd, nx, nz;
    int *xc, *zc, *zsup, *zsup_n, *obsq, nobs;
} mem_layout;

static void layout_alloc(mem_layout *Y, int nd, int nx, int nz, int nobs)
{
    Y->nd = nd; Y->nx = nx; Y->nz = nz; Y->nobs = nobs;
    Y->xc = malloc(sizeof(int) * 4 * (nx + 1));
    Y->zc = malloc(sizeof(int) * 4 * (nz + 1));
    Y->zsup = malloc(sizeof(int) * 4 * (nz + 1));
    Y->zsup_n = calloc(nz + 1, sizeof(int));
    Y->obsq = malloc(sizeof(int) * (nobs + 1));
}

static void layout_free(mem_layout *Y)
{
    free(Y->xc); free(Y->zc); free(Y->zsup); free(Y->zsup_n); free(Y->obsq);
}

static int memory_circuit(const mem_layout *Y, int rounds, double p, or_dem *out,
                          int32_t *n_hyper_out, int32_t *n_gauge_bad_out);

int or_build_memory_z(int d, int rounds, double p, or_dem *out,
                      int32_t *n_hyper_out, int32_t *n_gauge_bad_out)
{
    if (d < 3 || (d & 1) == 0 || rounds < 1 || !(p > 0.0) || p >= 0.5) return -1;

    /* stabilizer plaquettes */
    int nx = 0, nz = 0;
    int (*xs)[2] = malloc(sizeof(int[2]) * (d + 1) * (d + 1));
    int (*zs)[2] = malloc(sizeof(int[2]) * (d + 1) * (d + 1));
    for (int r = -1; r <= d - 1; ++r)
        for (int c = -1; c <= d - 1; ++c) {
            if (plaquette_valid(d, r, c, 1)) { xs[nx][0] = r; xs[nx][1] = c; nx++; }
            if (plaquette_valid(d, r, c, 0)) { zs[nz][0] = r; zs[nz][1] = c; nz++; }
        }
    mem_layout Y;
    layout_alloc(&Y, d * d, nx, nz, d);
    /* corner order per layer: X checks TL, TR, BL, BR; Z checks TL, BL, TR, BR */
    const int xo[4][2] = {{0, 0}, {0, 1}, {1, 0}, {1, 1}};
    const int zo[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
    for (int i = 0; i < nx; ++i)
        for (int k = 0; k < 4; ++k) {
            int r = xs[i][0] + xo[k][0], c = xs[i][1] + xo[k][1];
            Y.xc[4 * i + k] = (r < 0 || r >= d || c < 0 || c >= d) ? -1 : r * d + c;
        }
    for (int i = 0; i < nz; ++i)
        for (int k = 0; k < 4; ++k) {
            int r = zs[i][0] + zo[k][0], c = zs[i][1] + zo[k][1];
            int q = (r < 0 || r >= d || c < 0 || c >= d) ? -1 : r * d + c;
            Y.zc[4 * i + k] = q;
            if (q >= 0) Y.zsup[4 * i + Y.zsup_n[i]++] = q;
        }
    for (int c = 0; c < d; ++c) Y.obsq[c] = c;          /* Z logical: data row 0 */
    int rc = memory_circuit(&Y, rounds, p, out, n_hyper_out, n_gauge_bad_out);
    layout_free(&Y);
    free(xs); free(zs);
    return rc;
}

/* Unrotated code: on the (2d-1) x (2d-1) grid, data at r + c even (row-major
 * numbering), X stabilizers at (odd, even), Z stabilizers at (even, odd),
 * each numbered row-major.  Layers visit the neighbours N, W, E, S (X) and
 * N, E, W, S (Z).  Observable: Z readout of the data of column 0. */
static int unrot_data(int d, int r, int c)
{
    int n = 2 * d - 1;
    if (r < 0 || r >= n || c < 0 || c >= n || ((r + c) & 1)) return -1;
    int before = 0;
    for (int rr = 0; rr < r; ++rr) before += (rr & 1) ? d - 1 : d;
    return before + c / 2;                    /* c / 2 == (c - 1) / 2 on odd rows */
}

int or_build_memory_z_unrotated(int d, int rounds, double p, or_dem *out,
                                int32_t *n_hyper_out, int32_t *n_gauge_bad_out)
{
    if (d < 2 || rounds < 1 || !(p > 0.0) || p >= 0.5) return -1;
    const int n = 2 * d - 1;
    const int xn[4][2] = {{-1, 0}, {0, -1}, {0, 1}, {1, 0}};    /* N W E S */
    const int zn[4][2] = {{-1, 0}, {0, 1}, {0, -1}, {1, 0}};    /* N E W S */
    mem_layout Y;
    layout_alloc(&Y, d * d + (d - 1) * (d - 1), d * (d - 1), d * (d - 1), d);
    int i = 0;
    for (int r = 1; r < n; r += 2)
        for (int c = 0; c < n; c += 2, ++i)
            for (int k = 0; k < 4; ++k) Y.xc[4 * i + k] = unrot_data(d, r + xn[k][0], c + xn[k][1]);
    i = 0;
    for (int r = 0; r < n; r += 2)
        for (int c = 1; c < n; c += 2, ++i)
            for (int k = 0; k < 4; ++k) {
                int q = unrot_data(d, r + zn[k][0], c + zn[k][1]);
                Y.zc[4 * i + k] = q;
                if (q >= 0) Y.zsup[4 * i + Y.zsup_n[i]++] = q;
            }
    for (int a = 0; a < d; ++a) Y.obsq[a] = unrot_data(d, 2 * a, 0);
    int rc = memory_circuit(&Y, rounds, p, out, n_hyper_out, n_gauge_bad_out);
    layout_free(&Y);
    return rc;
}

/* Reset everything (X flip p), then per round: depolarize the data, H on the
 * X ancillas (+depolarize), four CNOT layers (each followed by two-qubit
 * depolarizing noise), H on the X ancillas (+depolarize), flip-measure-
 * reset-flip the ancillas; finally flip and measure the data.  Detectors: Z
 * stabilizers per round (vs. the previous round) and at the final readout.
 * Symptoms by forward propagation of one generator per noise component. */
static int memory_circuit(const mem_layout *Y, int rounds, double p, or_dem *out,
                          int32_t *n_hyper_out, int32_t *n_gauge_bad_out)
{
    memset(out, 0, sizeof(*out));
    const int nd = Y->nd, nx = Y->nx, nz = Y->nz;
    int nq = nd + nx + nz;               /* data, X ancillas, Z ancillas */

    /* ---- circuit ---- */
    oplist C = {0};
    int n_meas = 0;
    for (int q = 0; q < nd; ++q) { push(&C, OP_R, q, 0); push(&C, OP_XERR, q, 0); }
    for (int q = nd; q < nq; ++q) { push(&C, OP_R, q, 0); push(&C, OP_XERR, q, 0); }
    int *zmeas = malloc(sizeof(int) * (size_t)rounds * nz);   /* record index */
    int (*pairs)[2] = malloc(sizeof(int[2]) * (nx + nz + 1));
    for (int t = 0; t < rounds; ++t) {
        for (int q = 0; q < nd; ++q) push(&C, OP_DEP1, q, 0);
        for (int i = 0; i < nx; ++i) { push(&C, OP_H, nd + i, 0); push(&C, OP_DEP1, nd + i, 0); }
        for (int k = 0; k < 4; ++k) {
            int np = 0;
            for (int i = 0; i < nx; ++i) {
                int q = Y->xc[4 * i + k];
                if (q < 0) continue;
                pairs[np][0] = nd + i; pairs[np][1] = q; np++;
            }
            for (int i = 0; i < nz; ++i) {
                int q = Y->zc[4 * i + k];
                if (q < 0) continue;
                pairs[np][0] = q; pairs[np][1] = nd + nx + i; np++;
            }
            for (int j = 0; j < np; ++j) push(&C, OP_CX, pairs[j][0], pairs[j][1]);
            for (int j = 0; j < np; ++j) push(&C, OP_DEP2, pairs[j][0], pairs[j][1]);
        }
        for (int i = 0; i < nx; ++i) { push(&C, OP_H, nd + i, 0); push(&C, OP_DEP1, nd + i, 0); }
        for (int q = nd; q < nq; ++q) push(&C, OP_XERR, q, 0);
        for (int q = nd; q < nq; ++q) {
            if (q >= nd + nx) zmeas[t * nz + (q - nd - nx)] = n_meas;
            push(&C, OP_M, q, n_meas++);
        }
        for (int q = nd; q < nq; ++q) { push(&C, OP_R, q, 0); push(&C, OP_XERR, q, 0); }
    }
    free(pairs);
    for (int q = 0; q < nd; ++q) push(&C, OP_XERR, q, 0);
    int *dmeas = malloc(sizeof(int) * nd);
    for (int q = 0; q < nd; ++q) { dmeas[q] = n_meas; push(&C, OP_M, q, n_meas++); }

    /* ---- generators: per noise op, the X and Z generators of its qubits;
     *      gauge generators: Z after every reset and every measurement ---- */
    int n_gen = 0;
    for (int i = 0; i < C.n; ++i) {
        switch (C.v[i].kind) {
        case OP_DEP1: n_gen += 2; break;
        case OP_DEP2: n_gen += 4; break;
        case OP_XERR: n_gen += 1; break;
        case OP_R: case OP_M: n_gen += 1; break;
        default: break;
        }
    }
    int W = (n_gen + 63) / 64;
    word *fx = calloc((size_t)nq * W, sizeof(word));
    word *fz = calloc((size_t)nq * W, sizeof(word));
    word *rec = calloc((size_t)n_meas * W, sizeof(word));
    int *gen_op = malloc(sizeof(int) * n_gen);   /* op index of each generator */
    int g = 0;
#define SETBIT(row, gi) ((row)[(gi) >> 6] |= (word)1 << ((gi) & 63))
    for (int i = 0; i < C.n; ++i) {
        op_t o = C.v[i];
        switch (o.kind) {
        case OP_R:
            memset(fx + (size_t)o.a * W, 0, sizeof(word) * W);
            memset(fz + (size_t)o.a * W, 0, sizeof(word) * W);
            gen_op[g] = i; SETBIT(fz + (size_t)o.a * W, g); g++;
            break;
        case OP_H: {
            word *x = fx + (size_t)o.a * W, *z = fz + (size_t)o.a * W;
            for (int w = 0; w < W; ++w) { word t = x[w]; x[w] = z[w]; z[w] = t; }
            break; }
        case OP_CX: {
            word *xc = fx + (size_t)o.a * W, *xt = fx + (size_t)o.b * W;
            word *zc = fz + (size_t)o.a * W, *zt = fz + (size_t)o.b * W;
            for (int w = 0; w < W; ++w) { xt[w] ^= xc[w]; zc[w] ^= zt[w]; }
            break; }
        case OP_M:
            memcpy(rec + (size_t)o.b * W, fx + (size_t)o.a * W, sizeof(word) * W);
            gen_op[g] = i; SETBIT(fz + (size_t)o.a * W, g); g++;
            break;
        case OP_DEP1:
            gen_op[g] = i; SETBIT(fx + (size_t)o.a * W, g); g++;
            gen_op[g] = i; SETBIT(fz + (size_t)o.a * W, g); g++;
            break;
        case OP_DEP2:
            gen_op[g] = i; SETBIT(fx + (size_t)o.a * W, g); g++;
            gen_op[g] = i; SETBIT(fz + (size_t)o.a * W, g); g++;
            gen_op[g] = i; SETBIT(fx + (size_t)o.b * W, g); g++;
            gen_op[g] = i; SETBIT(fz + (size_t)o.b * W, g); g++;
            break;
        case OP_XERR:
            gen_op[g] = i; SETBIT(fx + (size_t)o.a * W, g); g++;
            break;
        }
    }

    /* ---- detectors and observable as rows over generators ---- */
    int n_det = (rounds + 1) * nz;
    word *det = calloc((size_t)(n_det + 1) * W, sizeof(word));   /* last row = observable */
    for (int t = 0; t <= rounds; ++t)
        for (int i = 0; i < nz; ++i) {
            word *row = det + (size_t)(t * nz + i) * W;
            if (t < rounds) {
                const word *a = rec + (size_t)zmeas[t * nz + i] * W;
                for (int w = 0; w < W; ++w) row[w] ^= a[w];
                if (t > 0) {
                    const word *b = rec + (size_t)zmeas[(t - 1) * nz + i] * W;
                    for (int w = 0; w < W; ++w) row[w] ^= b[w];
                }
            } else {
                const word *a = rec + (size_t)zmeas[(rounds - 1) * nz + i] * W;
                for (int w = 0; w < W; ++w) row[w] ^= a[w];
                for (int k = 0; k < Y->zsup_n[i]; ++k) {
                    const word *b = rec + (size_t)dmeas[Y->zsup[4 * i + k]] * W;
                    for (int w = 0; w < W; ++w) row[w] ^= b[w];
                }
            }
        }
    {
        word *row = det + (size_t)n_det * W;
        for (int k = 0; k < Y->nobs; ++k) {
            const word *b = rec + (size_t)dmeas[Y->obsq[k]] * W;
            for (int w = 0; w < W; ++w) row[w] ^= b[w];
        }
    }

    /* ---- per-generator symptoms (transpose) ---- */
    int *gcount = calloc(n_gen, sizeof(int));
    uint8_t *gobs = calloc(n_gen, 1);
    for (int k = 0; k < n_det; ++k) {
        const word *row = det + (size_t)k * W;
        for (int gi = 0; gi < n_gen; ++gi)
            if ((row[gi >> 6] >> (gi & 63)) & 1) gcount[gi]++;
    }
    for (int gi = 0; gi < n_gen; ++gi)
        gobs[gi] = (det[(size_t)n_det * W + (gi >> 6)] >> (gi & 63)) & 1;
    int *goff = malloc(sizeof(int) * (n_gen + 1));
    goff[0] = 0;
    for (int gi = 0; gi < n_gen; ++gi) goff[gi + 1] = goff[gi] + gcount[gi];
    int32_t *gdet = malloc(sizeof(int32_t) * (goff[n_gen] + 1));
    int *fill = calloc(n_gen, sizeof(int));
    for (int k = 0; k < n_det; ++k) {                    /* ascending k => sorted lists */
        const word *row = det + (size_t)k * W;
        for (int gi = 0; gi < n_gen; ++gi)
            if ((row[gi >> 6] >> (gi & 63)) & 1) gdet[goff[gi] + fill[gi]++] = k;
    }

    /* ---- gauge check: Z after reset / measurement must flip nothing ---- */
    int gauge_bad = 0;
    for (int gi = 0; gi < n_gen; ++gi) {
        int kind = C.v[gen_op[gi]].kind;
        if ((kind == OP_R || kind == OP_M) && (gcount[gi] || gobs[gi])) gauge_bad++;
    }

    /* ---- channel outcomes -> contributions ---- */
    int cap = 0;
    for (int i = 0; i < C.n; ++i) {
        int kd = C.v[i].kind;
        cap += kd == OP_DEP1 ? 3 : kd == OP_DEP2 ? 15 : kd == OP_XERR ? 1 : 0;
    }
    contrib *cs = malloc(sizeof(contrib) * (cap + 1));
    int ncs = 0;
    int32_t *tmp = malloc(sizeof(int32_t) * (4 * (size_t)n_det + 8));
    g = 0;
    for (int i = 0; i < C.n; ++i) {
        int kd = C.v[i].kind;
        int ng = kd == OP_DEP1 ? 2 : kd == OP_DEP2 ? 4 : kd == OP_XERR ? 1 : (kd == OP_R || kd == OP_M) ? 1 : 0;
        if (kd == OP_DEP1 || kd == OP_DEP2 || kd == OP_XERR) {
            int cls = kd == OP_XERR ? 0 : kd == OP_DEP1 ? 1 : 2;
            int nout = kd == OP_XERR ? 1 : kd == OP_DEP1 ? 3 : 15;
            for (int mask = 1; mask <= nout; ++mask) {
                /* outcome = XOR of the generators selected by mask's bits */
                int n = 0, ob = 0;
                for (int b = 0; b < ng; ++b) {
                    if (!((mask >> b) & 1)) continue;
                    int gi = g + b;
                    for (int e = goff[gi]; e < goff[gi + 1]; ++e) tmp[n++] = gdet[e];
                    ob ^= gobs[gi];
                }
                qsort(tmp, n, sizeof(int32_t), cmp_i32);
                int m = 0;   /* cancel pairs */
                for (int e = 0; e < n; ) {
                    if (e + 1 < n && tmp[e] == tmp[e + 1]) { e += 2; continue; }
                    tmp[m++] = tmp[e++];
                }
                if (m == 0 && ob == 0) continue;
                cs[ncs].d = malloc(sizeof(int32_t) * (m ? m : 1));
                memcpy(cs[ncs].d, tmp, sizeof(int32_t) * m);
                cs[ncs].n = m; cs[ncs].obs = (uint8_t)ob; cs[ncs].cls = (uint8_t)cls;
                ncs++;
            }
        }
        g += ng;
    }
    qsort(cs, ncs, sizeof(contrib), cmp_contrib);

    /* ---- merge ---- */
    double fX = 1.0 - 2.0 * p;
    double f1 = sqrt(1.0 - (4.0 * p) / 3.0);
    double f2 = sqrt(sqrt(sqrt(1.0 - (16.0 * p) / 15.0)));
    int nm = 0, total_dets = 0;
    for (int i = 0; i < ncs; ) {
        int j = i;
        while (j < ncs && cmp_contrib(&cs[i], &cs[j]) == 0) ++j;
        nm++; total_dets += cs[i].n; i = j;
    }
    out->n_det = n_det;
    out->n_mech = nm;
    out->off = malloc(sizeof(int32_t) * (nm + 1));
    out->dets = malloc(sizeof(int32_t) * (total_dets + 1));
    out->obs = malloc(nm + 1);
    out->q = malloc(sizeof(double) * (nm + 1));
    int n_hyper = 0, m = 0, nd_out = 0;
    for (int i = 0; i < ncs; ) {
        int j = i, cnt[3] = {0, 0, 0};
        while (j < ncs && cmp_contrib(&cs[i], &cs[j]) == 0) { cnt[cs[j].cls]++; ++j; }
        double y = 1.0;
        for (int k = 0; k < cnt[0]; ++k) y *= fX;
        for (int k = 0; k < cnt[1]; ++k) y *= f1;
        for (int k = 0; k < cnt[2]; ++k) y *= f2;
        out->off[m] = nd_out;
        memcpy(out->dets + nd_out, cs[i].d, sizeof(int32_t) * cs[i].n);
        nd_out += cs[i].n;
        out->obs[m] = cs[i].obs;
        out->q[m] = 0.5 * (1.0 - y);
        if (cs[i].n > 2 || cs[i].n == 0) n_hyper++;
        m++; i = j;
    }
    out->off[nm] = nd_out;

    if (n_hyper_out) *n_hyper_out = n_hyper;
    if (n_gauge_bad_out) *n_gauge_bad_out = gauge_bad;

    for (int i = 0; i < ncs; ++i) free(cs[i].d);
    free(cs); free(tmp); free(goff); free(gdet); free(fill); free(gcount); free(gobs);
    free(det); free(rec); free(fx); free(fz); free(gen_op); free(dmeas); free(zmeas);
    free(C.v);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Tanner graphs of the code-capacity codes (both check types)               */
/* ------------------------------------------------------------------------- */

void or_tanner_free(or_tanner *t)
{
    free(t->qx); free(t->qz); free(t->qobs); free(t->qmech); free(t->cq);
    memset(t, 0, sizeof(*t));
}

/* Append check id to a qubit's list of up to 2 (kept ascending). */
static void add_check(int32_t *list, int id)
{
    if (list[0] < 0) { list[0] = id; return; }
    if (list[1] >= 0) return;                       /* never more than two */
    if (id < list[0]) { list[1] = list[0]; list[0] = id; }
    else list[1] = id;
}

int or_build_tanner_code_capacity(int d, int unrotated, const or_dem *dem, or_tanner *t)
{
    memset(t, 0, sizeof(*t));
    int nq, nxc, nzc;
    if (unrotated) {
        if (d < 2) return -1;
        nq = d * d + (d - 1) * (d - 1); nxc = d * (d - 1); nzc = d * (d - 1);
    } else {
        if (d < 3 || (d & 1) == 0) return -1;
        nq = d * d; nxc = (d * d - 1) / 2; nzc = (d * d - 1) / 2;
    }
    if (dem->n_det != nxc || dem->n_mech != nq) return -2;
    t->n_q = nq; t->n_xc = nxc; t->n_zc = nzc;
    t->qx = malloc(sizeof(int32_t) * 2 * nq);
    t->qz = malloc(sizeof(int32_t) * 2 * nq);
    t->qobs = calloc(nq, 1);
    t->qmech = malloc(sizeof(int32_t) * nq);
    t->cq = malloc(sizeof(int32_t) * 4 * (nxc + nzc));
    for (int i = 0; i < 2 * nq; ++i) { t->qx[i] = -1; t->qz[i] = -1; }
    for (int i = 0; i < 4 * (nxc + nzc); ++i) t->cq[i] = -1;
    if (unrotated) {
        const int n = 2 * d - 1;
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
                if ((r + c) & 1) continue;
                int v = unrot_data(d, r, c);
                const int nb[4][2] = {{r - 1, c}, {r + 1, c}, {r, c - 1}, {r, c + 1}};
                for (int k = 0; k < 4; ++k) {
                    int a = nb[k][0], b = nb[k][1];
                    if (a < 0 || a >= n || b < 0 || b >= n) continue;
                    if ((a & 1) && !(b & 1)) add_check(t->qx + 2 * v, ((a - 1) / 2) * d + b / 2);
                    if (!(a & 1) && (b & 1)) add_check(t->qz + 2 * v, (a / 2) * (d - 1) + (b - 1) / 2);
                }
                t->qobs[v] = r == 0;                 /* X logical on data row 0 */
            }
    } else {
        for (int r = 0; r < d; ++r)
            for (int c = 0; c < d; ++c) {
                int v = r * d + c;
                for (int a = r - 1; a <= r; ++a)
                    for (int b = c - 1; b <= c; ++b) {
                        int ix = plaquette_index(d, a, b, 1), iz = plaquette_index(d, a, b, 0);
                        if (ix >= 0) add_check(t->qx + 2 * v, ix);
                        if (iz >= 0) add_check(t->qz + 2 * v, iz);
                    }
                t->qobs[v] = c == 0;                 /* X logical on data column 0 */
            }
    }
    /* checks' qubit lists, ascending by qubit */
    int *fill = calloc(nxc + nzc, sizeof(int));
    for (int v = 0; v < nq; ++v)
        for (int k = 0; k < 2; ++k) {
            int x = t->qx[2 * v + k], z = t->qz[2 * v + k];
            if (x >= 0) t->cq[4 * x + fill[x]++] = v;
            if (z >= 0) t->cq[4 * (nxc + z) + fill[nxc + z]++] = v;
        }
    free(fill);
    /* the DEM mechanism of each qubit's Z error: same X checks and observable
     * (the rotated code lists its mechanisms in qubit order, and there two
     * boundary qubits of the same check can be parallel edges; the unrotated
     * code's edges are all distinct) */
    for (int v = 0; v < nq; ++v) {
        int32_t want[2]; int nw = 0;
        for (int k = 0; k < 2; ++k) if (t->qx[2 * v + k] >= 0) want[nw++] = t->qx[2 * v + k];
        int found = -1;
        for (int m = unrotated ? 0 : v; m < (unrotated ? nq : v + 1); ++m) {
            int k0 = dem->off[m], k1 = dem->off[m + 1];
            if (k1 - k0 != nw || dem->obs[m] != t->qobs[v]) continue;
            int same = 1;
            for (int k = 0; k < nw; ++k) same &= dem->dets[k0 + k] == want[k];
            if (same) { if (found >= 0) { or_tanner_free(t); return -3; } found = m; }
        }
        if (found < 0) { or_tanner_free(t); return -4; }
        t->qmech[v] = found;
    }
    return 0;
}
