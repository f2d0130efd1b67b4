/*
 * Shortest paths and priors on the detector graph -- TEST INFRASTRUCTURE
 * ONLY (see oracle.h).
 *
 * The decoding-graph weight w_ij of a pair of defects is the weight of the
 * lowest-weight error that joins them; w_ii joins defect i to the boundary
 * (Fig. 1 caption; Sec. II.A after the prior equation).  With per-mechanism
 * probabilities q_e the weight of a path is the sum of W_e = ln((1-q_e)/q_e),
 * and the prior of the decoding-graph edge is rho(1) = exp(-D) for path
 * weight D, which is (p/(1-p))^w when all q_e are equal.  Its log-likelihood
 * ratio (Sec. II.B, prior LLR) is  l = ln(rho(1)/rho(0)) = -D - ln(1 - exp(-D)).
 *
 * Conventions fixed here (the paper does not state them):
 *  - W_e is stored in fixed point, round(W_e * 2^32), so path sums are exact
 *    integers and ties are exact.
 *  - The boundary is a sink: a path may end at it but never passes through
 *    it (Sec. II.E prefers the graph that keeps boundary-crossing paths out).
 *  - Among equal-weight paths the one with fewer edges wins; among those the
 *    predecessor is the smallest (node, edge id) that attains the optimum.
 *  - Entry [u][v] is computed from source u; the decoder reads pairs as
 *    [min][max].  Entry [u][u] holds the path from u to the boundary.
 *
 * The search is Dijkstra's algorithm with a binary heap on (weight, hops).
 */
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include "oracle.h"

int64_t or_fixed_weight(double q)
{
    double w = log((1.0 - q) / q);
    int64_t f = (int64_t)llround(w * 4294967296.0);
    return f < 1 ? 1 : f;
}

double or_prior_llr(int64_t dist_fixed)
{
    double D = ldexp((double)dist_fixed, -32);
    double e = exp(-D);
    double t = log1p(-e);
    return (-D) - t;
}

typedef struct { int64_t w; int32_t h; int32_t v; } hitem;

static int hless(const hitem *a, const hitem *b)
{
    if (a->w != b->w) return a->w < b->w;
    if (a->h != b->h) return a->h < b->h;
    return a->v < b->v;
}

static void hpush(hitem *H, int *n, hitem x)
{
    int i = (*n)++;
    H[i] = x;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (!hless(&H[i], &H[p])) break;
        hitem t = H[i]; H[i] = H[p]; H[p] = t; i = p;
    }
}

static hitem hpop(hitem *H, int *n)
{
    hitem top = H[0];
    H[0] = H[--(*n)];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, s = i;
        if (l < *n && hless(&H[l], &H[s])) s = l;
        if (r < *n && hless(&H[r], &H[s])) s = r;
        if (s == i) break;
        hitem t = H[i]; H[i] = H[s]; H[s] = t; i = s;
    }
    return top;
}

void or_tables_free(or_tables *t)
{
    free(t->dist); free(t->hops); free(t->par); free(t->pred); free(t->llr);
    memset(t, 0, sizeof(*t));
}

int or_build_tables(const or_dem *g, or_tables *t)
{
    return or_build_tables_w(g, NULL, t);
}

int or_build_tables_w(const or_dem *g, const int64_t *w, or_tables *t)
{
    int N = g->n_det, B = N;
    memset(t, 0, sizeof(*t));
    /* edges: every mechanism must be graphlike (1 or 2 detectors) */
    int E = g->n_mech;
    int *eu = malloc(sizeof(int) * E), *ev = malloc(sizeof(int) * E);
    int64_t *ew = malloc(sizeof(int64_t) * E);
    for (int e = 0; e < E; ++e) {
        int k = g->off[e + 1] - g->off[e];
        if (k < 1 || k > 2) { free(eu); free(ev); free(ew); return -2; }
        eu[e] = g->dets[g->off[e]];
        ev[e] = k == 2 ? g->dets[g->off[e] + 1] : B;
        ew[e] = w ? w[e] : or_fixed_weight(g->q[e]);
    }
    /* adjacency over nodes 0..N (B included as a target only) */
    int *deg = calloc(N + 1, sizeof(int));
    for (int e = 0; e < E; ++e) { deg[eu[e]]++; deg[ev[e]]++; }
    int *aoff = malloc(sizeof(int) * (N + 2));
    aoff[0] = 0;
    for (int v = 0; v <= N; ++v) aoff[v + 1] = aoff[v] + deg[v];
    int *adj_n = malloc(sizeof(int) * aoff[N + 1]);
    int *adj_e = malloc(sizeof(int) * aoff[N + 1]);
    int *fill = calloc(N + 1, sizeof(int));
    for (int e = 0; e < E; ++e) {
        int a = eu[e], b = ev[e];
        adj_n[aoff[a] + fill[a]] = b; adj_e[aoff[a] + fill[a]++] = e;
        adj_n[aoff[b] + fill[b]] = a; adj_e[aoff[b] + fill[b]++] = e;
    }

    size_t NN = (size_t)N * N;
    t->n = N;
    t->dist = malloc(sizeof(int64_t) * NN);
    t->hops = malloc(sizeof(int32_t) * NN);
    t->par = malloc(NN);
    t->pred = malloc(sizeof(int32_t) * NN);
    t->llr = malloc(sizeof(double) * NN);

    int64_t *dist = malloc(sizeof(int64_t) * (N + 1));
    int32_t *hops = malloc(sizeof(int32_t) * (N + 1));
    int32_t *pred = malloc(sizeof(int32_t) * (N + 1));
    uint8_t *par = malloc(N + 1);
    uint8_t *done = malloc(N + 1);
    int32_t *order = malloc(sizeof(int32_t) * (N + 1));
    hitem *H = malloc(sizeof(hitem) * (aoff[N + 1] + N + 2));
    int rc = 0;

    for (int u = 0; u < N && rc == 0; ++u) {
        for (int v = 0; v <= N; ++v) { dist[v] = INT64_MAX; hops[v] = INT32_MAX; done[v] = 0; pred[v] = -1; }
        int hn = 0, no = 0;
        dist[u] = 0; hops[u] = 0;
        hpush(H, &hn, (hitem){0, 0, u});
        while (hn) {
            hitem x = hpop(H, &hn);
            if (done[x.v] || x.w != dist[x.v] || x.h != hops[x.v]) continue;
            done[x.v] = 1;
            order[no++] = x.v;
            if (x.v == B) continue;                 /* the boundary is a sink */
            for (int a = aoff[x.v]; a < aoff[x.v + 1]; ++a) {
                int y = adj_n[a];
                int64_t nw = dist[x.v] + ew[adj_e[a]];
                int32_t nh = hops[x.v] + 1;
                if (nw < dist[y] || (nw == dist[y] && nh < hops[y])) {
                    dist[y] = nw; hops[y] = nh;
                    hpush(H, &hn, (hitem){nw, nh, y});
                }
            }
        }
        if (no != N + 1) { rc = -3; break; }       /* graph must be connected */
        /* canonical predecessor: smallest (node, edge) attaining the optimum */
        for (int y = 0; y <= N; ++y) {
            if (y == u) continue;
            int bx = INT32_MAX, be = INT32_MAX;
            for (int a = aoff[y]; a < aoff[y + 1]; ++a) {
                int x = adj_n[a], e = adj_e[a];
                if (x == B || dist[x] == INT64_MAX) continue;
                if (dist[x] + ew[e] == dist[y] && hops[x] + 1 == hops[y])
                    if (x < bx || (x == bx && e < be)) { bx = x; be = e; }
            }
            pred[y] = be;
        }
        /* parity along the predecessor tree, in order of increasing key */
        par[u] = 0;
        for (int i = 0; i < no; ++i) {
            int y = order[i];
            if (y == u) continue;
            int e = pred[y];
            int x = (eu[e] == y) ? ev[e] : eu[e];
            par[y] = par[x] ^ g->obs[e];
        }
        for (int v = 0; v < N; ++v) {
            size_t k = (size_t)u * N + v;
            int src = (v == u) ? B : v;
            t->dist[k] = dist[src];
            t->hops[k] = hops[src];
            t->par[k] = par[src];
            t->pred[k] = pred[src];
            t->llr[k] = or_prior_llr(dist[src]);
        }
    }
    free(dist); free(hops); free(pred); free(par); free(done); free(order); free(H);
    free(eu); free(ev); free(ew); free(deg); free(aoff); free(adj_n); free(adj_e); free(fill);
    if (rc) or_tables_free(t);
    return rc;
}
