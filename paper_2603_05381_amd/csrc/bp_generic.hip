// BP4M / BP4MF for shots of any size: one workgroup per shot, one thread per
// factor row (rows strided over the workgroup), messages double-buffered in
// the workgroup's slot of the caller's workspace.
//
// Factor graph (Sec. II.A): for s defects, variables v_ij (i <= j) are the
// decoding-graph edges (v_ii = defect i to the boundary) with prior LLR
// l_ij; factor c_i requires exactly one of v_i1..v_is to be 1.  The state is
// M[i][j] = message c_i -> v_ij.  One flooding iteration (Sec. II.B):
//   X_i[k] = l_ik + M[k][i] / alpha   (k != i: v_ik's only other factor is c_k)
//   X_i[i] = l_ii                     (v_ii has no other factor)
//   M'[i][j] = -max*_{k != j} X_i[k]  (leave-one-out soft maximum)
// and the posterior lambda_ij = l_ij + (M'[i][j] + M'[j][i]),
// lambda_ii = l_ii + M'[i][i].  Marginalization keeps v iff lambda_v > 0 and
// has converged iff every factor keeps exactly one variable (Sec. II.C-D).
//
// Two arithmetic modes:
//  - FP64 fixed order: the leave-one-out soft maximum is the pairwise
//    Jacobian fold of prefixes A_k = max*(A_{k-1}, X_k) and suffixes
//    B_k = max*(X_k, B_{k+1}), LOO_j = max*(A_{j-1}, B_{j+1}), with the
//    fixed-order exp/log1p of spec_math.hpp, so results are reproducible bit
//    for bit by any implementation of the same order.
//  - FP32: the exact leave-one-out log-sum-exp computed from the row's top
//    two values m1 >= m2 (argmax a) in base 2:
//      LOO_a = m2 + log2(S2),  S2 = sum_{k != a} 2^(X_k - m2)
//      LOO_j = m1 + log2(1 + 2^(m2 - m1) (S2 - 2^(X_j - m2)))   (j != a)
//    Every term is <= 1 after its shift, so nothing overflows, and the
//    argmax's own sum never underflows (it contains 2^0).  Messages may be
//    stored as FP16 or BF16 (rounded once, when written; both readers use
//    the rounded value).
//
// Forced convergence (Sec. II.D) takes variables in order of decreasing
// lambda (ties: smaller (i, j)) and accepts each one whose factors are still
// free.  It is computed here by rounds of locally dominant choices: every
// free factor picks its best variable among free partners; a pick that is
// mutual (or a boundary pick) is accepted.  With a strict total order this
// accepts exactly the variables the sequential greedy accepts.

#include <hip/hip_runtime.h>
#include <cfloat>
#include <cstdint>

#include "device_common.hpp"
#include "spec_math.hpp"

namespace bpm {

constexpr int kGenericThreads = 256;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// T: arithmetic type, TM: message storage type
template <typename T, typename TM>
struct SlotView {
    T *L;       // [s_cap * s_cap] priors (FP32 mode: base-2 units)
    T *P;       // [s_cap * s_cap] FP64 mode: prefix folds; FP32 mode: row exps
    TM *M0;     // [s_cap * s_cap] messages, buffer 0
    TM *M1;     // [s_cap * s_cap] messages, buffer 1
};

template <typename T, typename TM>
__host__ __device__ inline size_t generic_slot_bytes(int s_cap) {
    size_t ss = (size_t)s_cap * s_cap;
    size_t b = 2 * ss * sizeof(T) + 2 * ss * sizeof(TM);
    return (b + 255) & ~(size_t)255;
}

template <typename T, typename TM>
__device__ inline SlotView<T, TM> slot_view(void *base, int s_cap) {
    size_t ss = (size_t)s_cap * s_cap;
    T *p = (T *)base;
    TM *m = (TM *)(p + 2 * ss);
    return SlotView<T, TM>{p, p + ss, m, m + ss};
}

// Strict order of forced convergence: larger lambda first, then smaller
// (min(i,j), max(i,j)).
template <typename T>
__device__ inline bool fc_before(T la, int ia, int ja, T lb, int ib, int jb) {
    if (la != lb) return la > lb;
    int a0 = min(ia, ja), a1 = max(ia, ja), b0 = min(ib, jb), b1 = max(ib, jb);
    if (a0 != b0) return a0 < b0;
    return a1 < b1;
}

template <typename T, typename TM>
__device__ inline T posterior(const T *L, const TM *M, int s, int i, int j) {
    if (i == j) return L[i * s + i] + (T)M[i * s + i];
    return L[i * s + j] + ((T)M[i * s + j] + (T)M[j * s + i]);
}

// FP64 factor update of every row (fixed order): with X_k the row's inputs,
// prefix folds A_0 = X_0, A_k = max*(A_{k-1}, X_k), suffix folds
// B_{s-1} = X_{s-1}, B_k = max*(X_k, B_{k+1}), and the leave-one-out soft
// maximum of column j is max*(A_{j-1}, B_{j+1}) (B_1 for j = 0, A_{s-2} for
// j = s-1); the message is its negation.  Two steps with a workgroup barrier
// between them.  Step 1, two threads per row: the prefix and the suffix
// folds, stored shifted so that column j finds both at position j:
// P[i][j] = A_{j-1} (j >= 1) and Mnew[i][j] = B_{j+1} (j <= s-2).
template <int NT>
__device__ inline void fold_rows(const SlotView<double, double> &v, const double *Mold, double *Mnew, int s,
                                 double inv_alpha) {
    using namespace specmath;
    for (int t = threadIdx.x; t < 2 * s; t += NT) {
        const int i = t >> 1;
        const double *Li = v.L + (size_t)i * s;
        auto X = [&](int k) -> double { return k == i ? Li[i] : Li[k] + Mold[(size_t)k * s + i] * inv_alpha; };
        // (s >= 2; each step's next input is loaded before its max*)
        if ((t & 1) == 0) {
            double *Ai = v.P + (size_t)i * s;
            double a = X(0), xk = X(1);
            for (int k = 1; k < s; ++k) {
                Ai[k] = a;                          // A_{k-1}
                if (k + 1 < s) {
                    const double xn = X(k + 1);
                    a = maxstar(a, xk);
                    xk = xn;
                }
            }
        } else {
            double *Bi = Mnew + (size_t)i * s;
            double b = X(s - 1);                    // B_{s-1}
            Bi[s - 2] = b;
            double xk = X(s - 2);
            for (int k = s - 2; k >= 1; --k) {
                const double xn = X(k > 1 ? k - 1 : 0);
                b = maxstar(xk, b);                 // B_k
                Bi[k - 1] = b;
                xk = xn;
            }
        }
    }
}
// Step 2, one thread per message: M'[i][j] = -max*(A_{j-1}, B_{j+1}), or
// -B_1 / -A_{s-2} at the ends; each element is read and rewritten by the
// thread that owns it.
template <int NT>
__device__ inline void fold_messages(const SlotView<double, double> &v, double *Mnew, int s) {
    using namespace specmath;
    for (int e = threadIdx.x; e < s * s; e += NT) {
        const int j = e % s;
        Mnew[e] = j == 0 ? -Mnew[e] : j == s - 1 ? -v.P[e] : -maxstar(v.P[e], Mnew[e]);
    }
}

// Lanes per factor row in the row scans of one shot: the largest power of
// two up to 8 with s rows still fitting the workgroup (consecutive lanes of
// one wave, combined with lane shuffles).
template <int NT>
__device__ inline int lanes_per_row(int s) {
    int k = 1;
    while (k < 8 && 2 * k * s <= NT) k *= 2;
    return k;
}

template <typename TM>
__device__ inline void row_update(const SlotView<float, TM> &v, const TM *Mold, TM *Mnew, int s, int i,
                                  double inv_alpha_d) {
    const float inv_alpha = (float)inv_alpha_d;
    const float *Li = v.L + (size_t)i * s;
    float *E = v.P + (size_t)i * s;
    auto X = [&](int k) -> float { return k == i ? Li[i] : Li[k] + (float)Mold[(size_t)k * s + i] * inv_alpha; };
    float m1 = -FLT_MAX, m2 = -FLT_MAX;
    int a = 0;
    for (int k = 0; k < s; ++k) {
        float x = X(k);
        E[k] = x;
        if (x > m1) { m2 = m1; m1 = x; a = k; }
        else if (x > m2) { m2 = x; }
    }
    float S2 = 0.0f;
    for (int k = 0; k < s; ++k) {
        float e = __builtin_amdgcn_exp2f(E[k] - m2);
        E[k] = e;
        if (k != a) S2 += e;
    }
    const float c = __builtin_amdgcn_exp2f(m2 - m1);
    TM *Mi = Mnew + (size_t)i * s;
    for (int j = 0; j < s; ++j) {
        float loo;
        if (j == a) loo = m2 + __log2f(S2);
        else loo = m1 + __log2f(fmaf(c, S2 - E[j], 1.0f));
        Mi[j] = (TM)(-loo);
    }
}

// Workgroup scratch of one shot's decode (LDS arrays of thread-
// strided rows, s <= 1024).
struct ShotScratch {
    int32_t *fr, *cand, *best, *pick;
    int *flag_all, *any_free;
    unsigned long long *wsum;
};

// Path weight and observable parity of the decoding-graph edge joining
// defects i and p (p == i: i's boundary path), from the graph's tables ...
struct GraphPairs {
    const DevGraph *g;
    const uint16_t *def;
    int N;
    __device__ int64_t dist(int i, int p) const { return g->dist[(size_t)def[i] * N + def[p]]; }
    __device__ int par(int i, int p) const { return g->par[(size_t)def[i] * N + def[p]]; }
};

// ... or from per-shot tables [s][s] (entries [i][p] with i <= p).
struct SlotPairs {
    const int64_t *D;
    const uint8_t *P;
    int s;
    __device__ int64_t dist(int i, int p) const { return D[i * s + p]; }
    __device__ int par(int i, int p) const { return P[i * s + p]; }
};

// BP4M (variant 0) / BP4MF (variant 1) on one shot whose s x s priors are
// in v.L: T iterations of flooding BP with the memory factor, the
// marginal candidate of every converged iteration, forced convergence at the
// last iteration (BP4M) or at every non-converged one (BP4MF), and the
// lowest-weight candidate (Sec. III.A-B).  Every thread of the workgroup
// calls it; it leaves the chosen matching in sh.best and the final messages
// in *Mfinal, and returns the shot's kConvergedAny / kFcRan / kFcChosen bits.
template <int NT, typename T, typename TM, typename Pairs>
__device__ int bp4m_shot(const SlotView<T, TM> &v, int s, int max_iters, int variant, double inv_alpha,
                         const Pairs &pairs, const ShotScratch &sh, const TM **Mfinal) {
    const int tid = threadIdx.x;
    const int K = lanes_per_row<NT>(s);
    for (int e = tid; e < s * s; e += NT) v.M0[e] = (TM)0.0f;
    __syncthreads();
    TM *Mold = v.M0, *Mnew = v.M1;
    int have_best = 0, best_fc = 0, conv = 0, flags = 0;
    long long best_w = 0;

    // weight of the candidate in cand[] (all threads call)
    auto cand_weight = [&]() -> long long {
        if (tid == 0) *sh.wsum = 0ull;
        __syncthreads();
        unsigned long long part = 0;
        for (int i = tid; i < s; i += NT) {
            int p = sh.cand[i];
            if (p >= i) part += (unsigned long long)pairs.dist(i, p);
        }
        atomicAdd(sh.wsum, part);
        __syncthreads();
        long long w = (long long)*sh.wsum;
        __syncthreads();
        return w;
    };
    // forced convergence on the posteriors of M -> cand[]
    auto forced = [&](const TM *M) {
        for (int i = tid; i < s; i += NT) sh.fr[i] = 1;
        __syncthreads();
        // each round accepts at least the best free variable: s rounds
        // always suffice; the bound only guards the loop
        for (int round = 0;; ++round) {
            if (K == 1) {
                for (int i = tid; i < s; i += NT) {
                    if (!sh.fr[i]) continue;
                    int bj = i;
                    T bl = posterior(v.L, M, s, i, i);
                    for (int j = 0; j < s; ++j) {
                        if (j == i || !sh.fr[j]) continue;
                        T l = posterior(v.L, M, s, i, j);
                        if (fc_before(l, i, j, bl, i, bj)) { bl = l; bj = j; }
                    }
                    sh.pick[i] = bj;
                }
            } else if (tid < s * K) {
                // the row's free variables split over its K lanes; the
                // order is strict and total, so the combined best is the
                // sequential scan's
                const int i = tid / K, h = tid - i * K;
                if (sh.fr[i]) {
                    int bj = -1;
                    T bl = (T)0;
                    if (h == 0) { bj = i; bl = posterior(v.L, M, s, i, i); }
                    for (int j = h; j < s; j += K) {
                        if (j == i || !sh.fr[j]) continue;
                        T l = posterior(v.L, M, s, i, j);
                        if (bj < 0 || fc_before(l, i, j, bl, i, bj)) { bl = l; bj = j; }
                    }
                    for (int m = 1; m < K; m <<= 1) {
                        const T ol = __shfl_xor(bl, m, K);
                        const int oj = __shfl_xor(bj, m, K);
                        if (oj >= 0 && (bj < 0 || fc_before(ol, i, oj, bl, i, bj))) { bl = ol; bj = oj; }
                    }
                    if (h == 0) sh.pick[i] = bj;
                }
            }
            __syncthreads();
            if (tid == 0) *sh.any_free = 0;
            __syncthreads();
            for (int i = tid; i < s; i += NT) {
                if (!sh.fr[i]) continue;
                int j = sh.pick[i];
                if (j == i || sh.pick[j] == i) sh.cand[i] = j;
                else if (round >= s) { sh.cand[i] = i; sh.pick[i] = i; }
                else *sh.any_free = 1;
            }
            __syncthreads();
            for (int i = tid; i < s; i += NT)
                if (sh.fr[i] && (sh.pick[i] == i || sh.pick[sh.pick[i]] == i)) sh.fr[i] = 0;
            __syncthreads();
            if (!*sh.any_free) break;
        }
    };

    for (int t = 1; t <= max_iters; ++t) {
        if constexpr (sizeof(T) == 8) {
            fold_rows<NT>(v, Mold, Mnew, s, inv_alpha);
            __syncthreads();
            fold_messages<NT>(v, Mnew, s);
        } else {
            for (int i = tid; i < s; i += NT) row_update(v, Mold, Mnew, s, i, inv_alpha);
        }
        __syncthreads();
        { TM *sw = Mold; Mold = Mnew; Mnew = sw; }
        // marginalization and convergence check: the count of positive
        // posteriors of each row and its last positive column
        if (tid == 0) *sh.flag_all = 1;
        __syncthreads();
        if (K == 1) {
            for (int i = tid; i < s; i += NT) {
                int cnt = 0, p = -1;
                for (int j = 0; j < s; ++j)
                    if (posterior(v.L, Mold, s, i, j) > (T)0) { ++cnt; p = j; }
                sh.cand[i] = p;
                if (cnt != 1) *sh.flag_all = 0;
            }
        } else if (tid < s * K) {
            const int i = tid / K, h = tid - i * K;
            int cnt = 0, p = -1;
            for (int j = h; j < s; j += K)
                if (posterior(v.L, Mold, s, i, j) > (T)0) { ++cnt; p = j; }
            for (int m = 1; m < K; m <<= 1) {
                cnt += __shfl_xor(cnt, m, K);
                p = max(p, __shfl_xor(p, m, K));
            }
            if (h == 0) {
                sh.cand[i] = p;
                if (cnt != 1) *sh.flag_all = 0;
            }
        }
        __syncthreads();
        conv = *sh.flag_all;
        int consider = conv;
        if (!conv && variant == 1) {
            flags |= kFcRan;
            forced(Mold);
            consider = 1;
        }
        if (conv) flags |= kConvergedAny;
        if (consider) {
            long long w = cand_weight();
            if (!have_best || w < best_w) {
                for (int i = tid; i < s; i += NT) sh.best[i] = sh.cand[i];
                best_w = w; have_best = 1; best_fc = !conv;
            }
        }
        __syncthreads();
    }
    if (variant == 0 && !conv) {
        flags |= kFcRan;
        forced(Mold);
        long long w = cand_weight();
        if (!have_best || w < best_w) {
            for (int i = tid; i < s; i += NT) sh.best[i] = sh.cand[i];
            best_w = w; have_best = 1; best_fc = 1;
        }
        __syncthreads();
    }
    if (best_fc) flags |= kFcChosen;
    *Mfinal = Mold;
    return flags;
}

template <typename T, typename TM>
__global__ __launch_bounds__(kGenericThreads) void k_bp_generic(DecodeShared c, int cls, void *slots, int s_slot) {
    constexpr bool kSpec = sizeof(T) == 8;
    __shared__ int32_t fr[1024];        // free flags / scratch (s <= s_slot <= 1024)
    __shared__ int32_t cand[1024];
    __shared__ int32_t best[1024];
    __shared__ int32_t pick[1024];
    __shared__ int flag_all, any_free;
    __shared__ unsigned long long wsum;
    __shared__ int pred_x;

    const int tid = threadIdx.x;
    SlotView<T, TM> v =
        slot_view<T, TM>((char *)slots + (size_t)blockIdx.x * generic_slot_bytes<T, TM>(s_slot), s_slot);
    const ShotScratch sh{fr, cand, best, pick, &flag_all, &any_free, &wsum};
    const uint32_t count = c.class_count[cls];
    const uint32_t *list = c.class_list + (size_t)cls * c.total;

    for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
        const uint32_t x = list[item];             // global shot index
        const int ii = __builtin_amdgcn_readfirstlane(find_instance(c, x));
        DevGraph g;
        InstState st;
        uint64_t ibase, iblock0;
        load_instance(c, ii, g, st, ibase, iblock0);
        const int N = g.n_det;
        const uint64_t b = x - ibase;
        const int s = st.s[b];
        const uint16_t *def = st.defects + b * (uint64_t)c.s_cap;
        // priors
        for (int e = tid; e < s * s; e += kGenericThreads) {
            int i = e / s, j = e - i * s;
            size_t k = (size_t)def[i] * N + def[j];
            if constexpr (kSpec) v.L[e] = g.llr64[k];
            else v.L[e] = g.llr32[k] * kLog2e;
        }
        const GraphPairs pairs{&g, def, N};
        const TM *Mold = nullptr;
        int flags = bp4m_shot<kGenericThreads>(v, s, c.max_iters, c.variant, c.inv_alpha, pairs, sh, &Mold);
        // outputs
        if (tid == 0) pred_x = 0;
        __syncthreads();
        int px = 0;
        for (int i = tid; i < s; i += kGenericThreads) {
            int p = best[i];
            if (st.match) st.match[(size_t)b * st.match_stride + i] = p;
            if (p < i) continue;
            px ^= pairs.par(i, p);
            if (st.corr) emit_path(g, def[i], def[p], st.corr, st.W, b);
        }
        if (px) atomicXor(&pred_x, 1);
        if (st.lambda_out && s <= st.lambda_stride) {
            double *lo = st.lambda_out + (size_t)b * st.lambda_stride * st.lambda_stride;
            for (int e = tid; e < s * s; e += kGenericThreads) {
                int i = e / s, j = e - i * s;
                double l = (double)posterior(v.L, Mold, s, i, j);
                if constexpr (!kSpec) l *= (double)kLn2;
                lo[i * st.lambda_stride + j] = l;
            }
        }
        __syncthreads();
        if (tid == 0) {
            int ob = st.obs ? (int)((st.obs[b >> 6] >> (b & 63)) & 1) : 0;
            if (pred_x) flags |= kPred;
            if (pred_x != ob) flags |= kFail;
            st.flags[b] = (uint8_t)flags;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ B-BP4MF
//
// B-BP4MF for code-capacity depolarizing noise (Sec. III.D; correlated
// decoding, Sec. II.E), FP64 in a fixed operation order (written out with
// the oracle's, so that the two agree bit for bit):
//  1. quaternary BP on the Tanner graph, flooding, messages as log-ratios
//     ln P(commute)/P(anticommute) with the check's Pauli on the qubit:
//       qubit->check  L(E) = prior(E) - sum over the qubit's other checks c'
//                     (X checks, then Z checks, ascending) that anticommute
//                     with E of mu_c';  nu = max*(L over E commuting with the
//                     check's Pauli) - max*(L over the other two), in the
//                     orders (I, X | Y, Z) for X checks, (I, Z | X, Y) for Z;
//       check->qubit  t = product over the check's other qubits (ascending)
//                     of th(nu), th(x) = sign(x) (1 - e) / (1 + e),
//                     e = exp(-|x|); a = min(|t|, 1 - 2^-40);
//                     mu = +-log((1 + a) / (1 - a)), negative iff
//                     (t < 0) xor the syndrome bit;
//       posterior     L(E) = prior(E) - sum over anticommuting checks of mu,
//                     hard decision = first maximum over (I, X, Y, Z);
//     stopping at the first iteration whose hard decision has both
//     syndromes: its Z components are the correction;
//  2. otherwise the posterior probability of a Z component,
//     P = (e_Y + e_Z) / (((e_I + e_X) + e_Y) + e_Z), e_E = exp(L(E) - max L),
//     weights the qubit's decoding-graph edge: 1 (2^-32) if P >= 1/2, else
//     floor(log((1 - P) / P) 2^32 + 1/2) clamped to [1, 2^40];  each defect's
//     shortest paths (weight, then hops; the boundary a sink; the
//     predecessor the smallest (node, edge) attaining the optimum) follow
//     from synchronous Bellman-Ford rounds on keys weight * 2^11 + hops;
//     pair (i, j), i < j, takes defect i's tree; the prior of a path of
//     weight D is -D - log(1 - exp(-D));
//  3. BP4MF on those priors (bp4m_shot), its weights and parities from the
//     per-shot tables (BP4M instead if asked: the paper names that variant
//     too).
// One workgroup per shot; LDS holds quaternary BP's messages (up to
// kQbpMaxQubits qubits) and then BP4MF's arrays when the shot has up to
// kBbpLdsMaxS defects; the workgroup's slot holds the shot's path tables
// (and the BP arrays of larger shots).

constexpr int kQbpMaxQubits = 1024;
constexpr int kQbpMaxChecks = 2048;


__device__ inline bool bbp_anti(int E, bool xcheck) { return xcheck ? E >= 2 : (E == 1 || E == 2); }

__device__ inline double bbp_th(double x) {
    const double e = specmath::exp_fixed(-fabs(x));
    const double r = (1.0 - e) / (1.0 + e);
    return x < 0.0 ? -r : r;
}

__host__ __device__ inline size_t bbp_slot_bytes(int s_cap) {
    const size_t ss = (size_t)s_cap * s_cap;
    return generic_slot_bytes<double, double>(s_cap) + ((ss * 8 + 255) & ~(size_t)255) + ((ss + 255) & ~(size_t)255);
}

// LDS of the B-BP4MF kernel, reused stage by stage: quaternary BP's two
// message arrays; then path keys and edge weights; then, for shots of up to
// kBbpLdsMaxS defects, BP4MF's four s x s arrays (larger shots use the
// workgroup's global slot)
constexpr int kBbpLds = 16384;                      // doubles (128 KB)
constexpr int kBbpLdsMaxS = 64;                     // 4 s^2 <= kBbpLds
// int64 path keys per buffer (stage 2): the stage-1 message area and the
// qubit/check lists each hold one buffer
constexpr int kBbpKeys = 4096;
// threads of the B-BP4MF workgroup: its register count leaves room for two
// waves per SIMD, and its LDS for one workgroup per CU
constexpr int kBbpThreads = 512;
// neighbours of a detector node kept in registers by stage 2's relaxation
constexpr int kBfDeg = 8;
static_assert(kBbpKeys <= 4 * kQbpMaxQubits && 2 * kBbpKeys <= 4 * kQbpMaxQubits + 4 * kQbpMaxChecks,
              "key buffers inside the message area and the qubit/check lists");
static_assert(2 * kQbpMaxQubits * 4 <= kBbpLds && 4 * kBbpLdsMaxS * kBbpLdsMaxS <= kBbpLds, "LDS layout");

__global__ __launch_bounds__(kBbpThreads) void k_bbp4mf(BbpArgs a) {
    using namespace specmath;
    __shared__ double lbuf[kBbpLds];
    double *const mu = lbuf;                        // check -> qubit [v][slot]; later path keys
    double *const nu = lbuf + kQbpMaxQubits * 4;    // th of qubit -> check [v][slot]; later edge weights
    __shared__ uint8_t hard[kQbpMaxQubits];
    __shared__ uint8_t zb[kQbpMaxChecks];           // syndrome bits, X checks then Z checks
    __shared__ uint16_t def[1024];
    __shared__ int32_t fr[1024], cand[1024], best[1024], pick[1024];
    __shared__ int flag_all, any_free, ok_sh, chg[3], pred_x, s_sh;
    __shared__ unsigned long long wsum;

    const int tid = threadIdx.x;
    const TannerDev &tn = a.tn;
    const int nq = tn.n_q, nxc = tn.n_xc, nc = tn.n_xc + tn.n_zc, N = a.g.n_det;
    char *slot = a.slots + (size_t)blockIdx.x * a.slot_bytes;
    const ShotScratch sh{fr, cand, best, pick, &flag_all, &any_free, &wsum};
    int64_t *wgt = reinterpret_cast<int64_t *>(nu);  // [n_mech] edge weights of stage 2
    constexpr int64_t kInf = INT64_MAX;
    // the graphs' lists, copied into the upper half of lbuf at every shot
    // (stage 3 may overwrite it): qubit -> checks; check -> (qubit << 2 |
    // slot); node -> incident (neighbour << 11 | edge << 1 | observable bit)
    int32_t *const tq = reinterpret_cast<int32_t *>(lbuf + kBbpLds / 2);
    int32_t *const qcL = tq;                        // [4 n_q]  (n_q <= 1024)
    int32_t *const cqL = tq + 4 * kQbpMaxQubits;    // [4 nc]   (nc <= 2048)
    int32_t *const noffL = cqL + 4 * kQbpMaxChecks; // [N + 2]  (N <= 1023)
    int32_t *const adjL = noffL + 1040;             // [2 n_mech]
    static_assert(4 * kQbpMaxQubits + 4 * kQbpMaxChecks + 1040 + 2 * kQbpMaxQubits <= kBbpLds, "list layout");

    // posterior log-probabilities of qubit v from the current mu
    auto post = [&](int v, double L[4]) {
        for (int E = 0; E < 4; ++E) {
            L[E] = E == 0 ? a.pri_i : a.pri_p;
            for (int k = 0; k < 4; ++k) {
                const int c = qcL[4 * v + k];
                if (c >= 0 && bbp_anti(E, c < nxc)) L[E] = L[E] - mu[4 * v + k];
            }
        }
    };

    for (uint64_t b = blockIdx.x; b < a.n; b += gridDim.x) {
        const uint64_t w = b >> 6, bit = 1ull << (b & 63);
        for (int c = tid; c < nc; c += kBbpThreads)
            zb[c] = ((c < nxc ? a.synx[(uint64_t)c * a.W + w] : a.synz[(uint64_t)(c - nxc) * a.W + w]) & bit) != 0;
        for (int e = tid; e < 4 * nq; e += kBbpThreads) {
            mu[e] = 0.0;
            qcL[e] = tn.qc[e];
        }
        for (int e = tid; e < 4 * nc; e += kBbpThreads)
            cqL[e] = tn.cq[e] < 0 ? -1 : (tn.cq[e] << 2) | tn.cs[e];
        for (int u = tid; u <= N + 1; u += kBbpThreads) noffL[u] = tn.noff[u];
        for (int u = tid; u <= N; u += kBbpThreads)
            for (int q = tn.noff[u]; q < tn.noff[u + 1]; ++q) {
                const int e = tn.nedge[q];
                const int x0 = a.g.edge_u[e], x1 = a.g.edge_v[e] < 0 ? N : a.g.edge_v[e];
                adjL[q] = ((x0 == u ? x1 : x0) << 11) | (e << 1) | (int)a.g.mech_obs[e];
            }
        __syncthreads();
        if (tid == 0) {
            int s = 0;
            for (int c = 0; c < nxc; ++c)
                if (zb[c]) { if (s < a.s_cap) def[s] = (uint16_t)c; ++s; }
            s_sh = s;
        }
        // ---- stage 1: quaternary BP ----
        int conv = 0;
        for (int t = 1; t <= a.max_iters; ++t) {
            // qubit -> check, one thread per (qubit, slot); the message is
            // only ever used through th, so th(nu) is what is stored
            for (int e = tid; e < 4 * nq; e += kBbpThreads) {
                const int v = e >> 2, k = e & 3;
                const int c = qcL[e];
                if (c < 0) continue;
                double L[4];
                for (int E = 0; E < 4; ++E) {
                    L[E] = E == 0 ? a.pri_i : a.pri_p;
                    for (int k2 = 0; k2 < 4; ++k2) {
                        const int c2 = qcL[4 * v + k2];
                        if (k2 != k && c2 >= 0 && bbp_anti(E, c2 < nxc)) L[E] = L[E] - mu[4 * v + k2];
                    }
                }
                double cm, an;
                if (c < nxc) { cm = maxstar(L[0], L[1]); an = maxstar(L[2], L[3]); }
                else         { cm = maxstar(L[0], L[3]); an = maxstar(L[1], L[2]); }
                nu[e] = bbp_th(cm - an);
            }
            __syncthreads();
            // check -> qubit, one thread per (check, edge)
            for (int e = tid; e < 4 * nc; e += kBbpThreads) {
                const int c = e >> 2, i = e & 3;
                const int vs = cqL[e];                        // qubit << 2 | its slot
                if (vs < 0) continue;
                double tt = 1.0;
                for (int i2 = 0; i2 < 4; ++i2) {
                    const int vs2 = cqL[4 * c + i2];
                    if (i2 != i && vs2 >= 0) tt = tt * nu[vs2];   // th of 4 v + slot
                }
                double aa = fabs(tt);
                if (aa > 1.0 - 0x1p-40) aa = 1.0 - 0x1p-40;
                const double r = log_fixed((1.0 + aa) / (1.0 - aa));
                mu[vs] = ((tt < 0.0) != (zb[c] != 0)) ? -r : r;
            }
            __syncthreads();
            for (int v = tid; v < nq; v += kBbpThreads) {
                double L[4];
                post(v, L);
                int h = 0;
                for (int E = 1; E < 4; ++E) if (L[E] > L[h]) h = E;
                hard[v] = (uint8_t)h;
            }
            if (tid == 0) ok_sh = 1;
            __syncthreads();
            for (int c = tid; c < nc; c += kBbpThreads) {
                int par = 0;
                for (int i = 0; i < 4; ++i) {
                    const int vs = cqL[4 * c + i];
                    if (vs >= 0) par ^= (int)bbp_anti(hard[vs >> 2], c < nxc);
                }
                if (par != zb[c]) ok_sh = 0;
            }
            __syncthreads();
            conv = ok_sh;
            __syncthreads();
            if (conv) break;
        }
        const int s = s_sh;
        int flags = 0;
        if (tid == 0) pred_x = 0;
        __syncthreads();
        if (conv) {
            flags = kQbp | kConvergedAny;
            int px = 0;
            for (int v = tid; v < nq; v += kBbpThreads)
                if (hard[v] >= 2 && tn.qobs[v]) px ^= 1;
            if (px) atomicXor(&pred_x, 1);
        } else if (s > a.s_cap) {
            flags = kOverflow;
        } else {
            // ---- stage 2: re-weighted shortest paths of the shot's defects ----
            for (int v = tid; v < nq; v += kBbpThreads) {
                double L[4];
                post(v, L);
                double mx = L[0];
                for (int E = 1; E < 4; ++E) mx = fmax(mx, L[E]);
                double e[4];
                for (int E = 0; E < 4; ++E) e[E] = exp_fixed(L[E] - mx);
                const double P = (e[2] + e[3]) / (((e[0] + e[1]) + e[2]) + e[3]);
                int64_t wv = 1;
                if (P < 0.5) {
                    const double f = floor(log_fixed((1.0 - P) / P) * 4294967296.0 + 0.5);
                    wv = f < 1.0 ? 1 : f > 1099511627776.0 ? ((int64_t)1 << 40) : (int64_t)f;
                }
                wgt[tn.qmech[v]] = wv;               // nu is no longer read
            }
            __syncthreads();
            int64_t *Dt = reinterpret_cast<int64_t *>(slot + generic_slot_bytes<double, double>(a.s_cap));
            uint8_t *Pt = reinterpret_cast<uint8_t *>(Dt) + (((size_t)a.s_cap * a.s_cap * 8 + 255) & ~(size_t)255);
            // Bellman-Ford from a batch of defects at once: the keys of nb
            // sources, [source][node], ping-pong between the stage-1 message
            // area and the (now unused) qubit/check lists; one barrier per
            // synchronous round of the whole batch.  Labels only decrease and
            // reach the lexicographic (weight, hops) optimum of every source;
            // the boundary never relays a path.
            // Every detector node (at most kBbpThreads of them, at most
            // kBfDeg neighbours each: checked on the host) is relaxed by
            // thread (rep, u), which keeps node u's neighbours and their key
            // increments in registers and relaxes u for the sources rep,
            // rep + R, ...: one round of independent loads per node and
            // source.  The boundary, a sink, is left out of the rounds; its
            // keys are taken once they have converged (the minimum the rounds
            // would reach).
            const int NB1 = N + 1;
            const int per = kBbpKeys / NB1;           // sources per batch (>= 4)
            int64_t *const keyA = reinterpret_cast<int64_t *>(mu);
            int64_t *const keyB = reinterpret_cast<int64_t *>(lbuf + kBbpLds / 2);
            const int R = kBbpThreads / N;
            const int bu = tid % N, brep = tid / N;
            int xs[kBfDeg];
            int64_t ws[kBfDeg];
            if (brep < R) {
                const int q0 = noffL[bu], deg = noffL[bu + 1] - q0;
#pragma unroll
                for (int k = 0; k < kBfDeg; ++k) {
                    xs[k] = -1;
                    ws[k] = 0;
                    if (k < deg) {
                        const int aq = adjL[q0 + k], x = aq >> 11;
                        if (x != N) { xs[k] = x; ws[k] = (wgt[(aq >> 1) & 1023] << 11) + 1; }
                    }
                }
            }
            for (int i0 = 0; i0 < s; i0 += per) {
                const int nb = min(per, s - i0);
                for (int t = tid; t < nb * NB1; t += kBbpThreads) {
                    const int bi = t / NB1, u = t - bi * NB1;
                    keyA[t] = u == def[i0 + bi] ? 0 : kInf;
                    keyB[t] = kInf;
                }
                if (tid < 3) chg[tid] = 0;
                __syncthreads();
                const int64_t *cur = keyA;
                int64_t *nxt = keyB;
                for (int round = 0; round <= N + 1; ++round) {
                    // flag of this round; the one of the next round is cleared
                    // now (its last readers passed the previous barrier)
                    const int fr3 = round % 3;
                    if (tid == 0) chg[(round + 1) % 3] = 0;
                    int ch = 0;
                    for (int bi = brep; bi < nb && brep < R; bi += R) {
                        const int64_t *const kr = cur + bi * NB1;
                        const int64_t k0 = kr[bu];
                        int64_t bk = k0;
                        if (bu != def[i0 + bi]) {
#pragma unroll
                            for (int k = 0; k < kBfDeg; ++k) {
                                const bool on = xs[k] >= 0;
                                const int64_t kx = kr[on ? xs[k] : bu];
                                const int64_t ck = (on && kx != kInf) ? kx + ws[k] : kInf;
                                bk = ck < bk ? ck : bk;
                            }
                        }
                        nxt[bi * NB1 + bu] = bk;
                        if (bk != k0) ch = 1;
                    }
                    if (ch) chg[fr3] = 1;
                    __syncthreads();
                    const int any = chg[fr3];
                    const int64_t *const done = nxt;
                    nxt = const_cast<int64_t *>(cur);
                    cur = done;
                    if (!any) break;
                }
                // the boundary's keys from its converged neighbours
                for (int bi = tid; bi < nb; bi += kBbpThreads) {
                    int64_t *const kr = const_cast<int64_t *>(cur) + bi * NB1;
                    int64_t bk = kInf;
                    for (int q = noffL[N]; q < noffL[N + 1]; ++q) {
                        const int aq = adjL[q], e = (aq >> 1) & 1023, x = aq >> 11;
                        if (x == N || kr[x] == kInf) continue;
                        const int64_t ck = kr[x] + (wgt[e] << 11) + 1;
                        if (ck < bk) bk = ck;
                    }
                    kr[N] = bk;
                }
                __syncthreads();
                // paths of source i = i0 + bi to the defects j > i and to the
                // boundary (j == i)
                for (int t = tid; t < nb * s; t += kBbpThreads) {
                    const int bi = t / s, j = t - bi * s, i = i0 + bi;
                    if (j < i) continue;
                    const int src = def[i];
                    const int64_t *const kr = cur + bi * NB1;
                    int y = j == i ? N : def[j];
                    const int64_t D = kr[y] == kInf ? ((int64_t)1 << 50) : kr[y] >> 11;
                    int par = 0;
                    // every reached node other than the source has an optimal
                    // predecessor; the checks only keep a malformed graph in bounds
                    for (int hop = 0; y != src && kr[y] != kInf && hop <= N; ++hop) {
                        int bx = INT32_MAX, be = INT32_MAX, bo = 0;
                        for (int q = noffL[y]; q < noffL[y + 1]; ++q) {
                            const int aq = adjL[q], e = (aq >> 1) & 1023, x = aq >> 11;
                            if (x == N || kr[x] == kInf) continue;
                            if (kr[x] + (wgt[e] << 11) + 1 == kr[y] && (x < bx || (x == bx && e < be))) {
                                bx = x; be = e; bo = aq & 1;
                            }
                        }
                        if (be == INT32_MAX) break;
                        par ^= bo;
                        y = bx;
                    }
                    Dt[i * s + j] = D;
                    Pt[i * s + j] = (uint8_t)par;
                }
                __syncthreads();
            }
            // the shot's BP arrays: in LDS (keys and weights are done with)
            // when they fit, else in the slot; priors of the new paths
            SlotView<double, double> v = slot_view<double, double>(slot, s > 0 ? s : 1);
            if (s <= kBbpLdsMaxS) {
                const int ss = s * s;
                v = SlotView<double, double>{lbuf, lbuf + ss, lbuf + 2 * ss, lbuf + 3 * ss};
            }
            for (int e = tid; e < s * s; e += kBbpThreads) {
                const int i = e / s, j = e - i * s;
                const double Df = ldexp((double)Dt[min(i, j) * s + max(i, j)], -32);
                v.L[e] = (-Df) - log_fixed(1.0 - exp_fixed(-Df));
            }
            __syncthreads();
            if (s == 0) {
                flags = kConvergedAny;
            } else if (s == 1) {
                flags = kConvergedAny;
                if (tid == 0) {
                    best[0] = 0;
                    pred_x = Pt[0];
                }
            } else {
                // ---- stage 3: BP4MF on the re-weighted priors ----
                const SlotPairs pairs{Dt, Pt, s};
                const double *Mfin = nullptr;
                flags = bp4m_shot<kBbpThreads>(v, s, a.max_iters, a.variant, a.inv_alpha, pairs, sh, &Mfin);
                int px = 0;
                for (int i = tid; i < s; i += kBbpThreads) {
                    const int q = best[i];
                    if (q >= i) px ^= pairs.par(i, q);
                }
                if (px) atomicXor(&pred_x, 1);
            }
            __syncthreads();
            if (a.match)
                for (int i = tid; i < s; i += kBbpThreads) a.match[b * (uint64_t)a.match_stride + i] = best[i];
        }
        __syncthreads();
        if (tid == 0) {
            const int ob = a.obs ? (int)((a.obs[w] >> (b & 63)) & 1) : 0;
            if (!(flags & kOverflow)) {
                if (pred_x) flags |= kPred;
                if (pred_x != ob) flags |= kFail;
            }
            a.flags[b] = (uint8_t)flags;
            a.s_out[b] = s;
        }
        __syncthreads();
    }
}

hipError_t launch_bbp4mf(const BbpArgs &a, int n_slots, hipStream_t stream) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bbp4mf, dim3(n_slots), dim3(kBbpThreads), 0, stream, a);
    return hipGetLastError();
}

size_t bbp4mf_slot_bytes_host(int s_cap) { return bbp_slot_bytes(s_cap); }

void bbp4mf_graph_limits(int *max_nodes, int *max_degree) {
    *max_nodes = kBbpThreads;
    *max_degree = kBfDeg;
}

size_t generic_slot_bytes_host(bool spec, int store, int s_cap) {
    if (spec) return generic_slot_bytes<double, double>(s_cap);
    return store == 0 ? generic_slot_bytes<float, float>(s_cap) : generic_slot_bytes<float, _Float16>(s_cap);
}

hipError_t launch_bp_generic(bool spec, const DecodeShared &c, int cls, void *slots, int s_slot, int n_slots,
                             hipStream_t stream) {
    const dim3 grid(n_slots), block(kGenericThreads);
    if (spec)
        hipLaunchKernelGGL((k_bp_generic<double, double>), grid, block, 0, stream, c, cls, slots, s_slot);
    else if (c.store == 1)
        hipLaunchKernelGGL((k_bp_generic<float, _Float16>), grid, block, 0, stream, c, cls, slots, s_slot);
    else if (c.store == 2)
        hipLaunchKernelGGL((k_bp_generic<float, __bf16>), grid, block, 0, stream, c, cls, slots, s_slot);
    else
        hipLaunchKernelGGL((k_bp_generic<float, float>), grid, block, 0, stream, c, cls, slots, s_slot);
    return hipGetLastError();
}

}  // namespace bpm
