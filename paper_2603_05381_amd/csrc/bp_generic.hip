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

// One iteration of factor updates for row i: reads Mold, writes Mnew row i.
__device__ inline void row_update(const SlotView<double, double> &v, const double *Mold, double *Mnew, int s,
                                  int i, double inv_alpha) {
    using namespace specmath;
    const double *Li = v.L + (size_t)i * s;
    double *A = v.P + (size_t)i * s;
    auto X = [&](int k) -> double { return k == i ? Li[i] : Li[k] + Mold[(size_t)k * s + i] * inv_alpha; };
    double a = X(0);
    A[0] = a;
    for (int k = 1; k < s; ++k) { a = maxstar(a, X(k)); A[k] = a; }
    double *Mi = Mnew + (size_t)i * s;
    double b = X(s - 1);        // B_{s-1}
    Mi[s - 1] = -A[s - 2];
    for (int j = s - 2; j >= 0; --j) {
        // here b = B_{j+1}
        double loo = (j == 0) ? b : maxstar(A[j - 1], b);
        Mi[j] = -loo;
        b = maxstar(X(j), b);
    }
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
        // priors and zero messages
        for (int e = tid; e < s * s; e += kGenericThreads) {
            int i = e / s, j = e - i * s;
            size_t k = (size_t)def[i] * N + def[j];
            if constexpr (kSpec) v.L[e] = g.llr64[k];
            else v.L[e] = g.llr32[k] * kLog2e;
            v.M0[e] = (TM)0.0f;
        }
        __syncthreads();
        TM *Mold = v.M0, *Mnew = v.M1;
        int have_best = 0, best_fc = 0, conv = 0, flags = 0;
        long long best_w = 0;

        // weight of the candidate in cand[] (all threads call)
        auto cand_weight = [&]() -> long long {
            if (tid == 0) wsum = 0ull;
            __syncthreads();
            unsigned long long part = 0;
            for (int i = tid; i < s; i += kGenericThreads) {
                int p = cand[i];
                if (p >= i) part += (unsigned long long)g.dist[(size_t)def[i] * N + def[p]];
            }
            atomicAdd(&wsum, part);
            __syncthreads();
            long long w = (long long)wsum;
            __syncthreads();
            return w;
        };
        // forced convergence on the posteriors of M -> cand[]
        auto forced = [&](const TM *M) {
            for (int i = tid; i < s; i += kGenericThreads) fr[i] = 1;
            __syncthreads();
            // each round accepts at least the best free variable: s rounds
            // always suffice; the bound only guards the loop
            for (int round = 0;; ++round) {
                for (int i = tid; i < s; i += kGenericThreads) {
                    if (!fr[i]) continue;
                    int bj = i;
                    T bl = posterior(v.L, M, s, i, i);
                    for (int j = 0; j < s; ++j) {
                        if (j == i || !fr[j]) continue;
                        T l = posterior(v.L, M, s, i, j);
                        if (fc_before(l, i, j, bl, i, bj)) { bl = l; bj = j; }
                    }
                    pick[i] = bj;
                }
                __syncthreads();
                if (tid == 0) any_free = 0;
                __syncthreads();
                for (int i = tid; i < s; i += kGenericThreads) {
                    if (!fr[i]) continue;
                    int j = pick[i];
                    if (j == i || pick[j] == i) cand[i] = j;
                    else if (round >= s) { cand[i] = i; pick[i] = i; }
                    else any_free = 1;
                }
                __syncthreads();
                for (int i = tid; i < s; i += kGenericThreads)
                    if (fr[i] && (pick[i] == i || pick[pick[i]] == i)) fr[i] = 0;
                __syncthreads();
                if (!any_free) break;
            }
        };

        for (int t = 1; t <= c.max_iters; ++t) {
            for (int i = tid; i < s; i += kGenericThreads) row_update(v, Mold, Mnew, s, i, c.inv_alpha);
            __syncthreads();
            { TM *sw = Mold; Mold = Mnew; Mnew = sw; }
            // marginalization and convergence check
            if (tid == 0) flag_all = 1;
            __syncthreads();
            for (int i = tid; i < s; i += kGenericThreads) {
                int cnt = 0, p = -1;
                for (int j = 0; j < s; ++j)
                    if (posterior(v.L, Mold, s, i, j) > (T)0) { ++cnt; p = j; }
                cand[i] = p;
                if (cnt != 1) flag_all = 0;
            }
            __syncthreads();
            conv = flag_all;
            int consider = conv;
            if (!conv && c.variant == 1) {
                flags |= kFcRan;
                forced(Mold);
                consider = 1;
            }
            if (conv) flags |= kConvergedAny;
            if (consider) {
                long long w = cand_weight();
                if (!have_best || w < best_w) {
                    for (int i = tid; i < s; i += kGenericThreads) best[i] = cand[i];
                    best_w = w; have_best = 1; best_fc = !conv;
                }
            }
            __syncthreads();
        }
        if (c.variant == 0 && !conv) {
            flags |= kFcRan;
            forced(Mold);
            long long w = cand_weight();
            if (!have_best || w < best_w) {
                for (int i = tid; i < s; i += kGenericThreads) best[i] = cand[i];
                best_w = w; have_best = 1; best_fc = 1;
            }
            __syncthreads();
        }
        if (best_fc) flags |= kFcChosen;
        // outputs
        if (tid == 0) pred_x = 0;
        __syncthreads();
        int px = 0;
        for (int i = tid; i < s; i += kGenericThreads) {
            int p = best[i];
            if (st.match) st.match[(size_t)b * st.match_stride + i] = p;
            if (p < i) continue;
            px ^= g.par[(size_t)def[i] * N + def[p]];
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
