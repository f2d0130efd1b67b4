// FP32 BP4M / BP4MF for shots with at most 128 defects: a group of S lanes
// per shot (S in {16, 32, 64, 96, 128}), one factor row per lane, the row in
// registers.
//
// Iteration (flooding schedule, Sec. II.B), for factor i = the lane's row:
//   X_i[k] = l_ik + M[k][i] / alpha (k != i),  X_i[i] = l_ii,
//   M'[i][j] = -LSE_{k != j} X_i[k],
//   lambda_ij = l_ij + (M'[i][j] + M'[j][i]),  lambda_ii = l_ii + M'[i][i],
// computed in base 2 (l scaled by log2 e) with the exact leave-one-out
// log-sum-exp, shifted by the row maximum m:
//   g_k = 2^(X_k - m) in [0, 1] (exactly 1 for every maximal entry),
//   H = sum_k fract(g_k) (the non-maximal terms), n = number of maximal terms,
//   LOO_r = m + log2(H + (n - g_r)).
// For a non-maximal r this is the sum of every other term; for a maximal r,
// n - 1 is exact and H carries the small remainder without cancellation, so
// the message to a dominant variable keeps full relative accuracy.  H is
// kept >= 2^-120 so that a variable whose competitors all underflow gets a
// large finite message instead of an infinite one.
//
// Register layout: lane i keeps its row rotated, entry r = column
// (i + r) mod S, so every register index in the unrolled loops is a
// compile-time constant.  The transpose every iteration needs (row i reads
// column i of M) goes through an LDS tile: lane i writes its rotated row to
// tile row i, and reads for entry r the message of row k = (i + r) mod S to
// column i, i.e. tile[k][S - r].  With DUP the tile holds every row twice
// (rows i and i + S), so that address is tile[i + r][S - r] = a per-lane base
// plus a compile-time offset; without DUP (S = 128, to stay within LDS) the
// wrap-around is selected per entry.  The odd row stride S + 1 keeps row
// writes and transposed reads free of bank conflicts.  Columns or rows >= s
// are padding: priors make them never win a maximum and add 0 to any sum.
//
// Marginalization and the convergence check (Sec. II.C-D) run in the same
// pass as the transpose.  Forced convergence (Sec. II.D) picks variables by
// decreasing lambda (ties: smaller (i, j)); it runs as rounds of locally
// dominant choices, which accept exactly the variables of the sequential
// greedy.  Candidate bookkeeping follows BP4M / BP4MF (Sec. III.A-B).

#include <hip/hip_runtime.h>
#include <cfloat>
#include <cstdint>

#include "device_common.hpp"

namespace bpm {

namespace {

constexpr float kLog2eF = 1.4426950408889634f;
constexpr float kLn2F = 0.6931471805599453f;
constexpr float kPadPrior = -1.0e30f;
constexpr int kChunk = 16;

template <int S>
struct GroupShape {
    static constexpr int kThreads = S <= 64 ? 64 : ((S + 63) / 64) * 64;
    static constexpr int kGroups = kThreads / S;
    static constexpr int kStride = S + 1;               // odd: conflict-free
    static constexpr bool kDup = S <= 96;               // duplicated tile rows
    static constexpr int kRows = kDup ? 2 * S : S;
};

// Hides a value from loop-invariant code motion, so that per-entry column
// indices are recomputed where they are used instead of being hoisted into
// (and occupying) one register each.
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ bool fc_before(float la, int ia, int ja, float lb, int ib, int jb) {
    if (la != lb) return la > lb;
    int a0 = min(ia, ja), a1 = max(ia, ja), b0 = min(ib, jb), b1 = max(ib, jb);
    if (a0 != b0) return a0 < b0;
    return a1 < b1;
}

}  // namespace

template <int S, bool kMemory>
__global__ __launch_bounds__(GroupShape<S>::kThreads) void k_bp_group(DevGraph g, DecodeState st, int cls) {
    using Shape = GroupShape<S>;
    constexpr int G = Shape::kGroups;
    constexpr int ST = Shape::kStride;
    constexpr bool DUP = Shape::kDup;
    __shared__ float tile[G][Shape::kRows * ST];
    __shared__ uint16_t sdef[G][S];
    __shared__ int32_t pick[G][S];
    __shared__ int32_t freef[G][S];
    __shared__ unsigned long long gw[2][G];
    __shared__ int gnc[2][G];
    __shared__ int gpred[G];
    __shared__ int block_any;

    const int tid = threadIdx.x;
    const int grp = tid / S;                      // == G for spare lanes
    const bool in_group = grp < G;
    const int gi = in_group ? grp : 0;
    const int j = in_group ? tid - grp * S : 0;   // row = lane within group
    const int N = g.n_det;
    const uint32_t count = st.class_count[cls];
    const uint32_t *list = st.class_list + (size_t)cls * st.n_shots;
    const float inv_alpha = (float)st.inv_alpha;
    float *const T = tile[gi];
    float *const Trow = T + j * ST;               // own row
    float *const Tdup = T + (j + S) * ST;         // its copy (DUP)
    // transposed read of entry r: DUP: T[(j + r) * ST + S - r] = Tt + r * S
    const float *const Tt = T + j * ST + S;

    auto recv_at = [&](int jj, int r) -> float {
        if constexpr (DUP) {
            return Tt[r * S];
        } else {
            const int k = (jj + r >= S) ? jj + r - S : jj + r;
            return T[k * ST + (S - r)];
        }
    };

    for (uint32_t base = blockIdx.x * (uint32_t)G; base < count; base += gridDim.x * (uint32_t)G) {
        const uint32_t item = base + (uint32_t)gi;
        const bool live = in_group && item < count;
        uint32_t b = 0;
        int s = 0;
        if (live) {
            b = list[item];
            s = st.s[b];
        }
        const bool row = live && j < s;
        if (in_group) sdef[gi][j] = row ? st.defects[(size_t)b * st.s_cap + j] : 0;
        if (tid < G) { gw[0][tid] = 0; gw[1][tid] = 0; gnc[0][tid] = 0; gnc[1][tid] = 0; gpred[tid] = 0; }
        __syncthreads();
        const int myd = sdef[gi][j];

        // priors, rotated: entry r = column (j + r) mod S
        float Lr[S], A[S];
        const int jg = opaque(j);
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const int k = (jg + r >= S) ? jg + r - S : jg + r;
            float l;
            if (!row) l = 0.0f;
            else if (k >= s) l = kPadPrior;
            else l = g.llr32[(size_t)myd * N + sdef[gi][k]] * kLog2eF;
            Lr[r] = l;
            A[r] = l;                                 // X while all messages are 0
        }

        int have_best = 0, best_fc = 0, conv = 0, flags = 0, best_p = j;
        long long best_w = 0;
        int cand = j;

        // posterior of (row j, entry r) from the tile
        auto lam_at = [&](int jj, int r) -> float {
            if (r == 0) return Lr[0] + Trow[0];
            return Lr[r] + (Trow[r] + recv_at(jj, r));
        };

        // forced convergence on the tile's messages -> cand (block-uniform)
        auto forced = [&](bool want) {
            if (in_group) freef[gi][j] = (want && row) ? 1 : 0;
            __syncthreads();
            // every round accepts at least the best free variable, so S
            // rounds always suffice; the bound only guards the loop
            for (int round = 0;; ++round) {
                if (in_group && freef[gi][j]) {
                    const int jj = opaque(j);
                    int bk = j;
                    float bl = lam_at(jj, 0);
#pragma unroll
                    for (int r = 1; r < S; ++r) {
                        const int k = (jj + r >= S) ? jj + r - S : jj + r;
                        if (k < s && freef[gi][k]) {
                            const float l = lam_at(jj, r);
                            if (fc_before(l, j, k, bl, j, bk)) { bl = l; bk = k; }
                        }
                    }
                    pick[gi][j] = bk;
                }
                if (tid == 0) block_any = 0;
                __syncthreads();
                if (in_group && freef[gi][j]) {
                    const int k = pick[gi][j];
                    if (k == j || pick[gi][k] == j) cand = k;
                    else if (round >= S) { cand = j; pick[gi][j] = j; }
                    else block_any = 1;
                }
                __syncthreads();
                if (in_group && freef[gi][j]) {
                    const int k = pick[gi][j];
                    if (k == j || pick[gi][k] == j) freef[gi][j] = 0;
                }
                const bool again = block_any != 0;
                __syncthreads();
                if (!again) break;
            }
        };

        // total weight of `cand` over the group (block-uniform)
        auto cand_weight = [&](int slot) -> long long {
            if (row && cand >= j)
                atomicAdd(&gw[slot][gi], (unsigned long long)g.dist[(size_t)myd * N + sdef[gi][cand]]);
            __syncthreads();
            const long long w = (long long)gw[slot][gi];
            __syncthreads();
            if (tid < G) gw[slot][tid] = 0;
            return w;
        };

        for (int t = 1; t <= st.max_iters; ++t) {
            const int par = t & 1;
            // ---- factor update of row j ----
            float m = -FLT_MAX;
#pragma unroll
            for (int r = 0; r < S; ++r) m = fmaxf(m, A[r]);
            float esum = 0.0f, hsum = 0.0f;
#pragma unroll
            for (int r = 0; r < S; ++r) {
                const float e = __builtin_amdgcn_exp2f(A[r] - m);
                A[r] = e;
                esum += e;
                hsum += __builtin_amdgcn_fractf(e);
            }
            const float n_max = rintf(esum - hsum);
            hsum = fmaxf(hsum, 0x1p-120f);
#pragma unroll
            for (int r = 0; r < S; ++r) {
                const float v = hsum + (n_max - A[r]);
                const float msg = -m - __builtin_amdgcn_logf(v);
                A[r] = msg;
                if (in_group) {
                    Trow[r] = msg;
                    if constexpr (DUP) Tdup[r] = msg;
                }
            }
            __syncthreads();
            // ---- transpose, marginalization, next X ----
            int cnt = 0, pr = 0;
            const int jd = opaque(j);
            {
                const float lam0 = Lr[0] + A[0];
                cnt += lam0 > 0.0f;
                A[0] = Lr[0];
            }
#pragma unroll
            for (int r = 1; r < S; ++r) {
                const float recv = recv_at(jd, r);
                const float lam = Lr[r] + (A[r] + recv);
                const bool on = lam > 0.0f;
                cnt += on;
                pr = on ? r : pr;
                if constexpr (kMemory) A[r] = fmaf(recv, inv_alpha, Lr[r]);
                else A[r] = Lr[r] + recv;
                // keep at most kChunk transposed reads in flight
                if ((r & (kChunk - 1)) == kChunk - 1) __builtin_amdgcn_sched_barrier(0);
            }
            cand = (j + pr >= S) ? j + pr - S : j + pr;
            if (row && cnt != 1) gnc[par][gi] = 1;
            if (row && cnt == 1 && cand >= j)
                atomicAdd(&gw[par][gi], (unsigned long long)g.dist[(size_t)myd * N + sdef[gi][cand]]);
            __syncthreads();
            conv = gnc[par][gi] == 0;
            const long long w = (long long)gw[par][gi];
            if (tid < G) { gnc[par ^ 1][tid] = 0; gw[par ^ 1][tid] = 0; }
            if (conv) {
                flags |= kConvergedAny;
                if (!have_best || w < best_w) { best_p = cand; best_w = w; have_best = 1; best_fc = 0; }
            }
            if (st.variant == 1) {
                forced(!conv);                 // where marginalization failed
                if (!conv) flags |= kFcRan;
                const long long wf = cand_weight(par ^ 1);
                if (!conv && (!have_best || wf < best_w)) { best_p = cand; best_w = wf; have_best = 1; best_fc = 1; }
                __syncthreads();               // the tile is rewritten next
            }
        }
        if (st.variant == 0) {
            forced(!conv);
            if (!conv) flags |= kFcRan;
            const long long wf = cand_weight((st.max_iters + 1) & 1);
            if (!conv && (!have_best || wf < best_w)) { best_p = cand; best_w = wf; have_best = 1; best_fc = 1; }
        }
        if (best_fc) flags |= kFcChosen;
        // ---- outputs ----
        if (row) {
            const int p = best_p;
            if (st.match) st.match[(size_t)b * st.match_stride + j] = p;
            if (p >= j) {
                const int dp = sdef[gi][p];
                if (g.par[(size_t)myd * N + dp]) atomicXor(&gpred[gi], 1);
                if (st.corr) emit_path(g, myd, dp, st.corr, st.W, b);
            }
            if (st.lambda_out && s <= st.lambda_stride) {
                double *lo = st.lambda_out + (size_t)b * st.lambda_stride * st.lambda_stride +
                             (size_t)j * st.lambda_stride;
                const int jj = opaque(j);
#pragma unroll
                for (int r = 0; r < S; ++r) {
                    const int k = (jj + r >= S) ? jj + r - S : jj + r;
                    if (k < s) lo[k] = (double)lam_at(jj, r) * (double)kLn2F;
                }
            }
        }
        __syncthreads();
        if (live && j == 0) {
            const int px = gpred[gi];
            const int ob = (int)((st.obs[b >> 6] >> (b & 63)) & 1);
            if (px) flags |= kPred;
            if (px != ob) flags |= kFail;
            st.flags[b] = (uint8_t)flags;
        }
        __syncthreads();
    }
}

namespace {

template <int S>
hipError_t launch_s(const DevGraph &g, const DecodeState &st, int cls, hipStream_t stream) {
    // persistent grid: enough workgroups for several per CU; each walks the
    // class list with a grid stride (the count is read on the device)
    const int blocks = 256 * (S <= 64 ? 16 : 4);
    if (st.inv_alpha == 1.0)
        hipLaunchKernelGGL((k_bp_group<S, false>), dim3(blocks), dim3(GroupShape<S>::kThreads), 0, stream, g, st, cls);
    else
        hipLaunchKernelGGL((k_bp_group<S, true>), dim3(blocks), dim3(GroupShape<S>::kThreads), 0, stream, g, st, cls);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bp_group(const DevGraph &g, const DecodeState &st, int cls, hipStream_t stream) {
    switch (class_max_s(cls)) {
    case 16: return launch_s<16>(g, st, cls, stream);
    case 32: return launch_s<32>(g, st, cls, stream);
    case 64: return launch_s<64>(g, st, cls, stream);
    case 96: return launch_s<96>(g, st, cls, stream);
    default: return launch_s<128>(g, st, cls, stream);
    }
}

}  // namespace bpm
