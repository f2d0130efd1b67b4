// BP4M / BP4MF with FP32 arithmetic for shots with 257..512 defects: one
// workgroup of 1024 lanes per shot, two lanes per factor row, each lane
// walking its half of the row (up to 256 entries) in loops.  The same
// iteration as the group kernels (flooding schedule, Sec. II.B; the exact
// base-2 leave-one-out log-sum-exp; marginalization and convergence check,
// Sec. II.C-D; forced convergence and the BP4M / BP4MF candidate rules,
// Sec. III.A-B), with the row's values in global memory instead of
// registers: per workgroup a slot holds
//   X[e/4][lane][4]  the lane's entries of X,
//   L[e/4][lane][4]  the lane's priors (base 2),
// both in 16-byte pieces of four entries interleaved by lane, so that a
// lane loads four entries at once and a wave's piece covers one contiguous
// kilobyte, and
// the message tile T[S][ST] (row j writes T[j][k], reads column j as
// T[k][j]; the diagonal is zeroed so column j yields X_j[j] = l_jj).  The
// maximum of a row for the next iteration is taken while its X is written.

#include "bp_group_impl.hpp"

namespace bpm {

namespace {

constexpr int kStreamLanes = 1024;
constexpr int kStreamRows = kStreamLanes / 2;       // two lanes per row

// entries per lane: half a row rounded up to a multiple of 8, so that each
// lane's columns of a tile row start on a 16-byte boundary and its 16-byte
// stores never reach the other lane's columns; the tile row stride is a
// multiple of 32 elements, so that every row starts on a 128-byte cache line
// and a half-wave's column read (32 consecutive rows' entries of one column)
// covers one line (FP32) or half of one (16-bit) instead of straddling two
__host__ __device__ constexpr int stream_entries(int s) { return ((s + 1) / 2 + 7) & ~7; }
__host__ __device__ constexpr int stream_stride(int s) { return (2 * stream_entries(s) + 8 + 31) & ~31; }
constexpr int kStreamMaxE = stream_entries(kStreamMaxS);

template <typename TS>
__host__ __device__ constexpr uint64_t stream_slot_bytes_t() {
    return ((uint64_t)2 * kStreamLanes * kStreamMaxE * 4 +
            (uint64_t)kStreamMaxS * stream_stride(kStreamMaxS) * sizeof(TS) + 255) & ~(uint64_t)255;
}

}  // namespace

template <int kVariant, typename TS>
__global__ __launch_bounds__(kStreamLanes) void k_bp_stream(DecodeShared c, int cls) {
    using MS = MsgStore<TS>;
    __shared__ uint16_t sdef[kStreamRows];
    __shared__ int32_t pick[kStreamRows];
    __shared__ int32_t freef[kStreamRows];
    // path weights: three rotating slots for the marginal candidates, slot 3
    // for forced-convergence candidates (cleared after each read)
    __shared__ unsigned long long gw[4];
    __shared__ int gnc[3];
    __shared__ int gpred;
    __shared__ int block_any;

    const int tid = threadIdx.x;
    const int j = tid >> 1;                       // factor row
    const int h = tid & 1;                        // half of the row
    const bool lead = h == 0;
    const uint32_t count = c.class_count[cls];
    const uint32_t *list = c.class_list + (size_t)cls * c.total;
    const float inv_alpha = (float)c.inv_alpha;
    char *const slot = c.sslot + (size_t)blockIdx.x * c.sslot_stride;
    float *const Xb = reinterpret_cast<float *>(slot);
    float *const Lb = Xb + (size_t)kStreamLanes * kStreamMaxE;
    TS *const T = reinterpret_cast<TS *>(Lb + (size_t)kStreamLanes * kStreamMaxE);
    // entry e of this lane, and its piece p (entries 4p .. 4p+3)
    auto xat = [&](int e) -> float & { return Xb[((e >> 2) * kStreamLanes + tid) * 4 + (e & 3)]; };
    auto lat = [&](int e) -> float & { return Lb[((e >> 2) * kStreamLanes + tid) * 4 + (e & 3)]; };
    float4 *const X4 = reinterpret_cast<float4 *>(Xb);
    const float4 *const L4 = reinterpret_cast<const float4 *>(Lb);
    // the C entries of chunk e0 (a multiple of C) from a piece array, whole
    // pieces below piece np (values past the lane's last entry inside them
    // are never used), `fill` beyond
    auto load_chunk = [&](const float4 *A, int e0, int np, float fill, float *v) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            float4 a = make_float4(fill, fill, fill, fill);
            if ((e0 >> 2) + w < np) a = A[((e0 >> 2) + w) * kStreamLanes + tid];
            v[4 * w] = a.x; v[4 * w + 1] = a.y; v[4 * w + 2] = a.z; v[4 * w + 3] = a.w;
        }
    };

    for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
        const uint32_t x = list[item];
        const int ii = __builtin_amdgcn_readfirstlane(find_instance(c, x));
        DevGraph g;
        InstState st;
        uint64_t ibase, iblock0;
        load_instance(c, ii, g, st, ibase, iblock0);
        const int N = g.n_det;
        const uint64_t b = x - ibase;
        const int s = st.s[b];
        const int E = stream_entries(s);          // entries per lane
        const int ST = stream_stride(s);          // tile row stride (> 2E, multiple of 32)
        const int k0 = h * E;
        const int kend = min(k0 + E, s);          // columns [k0, kend)
        const int ne = kend - k0;
        const int np = (ne + 3) >> 2;             // pieces of X and the priors in use
        const bool row = j < s;
        if (lead && row) sdef[j] = st.defects[b * (uint64_t)c.s_cap + j];
        if (tid < 4) gw[tid] = 0;
        if (tid < 3) gnc[tid] = 0;
        if (tid == 0) gpred = 0;
        __syncthreads();
        const int myd = row ? sdef[j] : 0;
        const float Ljj = row ? g.llr32[(size_t)myd * N + myd] * kLog2eF : 0.0f;

        // priors and initial X; the row maximum of X.  Every pass below
        // walks the lane's entries in chunks of C, issuing the chunk's loads
        // before using them
        constexpr int C = 16;
        float mx = -FLT_MAX;
        if (row) {
            for (int e0 = 0; e0 < ne; e0 += C) {
                float v[C];
#pragma unroll
                for (int u = 0; u < C; ++u)
                    v[u] = e0 + u < ne ? g.llr32[(size_t)myd * N + sdef[k0 + e0 + u]] * kLog2eF : -FLT_MAX;
#pragma unroll
                for (int u = 0; u < C; ++u) {
                    if (e0 + u < ne) {
                        lat(e0 + u) = v[u];
                        xat(e0 + u) = v[u];
                    }
                    mx = fmaxf(mx, v[u]);
                }
            }
        }

        int have_best = 0, best_fc = 0, conv = 0, flags = 0, best_p = j, cand = j;
        long long best_w = 0;
        float mdiag = 0.0f;

        // posterior of (row j, column k), k != j, from the tile
        auto lam = [&](int e) -> float {
            const int k = k0 + e;
            return lat(e) + (MS::get(T[(size_t)j * ST + k]) + MS::get(T[(size_t)k * ST + j]));
        };

        auto forced = [&](bool want) {
            if (lead) freef[j] = (want && row) ? 1 : 0;
            __syncthreads();
            // the lane's best among the boundary variable and its free
            // columns, kept across rounds and rescanned only once its own
            // column is taken (checks only ever stop being free)
            float bl = -FLT_MAX;
            int bk = j;
            auto scan = [&]() {
                bl = Ljj + mdiag;
                bk = j;
                for (int e = 0; e < ne; ++e) {
                    const int k = k0 + e;
                    if (k != j && freef[k]) {
                        const float lv = lam(e);
                        if (fc_row_before(lv, k, bl, bk)) { bl = lv; bk = k; }
                    }
                }
            };
            if (row && freef[j]) scan();
            for (int round = 0;; ++round) {
                const bool mine = row && freef[j];
                if (mine && bk != j && !freef[bk]) scan();
                float rl = mine ? bl : -FLT_MAX;
                int rk = mine ? bk : j;
                {
                    const float ol = dpp_x1(rl);
                    const int ok = dpp_x1(rk);
                    if (fc_row_before(ol, ok, rl, rk)) { rl = ol; rk = ok; }
                }
                if (mine && lead) pick[j] = rk;
                if (tid == 0) block_any = 0;
                __syncthreads();
                if (mine) {
                    const int k = pick[j];
                    if (k == j || pick[k] == j) cand = k;
                    else if (round >= kStreamRows) cand = j;
                    else block_any = 1;
                }
                __syncthreads();
                if (mine && lead) {
                    const int k = pick[j];
                    if (k == j || pick[k] == j || round >= kStreamRows) freef[j] = 0;
                }
                const bool again = block_any != 0;
                __syncthreads();
                if (!again) break;
            }
        };
        auto cand_weight = [&](int q) -> long long {
            if (row && lead && cand >= j) atomicAdd(&gw[q], (unsigned long long)g.dist[(size_t)myd * N + sdef[cand]]);
            __syncthreads();
            const long long w = (long long)gw[q];
            __syncthreads();
            if (tid == 0) gw[q] = 0;
            return w;
        };

        for (int t = 1; t <= c.max_iters; ++t) {
            const int q = t % 3;
            // ---- factor update of row j ----
            const float m = fmaxf(mx, dpp_x1(mx));
            float es0 = 0.0f, es1 = 0.0f, hs0 = 0.0f, hs1 = 0.0f;
            if (row) {
                for (int e0 = 0; e0 < ne; e0 += C) {
                    float v[C];
                    load_chunk(X4, e0, np, -FLT_MAX, v);
#pragma unroll
                    for (int u = 0; u < C; ++u) v[u] = e0 + u < ne ? v[u] : -FLT_MAX;
#pragma unroll
                    for (int u = 0; u < C; ++u) {
                        const float gv = __builtin_amdgcn_exp2f(v[u] - m);   // 0 past the row's end
                        if (u & 1) { es1 += gv; hs1 += __builtin_amdgcn_fractf(gv); }
                        else { es0 += gv; hs0 += __builtin_amdgcn_fractf(gv); }
                    }
                }
            }
            float esum = es0 + es1, hsum = hs0 + hs1;
            esum = esum + dpp_x1(esum);
            hsum = hsum + dpp_x1(hsum);
            const float n_max = rintf(esum - hsum);
            hsum = fmaxf(hsum, 0x1p-120f);
            if (row) {
                // the row's messages go to the tile in 16-byte pieces (the
                // columns past the row's end inside a piece are padding)
                constexpr int V = 16 / (int)sizeof(TS);
                using TSV = TS __attribute__((ext_vector_type(V)));
                TS *const trow = T + (size_t)j * ST + k0;
                for (int e0 = 0; e0 < ne; e0 += C) {
                    // 2^(X - m) again (cheaper than storing and re-reading it)
                    float v[C];
                    load_chunk(X4, e0, np, -FLT_MAX, v);
#pragma unroll
                    for (int u = 0; u < C; ++u) v[u] = e0 + u < ne ? v[u] : -FLT_MAX;
                    TS q[C];
#pragma unroll
                    for (int u = 0; u < C; ++u)
                        q[u] = MS::put(-m - __builtin_amdgcn_logf(hsum + (n_max - __builtin_amdgcn_exp2f(v[u] - m))));
#pragma unroll
                    for (int w = 0; w < C / V; ++w) {
                        if (e0 + w * V < ne) {
                            TSV pv;
#pragma unroll
                            for (int u = 0; u < V; ++u) pv[u] = q[w * V + u];
                            *reinterpret_cast<TSV *>(trow + e0 + w * V) = pv;
                        }
                    }
                }
                const float gjj = __builtin_amdgcn_exp2f(Ljj - m);
                mdiag = MS::get(MS::put(-m - __builtin_amdgcn_logf(hsum + (n_max - gjj))));
                T[(size_t)j * ST + j] = MS::put(0.0f);   // both lanes, after their own writes
            }
            __syncthreads();
            // ---- transpose, marginalization, next X (and its maximum) ----
            int hi = -1, lo = kStreamMaxS;
            mx = -FLT_MAX;
            if (row) {
                // the row's own messages come back from its tile row (16-byte
                // pieces), except at the diagonal, which the tile holds as 0:
                // there the own message is M'[j][j]
                constexpr int V = 16 / (int)sizeof(TS);
                using TSV = TS __attribute__((ext_vector_type(V)));
                const TS *const trow = T + (size_t)j * ST + k0;
                for (int e0 = 0; e0 < ne; e0 += C) {
                    // whole pieces (the own row's inside its stride); entries
                    // past the row's end are masked
                    float rv[C], ow[C], lv[C], xv[C];
#pragma unroll
                    for (int w = 0; w < C / V; ++w) {
                        const TSV pv = *reinterpret_cast<const TSV *>(trow + e0 + w * V);
#pragma unroll
                        for (int u = 0; u < V; ++u) ow[w * V + u] = MS::get(pv[u]);
                    }
                    load_chunk(L4, e0, np, 0.0f, lv);
#pragma unroll
                    for (int u = 0; u < C; ++u) {
                        const int k = min(k0 + e0 + u, s - 1);      // any row past the end
                        rv[u] = MS::get(T[k * ST + j]);
                        if (k0 + e0 + u == j) ow[u] = mdiag;
                    }
#pragma unroll
                    for (int u = 0; u < C; ++u) {
                        const bool in = e0 + u < ne;
                        const int k = k0 + e0 + u;
                        const bool pos = in && ow[u] + rv[u] > -lv[u];
                        hi = pos ? k : hi;
                        lo = pos ? min(lo, k) : lo;
                        xv[u] = fmaf(rv[u], inv_alpha, lv[u]);
                        mx = in ? fmaxf(mx, xv[u]) : mx;
                    }
#pragma unroll
                    for (int w = 0; w < 4; ++w)
                        if ((e0 >> 2) + w < np)
                            X4[((e0 >> 2) + w) * kStreamLanes + tid] =
                                make_float4(xv[4 * w], xv[4 * w + 1], xv[4 * w + 2], xv[4 * w + 3]);
                }
            }
            hi = max(hi, dpp_x1(hi));
            lo = min(lo, dpp_x1(lo));
            const bool one = hi >= 0 && hi == lo;
            cand = hi < 0 ? j : hi;
            if (row && lead && !one) gnc[q] = 1;
            if (row && lead && one && cand >= j)
                atomicAdd(&gw[q], (unsigned long long)g.dist[(size_t)myd * N + sdef[cand]]);
            __syncthreads();
            conv = gnc[q] == 0;
            const long long w = (long long)gw[q];
            if (conv) {
                flags |= kConvergedAny;
                if (!have_best || w < best_w) { best_p = cand; best_w = w; have_best = 1; best_fc = 0; }
            }
            if (tid == 0) { gnc[(t + 1) % 3] = 0; gw[(t + 1) % 3] = 0; }
            if constexpr (kVariant == 1) {
                forced(!conv);
                if (!conv) flags |= kFcRan;
                const long long wf = cand_weight(3);
                if (!conv && (!have_best || wf < best_w)) { best_p = cand; best_w = wf; have_best = 1; best_fc = 1; }
            }
            __syncthreads();                       // the tile is rewritten next
        }
        if constexpr (kVariant == 0) {
            forced(!conv);
            if (!conv) flags |= kFcRan;
            const long long wf = cand_weight(3);
            if (!conv && (!have_best || wf < best_w)) { best_p = cand; best_w = wf; have_best = 1; best_fc = 1; }
        }
        if (best_fc) flags |= kFcChosen;
        // ---- outputs ----
        if (row && lead) {
            const int p = best_p;
            if (st.match) st.match[(size_t)b * st.match_stride + j] = p;
            if (p >= j) {
                const int dp = sdef[p];
                if (g.par[(size_t)myd * N + dp]) atomicXor(&gpred, 1);
                if (st.corr) emit_path(g, myd, dp, st.corr, st.W, b);
            }
        }
        if (row && st.lambda_out && s <= st.lambda_stride) {
            double *lout = st.lambda_out + (size_t)b * st.lambda_stride * st.lambda_stride + (size_t)j * st.lambda_stride;
            for (int e = 0; e < ne; ++e) {
                const int k = k0 + e;
                lout[k] = (double)(k == j ? Ljj + mdiag : lam(e)) * (double)kLn2F;
            }
        }
        __syncthreads();
        if (tid == 0) {
            const int ob = st.obs ? (int)((st.obs[b >> 6] >> (b & 63)) & 1) : 0;
            if (gpred) flags |= kPred;
            if (gpred != ob) flags |= kFail;
            st.flags[b] = (uint8_t)flags;
        }
        __syncthreads();
    }
}

uint64_t stream_slot_bytes(int store) {
    return store == 0 ? stream_slot_bytes_t<float>() : stream_slot_bytes_t<_Float16>();
}

hipError_t launch_bp_stream(const DecodeShared &c, int cls, hipStream_t stream) {
    if (!c.sslot || c.n_sslots < 1) return hipErrorInvalidValue;
    int blocks = device_cus();
    if (blocks > c.n_sslots) blocks = c.n_sslots;
    const dim3 grid(blocks), block(kStreamLanes);
    const bool v1 = c.variant == 1;
    switch (c.store) {
    case 1:
        if (v1) hipLaunchKernelGGL((k_bp_stream<1, _Float16>), grid, block, 0, stream, c, cls);
        else hipLaunchKernelGGL((k_bp_stream<0, _Float16>), grid, block, 0, stream, c, cls);
        break;
    case 2:
        if (v1) hipLaunchKernelGGL((k_bp_stream<1, __bf16>), grid, block, 0, stream, c, cls);
        else hipLaunchKernelGGL((k_bp_stream<0, __bf16>), grid, block, 0, stream, c, cls);
        break;
    default:
        if (v1) hipLaunchKernelGGL((k_bp_stream<1, float>), grid, block, 0, stream, c, cls);
        else hipLaunchKernelGGL((k_bp_stream<0, float>), grid, block, 0, stream, c, cls);
    }
    return hipGetLastError();
}

}  // namespace bpm
