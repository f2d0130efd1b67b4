// BP4M / BP4MF with FP32 arithmetic for shots with at most 192 defects: one
// group of S*K lanes per shot, K lanes per factor row (S in 16..192 by size
// class), each lane holding E = S/K entries of its row in registers.
// Messages are stored as TS (FP32, FP16 or BF16): a message is rounded to TS
// once, when it is written, and both of its readers (the row that computed
// it and the row it is sent to) use the rounded value.
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
// Layout: lane (row i, part h) owns columns k = h*E + e, e = 0..E-1, so every
// register index in the unrolled loops is a compile-time constant.  Messages
// go through an LDS tile T: row i writes M'[i][k] to T(i, k), and reads
// M'[k][i] back as T(k, i) -- a per-lane base plus a compile-time offset.
// The tile layout (layout32 below for FP32; rows of S + 2 16-bit halves,
// written two at a time) keeps bank conflicts of both low.  The
// diagonal T[i][i] is zeroed after the write, so the read of column i yields
// X_i[i] = l_ii and lambda_ii = l_ii + M'[i][i] without a per-entry test.
// Row reductions over the K lanes of a row use DPP lane permutations.
// Columns or rows >= s are padding: priors make them never win a maximum and
// add 0 to every sum.
//
// Marginalization and the convergence check (Sec. II.C-D) run in the same
// pass as the transpose.  Forced convergence (Sec. II.D) picks variables by
// decreasing lambda (ties: smaller (i, j)); it runs as rounds of locally
// dominant choices, which accept exactly the variables of the sequential
// greedy.  Candidate bookkeeping follows BP4M / BP4MF (Sec. III.A-B).

#pragma once

#include <hip/hip_runtime.h>
#include <cfloat>
#include <cstdint>

#include "device_common.hpp"

namespace bpm {

namespace {

constexpr float kLog2eF = 1.4426950408889634f;
constexpr float kLn2F = 0.6931471805599453f;
constexpr float kPadPrior = -1.0e30f;

// Message storage: put rounds an FP32 message to TS, get widens it back.
// For 16-bit storage, lo / hi widen the two halves of a packed pair from its
// bits, so that the row's rounded copies come from the pair just stored
// rather than from a second rounding of the FP32 values.
template <typename TS>
struct MsgStore {
    static __device__ __forceinline__ TS put(float x) { return (TS)x; }
    static __device__ __forceinline__ float get(TS v) { return (float)v; }
    static __device__ __forceinline__ float lo(uint32_t b) {
        if constexpr (sizeof(TS) == 2 && __is_same(TS, __bf16)) return __uint_as_float(b << 16);
        else return (float)__builtin_bit_cast(TS, (uint16_t)b);
    }
    static __device__ __forceinline__ float hi(uint32_t b) {
        if constexpr (sizeof(TS) == 2 && __is_same(TS, __bf16)) return __uint_as_float(b & 0xffff0000u);
        else return (float)__builtin_bit_cast(TS, (uint16_t)(b >> 16));
    }
};

// FP32 tile layout for S columns split over K lanes per row (E = S/K per
// lane), B workgroups per CU: element (r, c) sits at
// r*ST + (r/E)*Q + c + (c/E)*P, i.e. rows of stride ST >= S + (K-1)*P, with
// P extra words between the column parts of a row and Q between the row
// parts of the tile.  Lane (j, h) writes its row at (j, h*E + e) and reads
// column j at (h*E + e, j); with 32 LDS banks of 4 bytes serving 32 lanes per
// cycle, a plain S + 1 stride leaves 2-way (4-way where E is a multiple of
// 32) conflicts on one or both accesses for most splits.  The entries below
// minimise the mean conflict degree of both accesses over all half-waves
// under that bank model (1.0 to 1.33 per access; 2.0 for the row writes of
// the three-workgroup 80 classes, whose LDS leaves no room) while the B
// workgroups keep their double-buffered tiles.  The 88-column split over 8
// lanes keeps stride 92 (2-way writes, conflict-free reads): its modelled
// optimum (stride 88, Q = 4) measured 3% slower.
struct TileLayout32 {
    int st, p, q;
};
constexpr TileLayout32 layout32(int S, int K, int B) {
    return (S == 48 && K == 4)                ? TileLayout32{51, 0, 4}
           : (S == 64 && K == 4)              ? TileLayout32{68, 1, 8}
           : (S == 64 && K == 8)              ? TileLayout32{72, 1, 4}
           : (S == 72 && K == 4)              ? TileLayout32{76, 1, 0}
           : (S == 72 && K == 8)              ? TileLayout32{72, 0, 4}
           : (S == 80 && (K == 4 || B == 3))  ? TileLayout32{S == 80 && K == 4 ? 81 : 80, 0, 4}
           : (S == 80 && K == 8)              ? TileLayout32{88, 1, 4}
           : (S == 88 && K == 4)              ? TileLayout32{92, 1, 0}
           : (S == 88 && K == 8)              ? TileLayout32{92, 0, 0}
           : (S == 104 && K == 4)             ? TileLayout32{108, 1, 0}
           : (S == 104 && K == 8)             ? TileLayout32{104, 0, 4}
           : (S == 112 && K == 4)             ? TileLayout32{116, 1, 8}
           : (S == 112 && K == 8)             ? TileLayout32{120, 1, 4}
           : (S == 120 && K == 4)             ? TileLayout32{124, 1, 0}
           : (S == 120 && K == 8)             ? TileLayout32{120, 0, 4}
           : (S == 128 && K == 4)             ? TileLayout32{132, 1, 8}
           : (S == 128 && K == 8)             ? TileLayout32{136, 1, 4}
           : (S == 192 && K == 4)             ? TileLayout32{196, 1, 8}
                                              : TileLayout32{S + 1, 0, 0};
}

// Shape of one workgroup for size class S, K lanes per factor row, a target
// of B resident workgroups per CU, and messages stored as TS.
template <int S, int K, int B, typename TS>
struct GroupShape {
    static_assert(S % K == 0, "row split");
    static constexpr int kE = S / K;                    // entries per lane
    static constexpr int kLanes = S * K;                // lanes per shot
    static constexpr int kThreads = kLanes <= 64 ? 64 : ((kLanes + 63) / 64) * 64;
    static constexpr int kGroups = kThreads / kLanes;
    static_assert(sizeof(TS) == 4 || sizeof(TS) == 2, "32- or 16-bit messages");
    // above kLdsMaxS the tiles and the priors live in a global-memory slot
    static constexpr bool kGlobal = S > kLdsMaxS;
    // tile layout in elements (16-bit: rows of an odd number of 32-bit words;
    // the global-slot classes keep plain rows of S + 1)
    static constexpr TileLayout32 kL32 = kGlobal ? TileLayout32{S + 1, 0, 0} : layout32(S, K, B);
    static constexpr int kStride = sizeof(TS) == 4 ? kL32.st : S + 2;
    static constexpr int kPadP = sizeof(TS) == 4 ? kL32.p : 0;
    static constexpr int kPadQ = sizeof(TS) == 4 ? kL32.q : 0;
    // elements of one tile: up to the last element (S-1, S-1), at least S rows
    static constexpr int kTileElems = (S - 1) * kStride + S + (K - 1) * (kPadP + kPadQ) > S * kStride
                                          ? (S - 1) * kStride + S + (K - 1) * (kPadP + kPadQ)
                                          : S * kStride;
    static constexpr int kTileBytes = kGroups * kTileElems * (int)sizeof(TS);
    static_assert(kStride >= S + (K - 1) * kPadP, "rows of a tile must not overlap");
    static_assert(!kGlobal || (kGroups == 1 && B == 1 && S <= kGlobalMaxS), "global-slot classes");
    // double-buffer the message tile when B workgroups with two copies each
    // fit in the 160 KB of LDS next to the per-row arrays; FP32 tiles split
    // over four lanes per row at two workgroups per CU stay single (the only
    // such pairs that would fit two, the 88 and 96 classes, ran 17% faster
    // with one: the pipelined verdict's registers cost more than the second
    // barrier)
    static constexpr int kBuffers = kGlobal                                       ? 2
                                    : (sizeof(TS) == 4 && K == 4 && B == 2)       ? 1
                                    : B * (2 * kTileBytes + 1024) <= 156 * 1024 ? 2
                                                                                : 1;
    // waves per SIMD needed for B resident workgroups, for which the
    // compiler keeps the register count low enough.  A workgroup's waves are
    // spread over the 4 SIMDs of a CU with up to ceil(waves / 4) on one of
    // them, so B workgroups need B of those on a SIMD, not the average (at
    // the average's register count, 9-wave workgroups of 82 registers fitted
    // one to a CU instead of two).  That count is asked for where the
    // compiler can grant it (no more than the average occupancy that the 32
    // wave slots of a CU allow for workgroups of this size); otherwise the
    // average.
    static constexpr int kWaves = kThreads / 64;
    static constexpr int kWavesAvg = (B * kWaves + 3) / 4 < 1 ? 1 : (B * kWaves + 3) / 4;
    static constexpr int kWavesOnOneSimd = B * ((kWaves + 3) / 4);
    static constexpr int kWavesSlotLimit = (32 / kWaves) * kWaves / 4;
    static constexpr int kWavesPerEu = kWavesOnOneSimd <= 8 && kWavesOnOneSimd <= kWavesSlotLimit &&
                                               kWavesOnOneSimd > kWavesAvg
                                           ? kWavesOnOneSimd
                                           : kWavesAvg;
};

// Exchange with the lane whose index differs in bit 0 / bit 1 (DPP quad
// permutations [1,0,3,2] and [2,3,0,1]), and with the mirror lane in the
// other half of an aligned group of 8 (DPP row_half_mirror, lane i <-> 7 - i).
// Every lane of a row takes part, so the bound control never applies; it is
// set so that the compiler can fold the move into the operation using it.
__device__ __forceinline__ int dpp_x1(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_x2(int v) { return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_m8(int v) { return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true); }
__device__ __forceinline__ float dpp_x1(float v) { return __int_as_float(dpp_x1(__float_as_int(v))); }
__device__ __forceinline__ float dpp_x2(float v) { return __int_as_float(dpp_x2(__float_as_int(v))); }
__device__ __forceinline__ float dpp_m8(float v) { return __int_as_float(dpp_m8(__float_as_int(v))); }

template <int K, typename T, typename F>
__device__ __forceinline__ T row_reduce(T v, F op) {
    static_assert(K == 1 || K == 2 || K == 4 || K == 8, "K in {1,2,4,8}");
    if constexpr (K >= 2) v = op(v, dpp_x1(v));
    if constexpr (K >= 4) v = op(v, dpp_x2(v));
    if constexpr (K >= 8) v = op(v, dpp_m8(v));
    return v;
}

// Strict order of forced convergence: larger lambda first, then smaller
// (min(i,j), max(i,j)).  Between two variables (j, ka) and (j, kb) of one
// row j (k = j: the row's boundary variable) the pairs (min, max) ascend
// with k: (k, j) for k < j, then (j, j), then (j, k) for k > j; so a tie
// goes to the smaller k.
__device__ __forceinline__ bool fc_row_before(float la, int ka, float lb, int kb) {
    return la > lb || (la == lb && ka < kb);
}

}  // namespace

template <int S, int K, int kVariant, int B, typename TS>
__global__ __launch_bounds__((GroupShape<S, K, B, TS>::kThreads))
__attribute__((amdgpu_waves_per_eu(GroupShape<S, K, B, TS>::kWavesPerEu, 8)))
void k_bp_group(DecodeShared c, int cls) {
    using Shape = GroupShape<S, K, B, TS>;
    using MS = MsgStore<TS>;
    using TS2 = TS __attribute__((ext_vector_type(2)));
    constexpr int G = Shape::kGroups;
    constexpr int ST = Shape::kStride;
    constexpr int PP = Shape::kPadP, PQ = Shape::kPadQ;
    constexpr int TE = Shape::kTileElems;
    constexpr int E = Shape::kE;
    constexpr int LANES = Shape::kLanes;
    constexpr int NB = Shape::kBuffers;
    constexpr bool kAllIn = G * LANES == Shape::kThreads;   // no spare lanes
    constexpr int NC = 8 / K;                     // summation chunks per lane
    constexpr int CH = E / NC;                    // columns per chunk (S / 8)
    static_assert(K <= 8 && S % 8 == 0 && NC * CH == E, "canonical summation order");
    constexpr bool KG = Shape::kGlobal;
    __shared__ TS tile_lds[KG ? 1 : NB][KG ? 1 : G][KG ? 1 : TE];
    // message tiles [NB][G][TE]: LDS, or this workgroup's global slot,
    // followed there by the shot's S x S prior matrix
    TS *const tiles = KG ? reinterpret_cast<TS *>(c.gslot + ((size_t)(cls - kFirstGlobalClass) * c.n_gslots + blockIdx.x) *
                                                                  c.gslot_stride)
                         : &tile_lds[0][0][0];
    float *const Lsh = KG ? reinterpret_cast<float *>(tiles + (size_t)NB * G * TE) : nullptr;
    auto tile = [&](int nb, int gg) -> TS * { return tiles + ((size_t)nb * G + gg) * TE; };
    static_assert(!KG || (uint64_t)NB * TE * sizeof(TS) + (uint64_t)S * S * 4 <= global_slot_bytes(sizeof(TS) == 4 ? 0 : 1),
                  "global slot size");
    // position of element (r, c) in a tile
    auto toff = [](int r, int c) -> int { return r * ST + (r / E) * PQ + c + (c / E) * PP; };
    // The global-slot classes exchange messages through LDS, not the slot.  A
    // 16-bit tile fits whole and is exchanged in one phase.  An FP32 tile fits
    // by halves: it splits into four (S/2) x (S/2) blocks; lanes whose columns
    // lie in their own row half (diagonal blocks) exchange first, the
    // off-diagonal pair second, each phase holding two blocks.  Element (r, c)
    // sits in region r/HS at rr*XST + (rr/E)*XQ + cc + (cc/E)*XP (rr, cc taken
    // mod HS; HS = S in one phase).  The strides and gaps put the row writes
    // and the column reads of the active lanes of a half-wave in distinct
    // banks.  The slot tile is still written for the readers outside the
    // exchange (forced convergence, the posterior export): by every iteration
    // under BP4MF, whose forced convergence runs each iteration, by the last
    // one under BP4M.
    constexpr bool kXch = KG && K == 4;
    constexpr bool kSplit = kXch && sizeof(TS) == 4;
    static_assert(!KG || kXch, "global-slot classes split rows over 4 lanes");
    constexpr int HS = kSplit ? S / 2 : S;
    constexpr int XST = kSplit ? (HS % 32 == 0 ? HS + 17 : HS + 1) : S + 8;
    constexpr int XP = kSplit ? (HS % 32 == 0 ? 16 : 0) : 2;
    constexpr int XQ = kSplit ? XP : 8;
    constexpr int XREG = (HS - 1) * XST + ((HS - 1) / E) * (XQ + XP) + HS;
    static_assert(!kXch || (HS % E == 0 && XST >= HS + (HS / E - 1) * XP && (kSplit || XST % 2 == 0)),
                  "exchange geometry");
    __shared__ __attribute__((aligned(16))) TS xch[kXch ? (kSplit ? 2 : 1) * XREG : 1];
    auto xoff = [](int r, int c) -> int {
        const int rr = r % HS, cc = c % HS;
        return (r / HS) * XREG + rr * XST + (rr / E) * XQ + cc + (cc / E) * XP;
    };
    __shared__ uint16_t sdef[G][S];
    __shared__ int32_t pick[2][G][S];
    __shared__ int32_t freef[G][S];
    // path weights: four rotating slots for the marginal candidates, and
    // slot kFcSlot for forced-convergence candidates (cleared after each read)
    constexpr int kFcSlot = 4;
    __shared__ unsigned long long gw[5][G];
    __shared__ int gnc[4][G];
    __shared__ int gpred[G];
    __shared__ int block_any[2];

    const int tid = threadIdx.x;
    const int grp = tid / LANES;                  // == G for spare lanes
    const bool in_group = grp < G;
    // (one shot per workgroup: gi is the constant 0, so that per-group LDS
    // addresses are uniform and need no registers)
    const int gi = (G == 1 || !in_group) ? 0 : grp;
    const int l = in_group ? tid - gi * LANES : 0;
    const int j = l / K;                          // factor row
    const int h = l - j * K;                      // part of the row
    const bool lead = in_group && h == 0;         // one lane per row
    const bool gl0 = in_group && l == 0;          // one lane per group
    // clear weight slot q of the group.  The zero is made opaque where it is
    // stored: as a plain constant the compiler keeps one register pair of
    // zeros alive across the iterations, and spills it.
    auto clear_gw = [&](int q) {
        unsigned long long z = 0;
        __asm__ volatile("" : "+v"(z));
        gw[q][gi] = z;
    };
    const int k0 = h * E;                         // first column owned
    const uint32_t count = c.class_count[cls];
    const uint32_t *list = c.class_list + (size_t)cls * c.total;
    const float inv_alpha = (float)c.inv_alpha;
    // within a tile: own row, own columns at + e; column j of own rows at + e*ST
    // (the entries of one part share its offsets)
    const int row_off = toff(j, k0);
    const int col_off = toff(k0, j);
    // split exchange: own row / column j of own rows, and the lane's phase
    const int xrow = kXch ? xoff(j, k0) : 0;
    const int xcol = kXch ? xoff(k0, j) : 0;
    const int xdiag = kXch ? xoff(j, j) : 0;
    const int xph = kSplit && j / HS != h / 2 ? 1 : 0;
    // BP4M consumes the verdict of iteration t at iteration t + 2: rows load
    // their candidate's path weight at t, add it at t + 1 (the load's
    // latency hidden behind a factor update), and the sum is read at t + 2.
    // BP4MF needs each verdict at once (forced convergence runs in the same
    // iteration).  Flag slots rotate over 4 iterations.
    constexpr bool pipelined = kVariant == 0 && NB == 2;

    for (uint32_t base = blockIdx.x * (uint32_t)G; base < count; base += gridDim.x * (uint32_t)G) {
        const uint32_t item = base + (uint32_t)gi;
        const bool live = in_group && item < count;
        const uint32_t x = live ? list[item] : 0u;   // global shot index
        int ii = find_instance(c, x);
        // one shot per workgroup: the instance is workgroup-uniform (lane 0
        // of every wave belongs to the group), so its fields load as scalars
        if constexpr (G == 1) ii = __builtin_amdgcn_readfirstlane(ii);
        DevGraph g;
        InstState st;
        uint64_t ibase, iblock0;
        load_instance(c, ii, g, st, ibase, iblock0);
        const int N = g.n_det;
        const uint64_t b = live ? x - ibase : 0;      // shot within the instance
        const int s = live ? st.s[b] : 0;
        const bool row = live && j < s;
        if (lead) sdef[gi][j] = row ? st.defects[b * (uint64_t)c.s_cap + j] : 0;
        if (gl0) {
            // slots 3 and 0 stand for iterations -1 and 0: not converged
            for (int q = 0; q < 4; ++q) { gw[q][gi] = 0; gnc[q][gi] = q == 0 || q == 3; }
            gw[kFcSlot][gi] = 0;
            gpred[gi] = 0;
        }
        __syncthreads();
        const int myd = sdef[gi][j];
        // the row of the packed upper-triangle prior table (2.8 MB at d = 13,
        // small enough to stay in one XCD's L2, where the square table is not)
        const uint32_t myrow = tri_row((uint32_t)N, (uint32_t)myd);
        const float Ljj = row ? g.llr32u[myrow + myd] * kLog2eF : 0.0f;

        // prior of (row j, column k): the same value wherever it is read.
        // Defects ascend, so the columns k >= j lie in the row's own part of
        // the triangle and the columns k < j in their rows' parts.
        auto prior = [&](int k) -> float {
            if (!row) return 0.0f;
            if (k >= s) return kPadPrior;
            const uint32_t dk = sdef[gi][k];
            return g.llr32u[k >= j ? myrow + dk : tri_index((uint32_t)N, dk, (uint32_t)myd)] * kLog2eF;
        };
        // the row's priors: in registers with compile-time offsets, staged
        // through lane-private slots of the (still unused) LDS tile, P entries
        // per pass; or, for the global-slot classes, in the shot's prior
        // matrix, re-read every iteration
        float nL[KG ? 1 : E], A[E];                   // -priors; X, then messages
        float *const Lrow = KG ? Lsh + (size_t)j * S + k0 : nullptr;
        if constexpr (KG) {
            if (kAllIn || in_group) {
#pragma unroll 4
                for (int e = 0; e < E; ++e) Lrow[e] = prior(k0 + e);
            }
#pragma unroll
            for (int e = 0; e < E; ++e) A[e] = Lrow[e];   // X while all messages are 0
        } else if constexpr (sizeof(tile_lds) >= (size_t)4 * G * S * S) {
            // the prior matrix is symmetric: each lane loads the entries of
            // its columns at or above the diagonal (each pair once) and
            // writes them to both halves of an S x S matrix in the tile
            float *const Pm = reinterpret_cast<float *>(tiles) + (size_t)gi * S * S;
            if (kAllIn || in_group) {
#pragma unroll 4
                for (int e = 0; e < E; ++e) {
                    const int k = k0 + e;
                    if (k >= j) {
                        const float v = prior(k);
                        Pm[j * S + k] = v;
                        Pm[k * S + j] = v;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) {
                nL[e] = -Pm[j * S + k0 + e];
                A[e] = -nL[e];                        // X while all messages are 0
            }
        } else {
            constexpr int kSlots = (int)(sizeof(tile_lds) / sizeof(float)) / (G * LANES);
            constexpr int P = kSlots < E ? kSlots : E;
            static_assert(P >= 1, "staging room");
            float *const stage = reinterpret_cast<float *>(tiles) + (size_t)(in_group ? tid : 0) * P;
#pragma unroll
            for (int p0 = 0; p0 < E; p0 += P) {
                if (kAllIn || in_group) {             // spare lanes only read
#pragma unroll 4
                    for (int e = p0; e < p0 + P && e < E; ++e) stage[e - p0] = prior(k0 + e);
                }
#pragma unroll
                for (int e = p0; e < p0 + P && e < E; ++e) {
                    nL[e] = -stage[e - p0];
                    A[e] = -nL[e];                    // X while all messages are 0
                }
            }
        }
        // -prior of entry e
        auto negl = [&](int e) -> float {
            if constexpr (KG) return -Lrow[e];
            else return nL[e];
        };
        __syncthreads();                              // staging reads done

        int have_best = 0, best_fc = 0, conv = 0, flags = 0, best_p = j;
        long long best_w = 0;
        int cand = j;
        // pipelined BP4M: candidates of the last two iterations, whether the
        // last one had exactly one positive variable, and its path weight;
        // BP4MF: the last iteration's candidate and its path weight
        int cand1 = j, cand2 = j;
        bool one1 = false;
        unsigned long long pend = 0;
        float mdiag = 0.0f;                           // M'[j][j] of the current tile
        const TS *Tcur = tile(0, gi);                 // tile of the last iteration

        // posterior of (row j, column k) from the current tile, for the
        // rolled loops below (forced convergence, posterior export)
        auto lam_at = [&](int k) -> float {
            if (k == j) return Ljj + mdiag;
            return prior(k) + (MS::get(Tcur[toff(j, k)]) + MS::get(Tcur[toff(k, j)]));
        };

        // forced convergence on the current tile -> cand (block-uniform)
        // posterior of the row's entry e (column k0 + e != j) from the
        // current tile and the priors in registers
        auto lam_e = [&](int e) -> float {
            return -negl(e) + (MS::get(Tcur[row_off + e]) + MS::get(Tcur[col_off + e * ST]));
        };
        // BP4MF: the lane's best variable of this iteration's posteriors
        // (the boundary variable and its columns), found in the exchange
        // pass in the order a first scan would take, so that forced
        // convergence starts without one
        float bl0 = -FLT_MAX;
        int bk0 = j;
        // the row's best of its lanes' candidates (lanes that are not
        // candidates offer nothing), the same value on every lane of the row
        auto row_pick = [&](bool mine, float bl_, int bk_) -> int {
            float rl = mine ? bl_ : -FLT_MAX;
            int rk = mine ? bk_ : j;
            if constexpr (K >= 2) {
                const float ol = dpp_x1(rl);
                const int ok = dpp_x1(rk);
                if (fc_row_before(ol, ok, rl, rk)) { rl = ol; rk = ok; }
            }
            if constexpr (K >= 4) {
                const float ol = dpp_x2(rl);
                const int ok = dpp_x2(rk);
                if (fc_row_before(ol, ok, rl, rk)) { rl = ol; rk = ok; }
            }
            if constexpr (K >= 8) {
                const float ol = dpp_m8(rl);
                const int ok = dpp_m8(rk);
                if (fc_row_before(ol, ok, rl, rk)) { rl = ol; rk = ok; }
            }
            return rk;
        };
        // BP4MF passes the flag slot of the iteration (qv >= 0): every row is
        // marked free, and the verdict read after the first barrier decides
        // whether the rounds run (returns whether they did)
        auto forced = [&](bool want, int qv) -> bool {
            // BP4MF: the row's own free flag is also kept in a register by
            // every lane of the row (they all see the same picks), so that a
            // round reads only the other rows' flags
            bool free_me = (qv >= 0 || want) && row;
            if (lead) freef[gi][j] = free_me ? 1 : 0;
            auto own_free = [&]() -> bool {
                if constexpr (kVariant == 1) return free_me;
                else return freef[gi][j] != 0;
            };
            // BP4MF: likewise the row's own pick of the round
            int my_pick = j;
            if (tid == 0) block_any[0] = 0;
            // BP4M runs this once, after the last iteration: the row's
            // posteriors are fixed during the rounds and A is free to hold them
            if constexpr (kVariant == 0) {
#pragma unroll
                for (int e = 0; e < E; ++e) A[e] = lam_e(e);
            }
            // BP4MF: the first round's picks before the first barrier (every
            // row is free then, and each lane's best is known from the
            // exchange pass), so that this barrier also serves that round
            if constexpr (kVariant == 1) {
                if (qv >= 0) {
                    const int rk = row_pick(in_group && row, bl0, bk0);
                    if (in_group && row && lead) pick[0][gi][j] = rk;
                    my_pick = rk;
                }
            }
            __syncthreads();
            // (per group: a workgroup of several groups runs the rounds, and
            // their barriers, for all of them; one group may leave at once)
            const bool want_g = qv < 0 || gnc[qv][gi] != 0;
            if constexpr (G == 1) {
                if (!want_g) return false;                     // marginalization converged
            }
            // The lane's best variable among the row's boundary variable and
            // its own free columns.  A check only ever stops being free, so
            // the best stays the best until its own column is taken; only
            // then is the lane's range scanned again (the posteriors are fixed
            // during the rounds).  Columns >= s are never free.
            float bl = -FLT_MAX;
            int bk = j;
            auto scan = [&]() {
                if constexpr (kVariant == 0) {
                    bl = Ljj + mdiag;
                    bk = j;
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int k = k0 + e;
                        if (k != j && freef[gi][k]) {
                            if (fc_row_before(A[e], k, bl, bk)) { bl = A[e]; bk = k; }
                        }
                    }
                } else {
                    // BP4MF rescans run in every round: four entries' flags
                    // and posteriors are read together, then chosen without
                    // branches (the first of equal values stays, as the
                    // columns ascend), and the boundary variable joins last
                    float cl = -FLT_MAX;
                    int ce = 0;
#pragma unroll
                    for (int c = 0; c < E; c += 4) {
                        int fr[4];
                        float lv[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (c + i < E) { fr[i] = freef[gi][k0 + c + i]; lv[i] = lam_e(c + i); }
                        }
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (c + i < E) {
                                const bool take = (k0 + c + i != j) & (fr[i] != 0) & (lv[i] > cl);
                                cl = take ? lv[i] : cl;
                                ce = take ? c + i : ce;
                            }
                        }
                    }
                    bl = cl;
                    bk = k0 + ce;
                    const float lb = Ljj + mdiag;
                    if (fc_row_before(lb, j, bl, bk)) { bl = lb; bk = j; }
                }
            };
            if (in_group && want_g && own_free()) {
                // every column below s is free at the start, and the padding
                // columns' posteriors never beat the boundary variable's
                if constexpr (kVariant == 1) { bl = bl0; bk = bk0; }
                else scan();
            }
            // every round accepts at least the best free variable, so S
            // rounds always suffice; the bound only guards the loop.  Two
            // barriers per round: the picks and the any-left flag alternate
            // between two buffers, so a round's writes never meet the
            // previous round's reads.
            for (int round = 0;; ++round) {
                const int rb = round & 1;
                const bool mine = in_group && want_g && own_free();
                if (!(kVariant == 1 && qv >= 0 && round == 0)) {
                    if (mine && bk != j && !freef[gi][bk]) scan();
                    const int rk = row_pick(mine, bl, bk);
                    if (mine && lead) pick[rb][gi][j] = rk;
                    if constexpr (kVariant == 1) my_pick = rk;
                    __syncthreads();
                }
                // (the next round's flag was last read before this barrier)
                if (tid == 0) block_any[rb ^ 1] = 0;
                if (mine) {
                    int k;
                    if constexpr (kVariant == 1) k = my_pick;
                    else k = pick[rb][gi][j];
                    const bool mutual = k == j || pick[rb][gi][k] == j;
                    if (mutual) cand = k;
                    else if (round >= S) cand = j;
                    else block_any[rb] = 1;
                    // (no row reads the free flags between the two barriers)
                    if (mutual || round >= S) {
                        if constexpr (kVariant == 1) free_me = false;
                        if (lead) freef[gi][j] = 0;
                    }
                }
                __syncthreads();
                if (block_any[rb] == 0) break;
            }
            return want_g;
        };

        // total weight of `cand` over the group, in weight slot q, which is
        // zero on entry and cleared again before return (block-uniform)
        auto cand_weight = [&](int q) -> long long {
            if (row && lead && cand >= j)
                atomicAdd(&gw[q][gi], (unsigned long long)g.dist[(size_t)myd * N + sdef[gi][cand]]);
            __syncthreads();
            const long long w = (long long)gw[q][gi];
            __syncthreads();
            if (gl0) gw[q][gi] = 0;
            return w;
        };

        // verdict of an iteration from flag slot q, with that iteration's
        // marginal candidate c
        auto consume = [&](int q, int c) {
            conv = gnc[q][gi] == 0;
            const long long w = (long long)gw[q][gi];
            if (conv) {
                flags |= kConvergedAny;
                if (!have_best || w < best_w) { best_p = c; best_w = w; have_best = 1; best_fc = 0; }
            }
        };

        // BP4MF: the verdict of an iteration from flag slot q, with its
        // candidate c (marginal if it converged, forced otherwise)
        auto decide = [&](int q, int c) {
            const bool cv = gnc[q][gi] == 0;
            const long long w = (long long)gw[q][gi];
            if (cv) flags |= kConvergedAny;
            else flags |= kFcRan;
            if (!have_best || w < best_w) { best_p = c; best_w = w; have_best = 1; best_fc = cv ? 0 : 1; }
        };
        for (int t = 1; t <= c.max_iters; ++t) {
            TS *const Tb = tile(NB == 2 ? (t & 1) : 0, gi);
            const int q = t % 4;                      // this iteration's flag slot
            // ---- factor update of row j ----
            // (four running maxima, started from the first entries: a start
            // at -FLT_MAX costs a move each and changes nothing)
            float m4[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) m4[c] = A[c < E ? c : 0];
#pragma unroll
            for (int e = 4; e < E; ++e) m4[e & 3] = fmaxf(m4[e & 3], A[e]);
            float m = fmaxf(fmaxf(m4[0], m4[1]), fmaxf(m4[2], m4[3]));
            m = row_reduce<K>(m, [](float a, float c) { return fmaxf(a, c); });
            // row sums in one fixed order for every K: eight chunks of S/8
            // columns (two interleaved partial sums each), combined pairwise
            // in a binary tree, first inside the lane, then across lanes
            float es[NC][2], hs[NC][2];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const float gv = __builtin_amdgcn_exp2f(A[e] - m);
                A[e] = gv;
                const float fv = __builtin_amdgcn_fractf(gv);
                // the first term of each partial sum starts it (0 + x is not
                // folded to x under strict FP): same value, one add fewer
                if ((e % CH) < 2) { es[e / CH][(e % CH) & 1] = gv; hs[e / CH][(e % CH) & 1] = fv; }
                else { es[e / CH][(e % CH) & 1] += gv; hs[e / CH][(e % CH) & 1] += fv; }
            }
            float ep[NC], hp[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) { ep[c] = es[c][0] + es[c][1]; hp[c] = hs[c][0] + hs[c][1]; }
#pragma unroll
            for (int w = 1; w < NC; w *= 2) {
#pragma unroll
                for (int c = 0; c < NC; c += 2 * w) { ep[c] = ep[c] + ep[c + w]; hp[c] = hp[c] + hp[c + w]; }
            }
            const float esum = row_reduce<K>(ep[0], [](float a, float c) { return a + c; });
            float hsum = row_reduce<K>(hp[0], [](float a, float c) { return a + c; });
            const float n_max = rintf(esum - hsum);
            hsum = fmaxf(hsum, 0x1p-120f);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const float v = hsum + (n_max - A[e]);
                A[e] = -m - __builtin_amdgcn_logf(v);
            }
            // store, rounded to TS; the row keeps the rounded values
            const bool gst = !kXch || kVariant != 0 || t == c.max_iters;
            if constexpr (sizeof(TS) == 2 && E % 2 == 0) {
#pragma unroll
                for (int e = 0; e < E; e += 2) {
                    const TS2 pr2 = {MS::put(A[e]), MS::put(A[e + 1])};
                    if ((kAllIn || in_group) && gst) *reinterpret_cast<TS2 *>(&Tb[row_off + e]) = pr2;
                    if constexpr (kXch) {
                        if (kAllIn || in_group) *reinterpret_cast<TS2 *>(&xch[xrow + e]) = pr2;
                    }
                    uint32_t bits = __builtin_bit_cast(uint32_t, pr2);
                    // (an empty register constraint: the halves are widened from
                    // these bits, not recomputed from A by the compiler)
                    if constexpr (!__is_same(TS, __bf16)) __asm__ volatile("" : "+v"(bits));
                    A[e] = MS::lo(bits);
                    A[e + 1] = MS::hi(bits);
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const TS q1 = MS::put(A[e]);
                    if ((kAllIn || in_group) && gst) Tb[row_off + e] = q1;
                    A[e] = MS::get(q1);
                }
            }
            {
                const float gjj = __builtin_amdgcn_exp2f(Ljj - m);
                mdiag = MS::get(MS::put(-m - __builtin_amdgcn_logf(hsum + (n_max - gjj))));
            }
            if ((kAllIn || in_group) && gst) Tb[toff(j, j)] = MS::put(0.0f);
            // (the diagonal element belongs to a diagonal block: phase 0 only)
            auto xwrite = [&](bool diag) {
#pragma unroll
                for (int e = 0; e < E; ++e) xch[xrow + e] = A[e];
                if (diag) xch[xdiag] = 0.0f;
            };
            if constexpr (kSplit) {
                if ((kAllIn || in_group) && xph == 0) xwrite(true);
            } else if constexpr (kXch) {
                if (kAllIn || in_group) xch[xdiag] = MS::put(0.0f);   // row already written
            }
            if constexpr (kVariant == 1) {
                if (t > 1 && pend) atomicAdd(&gw[(t + 3) % 4][gi], pend);   // iteration t - 1
            }
            __syncthreads();
            Tcur = Tb;
            // the verdict taken in this iteration (pipelined BP4M: of
            // iteration t - 2; BP4MF: of t - 1) is read before the column
            // reads, so that waiting for it does not wait for them
            int pre_nc = 0;
            unsigned long long pre_w = 0;
            if constexpr (pipelined || kVariant == 1) {
                constexpr int back = pipelined ? 2 : 3;
                pre_nc = gnc[(t + back) % 4][gi];
                pre_w = gw[(t + back) % 4][gi];
                __asm__ volatile("" ::: "memory");
            }
            // column j of the new tile: the reads are issued before the
            // verdict bookkeeping, which hides part of their latency
            float rv[kXch ? 1 : E];
            if constexpr (!kXch) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    rv[e] = MS::get(Tb[col_off + e * ST]);
                    // With four lanes per row, one read per entry at an
                    // immediate offset from one base: left to itself the
                    // compiler pairs the reads and spends an address add per
                    // pair (the 104 class 5% faster without; no gain at eight
                    // lanes per row, which keep the pairs)
                    if constexpr (K == 4) __asm__ volatile("" ::: "memory");
                }
            }
            if constexpr (kVariant == 1) {
                // BP4MF: the verdict of iteration t - 1, whose candidate's
                // weight was added before this iteration's barrier
                if (t > 1) {
                    const bool cv = pre_nc == 0;
                    const long long w = (long long)pre_w;
                    if (cv) flags |= kConvergedAny;
                    else flags |= kFcRan;
                    if (!have_best || w < best_w) { best_p = cand1; best_w = w; have_best = 1; best_fc = cv ? 0 : 1; }
                }
                if (gl0) { gnc[(t + 1) % 4][gi] = 0; clear_gw((t + 1) % 4); }
            }
            if constexpr (pipelined) {
                conv = pre_nc == 0;                       // verdict of iteration t - 2
                if (conv) {
                    flags |= kConvergedAny;
                    if (!have_best || (long long)pre_w < best_w) {
                        best_p = cand2; best_w = (long long)pre_w; have_best = 1; best_fc = 0;
                    }
                }
                if (row && lead && one1 && cand1 >= j)    // weight of iteration t - 1
                    atomicAdd(&gw[(t + 3) % 4][gi], pend);
                if (gl0) { gnc[(t + 1) % 4][gi] = 0; clear_gw((t + 1) % 4); }
            }
            // ---- transpose, marginalization, next X ----
            // lambda_jk > 0  <=>  M'[j][k] + M'[k][j] > -l_jk (the rounded sum
            // l + t is positive exactly when t > -l); the row converged iff
            // exactly one of its variables is positive (a count per lane, not
            // a flag per entry: no per-entry lane masks stay live)
            // last positive entry, as an offset from k0 (-1 - k0: none), and
            // the positives
            int hi = -1 - k0, npos = 0;
            // (BP4MF) the lane's best posterior in forced convergence's order
            // (larger first, then the smaller column), its columns taken in
            // increasing order so that the first of equal values stays: one
            // compare per entry.  The diagonal entry's posterior is exactly
            // the boundary variable's (its column message is the zeroed
            // diagonal, its own message M'[j][j], its prior l_jj), so the
            // boundary takes part at its own place, column j; lanes without
            // column j meet it after the pass.
            int be0 = 0;
            if constexpr (kVariant == 1) bl0 = -FLT_MAX;
            auto track = [&](float lv, int e) {
                const bool take = lv > bl0;
                bl0 = take ? lv : bl0;
                be0 = take ? e : be0;
            };
            if constexpr (kXch) {
                auto xread = [&]() {
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const float recv = MS::get(xch[xcol + e * XST]);
                        const float nl = negl(e);
                        const float tt = A[e] + recv;
                        const bool pos = tt > nl;
                        hi = pos ? e : hi;
                        npos += pos ? 1 : 0;
                        if constexpr (kVariant == 1) track(-nl + tt, e);
                        A[e] = fmaf(recv, inv_alpha, -nl);
                    }
                };
                if (xph == 0) xread();
                __syncthreads();                      // phase-0 reads done
                if constexpr (kSplit) {
                    if ((kAllIn || in_group) && xph == 1) xwrite(false);
                    __syncthreads();
                    if (xph == 1) xread();
                    __syncthreads();                  // before the next phase-0 writes
                }
            } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const float recv = rv[e];
                const float nl = negl(e);
                const float tt = A[e] + recv;
                const bool pos = tt > nl;
                hi = pos ? e : hi;
                npos += pos ? 1 : 0;
                if constexpr (kVariant == 1) track(-nl + tt, e);
                A[e] = fmaf(recv, inv_alpha, -nl);
            }
            }
            if constexpr (kVariant == 1) {
                bk0 = k0 + be0;
                const float lb = Ljj + mdiag;
                if (fc_row_before(lb, j, bl0, bk0)) { bl0 = lb; bk0 = j; }
            }
            hi += k0;
            hi = row_reduce<K>(hi, [](int a, int c) { return max(a, c); });
            npos = row_reduce<K>(npos, [](int a, int c) { return a + c; });
            const bool one = npos == 1;
            cand = hi < 0 ? j : hi;
            if (row && lead && !one) gnc[q][gi] = 1;
            if constexpr (pipelined) {
                if (row && lead && one && cand >= j)      // added next iteration
                    pend = (unsigned long long)g.dist[(size_t)myd * N + sdef[gi][cand]];
                cand2 = cand1;
                cand1 = cand;
                one1 = one;
            } else if constexpr (kVariant == 1) {
                // forced convergence where marginalization failed; the
                // iteration's candidate (marginal or forced) has its path
                // weight loaded now and added before the next iteration's
                // barrier, after which the verdict is taken
                // (no end-of-iteration barrier: the rounds end with one after
                // their last tile reads, and a converged iteration reads the
                // tile only before the first)
                forced(false, q);
                pend = (row && lead && cand >= j) ? (unsigned long long)g.dist[(size_t)myd * N + sdef[gi][cand]] : 0ull;
                cand1 = cand;
            } else {
                if (row && lead && one && cand >= j)
                    atomicAdd(&gw[q][gi], (unsigned long long)g.dist[(size_t)myd * N + sdef[gi][cand]]);
                __syncthreads();
                consume(q, cand);
                if (gl0) { gnc[(t + 1) % 4][gi] = 0; clear_gw((t + 1) % 4); }
                __syncthreads();                   // the tile is rewritten next
            }
        }
        if constexpr (pipelined) {
            const int T = c.max_iters;
            __syncthreads();
            consume((T + 3) % 4, cand2);                  // iteration T - 1
            if (row && lead && one1 && cand1 >= j) atomicAdd(&gw[T % 4][gi], pend);
            __syncthreads();
            consume(T % 4, cand1);                        // iteration T
        }
        if constexpr (kVariant == 1) {
            const int T = c.max_iters;
            if (T >= 1) {
                if (pend) atomicAdd(&gw[T % 4][gi], pend);
                __syncthreads();
                decide(T % 4, cand1);
            }
        }
        if constexpr (kVariant == 0) {
            forced(!conv, -1);
            if (!conv) flags |= kFcRan;
            const long long wf = cand_weight(kFcSlot);
            if (!conv && (!have_best || wf < best_w)) { best_p = cand; best_w = wf; have_best = 1; best_fc = 1; }
        }
        if (best_fc) flags |= kFcChosen;
        // ---- outputs ----
        if (row && lead) {
            const int p = best_p;
            if (st.match) st.match[(size_t)b * st.match_stride + j] = p;
            if (p >= j) {
                const int dp = sdef[gi][p];
                if (g.par[(size_t)myd * N + dp]) atomicXor(&gpred[gi], 1);
                if (st.corr) emit_path(g, myd, dp, st.corr, st.W, b);
            }
        }
        if (row && st.lambda_out && s <= st.lambda_stride) {
            double *lo = st.lambda_out + (size_t)b * st.lambda_stride * st.lambda_stride +
                         (size_t)j * st.lambda_stride;
#pragma unroll 1
            for (int k = k0; k < k0 + E && k < s; ++k) lo[k] = (double)lam_at(k) * (double)kLn2F;
        }
        __syncthreads();
        if (live && l == 0) {
            const int px = gpred[gi];
            const int ob = st.obs ? (int)((st.obs[b >> 6] >> (b & 63)) & 1) : 0;
            if (px) flags |= kPred;
            if (px != ob) flags |= kFail;
            st.flags[b] = (uint8_t)flags;
        }
        __syncthreads();
    }
}

// Resident workgroups per CU for a kernel and block size (register, LDS
// and wave limits), from the runtime's occupancy calculator.
inline int blocks_per_cu(const void *kernel, int threads) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) {
        (void)hipGetLastError();
        nb = 1;
    }
    return nb;
}

inline int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) {
        (void)hipGetLastError();
        n = 256;
    }
    return n;
}

template <int S, int K, int B, int V, typename TS>
hipError_t launch_skbv(const DecodeShared &c, int cls, hipStream_t stream) {
    using Shape = GroupShape<S, K, B, TS>;
    // persistent grid: as many workgroups as stay resident, each walking
    // the class list with a grid stride (the count is read on the device)
    static const int per_cu = blocks_per_cu((const void *)&k_bp_group<S, K, V, B, TS>, Shape::kThreads);
    int blocks = device_cus() * per_cu;
    if (Shape::kGlobal) {
        if (!c.gslot || c.n_gslots < 1) return hipErrorInvalidValue;
        blocks = blocks < c.n_gslots ? blocks : c.n_gslots;
    }
    const dim3 grid(blocks), block(Shape::kThreads);
    hipLaunchKernelGGL((k_bp_group<S, K, V, B, TS>), grid, block, 0, stream, c, cls);
    return hipGetLastError();
}

template <int S, int K, int B, typename TS>
hipError_t launch_skb(const DecodeShared &c, int cls, hipStream_t stream) {
    return c.variant == 0 ? launch_skbv<S, K, B, 0, TS>(c, cls, stream) : launch_skbv<S, K, B, 1, TS>(c, cls, stream);
}

// Kernel configurations of each size class, as (lanes per row K, resident
// workgroups per CU B); the first is the default.  All give the same
// results: K and B only change how the work is spread over lanes and CUs.
// K fixes the unrolled entries per lane (E = S/K) and, for the small
// classes, the shots per workgroup (64-lane workgroups hold 64/(S K) shots:
// 4, 2 or 1 at S = 16, 2 or 1 at S = 32).
struct KB { int K, B; };
constexpr int kMaxCfg = 4;
struct ClassCfgs { int n; KB c[kMaxCfg]; };
constexpr ClassCfgs configs_of(int S) {
    switch (S) {
    case 16: return {3, {{1, 1}, {2, 1}, {4, 1}}};
    case 32: return {3, {{2, 1}, {1, 1}, {4, 1}}};
    case 48: return {2, {{4, 1}, {2, 1}}};
    case 64: return {2, {{4, 1}, {8, 1}}};
    case 72: return {4, {{8, 2}, {4, 3}, {8, 1}, {8, 3}}};
    case 80: return {4, {{8, 3}, {4, 3}, {8, 1}, {8, 2}}};
    case 88: return {3, {{8, 2}, {8, 1}, {4, 2}}};
    case 96: return {3, {{8, 2}, {8, 1}, {4, 2}}};
    case 104: return {3, {{4, 2}, {8, 1}, {8, 2}}};
    case 112: return {3, {{4, 2}, {8, 1}, {8, 2}}};
    case 120: return {3, {{4, 2}, {8, 1}, {8, 2}}};
    case 128: return {3, {{4, 2}, {8, 1}, {8, 2}}};
    case 160: return {1, {{4, 1}}};
    case 192: return {1, {{4, 1}}};
    case 224: return {1, {{4, 1}}};
    case 256: return {1, {{4, 1}}};
    default: return {0, {}};
    }
}

template <int S, int I, typename TS>
hipError_t launch_cfg(const DecodeShared &c, int cls, hipStream_t stream) {
    constexpr ClassCfgs cc = configs_of(S);
    if constexpr (I < cc.n) {
        return launch_skb<S, cc.c[I].K, cc.c[I].B, TS>(c, cls, stream);
    } else {
        return hipErrorInvalidValue;
    }
}

template <int S, typename TS>
hipError_t launch_class(const DecodeShared &c, int cls, int cfg, hipStream_t stream) {
    static_assert(configs_of(S).n >= 1 && configs_of(S).n <= kMaxCfg, "configuration table");
    switch (cfg) {
    case 0: return launch_cfg<S, 0, TS>(c, cls, stream);
    case 1: return launch_cfg<S, 1, TS>(c, cls, stream);
    case 2: return launch_cfg<S, 2, TS>(c, cls, stream);
    case 3: return launch_cfg<S, 3, TS>(c, cls, stream);
    default: return hipErrorInvalidValue;
    }
}

// Launch the group kernel of size class cls in configuration cfg, messages
// stored as TS.
template <typename TS>
hipError_t launch_group_ts(const DecodeShared &c, int cls, int cfg, hipStream_t stream) {
    if (cfg < 0 || cfg >= configs_of(class_max_s(cls)).n) return hipErrorInvalidValue;
    switch (class_max_s(cls)) {
    case 16: return launch_class<16, TS>(c, cls, cfg, stream);
    case 32: return launch_class<32, TS>(c, cls, cfg, stream);
    case 48: return launch_class<48, TS>(c, cls, cfg, stream);
    case 64: return launch_class<64, TS>(c, cls, cfg, stream);
    case 72: return launch_class<72, TS>(c, cls, cfg, stream);
    case 80: return launch_class<80, TS>(c, cls, cfg, stream);
    case 88: return launch_class<88, TS>(c, cls, cfg, stream);
    case 96: return launch_class<96, TS>(c, cls, cfg, stream);
    case 104: return launch_class<104, TS>(c, cls, cfg, stream);
    case 112: return launch_class<112, TS>(c, cls, cfg, stream);
    case 120: return launch_class<120, TS>(c, cls, cfg, stream);
    case 128: return launch_class<128, TS>(c, cls, cfg, stream);
    case 160: return launch_class<160, TS>(c, cls, cfg, stream);
    case 192: return launch_class<192, TS>(c, cls, cfg, stream);
    case 224: return launch_class<224, TS>(c, cls, cfg, stream);
    case 256: return launch_class<256, TS>(c, cls, cfg, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bpm
