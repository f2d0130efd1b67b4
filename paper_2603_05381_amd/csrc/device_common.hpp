// Device-side structures shared by the bpm kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bpm {

// Read-only tables of one graph, resident in device memory.
struct DevGraph {
    int32_t n_det, n_mech;
    const int32_t *mech_off;     // [n_mech + 1]
    const int32_t *mech_det;     // [mech_off[n_mech]]
    const uint8_t *mech_obs;     // [n_mech]
    const uint32_t *thr;         // [n_mech] firing thresholds
    const float *llr32;          // [N*N] prior LLR (natural log), FP32
    const double *llr64;         // [N*N] prior LLR, FP64
    const int64_t *dist;         // [N*N] fixed-point path weight
    const uint8_t *par;          // [N*N] observable parity of the path
    const int32_t *pred;         // [N*N] last edge of the path
    const int32_t *edge_u;       // [n_mech] first detector of an edge
    const int32_t *edge_v;       // [n_mech] second detector, -1 = boundary
};

// Per-call decode state in the caller's workspace.
struct DecodeState {
    uint64_t n_shots;
    int32_t s_cap;
    int32_t max_iters;
    int32_t variant;             // 0 BP4M, 1 BP4MF
    int32_t store;               // FP32 arithmetic: messages stored as 0 FP32, 1 FP16, 2 BF16
    double inv_alpha;
    const uint64_t *syn;         // [N][W]
    const uint64_t *obs;         // [W]
    uint64_t W;
    int32_t *s;                  // [n]
    uint16_t *defects;           // [n][s_cap], ascending detector ids
    uint8_t *flags;              // [n]
    uint32_t *class_count;       // [kClasses]
    uint32_t *class_list;        // [kClasses][n]
    // optional outputs
    uint64_t *corr;              // [n_mech][W]
    int32_t *match;              // [n][match_stride]
    int32_t match_stride;
    double *lambda_out;          // [n][lambda_stride^2]
    int32_t lambda_stride;
};

// Work classes by defect count: shots with 2 <= s <= class_max_s(c) (and
// above the previous bound) go to class c; larger ones to kClassGeneric.
constexpr int kGroupClasses = 14;
constexpr int kClassGeneric = kGroupClasses;
constexpr int kClasses = kGroupClasses + 1;
__host__ __device__ constexpr int class_max_s(int c) {
    switch (c) {
    case 0: return 16;   case 1: return 32;   case 2: return 48;   case 3: return 64;
    case 4: return 72;   case 5: return 80;   case 6: return 88;   case 7: return 96;
    case 8: return 104;  case 9: return 112;  case 10: return 120; case 11: return 128;
    case 12: return 160; case 13: return 192;
    default: return 0;
    }
}
__host__ __device__ inline int class_of(int s) {
    for (int c = 0; c < kGroupClasses; ++c)
        if (s <= class_max_s(c)) return c;
    return kClassGeneric;
}

enum : uint8_t {
    kConvergedAny = 1, kFcRan = 2, kFcChosen = 4, kPred = 8, kFail = 16, kOverflow = 32
};

// Toggle the edges of the shortest path between defects u <= v (v == u:
// u's boundary path) in the correction planes of batch shot b.
__device__ inline void emit_path(const DevGraph &g, int u, int v, uint64_t *corr, uint64_t W, uint64_t b) {
    const int N = g.n_det;
    const uint64_t bit = 1ull << (b & 63);
    const uint64_t word = b >> 6;
    int y = v;
    if (v == u) {
        int e = g.pred[(size_t)u * N + u];
        atomicXor((unsigned long long *)&corr[(uint64_t)e * W + word], (unsigned long long)bit);
        y = g.edge_u[e];
    }
    while (y != u) {
        int e = g.pred[(size_t)u * N + y];
        atomicXor((unsigned long long *)&corr[(uint64_t)e * W + word], (unsigned long long)bit);
        int a = g.edge_u[e], c = g.edge_v[e];
        y = (a == y) ? c : a;
    }
}

}  // namespace bpm
