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
    const float *llr32u;         // the same, packed upper triangle: (i, j >= i) at tri_index(N, i, j)
    const double *llr64;         // [N*N] prior LLR, FP64
    const int64_t *dist;         // [N*N] fixed-point path weight
    const uint8_t *par;          // [N*N] observable parity of the path
    const int32_t *pred;         // [N*N] last edge of the path
    const int32_t *edge_u;       // [n_mech] first detector of an edge
    const int32_t *edge_v;       // [n_mech] second detector, -1 = boundary
};

// Position of (i, j), i <= j, in a packed row-major upper triangle of an
// N x N symmetric matrix: row i holds columns i..N-1 after the N + (N-1) +
// ... + (N-i+1) entries of rows 0..i-1.
__host__ __device__ __forceinline__ uint32_t tri_row(uint32_t N, uint32_t i) { return i * N - i * (i + 1) / 2; }
__host__ __device__ __forceinline__ uint32_t tri_index(uint32_t N, uint32_t i, uint32_t j) { return tri_row(N, i) + j; }

// Tanner graph of a code-capacity code with both check types (B-BP4MF):
// qubit v's checks qc[4v..4v+3] are its X checks, then its Z checks (id
// n_xc + z), each ascending (-1 = none); check c's qubits cq[4c..] ascend
// (-1 = none) and cs[4c..] is c's slot in each of those qubits' lists.
// qobs[v]: a Z error on v flips the observable; qmech[v]: the decoding-graph
// edge that is v's Z error.  noff / nedge: the decoding graph's incident
// edges of node u (node n_det = the boundary), ascending.
struct TannerDev {
    int32_t n_q, n_xc, n_zc;
    const int32_t *qc;
    const int32_t *cq;
    const int32_t *cs;
    const uint8_t *qobs;
    const int32_t *qmech;
    const int32_t *noff;
    const int32_t *nedge;
};

// Arguments of the B-BP4MF kernel (one call, one graph).
struct BbpArgs {
    DevGraph g;                  // decoding graph (the X checks) with its tables
    TannerDev tn;
    const uint64_t *synx, *synz, *obs;   // [n_xc][W], [n_zc][W], [W]
    uint64_t n, W;
    int32_t variant, max_iters, s_cap;
    double inv_alpha;
    double pri_i, pri_p;         // ln(1 - p), ln(p / 3)
    char *slots;
    uint64_t slot_bytes;
    int32_t *s_out;              // [n] X-check defects
    uint8_t *flags;              // [n]
    int32_t *match;              // [n][match_stride] or NULL
    int32_t match_stride;
};

// One decoding instance of a call: a graph, its batch of shots, and that
// batch's per-shot state and outputs.  A call decodes one or several
// instances (up to kMaxInstances), each with its own graph.
struct InstState {
    uint64_t n_shots;
    uint64_t W;                  // words per bit plane, ceil(n_shots / 64)
    const uint64_t *syn;         // detector bit planes [N][W], or shot-major rows
                                 // [n_shots][rows_words] when rows_words > 0
    const uint64_t *obs;         // [W] sampled observable flips, or NULL
    int32_t rows_words;
    int32_t *s;                  // [n] defects per shot (workspace)
    uint16_t *defects;           // [n][s_cap], ascending detector ids (workspace)
    uint8_t *flags;              // [n] (workspace)
    // optional outputs
    uint64_t *corr;              // [n_mech][W]
    int32_t *match;              // [n][match_stride]
    int32_t match_stride;
    int32_t lambda_stride;
    double *lambda_out;          // [n][lambda_stride^2]
    uint64_t *obs_pred, *fail;   // [W]
    uint8_t *shot_flags;         // [n]
    int32_t *shot_s;             // [n]
    unsigned long long *counters;    // bpm_counters as 6 x u64
};

struct Instance {
    DevGraph g;
    InstState st;
    uint64_t base;               // global index of the instance's first shot
    uint64_t block0;             // first block of the per-shot launches
};

constexpr int kMaxInstances = 8;

// Options and work queues shared by the instances of a call.
struct DecodeShared {
    int32_t max_iters;
    int32_t variant;             // 0 BP4M, 1 BP4MF
    int32_t store;               // FP32 arithmetic: messages stored as 0 FP32, 1 FP16, 2 BF16
    int32_t s_cap;
    double inv_alpha;
    int32_t n_inst;
    uint64_t total;              // shots over all instances
    const Instance *inst;        // [n_inst], device
    uint32_t *class_count;       // [kClasses]
    uint32_t *class_list;        // [kClasses][total], global shot indices
    char *gslot;                 // workgroup slots of the size classes whose tiles
    uint64_t gslot_stride;       // live in global memory (S > 192):
    int32_t n_gslots;            // [kGlobalClasses][n_gslots][gslot_stride]
    char *sslot;                 // workgroup slots of the streaming class
    uint64_t sslot_stride;       // (257..kStreamMaxS defects): [n_sslots][stride]
    int32_t n_sslots;
};

// The instance table is read-only during a launch: reading it through the
// constant address space lets the compiler use scalar loads when the index
// is uniform.
using InstanceTab = const __attribute__((address_space(4))) Instance *;
__device__ __forceinline__ InstanceTab instance_tab(const DecodeShared &c) { return (InstanceTab)c.inst; }

// Copy of instance i's graph and state, field by field out of the constant
// address space.
__device__ __forceinline__ void load_instance(const DecodeShared &c, int i, DevGraph &g, InstState &st,
                                              uint64_t &base, uint64_t &block0) {
    InstanceTab t = instance_tab(c) + i;
    g.n_det = t->g.n_det; g.n_mech = t->g.n_mech;
    g.mech_off = t->g.mech_off; g.mech_det = t->g.mech_det; g.mech_obs = t->g.mech_obs; g.thr = t->g.thr;
    g.llr32 = t->g.llr32; g.llr32u = t->g.llr32u; g.llr64 = t->g.llr64; g.dist = t->g.dist; g.par = t->g.par; g.pred = t->g.pred;
    g.edge_u = t->g.edge_u; g.edge_v = t->g.edge_v;
    st.n_shots = t->st.n_shots; st.W = t->st.W; st.syn = t->st.syn; st.obs = t->st.obs;
    st.rows_words = t->st.rows_words; st.s = t->st.s; st.defects = t->st.defects; st.flags = t->st.flags;
    st.corr = t->st.corr; st.match = t->st.match; st.match_stride = t->st.match_stride;
    st.lambda_stride = t->st.lambda_stride; st.lambda_out = t->st.lambda_out;
    st.obs_pred = t->st.obs_pred; st.fail = t->st.fail; st.shot_flags = t->st.shot_flags;
    st.shot_s = t->st.shot_s; st.counters = t->st.counters;
    base = t->base;
    block0 = t->block0;
}

// Instance holding global shot index x (instances are in base order).
__device__ __forceinline__ int find_instance(const DecodeShared &c, uint64_t x) {
    int i = 0;
    while (i + 1 < c.n_inst && x >= instance_tab(c)[i + 1].base) ++i;
    return i;
}

// Instance owning block `blk` of a per-shot launch.
__device__ __forceinline__ int block_instance(const DecodeShared &c, uint64_t blk) {
    int i = 0;
    while (i + 1 < c.n_inst && blk >= instance_tab(c)[i + 1].block0) ++i;
    return i;
}

// Work classes by defect count: shots with 2 <= s <= class_max_s(c) (and
// above the previous bound) go to group class c < kGroupClasses; shots with
// up to kStreamMaxS defects to kClassStream; larger ones to kClassGeneric.
constexpr int kGroupClasses = 16;
constexpr int kClassStream = kGroupClasses;
constexpr int kClassGeneric = kGroupClasses + 1;
constexpr int kClasses = kGroupClasses + 2;
constexpr int kStreamMaxS = 512;
__host__ __device__ constexpr int class_max_s(int c) {
    switch (c) {
    case 0: return 16;   case 1: return 32;   case 2: return 48;   case 3: return 64;
    case 4: return 72;   case 5: return 80;   case 6: return 88;   case 7: return 96;
    case 8: return 104;  case 9: return 112;  case 10: return 120; case 11: return 128;
    case 12: return 160; case 13: return 192; case 14: return 224; case 15: return 256;
    case 16: return kStreamMaxS;
    default: return 0;
    }
}
__host__ __device__ inline int class_of(int s) {
    for (int c = 0; c < kGroupClasses; ++c)
        if (s <= class_max_s(c)) return c;
    return s <= kStreamMaxS ? kClassStream : kClassGeneric;
}

// Size classes above kLdsMaxS keep their message tiles (two FP32 or 16-bit
// S x (S+1|S+2) buffers) and their S x S FP32 prior matrix in a per-workgroup
// slot of global memory: kGlobalSlots slots per class (at most that many
// workgroups), a separate region for each such class so that classes may run
// concurrently.
constexpr int kLdsMaxS = 192;
constexpr int kGlobalMaxS = 256;
constexpr int kGlobalSlots = 256;
constexpr int kStreamSlots = 256;             // workgroups of the streaming class
constexpr int kFirstGlobalClass = 14;     // class_max_s(14) = 224
constexpr int kGlobalClasses = 2;
__host__ __device__ constexpr uint64_t global_slot_bytes(int store) {
    return ((uint64_t)2 * kGlobalMaxS * (store == 0 ? kGlobalMaxS + 1 : kGlobalMaxS + 2) * (store == 0 ? 4 : 2) +
            (uint64_t)kGlobalMaxS * kGlobalMaxS * 4 + 255) & ~(uint64_t)255;
}

enum : uint8_t {
    kConvergedAny = 1, kFcRan = 2, kFcChosen = 4, kPred = 8, kFail = 16, kOverflow = 32, kQbp = 64
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
