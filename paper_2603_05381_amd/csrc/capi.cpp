// C ABI of the bpm library: graph construction and upload, sampling and
// decoding launches, workspace layout and error reporting.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bpm.h"
#include "device_common.hpp"
#include "graph_internal.hpp"

namespace bpm {
hipError_t launch_sample(const DevGraph &g, uint64_t seed, uint64_t shot0, uint64_t n, uint64_t *syn,
                         uint64_t *obs, uint64_t *err, hipStream_t stream);
hipError_t launch_fill(uint64_t *p, uint64_t n, uint64_t v, hipStream_t stream);
uint64_t shot_blocks(uint64_t n_shots);
hipError_t launch_setup(const Instance *inst, int n, Instance *dst, hipStream_t stream);
hipError_t launch_extract(const DecodeShared &c, uint64_t blocks, hipStream_t stream);
hipError_t launch_finalize(const DecodeShared &c, uint64_t blocks, hipStream_t stream);
size_t generic_slot_bytes_host(bool spec, int store, int s_cap);
hipError_t launch_bp_generic(bool spec, const DecodeShared &c, int cls, void *slots, int s_slot, int n_slots,
                             hipStream_t stream);
int group_configs(int cls);
uint64_t stream_slot_bytes(int store);
hipError_t launch_bp_stream(const DecodeShared &c, int cls, hipStream_t stream);
hipError_t launch_bp_group_f32(const DecodeShared &c, int cls, int cfg, hipStream_t stream);
hipError_t launch_bp_group_f16(const DecodeShared &c, int cls, int cfg, hipStream_t stream);
hipError_t launch_bp_group_bf16(const DecodeShared &c, int cls, int cfg, hipStream_t stream);
hipError_t launch_sample_depol(const TannerDev &tn, uint64_t seed, uint64_t shot0, uint64_t n, uint32_t t1,
                               uint32_t t2, uint32_t t3, uint64_t *synx, uint64_t *synz, uint64_t *obs,
                               hipStream_t stream);
hipError_t launch_bbp4mf(const BbpArgs &a, int n_slots, hipStream_t stream);
size_t bbp4mf_slot_bytes_host(int s_cap);
void bbp4mf_graph_limits(int *max_nodes, int *max_degree);
}  // namespace bpm

using namespace bpm;

namespace {
thread_local std::string g_err;
}

bpm_status bpm::set_last_error(bpm_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

static_assert(kClasses + 2 <= BPM_MAX_STAGES, "stage events: extract, one per class, finalize");
static_assert(class_max_s(kFirstGlobalClass - 1) == kLdsMaxS && class_max_s(kFirstGlobalClass + kGlobalClasses - 1) == kGlobalMaxS &&
              kFirstGlobalClass + kGlobalClasses == kGroupClasses, "global-slot classes");
static_assert(sizeof(((bpm_decode_out *)nullptr)->stage_events) == 2 * BPM_MAX_STAGES * sizeof(void *), "");

struct bpm_graph {
    int32_t code, d, rounds;
    bpm_noise noise;
    MechanismList mech;
    PathTables tab;
    int32_t max_degree = 0;
    int device = 0;
    void *dev_mem = nullptr;      // one allocation holding every table
    size_t dev_bytes = 0;
    DevGraph dg{};
    TannerHost tanner;            // code capacity: both check types (B-BP4MF)
    void *tanner_mem = nullptr;
    TannerDev tn{};
};

namespace {

bpm_status fail(bpm_status st, const std::string &msg) { return set_last_error(st, msg); }

bpm_status hip_fail(hipError_t e, const char *what) {
    return fail(BPM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Number of resident workgroups used by the persistent decode kernels.
constexpr int kGenericSlotsFp32 = 512;
constexpr int kGenericSlotsFp64 = 256;

// message storage of the FP32 kernels: 0 FP32, 1 FP16, 2 BF16
int store_of(int precision) {
    return precision == BPM_FP16_STORE ? 1 : precision == BPM_BF16_STORE ? 2 : 0;
}

hipError_t launch_bp_group(const DecodeShared &c, int cls, int cfg, hipStream_t stream) {
    switch (c.store) {
    case 1: return launch_bp_group_f16(c, cls, cfg, stream);
    case 2: return launch_bp_group_bf16(c, cls, cfg, stream);
    default: return launch_bp_group_f32(c, cls, cfg, stream);
    }
}

// Workspace layout of a call: per instance s, defects and flags; shared
// instance table, class queues and generic-kernel slots.
struct Layout {
    size_t s[kMaxInstances], defects[kMaxInstances], flags[kMaxInstances];
    size_t table, class_count, class_list, slots, gslots, sslots, total;
    uint64_t n_total;
    int s_cap, s_slot, n_slots;
    bool generic;               // slots of the generic kernel are laid out
};

bool make_layout(const bpm_decode_item *items, int n_items, const bpm_decode_opts *o, Layout &L,
                 std::string &why) {
    int max_det = 1;
    uint64_t n_total = 0;
    for (int i = 0; i < n_items; ++i) {
        max_det = std::max(max_det, items[i].graph->mech.n_det);
        n_total += items[i].n_shots;
    }
    if (n_total > 0xFFFFFFFFull) { why = "at most 2^32 - 1 shots per call"; return false; }
    int s_cap = o->s_cap > 0 ? o->s_cap : std::min(max_det, 512);
    if (s_cap > max_det) s_cap = max_det;
    if (s_cap < 1) s_cap = 1;
    if (s_cap > 1024) { why = "s_cap must be <= 1024"; return false; }
    const bool spec = o->precision == BPM_FP64_SPEC;
    L.s_cap = s_cap;
    L.s_slot = s_cap;
    L.n_slots = spec ? kGenericSlotsFp64 : kGenericSlotsFp32;
    L.n_total = n_total;
    size_t off = 0;
    for (int i = 0; i < n_items; ++i) {
        const uint64_t n = items[i].n_shots;
        L.s[i] = off; off = align256(off + sizeof(int32_t) * n);
        L.defects[i] = off; off = align256(off + sizeof(uint16_t) * n * (size_t)s_cap);
        L.flags[i] = off; off = align256(off + n);
    }
    L.table = off; off = align256(off + sizeof(Instance) * (size_t)n_items);
    L.class_count = off; off = align256(off + sizeof(uint32_t) * kClasses);
    L.class_list = off; off = align256(off + sizeof(uint32_t) * kClasses * n_total);
    // the generic kernel decodes every shot in FP64 fixed order, and in the
    // FP32 modes only shots above the streaming class: no slots below that
    L.generic = spec || s_cap > kStreamMaxS;
    L.slots = off;
    if (L.generic) off += generic_slot_bytes_host(spec, store_of(o->precision), L.s_slot) * (size_t)L.n_slots;
    off = align256(off);
    L.gslots = off;
    if (!spec && s_cap > kLdsMaxS) off += global_slot_bytes(store_of(o->precision)) * kGlobalSlots * kGlobalClasses;
    off = align256(off);
    L.sslots = off;
    if (!spec && s_cap > kGlobalMaxS) off += stream_slot_bytes(store_of(o->precision)) * kStreamSlots;
    L.total = align256(off);
    return true;
}

bpm_status check_items(const bpm_decode_item *items, int n_items, bool need_device) {
    if (!items) return fail(BPM_EINVAL, "items is NULL");
    if (n_items < 1 || n_items > BPM_MAX_INSTANCES) return fail(BPM_EINVAL, "n_items must lie in [1, BPM_MAX_INSTANCES]");
    for (int i = 0; i < n_items; ++i) {
        const bpm_decode_item &it = items[i];
        if (!it.graph) return fail(BPM_EINVAL, "item graph is NULL");
        if (need_device && !it.graph->dev_mem) return fail(BPM_EDEVICE, "graph was built without a device");
        if (it.rows_words < 0 || (it.rows_words > 0 && it.rows_words < (it.graph->mech.n_det + 63) / 64))
            return fail(BPM_EINVAL, "rows_words must be 0 (bit planes) or >= ceil(n_det / 64)");
        if (it.n_shots > 0 && !it.syn) return fail(BPM_EINVAL, "syn must be a device buffer");
        if (it.rows_words == 0 && it.n_shots > 0 && !it.obs) return fail(BPM_EINVAL, "obs must be a device buffer");
        if (it.out.match && it.out.match_stride < 1) return fail(BPM_EINVAL, "match_stride must be >= 1");
        if (it.out.lambda_out && it.out.lambda_stride < 1) return fail(BPM_EINVAL, "lambda_stride must be >= 1");
        if (need_device && i > 0 && it.graph->device != items[0].graph->device)
            return fail(BPM_EINVAL, "all graphs of a call must live on one device");
    }
    return BPM_OK;
}

bpm_status check_opts(const bpm_decode_opts *o) {
    if (!o) return fail(BPM_EINVAL, "opts is NULL");
    if (o->max_iters < 1) return fail(BPM_EINVAL, "max_iters must be >= 1");
    if (o->variant != BPM_BP4M && o->variant != BPM_BP4MF) return fail(BPM_EINVAL, "unknown variant");
    if (o->precision != BPM_FP64_SPEC && o->precision != BPM_FP32 && o->precision != BPM_BF16_STORE &&
        o->precision != BPM_FP16_STORE)
        return fail(BPM_EUNSUPPORTED, "unknown precision");
    if (!(o->alpha > 0.0) || !std::isfinite(o->alpha)) return fail(BPM_EINVAL, "alpha must be > 0");
    if (o->s_cap < 0 || o->s_cap > 1024) return fail(BPM_EINVAL, "s_cap must lie in [0, 1024]");
    if (o->class_streams < 0 || o->class_streams > 8) return fail(BPM_EINVAL, "class_streams must lie in [0, 8]");
    return BPM_OK;
}

// Library-owned streams and events for concurrent size classes: one set per
// calling thread and device (so concurrent callers never share an event),
// default priority, released when the thread ends.
struct ClassStreams {
    int device = -1;
    hipStream_t aux[7] = {};
    hipEvent_t fork = nullptr, join[7] = {};
    int n = 0;                  // aux streams created
    ~ClassStreams() {
        for (int i = 0; i < n; ++i) {
            hipStreamDestroy(aux[i]);
            hipEventDestroy(join[i]);
        }
        if (fork) hipEventDestroy(fork);
    }
};

hipError_t class_streams_get(int want_aux, ClassStreams *&out) {
    thread_local ClassStreams pools[8];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    ClassStreams &p = pools[dev & 7];
    if (p.device != dev) {
        if (p.device >= 0) return hipErrorInvalidDevice;     // more than 8 devices per thread
        p.device = dev;
    }
    if (!p.fork) {
        e = hipEventCreateWithFlags(&p.fork, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    while (p.n < want_aux) {
        e = hipStreamCreateWithFlags(&p.aux[p.n], hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        e = hipEventCreateWithFlags(&p.join[p.n], hipEventDisableTiming);
        if (e != hipSuccess) { hipStreamDestroy(p.aux[p.n]); return e; }
        ++p.n;
    }
    out = &p;
    return hipSuccess;
}

// Kernel configuration of every stage (process-wide; index into the
// stage's configurations, 0 = default).
std::atomic<int> g_stage_cfg[BPM_MAX_STAGES];

int stage_configs(int stage) {
    if (stage >= 1 && stage <= kGroupClasses) return group_configs(stage - 1);
    return 1;
}

bpm_status decode_impl(const bpm_decode_item *items, int n_items, const bpm_decode_opts *opts,
                       void *const *stage_events, void *workspace, size_t workspace_bytes, void *stream,
                       const int *cfg);

}  // namespace

extern "C" {

const char *bpm_last_error(void) { return g_err.c_str(); }

int32_t bpm_stage_table(int32_t *max_s) {
    const int n = kClasses + 2;
    if (max_s) {
        for (int k = 0; k < BPM_MAX_STAGES; ++k) max_s[k] = 0;
        for (int c = 0; c < kGroupClasses; ++c) max_s[1 + c] = class_max_s(c);
        max_s[1 + kClassStream] = kStreamMaxS;
        max_s[1 + kClassGeneric] = INT32_MAX;
    }
    return n;
}

bpm_status bpm_build_graph(bpm_code code, int32_t d, int32_t rounds, const bpm_noise *noise, bpm_graph **out) {
    if (!out) return fail(BPM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!noise) return fail(BPM_EINVAL, "noise is NULL");
    if (code != BPM_ROTATED_SURFACE && code != BPM_UNROTATED_SURFACE) return fail(BPM_EUNSUPPORTED, "unknown code");
    bpm_graph *g = new (std::nothrow) bpm_graph();
    if (!g) return fail(BPM_ENOMEM, "host allocation failed");
    g->code = code; g->d = d; g->rounds = rounds; g->noise = *noise;
    std::string why;
    if (noise->kind == BPM_CODE_CAPACITY_DEPOL) {
        g->rounds = 1;
        why = code == BPM_UNROTATED_SURFACE ? build_code_capacity_unrotated(d, noise->p, g->mech)
                                            : build_code_capacity(d, noise->p, g->mech);
    } else if (noise->kind == BPM_CIRCUIT_MEMORY_Z) {
        why = code == BPM_UNROTATED_SURFACE ? build_memory_z_unrotated(d, rounds, noise->p, g->mech)
                                            : build_memory_z(d, rounds, noise->p, g->mech);
    } else {
        why = "unknown noise kind";
    }
    if (why.empty()) why = build_path_tables(g->mech, g->tab);
    if (why.empty() && noise->kind == BPM_CODE_CAPACITY_DEPOL)
        why = build_tanner_code_capacity(d, code == BPM_UNROTATED_SURFACE, g->mech, g->tanner);
    if (!why.empty()) { delete g; return fail(BPM_EINVAL, why); }
    const MechanismList &m = g->mech;
    const int N = m.n_det, E = m.size();
    if (N > 65535) { delete g; return fail(BPM_EUNSUPPORTED, "more than 65535 detectors"); }
    std::vector<int32_t> deg(N, 0);
    for (int e : m.dets) deg[e]++;
    for (int x : deg) g->max_degree = std::max(g->max_degree, x);

    // device layout: one allocation, 256-byte aligned pieces
    const size_t NN = (size_t)N * N;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const size_t o_off = take(sizeof(int32_t) * (E + 1)), o_det = take(sizeof(int32_t) * std::max<size_t>(m.dets.size(), 1));
    const size_t o_obs = take(E), o_thr = take(sizeof(uint32_t) * E);
    const size_t NU = (size_t)N * (N + 1) / 2;
    const size_t o_l32 = take(sizeof(float) * NN), o_l32u = take(sizeof(float) * NU), o_l64 = take(sizeof(double) * NN);
    const size_t o_dist = take(sizeof(int64_t) * NN), o_par = take(NN), o_pred = take(sizeof(int32_t) * NN);
    const size_t o_eu = take(sizeof(int32_t) * E), o_ev = take(sizeof(int32_t) * E);
    g->dev_bytes = off;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev == 0) {
        // no device: the host tables are complete; device calls will refuse
        (void)hipGetLastError();
        g->dev_bytes = 0;
        *out = g;
        return BPM_OK;
    }
    hipError_t he = hipGetDevice(&g->device);
    if (he != hipSuccess) { delete g; return hip_fail(he, "hipGetDevice"); }
    he = hipMalloc(&g->dev_mem, off);
    if (he != hipSuccess) { delete g; return fail(BPM_ENOMEM, "device allocation of the graph tables failed"); }
    std::vector<uint32_t> thr(E);
    std::vector<float> l32(NN);
    std::vector<int32_t> eu(E), ev(E);
    for (int e = 0; e < E; ++e) {
        thr[e] = fire_threshold(m.q[e]);
        int k = m.off[e + 1] - m.off[e];
        eu[e] = m.dets[m.off[e]];
        ev[e] = k == 2 ? m.dets[m.off[e] + 1] : -1;
    }
    for (size_t i = 0; i < NN; ++i) l32[i] = (float)g->tab.llr[i];
    std::vector<float> l32u(NU);
    for (int i = 0; i < N; ++i)
        for (int j = i; j < N; ++j) l32u[tri_index((uint32_t)N, (uint32_t)i, (uint32_t)j)] = l32[(size_t)i * N + j];

    char *base = (char *)g->dev_mem;
    struct Up { size_t o; const void *p; size_t n; } ups[] = {
        {o_off, m.off.data(), sizeof(int32_t) * (E + 1)},
        {o_det, m.dets.data(), sizeof(int32_t) * m.dets.size()},
        {o_obs, m.obs.data(), (size_t)E},
        {o_thr, thr.data(), sizeof(uint32_t) * E},
        {o_l32, l32.data(), sizeof(float) * NN},
        {o_l32u, l32u.data(), sizeof(float) * NU},
        {o_l64, g->tab.llr.data(), sizeof(double) * NN},
        {o_dist, g->tab.dist.data(), sizeof(int64_t) * NN},
        {o_par, g->tab.par.data(), NN},
        {o_pred, g->tab.pred.data(), sizeof(int32_t) * NN},
        {o_eu, eu.data(), sizeof(int32_t) * E},
        {o_ev, ev.data(), sizeof(int32_t) * E},
    };
    for (auto &u : ups) {
        if (u.n == 0) continue;
        he = hipMemcpy(base + u.o, u.p, u.n, hipMemcpyHostToDevice);
        if (he != hipSuccess) { hipFree(g->dev_mem); delete g; return hip_fail(he, "hipMemcpy of graph tables"); }
    }
    DevGraph &dg = g->dg;
    dg.n_det = N; dg.n_mech = E;
    dg.mech_off = (const int32_t *)(base + o_off);
    dg.mech_det = (const int32_t *)(base + o_det);
    dg.mech_obs = (const uint8_t *)(base + o_obs);
    dg.thr = (const uint32_t *)(base + o_thr);
    dg.llr32 = (const float *)(base + o_l32);
    dg.llr32u = (const float *)(base + o_l32u);
    dg.llr64 = (const double *)(base + o_l64);
    dg.dist = (const int64_t *)(base + o_dist);
    dg.par = (const uint8_t *)(base + o_par);
    dg.pred = (const int32_t *)(base + o_pred);
    dg.edge_u = (const int32_t *)(base + o_eu);
    dg.edge_v = (const int32_t *)(base + o_ev);
    if (g->tanner.n_q > 0) {
        const TannerHost &t = g->tanner;
        size_t toff = 0;
        auto ttake = [&](size_t bytes) { size_t o = toff; toff = align256(toff + bytes); return o; };
        const size_t o_qc = ttake(4 * t.qc.size()), o_cq = ttake(4 * t.cq.size()), o_cs = ttake(4 * t.cs.size());
        const size_t o_qo = ttake(t.qobs.size()), o_qm = ttake(4 * t.qmech.size());
        const size_t o_no = ttake(4 * t.noff.size()), o_ne = ttake(4 * std::max<size_t>(t.nedge.size(), 1));
        he = hipMalloc(&g->tanner_mem, toff);
        if (he != hipSuccess) { hipFree(g->dev_mem); delete g; return fail(BPM_ENOMEM, "device allocation of the Tanner graph failed"); }
        char *tb = (char *)g->tanner_mem;
        struct Up { size_t o; const void *p; size_t n; } tups[] = {
            {o_qc, t.qc.data(), 4 * t.qc.size()}, {o_cq, t.cq.data(), 4 * t.cq.size()},
            {o_cs, t.cs.data(), 4 * t.cs.size()}, {o_qo, t.qobs.data(), t.qobs.size()},
            {o_qm, t.qmech.data(), 4 * t.qmech.size()}, {o_no, t.noff.data(), 4 * t.noff.size()},
            {o_ne, t.nedge.data(), 4 * t.nedge.size()},
        };
        for (auto &u : tups) {
            if (u.n == 0) continue;
            he = hipMemcpy(tb + u.o, u.p, u.n, hipMemcpyHostToDevice);
            if (he != hipSuccess) {
                hipFree(g->tanner_mem); hipFree(g->dev_mem); delete g;
                return hip_fail(he, "hipMemcpy of the Tanner graph");
            }
        }
        TannerDev &tn = g->tn;
        tn.n_q = t.n_q; tn.n_xc = t.n_xc; tn.n_zc = t.n_zc;
        tn.qc = (const int32_t *)(tb + o_qc);
        tn.cq = (const int32_t *)(tb + o_cq);
        tn.cs = (const int32_t *)(tb + o_cs);
        tn.qobs = (const uint8_t *)(tb + o_qo);
        tn.qmech = (const int32_t *)(tb + o_qm);
        tn.noff = (const int32_t *)(tb + o_no);
        tn.nedge = (const int32_t *)(tb + o_ne);
    }
    *out = g;
    return BPM_OK;
}

bpm_status bpm_graph_info_get(const bpm_graph *g, bpm_graph_info *info) {
    if (!g || !info) return fail(BPM_EINVAL, "NULL argument");
    info->n_det = g->mech.n_det;
    info->n_mech = g->mech.size();
    info->n_edges = g->mech.size();
    info->d = g->d;
    info->rounds = g->rounds;
    info->max_degree = g->max_degree;
    info->p = g->noise.p;
    info->device_bytes = g->dev_bytes;
    return BPM_OK;
}

void bpm_graph_free(bpm_graph *g) {
    if (!g) return;
    if (g->dev_mem) {
        int cur = 0;
        hipGetDevice(&cur);
        hipSetDevice(g->device);
        hipFree(g->dev_mem);
        if (g->tanner_mem) hipFree(g->tanner_mem);
        hipSetDevice(cur);
    }
    delete g;
}

bpm_status bpm_graph_copy_mechanisms(const bpm_graph *g, int32_t *off, int32_t *dets, uint8_t *obs, double *q) {
    if (!g) return fail(BPM_EINVAL, "graph is NULL");
    const MechanismList &m = g->mech;
    if (off) std::memcpy(off, m.off.data(), sizeof(int32_t) * m.off.size());
    if (dets) std::memcpy(dets, m.dets.data(), sizeof(int32_t) * m.dets.size());
    if (obs) std::memcpy(obs, m.obs.data(), m.obs.size());
    if (q) std::memcpy(q, m.q.data(), sizeof(double) * m.q.size());
    return BPM_OK;
}

bpm_status bpm_graph_copy_tables(const bpm_graph *g, int64_t *dist, int32_t *hops, uint8_t *par, int32_t *pred,
                                 double *llr) {
    if (!g) return fail(BPM_EINVAL, "graph is NULL");
    const PathTables &t = g->tab;
    const size_t NN = (size_t)t.n * t.n;
    if (dist) std::memcpy(dist, t.dist.data(), sizeof(int64_t) * NN);
    if (hops) std::memcpy(hops, t.hops.data(), sizeof(int32_t) * NN);
    if (par) std::memcpy(par, t.par.data(), NN);
    if (pred) std::memcpy(pred, t.pred.data(), sizeof(int32_t) * NN);
    if (llr) std::memcpy(llr, t.llr.data(), sizeof(double) * NN);
    return BPM_OK;
}

bpm_status bpm_sample(const bpm_graph *g, uint64_t seed, uint64_t shot0, uint64_t n_shots, uint64_t *syn,
                      uint64_t *obs, uint64_t *err, void *stream) {
    if (!g) return fail(BPM_EINVAL, "graph is NULL");
    if (n_shots == 0) return BPM_OK;
    if (!g->dev_mem) return fail(BPM_EDEVICE, "graph was built without a device");
    if (!syn || !obs) return fail(BPM_EINVAL, "syn and obs must be device buffers");
    hipError_t e = launch_sample(g->dg, seed, shot0, n_shots, syn, obs, err, (hipStream_t)stream);
    return e == hipSuccess ? BPM_OK : hip_fail(e, "sample launch");
}

bpm_status bpm_decode_workspace_size(const bpm_graph *g, uint64_t n_shots, const bpm_decode_opts *opts,
                                     size_t *bytes) {
    if (!g || !bytes) return fail(BPM_EINVAL, "NULL argument");
    bpm_decode_item it{};
    it.graph = g;
    it.n_shots = n_shots;
    return bpm_decode_multi_workspace_size(&it, 1, opts, bytes);
}

bpm_status bpm_decode_multi_workspace_size(const bpm_decode_item *items, int32_t n_items,
                                           const bpm_decode_opts *opts, size_t *bytes) {
    if (!bytes) return fail(BPM_EINVAL, "bytes is NULL");
    bpm_status st = check_opts(opts);
    if (st != BPM_OK) return st;
    if (!items || n_items < 1 || n_items > BPM_MAX_INSTANCES)
        return fail(BPM_EINVAL, "n_items must lie in [1, BPM_MAX_INSTANCES]");
    for (int i = 0; i < n_items; ++i)
        if (!items[i].graph) return fail(BPM_EINVAL, "item graph is NULL");
    Layout L;
    std::string why;
    if (!make_layout(items, n_items, opts, L, why)) return fail(BPM_EINVAL, why);
    *bytes = L.total;
    return BPM_OK;
}

bpm_status bpm_decode(const bpm_graph *g, const uint64_t *syn, const uint64_t *obs, uint64_t n_shots,
                      const bpm_decode_opts *opts, const bpm_decode_out *out, void *workspace,
                      size_t workspace_bytes, void *stream) {
    if (!g || !out) return fail(BPM_EINVAL, "NULL argument");
    bpm_decode_item it{};
    it.graph = g;
    it.syn = syn;
    it.obs = obs;
    it.n_shots = n_shots;
    it.rows_words = 0;
    it.out = *out;
    if (n_shots > 0 && (!syn || !obs)) return fail(BPM_EINVAL, "syn and obs must be device buffers");
    int cfg[BPM_MAX_STAGES];
    for (int k = 0; k < BPM_MAX_STAGES; ++k) cfg[k] = g_stage_cfg[k].load(std::memory_order_relaxed);
    return decode_impl(&it, 1, opts, out->stage_events, workspace, workspace_bytes, stream, cfg);
}

bpm_status bpm_decode_multi(const bpm_decode_item *items, int32_t n_items, const bpm_decode_opts *opts,
                            void *const *stage_events, void *workspace, size_t workspace_bytes, void *stream) {
    int cfg[BPM_MAX_STAGES];
    for (int k = 0; k < BPM_MAX_STAGES; ++k) cfg[k] = g_stage_cfg[k].load(std::memory_order_relaxed);
    return decode_impl(items, n_items, opts, stage_events, workspace, workspace_bytes, stream, cfg);
}

}  // extern "C"

namespace {

bpm_status decode_impl(const bpm_decode_item *items, int n_items, const bpm_decode_opts *opts,
                       void *const *stage_events, void *workspace, size_t workspace_bytes, void *stream,
                       const int *cfg) {
    bpm_status st0 = check_opts(opts);
    if (st0 != BPM_OK) return st0;
    st0 = check_items(items, n_items, false);
    if (st0 != BPM_OK) return st0;
    uint64_t n_all = 0;
    for (int i = 0; i < n_items; ++i) n_all += items[i].n_shots;
    if (n_all == 0) return BPM_OK;
    st0 = check_items(items, n_items, true);
    if (st0 != BPM_OK) return st0;
    Layout L;
    std::string why;
    if (!make_layout(items, n_items, opts, L, why)) return fail(BPM_EINVAL, why);
    if (!workspace || workspace_bytes < L.total) return fail(BPM_EINVAL, "workspace missing or too small");
    if (((uintptr_t)workspace & 255) != 0) return fail(BPM_EINVAL, "workspace must be 256-byte aligned");
    for (int i = 0; i < n_items; ++i)
        if (items[i].out.match && items[i].out.match_stride < L.s_cap)
            return fail(BPM_EINVAL, "match_stride must be >= s_cap");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    Instance inst[kMaxInstances] = {};
    uint64_t base = 0, block0 = 0;
    for (int i = 0; i < n_items; ++i) {
        const bpm_decode_item &it = items[i];
        Instance &I = inst[i];
        InstState &d = I.st;
        I.g = it.graph->dg;
        I.base = base;
        I.block0 = block0;
        base += it.n_shots;
        block0 += shot_blocks(it.n_shots);
        d.n_shots = it.n_shots;
        d.W = (it.n_shots + 63) / 64;
        d.syn = it.syn;
        d.obs = it.obs;
        d.rows_words = it.rows_words;
        d.s = (int32_t *)(ws + L.s[i]);
        d.defects = (uint16_t *)(ws + L.defects[i]);
        d.flags = (uint8_t *)(ws + L.flags[i]);
        d.corr = it.out.corr;
        d.match = it.out.match;
        d.match_stride = it.out.match_stride;
        d.lambda_out = it.out.lambda_out;
        d.lambda_stride = it.out.lambda_stride;
        d.obs_pred = it.out.obs_pred;
        d.fail = it.out.fail;
        d.shot_flags = it.out.shot_flags;
        d.shot_s = it.out.shot_s;
        d.counters = (unsigned long long *)it.out.counters;
    }
    DecodeShared c{};
    c.max_iters = opts->max_iters;
    c.variant = opts->variant;
    c.store = store_of(opts->precision);
    c.s_cap = L.s_cap;
    c.inv_alpha = 1.0 / opts->alpha;
    c.n_inst = n_items;
    c.total = L.n_total;
    c.inst = (const Instance *)(ws + L.table);
    c.class_count = (uint32_t *)(ws + L.class_count);
    c.class_list = (uint32_t *)(ws + L.class_list);
    const bool spec = opts->precision == BPM_FP64_SPEC;
    if (!spec && L.s_cap > kLdsMaxS) {
        c.gslot = ws + L.gslots;
        c.gslot_stride = global_slot_bytes(c.store);
        c.n_gslots = kGlobalSlots;
    }
    if (!spec && L.s_cap > kGlobalMaxS) {
        c.sslot = ws + L.sslots;
        c.sslot_stride = stream_slot_bytes(c.store);
        c.n_sslots = kStreamSlots;
    }

    // streams for the message-passing stages: the caller's, plus n_aux
    // library streams forked after extraction and joined before packing
    const int n_str = spec ? 1 : std::max(1, (int)opts->class_streams);
    ClassStreams *cs = nullptr;
    if (n_str > 1) {
        hipError_t ep = class_streams_get(n_str - 1, cs);
        if (ep != hipSuccess) return hip_fail(ep, "class streams");
    }
    auto stream_of = [&](int k) -> hipStream_t { return k % n_str == 0 ? s : cs->aux[k % n_str - 1]; };
    auto mark_on = [&](int k, hipStream_t st) -> hipError_t {
        void *ev = stage_events ? stage_events[k] : nullptr;
        return ev ? hipEventRecord((hipEvent_t)ev, st) : hipSuccess;
    };
    auto mark = [&](int k) -> hipError_t { return mark_on(k, s); };
    hipError_t e = launch_setup(inst, n_items, (Instance *)(ws + L.table), s);
    if (e == hipSuccess) e = launch_fill((uint64_t *)c.class_count, (kClasses + 1) / 2, 0, s);
    for (int i = 0; i < n_items && e == hipSuccess; ++i)
        if (inst[i].st.corr)
            e = launch_fill(inst[i].st.corr, (uint64_t)items[i].graph->mech.size() * inst[i].st.W, 0, s);
    if (e == hipSuccess) e = mark(0);
    if (e == hipSuccess) e = launch_extract(c, block0, s);
    if (e == hipSuccess) e = mark(1);
    if (spec) {
        for (int k = 0; k < kGroupClasses && e == hipSuccess; ++k) {
            e = mark(2 + 2 * k);
            if (e == hipSuccess) e = mark(3 + 2 * k);
        }
        if (e == hipSuccess) e = mark(2 + 2 * kGroupClasses);
        for (int k = 0; k < kClasses && e == hipSuccess; ++k)
            e = launch_bp_generic(true, c, k, ws + L.slots, L.s_slot, L.n_slots, s);
        if (e == hipSuccess) e = mark(3 + 2 * kGroupClasses);
    } else {
        if (n_str > 1) {
            if (e == hipSuccess) e = hipEventRecord(cs->fork, s);
            for (int i = 0; i + 1 < n_str && e == hipSuccess; ++i) e = hipStreamWaitEvent(cs->aux[i], cs->fork, 0);
        }
        // largest classes first, so that concurrent streams start with the
        // longest work
        for (int k = kClasses - 1; k >= 0 && e == hipSuccess; --k) {
            hipStream_t st = stream_of(kClasses - 1 - k);
            e = mark_on(2 + 2 * k, st);
            if (k == kClassGeneric) {
                if (e == hipSuccess && L.generic)
                    e = launch_bp_generic(false, c, kClassGeneric, ws + L.slots, L.s_slot, L.n_slots, st);
            } else if (k == kClassStream) {
                if (e == hipSuccess && L.s_cap > kGlobalMaxS) e = launch_bp_stream(c, kClassStream, st);
            } else {
                // a class whose smallest size exceeds s_cap holds no shot
                const int lowest = k == 0 ? 2 : class_max_s(k - 1) + 1;
                if (e == hipSuccess && lowest <= L.s_cap) e = launch_bp_group(c, k, cfg[1 + k], st);
            }
            if (e == hipSuccess) e = mark_on(3 + 2 * k, st);
        }
        for (int i = 0; i + 1 < n_str && e == hipSuccess; ++i) {
            e = hipEventRecord(cs->join[i], cs->aux[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, cs->join[i], 0);
        }
    }
    if (e == hipSuccess) e = mark(2 * (kClasses + 1));
    if (e == hipSuccess) e = launch_finalize(c, block0, s);
    if (e == hipSuccess) e = mark(2 * (kClasses + 1) + 1);
    return e == hipSuccess ? BPM_OK : hip_fail(e, "decode launch");
}

}  // namespace

extern "C" {

int32_t bpm_stage_configs(int32_t stage) {
    if (stage < 0 || stage >= kClasses + 2) return 0;
    return stage_configs(stage);
}

bpm_status bpm_get_stage_config(int32_t *cfg) {
    if (!cfg) return fail(BPM_EINVAL, "cfg is NULL");
    for (int k = 0; k < BPM_MAX_STAGES; ++k) cfg[k] = g_stage_cfg[k].load();
    return BPM_OK;
}

bpm_status bpm_set_stage_config(const int32_t *cfg) {
    if (!cfg) return fail(BPM_EINVAL, "cfg is NULL");
    for (int k = 0; k < BPM_MAX_STAGES; ++k) {
        const int n = k < kClasses + 2 ? stage_configs(k) : 1;
        if (cfg[k] < 0 || cfg[k] >= n) return fail(BPM_EINVAL, "configuration index out of range");
    }
    for (int k = 0; k < BPM_MAX_STAGES; ++k) g_stage_cfg[k].store(cfg[k]);
    return BPM_OK;
}

bpm_status bpm_autotune(const bpm_graph *g, const bpm_decode_opts *opts, uint64_t n_shots, uint64_t seed,
                        float *stage_ms, void *stream) {
    if (!g) return fail(BPM_EINVAL, "graph is NULL");
    bpm_status st = check_opts(opts);
    if (st != BPM_OK) return st;
    if (!g->dev_mem) return fail(BPM_EDEVICE, "graph was built without a device");
    if (n_shots == 0 || n_shots > 0xFFFFFFFFull) return fail(BPM_EINVAL, "n_shots must lie in [1, 2^32)");
    if (stage_ms)
        for (int k = 0; k < BPM_MAX_CONFIGS * BPM_MAX_STAGES; ++k) stage_ms[k] = -1.0f;
    if (opts->precision == BPM_FP64_SPEC) return BPM_OK;     // one kernel, nothing to choose
    const int n_stages = kClasses + 2;
    int n_cfg = 1;
    for (int k = 0; k < n_stages; ++k) n_cfg = std::max(n_cfg, stage_configs(k));
    if (n_cfg > BPM_MAX_CONFIGS) return fail(BPM_EUNSUPPORTED, "more configurations than BPM_MAX_CONFIGS");
    bpm_decode_item it{};
    it.graph = g;
    it.n_shots = n_shots;
    Layout L;
    std::string why;
    if (!make_layout(&it, 1, opts, L, why)) return fail(BPM_EINVAL, why);
    const uint64_t W = (n_shots + 63) / 64;
    const size_t syn_bytes = sizeof(uint64_t) * W * (size_t)g->mech.n_det, obs_bytes = sizeof(uint64_t) * W;
    hipStream_t s = (hipStream_t)stream;
    char *buf = nullptr;
    const size_t o_syn = 0, o_obs = align256(syn_bytes), o_ws = o_obs + align256(obs_bytes);
    hipError_t e = hipMalloc((void **)&buf, o_ws + L.total);
    if (e != hipSuccess) return fail(BPM_ENOMEM, "autotune buffers");
    hipEvent_t ev[2 * BPM_MAX_STAGES] = {};
    void *evp[2 * BPM_MAX_STAGES] = {};
    int n_ev = 0;
    for (; n_ev < 2 * n_stages && e == hipSuccess; ++n_ev) e = hipEventCreate(&ev[n_ev]);
    for (int k = 0; k < n_ev; ++k) evp[k] = ev[k];
    it.syn = (uint64_t *)(buf + o_syn);
    it.obs = (uint64_t *)(buf + o_obs);
    if (e == hipSuccess)
        e = launch_sample(g->dg, seed, 0, n_shots, (uint64_t *)(buf + o_syn), (uint64_t *)(buf + o_obs), nullptr, s);
    std::vector<float> t((size_t)n_cfg * n_stages, -1.0f);
    bpm_status rs = BPM_OK;
    for (int c = 0; c < n_cfg && e == hipSuccess && rs == BPM_OK; ++c) {
        int cfg[BPM_MAX_STAGES];
        for (int k = 0; k < BPM_MAX_STAGES; ++k)
            cfg[k] = k < n_stages ? std::min(c, stage_configs(k) - 1) : 0;
        // first pass loads the kernels; the second is timed
        bpm_decode_opts o1 = *opts;
        o1.class_streams = 0;               // one stream: stage times are per kernel
        for (int rep = 0; rep < 2 && rs == BPM_OK; ++rep)
            rs = decode_impl(&it, 1, &o1, evp, buf + o_ws, L.total, stream, cfg);
        if (rs == BPM_OK) e = hipEventSynchronize(ev[2 * n_stages - 1]);
        for (int k = 0; k < n_stages && e == hipSuccess; ++k)
            if (c < stage_configs(k)) e = hipEventElapsedTime(&t[(size_t)c * n_stages + k], ev[2 * k], ev[2 * k + 1]);
    }
    if (e == hipSuccess && rs == BPM_OK) {
        for (int k = 0; k < n_stages; ++k) {
            int best = 0;
            for (int c = 1; c < stage_configs(k); ++c)
                if (t[(size_t)c * n_stages + k] < t[(size_t)best * n_stages + k]) best = c;
            g_stage_cfg[k].store(best);
            if (stage_ms)
                for (int c = 0; c < stage_configs(k); ++c) stage_ms[c * BPM_MAX_STAGES + k] = t[(size_t)c * n_stages + k];
        }
    }
    hipError_t e2 = hipStreamSynchronize(s);
    for (int k = 0; k < n_ev; ++k) hipEventDestroy(ev[k]);
    hipFree(buf);
    if (rs != BPM_OK) return rs;
    if (e == hipSuccess) e = e2;
    return e == hipSuccess ? BPM_OK : hip_fail(e, "autotune");
}

}  // extern "C"

// ------------------------------------------------------------------ B-BP4MF

namespace {

constexpr int kBbpSlots = 256;

bpm_status bbp_check(const bpm_graph *g, const bpm_decode_opts *opts, int32_t *s_cap) {
    if (!g) return fail(BPM_EINVAL, "graph is NULL");
    if (g->tanner.n_q == 0) return fail(BPM_EUNSUPPORTED, "B-BP4MF needs a code-capacity graph");
    bpm_status st = check_opts(opts);
    if (st != BPM_OK) return st;
    if (opts->precision != BPM_FP64_SPEC)
        return fail(BPM_EUNSUPPORTED, "B-BP4MF runs in BPM_FP64_SPEC (fixed-order FP64) only");
    const TannerHost &t = g->tanner;
    if (t.n_q > 1024 || t.n_xc + t.n_zc > 2048 || g->mech.n_det > 1023 || g->mech.size() > 1024)
        return fail(BPM_EUNSUPPORTED, "B-BP4MF handles codes of up to 1024 qubits");
    // the path search keeps each detector node's neighbours in registers
    int max_nodes = 0, max_degree = 0;
    bpm::bbp4mf_graph_limits(&max_nodes, &max_degree);
    if (g->mech.n_det < 1 || g->mech.n_det > max_nodes)
        return fail(BPM_EUNSUPPORTED, "B-BP4MF handles decoding graphs of up to " + std::to_string(max_nodes) +
                                          " detectors");
    for (int u = 0; u < g->mech.n_det; ++u)
        if (t.noff[u + 1] - t.noff[u] > max_degree)
            return fail(BPM_EUNSUPPORTED, "B-BP4MF needs detectors of at most " + std::to_string(max_degree) +
                                              " decoding-graph edges");
    int32_t sc = opts->s_cap > 0 ? opts->s_cap : std::min<int32_t>(g->mech.n_det, 256);
    if (sc > 1024) sc = 1024;
    *s_cap = sc;
    return BPM_OK;
}

struct BbpLayout {
    size_t table, s, flags, slots, slot_bytes, total;
};

BbpLayout bbp_layout(uint64_t n, int32_t s_cap) {
    BbpLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.table = take(sizeof(Instance));
    L.s = take(sizeof(int32_t) * std::max<uint64_t>(n, 1));
    L.flags = take(std::max<uint64_t>(n, 1));
    L.slot_bytes = align256(bbp4mf_slot_bytes_host(s_cap));
    L.slots = take(L.slot_bytes * kBbpSlots);
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

bpm_status bpm_sample_depolarizing(const bpm_graph *g, uint64_t seed, uint64_t shot0, uint64_t n_shots,
                                   uint64_t *syn_x, uint64_t *syn_z, uint64_t *obs, void *stream) {
    if (!g) return fail(BPM_EINVAL, "graph is NULL");
    if (g->tanner.n_q == 0) return fail(BPM_EUNSUPPORTED, "depolarizing sampling needs a code-capacity graph");
    if (n_shots == 0) return BPM_OK;
    if (!g->dev_mem) return fail(BPM_EDEVICE, "graph was built without a device");
    if (!syn_x || !syn_z || !obs) return fail(BPM_EINVAL, "syn_x, syn_z and obs must be device buffers");
    const double p = g->noise.p;
    hipError_t e = launch_sample_depol(g->tn, seed, shot0, n_shots, fire_threshold(1.0 * p / 3.0),
                                       fire_threshold(2.0 * p / 3.0), fire_threshold(p), syn_x, syn_z, obs,
                                       (hipStream_t)stream);
    return e == hipSuccess ? BPM_OK : hip_fail(e, "depolarizing sample launch");
}

bpm_status bpm_bbp4mf_workspace_size(const bpm_graph *g, uint64_t n_shots, const bpm_decode_opts *opts,
                                     size_t *bytes) {
    if (!bytes) return fail(BPM_EINVAL, "bytes is NULL");
    int32_t s_cap = 0;
    bpm_status st = bbp_check(g, opts, &s_cap);
    if (st != BPM_OK) return st;
    *bytes = bbp_layout(n_shots, s_cap).total;
    return BPM_OK;
}

bpm_status bpm_decode_bbp4mf(const bpm_graph *g, const uint64_t *syn_x, const uint64_t *syn_z, const uint64_t *obs,
                             uint64_t n_shots, const bpm_decode_opts *opts, const bpm_decode_out *out,
                             void *workspace, size_t workspace_bytes, void *stream) {
    int32_t s_cap = 0;
    bpm_status st = bbp_check(g, opts, &s_cap);
    if (st != BPM_OK) return st;
    if (!out) return fail(BPM_EINVAL, "out is NULL");
    if (out->corr || out->lambda_out) return fail(BPM_EUNSUPPORTED, "B-BP4MF writes no corrections or posteriors");
    if (out->match && out->match_stride < s_cap) return fail(BPM_EINVAL, "match_stride must be >= s_cap");
    if (n_shots == 0) return BPM_OK;
    if (!g->dev_mem) return fail(BPM_EDEVICE, "graph was built without a device");
    if (!syn_x || !syn_z) return fail(BPM_EINVAL, "syn_x and syn_z must be device buffers");
    const BbpLayout L = bbp_layout(n_shots, s_cap);
    if (!workspace || workspace_bytes < L.total) return fail(BPM_EINVAL, "workspace too small");
    if ((uintptr_t)workspace & 255) return fail(BPM_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    Instance I{};
    I.g = g->dg;
    I.base = 0;
    I.block0 = 0;
    InstState &d = I.st;
    d.n_shots = n_shots;
    d.W = (n_shots + 63) / 64;
    d.syn = syn_x;
    d.obs = obs;
    d.s = (int32_t *)(ws + L.s);
    d.flags = (uint8_t *)(ws + L.flags);
    d.obs_pred = out->obs_pred;
    d.fail = out->fail;
    d.shot_flags = out->shot_flags;
    d.shot_s = out->shot_s;
    d.counters = (unsigned long long *)out->counters;
    DecodeShared c{};
    c.max_iters = opts->max_iters;
    c.variant = opts->variant;
    c.s_cap = s_cap;
    c.inv_alpha = 1.0 / opts->alpha;
    c.n_inst = 1;
    c.total = n_shots;
    c.inst = (const Instance *)(ws + L.table);
    BbpArgs a{};
    a.g = g->dg;
    a.tn = g->tn;
    a.synx = syn_x;
    a.synz = syn_z;
    a.obs = obs;
    a.n = n_shots;
    a.W = d.W;
    a.variant = opts->variant;
    a.max_iters = opts->max_iters;
    a.s_cap = s_cap;
    a.inv_alpha = 1.0 / opts->alpha;
    a.pri_i = std::log1p(-g->noise.p);
    a.pri_p = std::log(g->noise.p / 3.0);
    a.slots = ws + L.slots;
    a.slot_bytes = L.slot_bytes;
    a.s_out = d.s;
    a.flags = d.flags;
    a.match = out->match;
    a.match_stride = out->match_stride;
    hipError_t e = launch_setup(&I, 1, (Instance *)(ws + L.table), s);
    if (e == hipSuccess) e = launch_bbp4mf(a, (int)std::min<uint64_t>(kBbpSlots, n_shots), s);
    if (e == hipSuccess) e = launch_finalize(c, shot_blocks(n_shots), s);
    return e == hipSuccess ? BPM_OK : hip_fail(e, "B-BP4MF launch");
}

}  // extern "C"
