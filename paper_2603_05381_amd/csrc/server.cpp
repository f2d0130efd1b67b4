// Decode server: continuous batching of small syndrome requests over
// resident graphs (the paper's decoder applied as a service; the batching is
// this library's design, not the paper's).
//
// Requests (1..64 shots of one graph, shot-major syndrome rows in host
// memory) are queued by bpm_server_submit.  A worker thread forms batches
// from whatever is pending (or, with one_graph_per_batch, from the pending
// requests of the oldest request's graph) whenever one of `slots` in-flight
// slots is free:
// it packs the requests' rows into the slot's pinned buffers, copies them to
// the device, decodes all graphs of the batch with one bpm_decode_multi
// launch sequence (or a captured HIP graph of it), and copies the per-shot
// flags back, all on the slot's own stream.  Several slots run at once, so
// requests that arrive while others are on the GPU are admitted as soon as
// a slot frees, and their work overlaps on the device.  Each shot's result
// depends only on its own syndrome.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "bpm.h"
#include "device_common.hpp"
#include "graph_internal.hpp"

using Clock = std::chrono::steady_clock;
using namespace bpm;

namespace {

struct Request {
    uint64_t id;
    int graph;
    uint32_t n;
    std::vector<uint64_t> rows;     // [n][words of the graph]
    Clock::time_point t_submit;
};

struct InFlight {
    int graph;
    uint32_t n, offset;             // shots, first row in the graph's batch
    uint64_t id;
    Clock::time_point t_submit;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    // per graph: pinned host rows and flags, device rows and flags
    std::vector<uint64_t *> h_rows, d_rows;
    std::vector<uint8_t *> h_flags, d_flags;
    void *d_ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<uint32_t> batch_n;  // shots of each graph in the current batch
    std::vector<InFlight> reqs;
    std::map<uint32_t, hipGraphExec_t> graphs;   // captured launch sequences by shot bucket
};

}  // namespace

struct bpm_server {
    std::vector<const bpm_graph *> graphs;
    std::vector<int> words;         // row words per graph
    std::vector<int> n_det;
    bpm_server_opts opts{};
    int device = 0;
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> pending;
    uint64_t pending_shots = 0;
    uint64_t pending_bytes = 0;     // device bytes the queued shots take in a slot
    std::vector<uint64_t> shot_bytes;   // per graph: device bytes per shot
    uint64_t fixed_bytes = 0;       // the slots' device buffers
    std::deque<bpm_server_result> done;
    bool stop = false;
    std::string worker_error;
    std::thread worker;

    std::atomic<uint64_t> n_requests{0}, n_shots{0}, n_batches{0};
};

namespace {

bpm_status sfail(bpm_status st, const std::string &m) { return set_last_error(st, m); }

// Shots decoded for a batch of n shots of one graph: exact without HIP
// graphs; rounded up to a power of 4 (>= 64) with them, so that a few
// captured sequences cover every batch.
uint32_t bucket_of(uint32_t n, bool graphs, uint32_t cap) {
    if (!graphs) return n;
    uint32_t b = 64;
    while (b < n) b *= 4;
    return std::min(b, cap);
}

// Build the decode items of a slot for per-graph shot counts n[g].
std::vector<bpm_decode_item> slot_items(bpm_server *S, Slot &sl, const std::vector<uint32_t> &n) {
    std::vector<bpm_decode_item> it;
    for (size_t g = 0; g < S->graphs.size(); ++g) {
        if (n[g] == 0) continue;
        bpm_decode_item x{};
        x.graph = S->graphs[g];
        x.syn = sl.d_rows[g];
        x.obs = nullptr;
        x.n_shots = n[g];
        x.rows_words = S->words[g];
        x.out.shot_flags = sl.d_flags[g];
        it.push_back(x);
    }
    return it;
}

// Enqueue copy-in, decode and copy-out of the slot's current batch.
hipError_t launch_batch(bpm_server *S, Slot &sl, uint32_t bucket, bool use_graph) {
    const size_t G = S->graphs.size();
    std::vector<uint32_t> n(G);
    for (size_t g = 0; g < G; ++g) n[g] = use_graph ? bucket : sl.batch_n[g];
    hipError_t e = hipSuccess;
    for (size_t g = 0; g < G && e == hipSuccess; ++g)
        if (n[g]) e = hipMemcpyAsync(sl.d_rows[g], sl.h_rows[g], sizeof(uint64_t) * S->words[g] * n[g],
                                     hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) return e;
    std::vector<bpm_decode_item> items = slot_items(S, sl, n);
    if (items.empty()) return hipSuccess;
    if (use_graph) {
        auto it = sl.graphs.find(bucket);
        if (it == sl.graphs.end()) {
            // one eager run first (kernel loading, occupancy queries), then capture
            if (bpm_decode_multi(items.data(), (int32_t)items.size(), &S->opts.decode, nullptr, sl.d_ws,
                                 sl.ws_bytes, sl.stream) != BPM_OK)
                return hipErrorUnknown;
            e = hipStreamSynchronize(sl.stream);
            if (e != hipSuccess) return e;
            hipGraph_t gr = nullptr;
            e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            const bpm_status st = bpm_decode_multi(items.data(), (int32_t)items.size(), &S->opts.decode, nullptr,
                                                   sl.d_ws, sl.ws_bytes, sl.stream);
            e = hipStreamEndCapture(sl.stream, &gr);
            if (st != BPM_OK && e == hipSuccess) e = hipErrorUnknown;
            hipGraphExec_t ex = nullptr;
            if (e == hipSuccess) e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            if (gr) hipGraphDestroy(gr);
            if (e != hipSuccess) return e;
            it = sl.graphs.emplace(bucket, ex).first;
        }
        e = hipGraphLaunch(it->second, sl.stream);
    } else {
        if (bpm_decode_multi(items.data(), (int32_t)items.size(), &S->opts.decode, nullptr, sl.d_ws, sl.ws_bytes,
                             sl.stream) != BPM_OK)
            return hipErrorUnknown;
    }
    for (size_t g = 0; g < G && e == hipSuccess; ++g)
        if (sl.batch_n[g])
            e = hipMemcpyAsync(sl.h_flags[g], sl.d_flags[g], sl.batch_n[g], hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    return e;
}

// Publish the results of a finished slot.
void complete(bpm_server *S, Slot &sl) {
    const auto now = Clock::now();
    std::vector<bpm_server_result> out;
    out.reserve(sl.reqs.size());
    for (const InFlight &r : sl.reqs) {
        bpm_server_result x{};
        x.req_id = r.id;
        x.graph = r.graph;
        x.n_shots = r.n;
        const uint8_t *f = sl.h_flags[r.graph] + r.offset;
        for (uint32_t i = 0; i < r.n; ++i) {
            if (f[i] & kPred) x.pred |= 1ull << i;
            if (f[i] & kFcChosen) x.fc_chosen |= 1ull << i;
            if (f[i] & kOverflow) x.overflow |= 1ull << i;
        }
        x.latency_us = std::chrono::duration<double, std::micro>(now - r.t_submit).count();
        out.push_back(x);
    }
    S->n_requests += sl.reqs.size();
    S->n_batches += 1;
    sl.reqs.clear();
    sl.busy = false;
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto &x : out) S->done.push_back(x);
}

void worker_main(bpm_server *S) {
    hipSetDevice(S->device);
    const size_t G = S->graphs.size();
    const uint32_t cap = (uint32_t)S->opts.max_batch_shots;
    const bool use_graph = S->opts.use_graphs != 0;
    for (;;) {
        // 1. retire finished slots
        for (Slot &sl : S->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) complete(S, sl);
            else if (q != hipErrorNotReady) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->worker_error = std::string("device error: ") + hipGetErrorString(q);
                S->stop = true;
            }
        }
        // 2. admit pending requests into a free slot
        Slot *free_slot = nullptr;
        for (Slot &sl : S->slots)
            if (!sl.busy) { free_slot = &sl; break; }
        std::vector<Request> batch;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop) break;
            bool any_busy = false;
            for (Slot &sl : S->slots) any_busy |= sl.busy;
            if (free_slot && S->pending.empty() && !any_busy) {
                S->cv.wait(lk, [&] { return S->stop || !S->pending.empty(); });
                if (S->stop) break;
            }
            if (free_slot) {
                std::vector<uint32_t> used(G, 0);
                const int only = S->opts.one_graph_per_batch && !S->pending.empty() ? S->pending.front().graph : -1;
                for (auto it = S->pending.begin(); it != S->pending.end();) {
                    if ((only >= 0 && it->graph != only) || used[it->graph] + it->n > cap) { ++it; continue; }
                    used[it->graph] += it->n;
                    S->pending_shots -= it->n;
                    S->pending_bytes -= S->shot_bytes[it->graph] * it->n;
                    batch.push_back(std::move(*it));
                    it = S->pending.erase(it);
                }
            }
        }
        if (free_slot && !batch.empty()) {
            Slot &sl = *free_slot;
            std::fill(sl.batch_n.begin(), sl.batch_n.end(), 0u);
            for (Request &r : batch) {
                const uint32_t off = sl.batch_n[r.graph];
                std::memcpy(sl.h_rows[r.graph] + (size_t)off * S->words[r.graph], r.rows.data(),
                            sizeof(uint64_t) * r.rows.size());
                sl.batch_n[r.graph] += r.n;
                sl.reqs.push_back(InFlight{r.graph, r.n, off, r.id, r.t_submit});
                S->n_shots += r.n;
            }
            uint32_t bucket = 0;
            for (size_t g = 0; g < G; ++g) bucket = std::max(bucket, bucket_of(sl.batch_n[g], use_graph, cap));
            if (use_graph)                      // empty rows for the padding shots
                for (size_t g = 0; g < G; ++g)
                    std::memset(sl.h_rows[g] + (size_t)sl.batch_n[g] * S->words[g], 0,
                                sizeof(uint64_t) * S->words[g] * (bucket - sl.batch_n[g]));
            sl.busy = true;
            const hipError_t e = launch_batch(S, sl, bucket, use_graph);
            if (e != hipSuccess) {
                std::lock_guard<std::mutex> lk(S->mu);
                S->worker_error = std::string("batch launch failed: ") + hipGetErrorString(e) + " " + bpm_last_error();
                S->stop = true;
                break;
            }
            continue;                           // try to fill another free slot at once
        }
        // 3. nothing admitted: poll again shortly.  (Blocking on one slot's
        // event would leave any other slot that finishes first idle, with
        // its results unpublished, until that one is done.)
        bool any_busy = false;
        for (Slot &sl : S->slots) any_busy |= sl.busy;
        if (any_busy) std::this_thread::sleep_for(std::chrono::microseconds(free_slot ? 20 : 10));
    }
    // drain: wait for every slot so that buffers can be freed safely
    for (Slot &sl : S->slots)
        if (sl.busy) { hipEventSynchronize(sl.done); complete(S, sl); }
}

void free_slot(Slot &sl) {
    for (auto &kv : sl.graphs) hipGraphExecDestroy(kv.second);
    for (auto *p : sl.h_rows) if (p) hipHostFree(p);
    for (auto *p : sl.h_flags) if (p) hipHostFree(p);
    for (auto *p : sl.d_rows) if (p) hipFree(p);
    for (auto *p : sl.d_flags) if (p) hipFree(p);
    if (sl.d_ws) hipFree(sl.d_ws);
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.stream) hipStreamDestroy(sl.stream);
}

void destroy(bpm_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (Slot &sl : S->slots) free_slot(sl);
    delete S;
}

}  // namespace

extern "C" {

bpm_status bpm_server_create(const bpm_graph *const *graphs, int32_t n_graphs, const bpm_server_opts *opts,
                             bpm_server **out) {
    if (!out) return sfail(BPM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!graphs || !opts) return sfail(BPM_EINVAL, "NULL argument");
    if (n_graphs < 1 || n_graphs > BPM_MAX_INSTANCES) return sfail(BPM_EINVAL, "n_graphs must lie in [1, BPM_MAX_INSTANCES]");
    if (opts->max_batch_shots < 64 || opts->max_batch_shots > 65536 || opts->max_batch_shots % 64)
        return sfail(BPM_EINVAL, "max_batch_shots must be a multiple of 64 in [64, 65536]");
    if (opts->max_pending_shots < 64) return sfail(BPM_EINVAL, "max_pending_shots must be >= 64");
    if (opts->slots < 1 || opts->slots > 8) return sfail(BPM_EINVAL, "slots must lie in [1, 8]");
    if (opts->use_graphs != 0 && opts->use_graphs != 1) return sfail(BPM_EINVAL, "use_graphs must be 0 or 1");
    if (opts->one_graph_per_batch != 0 && opts->one_graph_per_batch != 1)
        return sfail(BPM_EINVAL, "one_graph_per_batch must be 0 or 1");
    bpm_server *S = new (std::nothrow) bpm_server();
    if (!S) return sfail(BPM_ENOMEM, "host allocation failed");
    S->opts = *opts;
    for (int g = 0; g < n_graphs; ++g) {
        if (!graphs[g]) { delete S; return sfail(BPM_EINVAL, "graph is NULL"); }
        bpm_graph_info info;
        bpm_graph_info_get(graphs[g], &info);
        if (info.device_bytes == 0) { delete S; return sfail(BPM_EDEVICE, "graph was built without a device"); }
        S->graphs.push_back(graphs[g]);
        S->words.push_back((info.n_det + 63) / 64);
        S->n_det.push_back(info.n_det);
    }
    // validate the decode options and size the workspace for full batches
    const uint32_t cap = (uint32_t)opts->max_batch_shots;
    std::vector<bpm_decode_item> items(n_graphs);
    for (int g = 0; g < n_graphs; ++g) {
        items[g] = bpm_decode_item{};
        items[g].graph = graphs[g];
        items[g].n_shots = cap;
        items[g].rows_words = S->words[g];
    }
    size_t ws = 0;
    bpm_status st = bpm_decode_multi_workspace_size(items.data(), n_graphs, &opts->decode, &ws);
    if (st != BPM_OK) { delete S; return st; }
    // device bytes per shot of each graph in a slot: its rows and flags, and
    // the decode workspace that grows with the shot count
    S->shot_bytes.assign(n_graphs, 0);
    for (int g = 0; g < n_graphs; ++g) {
        bpm_decode_item one = items[g];
        size_t w_hi = 0, w_lo = 0;
        one.n_shots = cap;
        st = bpm_decode_multi_workspace_size(&one, 1, &opts->decode, &w_hi);
        one.n_shots = 64;
        if (st == BPM_OK) st = bpm_decode_multi_workspace_size(&one, 1, &opts->decode, &w_lo);
        if (st != BPM_OK) { delete S; return st; }
        const uint64_t per = cap > 64 ? ((uint64_t)(w_hi - w_lo) + (cap - 64) - 1) / (cap - 64) : (w_hi + 63) / 64;
        S->shot_bytes[g] = sizeof(uint64_t) * S->words[g] + 1 + per;
    }
    for (int g = 0; g < n_graphs; ++g) S->fixed_bytes += (sizeof(uint64_t) * S->words[g] + 1) * (uint64_t)cap;
    S->fixed_bytes = (S->fixed_bytes + ws + 256) * (uint64_t)opts->slots;
    if (opts->mem_budget && S->fixed_bytes > opts->mem_budget) {
        const uint64_t need = S->fixed_bytes;
        delete S;
        return sfail(BPM_ENOMEM, "mem_budget " + std::to_string(opts->mem_budget) + " bytes is below the " +
                                     std::to_string(need) + " bytes the slots need");
    }
    hipGetDevice(&S->device);
    S->slots.resize(opts->slots);
    hipError_t e = hipSuccess;
    for (Slot &sl : S->slots) {
        sl.h_rows.assign(n_graphs, nullptr); sl.d_rows.assign(n_graphs, nullptr);
        sl.h_flags.assign(n_graphs, nullptr); sl.d_flags.assign(n_graphs, nullptr);
        sl.batch_n.assign(n_graphs, 0);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        for (int g = 0; g < n_graphs && e == hipSuccess; ++g) {
            const size_t rb = sizeof(uint64_t) * S->words[g] * cap;
            e = hipHostMalloc((void **)&sl.h_rows[g], rb, hipHostMallocDefault);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_flags[g], cap, hipHostMallocDefault);
            if (e == hipSuccess) e = hipMalloc((void **)&sl.d_rows[g], rb);
            if (e == hipSuccess) e = hipMalloc((void **)&sl.d_flags[g], cap);
            if (e == hipSuccess) std::memset(sl.h_rows[g], 0, rb);
        }
        sl.ws_bytes = ws;
        if (e == hipSuccess) e = hipMalloc(&sl.d_ws, ws + 256);
    }
    if (e != hipSuccess) {
        for (Slot &sl : S->slots) free_slot(sl);
        delete S;
        return sfail(BPM_ENOMEM, std::string("server buffers: ") + hipGetErrorString(e));
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return BPM_OK;
}

bpm_status bpm_server_submit(bpm_server *S, int32_t graph_idx, const uint64_t *rows, uint32_t n_shots,
                             uint64_t req_id) {
    if (!S || !rows) return sfail(BPM_EINVAL, "NULL argument");
    if (graph_idx < 0 || graph_idx >= (int32_t)S->graphs.size()) return sfail(BPM_EINVAL, "graph index out of range");
    if (n_shots < 1 || n_shots > 64) return sfail(BPM_EINVAL, "a request holds 1 to 64 shots");
    Request r;
    r.id = req_id;
    r.graph = graph_idx;
    r.n = n_shots;
    const int w = S->words[graph_idx];
    r.rows.assign(rows, rows + (size_t)w * n_shots);
    // bits past n_det are not detectors: clear them
    const int n_det = S->n_det[graph_idx];
    if (n_det % 64)
        for (uint32_t i = 0; i < n_shots; ++i) r.rows[(size_t)i * w + w - 1] &= (1ull << (n_det % 64)) - 1;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->worker_error.empty()) return sfail(BPM_EDEVICE, S->worker_error);
        if (S->pending_shots + n_shots > (uint64_t)S->opts.max_pending_shots)
            return sfail(BPM_EAGAIN, "pending-shot budget full");
        const uint64_t nb = S->shot_bytes[graph_idx] * n_shots;
        if (S->opts.mem_budget && S->fixed_bytes + S->pending_bytes + nb > S->opts.mem_budget)
            return sfail(BPM_EAGAIN, "device-memory budget full");
        r.t_submit = Clock::now();
        S->pending_shots += n_shots;
        S->pending_bytes += nb;
        S->pending.push_back(std::move(r));
    }
    S->cv.notify_one();
    return BPM_OK;
}

int32_t bpm_server_poll(bpm_server *S, bpm_server_result *res, int32_t max_results) {
    if (!S || !res || max_results < 1) return 0;
    std::lock_guard<std::mutex> lk(S->mu);
    int32_t k = 0;
    while (k < max_results && !S->done.empty()) {
        res[k++] = S->done.front();
        S->done.pop_front();
    }
    return k;
}

bpm_status bpm_server_stats_get(bpm_server *S, bpm_server_stats *st) {
    if (!S || !st) return sfail(BPM_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    st->requests_done = S->n_requests.load();
    st->shots_done = S->n_shots.load();
    st->batches = S->n_batches.load();
    st->pending_shots = S->pending_shots;
    if (!S->worker_error.empty()) return sfail(BPM_EDEVICE, S->worker_error);
    return BPM_OK;
}

void bpm_server_destroy(bpm_server *S) { destroy(S); }

}  // extern "C"
