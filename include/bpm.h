/*
 * bpm -- belief propagation for matching (BP4M) on surface-code decoding
 * graphs, MI355X (gfx950) library.  C ABI.
 *
 * Paper: "Achieving Thresholds via Standalone Belief Propagation on Surface
 * Codes", arXiv 2603.05381.  The call sequence follows the paper's problem
 * statement (Sec. I.B): build the detector graph of a code and noise model,
 * sample errors and their syndromes, decode every syndrome by belief
 * propagation on its decoding graph (Sec. II), and report corrections and
 * logical failures.
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" are HIP device memory on the current device;
 *    "host" pointers are ordinary host memory.  The caller owns every buffer
 *    it passes; the library never frees or keeps caller memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  bpm_sample and
 *    bpm_decode only enqueue work on it: they return before the work is done.
 *  - Argument errors are reported before anything is enqueued; the message
 *    is available from bpm_last_error() (per thread).  Device faults surface
 *    at the caller's next synchronisation.
 *  - Bit planes: bit b of word w of a plane is shot 64*w + b of the batch;
 *    a plane of n shots has W = ceil(n / 64) words; bits past n are zero.
 */
#ifndef BPM_H
#define BPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bpm_graph bpm_graph;

typedef enum {
    BPM_OK = 0,
    BPM_EINVAL = -1,        /* bad argument                                  */
    BPM_ENOMEM = -2,        /* host or device allocation failed              */
    BPM_EDEVICE = -3,       /* a HIP call failed                              */
    BPM_EUNSUPPORTED = -4,  /* valid request outside what is implemented     */
    BPM_EAGAIN = -5         /* server admission budget full: retry later     */
} bpm_status;

typedef enum {
    /* Rotated surface code with boundary plaquettes of weight 2; d odd >= 3. */
    BPM_ROTATED_SURFACE = 0,
    /* Unrotated (planar) surface code: d^2 + (d-1)^2 data qubits, d(d-1)
     * stabilizers of each type, d >= 2.  The paper's code-capacity and most
     * of its circuit-level experiments use this layout (Sec. III.E).  Its
     * memory-Z circuit visits the stabilizers' neighbours in the orders
     * N, W, E, S (X type) and N, E, W, S (Z type). */
    BPM_UNROTATED_SURFACE = 1
} bpm_code;

typedef enum {
    /* Code capacity (Sec. III.E): depolarizing noise of strength p on every
     * data qubit; Z errors are decoded on the X checks with q = 2p/3.  Such
     * graphs also carry the code's Tanner graph (both check types) for
     * B-BP4MF (bpm_sample_depolarizing, bpm_decode_bbp4mf). */
    BPM_CODE_CAPACITY_DEPOL = 0,
    /* Circuit level (Sec. III.E): memory-Z experiment of `rounds` rounds
     * with depolarizing noise p after every 1- and 2-qubit gate and on the
     * data before each round, and flips p after resets / before readouts.
     * Detectors are the Z stabilizers of every round and the final readout. */
    BPM_CIRCUIT_MEMORY_Z = 1
} bpm_noise_kind;

typedef struct {
    bpm_noise_kind kind;
    double p;               /* physical error rate, 0 < p < 0.5 */
} bpm_noise;

typedef struct {
    int32_t n_det;          /* detectors (nodes of the detector graph)        */
    int32_t n_mech;         /* error mechanisms (sampled independently)       */
    int32_t n_edges;        /* decoding-graph edges (= n_mech; all graphlike) */
    int32_t d, rounds;
    int32_t max_degree;     /* largest number of mechanisms at one detector  */
    double p;
    uint64_t device_bytes;  /* device memory held by the graph's tables       */
} bpm_graph_info;

typedef enum {
    BPM_BP4M = 0,           /* Sec. III.A: forced convergence once, at the end */
    BPM_BP4MF = 1           /* Sec. III.B: forced convergence at every iteration */
} bpm_variant;

typedef enum {
    /* FP64 with the pairwise Jacobian-logarithm fold and the library's own
     * exp/log1p, evaluated in a fixed order: bit-reproducible. */
    BPM_FP64_SPEC = 0,
    /* FP32 messages, exact leave-one-out log-sum-exp by max shifting. */
    BPM_FP32 = 1,
    /* FP32 arithmetic with messages stored (and exchanged) rounded to
     * bfloat16 / IEEE half precision, round to nearest even: half the
     * message memory.  A message is rounded once, when it is written; both
     * of its readers use the rounded value. */
    BPM_BF16_STORE = 2,
    BPM_FP16_STORE = 3
} bpm_precision;

typedef struct {
    int32_t max_iters;      /* T >= 1 (paper: 25 code capacity, 50 circuit) */
    int32_t variant;        /* bpm_variant                                   */
    int32_t precision;      /* bpm_precision                                 */
    int32_t s_cap;          /* most defects per shot, <= 1024; 0 = min(n_det, 512).
                               Shots above it are flagged BPM_SHOT_OVERFLOW,
                               counted, and not decoded: they predict no flip
                               and count as logical failures (BPM_SHOT_FAIL),
                               so a failure count is an upper bound.        */
    double alpha;           /* memory factor (Sec. III.E, "BP Improvements"):
                               variable-to-factor messages use 1/alpha times
                               the incoming factor messages; 1 = plain BP   */
    int32_t class_streams;  /* 0 or 1: every kernel on the caller's stream.
                               2..8: the size-class kernels run concurrently
                               on that many streams (the caller's and
                               library-owned ones, joined back to the caller's
                               stream with events before the result packing);
                               the results are the same.                     */
} bpm_decode_opts;

/* Per-shot flag bits written to bpm_decode_out.shot_flags. */
enum {
    BPM_SHOT_CONVERGED_ANY = 1,  /* marginalization converged at some iteration */
    BPM_SHOT_FC_RAN = 2,         /* forced convergence was evaluated            */
    BPM_SHOT_FC_CHOSEN = 4,      /* the output came from forced convergence     */
    BPM_SHOT_PRED = 8,           /* predicted flip of the logical observable    */
    BPM_SHOT_FAIL = 16,          /* prediction differs from the sampled flip    */
    BPM_SHOT_OVERFLOW = 32,      /* more than s_cap defects: not decoded, and
                                    flagged BPM_SHOT_FAIL as well              */
    BPM_SHOT_QBP_CONVERGED = 64  /* B-BP4MF: quaternary BP reproduced both
                                    syndromes and gave the output              */
};

typedef struct {
    uint64_t shots;
    uint64_t failures;          /* logical failures, overflow shots included  */
    uint64_t never_converged;   /* shots with s >= 2 never converged (r_nc)   */
    uint64_t fc_chosen;         /* outputs taken from forced convergence      */
    uint64_t sum_s;             /* total defects                              */
    uint64_t overflow;          /* shots above s_cap                          */
} bpm_counters;

/* Outputs of bpm_decode; every pointer is device memory or NULL (= skip). */
typedef struct {
    uint64_t *obs_pred;     /* [W] predicted observable flip per shot         */
    uint64_t *fail;         /* [W] logical failure per shot                   */
    uint64_t *corr;         /* [n_edges][W] correction: edges of the matched
                               shortest paths, XORed                          */
    uint8_t *shot_flags;    /* [n] BPM_SHOT_* bits                            */
    int32_t *shot_s;        /* [n] defects per shot                           */
    int32_t *match;         /* [n][match_stride] partner of each defect in
                               ascending detector order (own index = matched
                               to the boundary); entries past s untouched     */
    int32_t match_stride;
    double *lambda_out;     /* [n][lambda_stride^2] posteriors after the last
                               iteration (row-major, diagonal = boundary) for
                               shots with 2 <= s <= lambda_stride             */
    int32_t lambda_stride;
    bpm_counters *counters; /* accumulated into (not reset)                  */
    /* Optional stage timing: if non-NULL, stage_events[2k] and
     * stage_events[2k+1] (hipEvent_t created by the caller) are recorded on
     * the stream before and after stage k of the table bpm_stage_table
     * describes (defect extraction, one message-passing kernel per size
     * class of shots, result packing). */
    void *stage_events[2 * 32];
} bpm_decode_out;

enum { BPM_MAX_STAGES = 32 };

/* Stages of bpm_decode, in launch order; returns their number n
 * (<= BPM_MAX_STAGES).  Stage 0 extracts the defects of every shot and sorts
 * shots into size classes; stage n-1 packs the results.  Stages 1..n-2 run
 * message passing for one size class each: with max_s non-NULL (room for
 * BPM_MAX_STAGES entries), max_s[k] is the largest defect count stage k
 * decodes (the class starts after the previous stage's bound; stage 1 at
 * 2 defects), INT32_MAX for stage n-2, which takes every larger shot and,
 * in BPM_FP64_SPEC, every shot; max_s[0] = max_s[n-1] = 0. */
int32_t bpm_stage_table(int32_t *max_s);

/* Build the detector graph, its decoding-graph path tables and priors, and
 * upload them to the current device (Sec. I.B; prior equation of Sec. II.A).
 * Host, synchronous.  *out is owned by the caller and released with
 * bpm_graph_free.  d odd >= 3; rounds >= 1 (ignored for code capacity).
 * On a machine without a HIP device the host tables are still built (and
 * can be copied out); bpm_sample / bpm_decode then return BPM_EDEVICE. */
bpm_status bpm_build_graph(bpm_code code, int32_t d, int32_t rounds,
                           const bpm_noise *noise, bpm_graph **out);
bpm_status bpm_graph_info_get(const bpm_graph *g, bpm_graph_info *info);
void bpm_graph_free(bpm_graph *g);

/* Copy the mechanism list to host arrays: off[n_mech+1], dets[off[n_mech]],
 * obs[n_mech], q[n_mech].  Mechanism m flips detectors dets[off[m]..off[m+1])
 * and the observable iff obs[m]; it fires with probability q[m].  Any array
 * may be NULL. */
bpm_status bpm_graph_copy_mechanisms(const bpm_graph *g, int32_t *off, int32_t *dets,
                                     uint8_t *obs, double *q);

/* Copy the N x N path tables (N = n_det, row-major, host arrays, any may be
 * NULL).  Entry [u][v] describes the shortest path u -> v (v != u), entry
 * [u][u] the shortest path from u to the boundary: dist in 2^-32 units of
 * sum ln((1-q)/q), hops, observable parity, the edge id of the path's last
 * edge, and the prior LLR l = -D - ln(1 - e^-D) (Sec. II.B prior LLR). */
bpm_status bpm_graph_copy_tables(const bpm_graph *g, int64_t *dist, int32_t *hops,
                                 uint8_t *par, int32_t *pred, double *llr);

/* Sample n_shots independent shots with global indices shot0 .. shot0+n-1
 * (the detector error model of Sec. III.E; the problem statement of
 * Sec. I.B: errors and their syndromes): every mechanism fires
 * independently (Philox4x32-10 keyed by seed, counter (m div 4, shot), word
 * m mod 4, compared with round(q * 2^32)).
 * syn: device [n_det][W] detector bit planes; obs: device [W] observable
 * flips; err: NULL, or device [n_mech][W] planes of the sampled error itself
 * (bit b of plane m: mechanism m fired in shot b).  All given planes are
 * fully overwritten.  syn is the XOR of the fired mechanisms' detectors and
 * obs of their observable bits. */
bpm_status bpm_sample(const bpm_graph *g, uint64_t seed, uint64_t shot0, uint64_t n_shots,
                      uint64_t *syn, uint64_t *obs, uint64_t *err, void *stream);

/* Bytes of device workspace bpm_decode needs for n_shots with these options. */
bpm_status bpm_decode_workspace_size(const bpm_graph *g, uint64_t n_shots,
                                     const bpm_decode_opts *opts, size_t *bytes);

/* Decode every shot of the batch: per shot, BP on the factor graph of its
 * decoding graph (Sec. II.A-II.B), marginalization and the convergence check
 * at every iteration (Sec. II.C-II.D), forced convergence per the variant
 * (Sec. III.A-III.B), then the observable prediction and failure flag.
 * syn/obs: device bit planes as written by bpm_sample.  workspace: device,
 * at least bpm_decode_workspace_size bytes, 256-byte aligned; its contents
 * are scratch.  Shots are independent: a shot's result does not depend on
 * the rest of the batch. */
bpm_status bpm_decode(const bpm_graph *g, const uint64_t *syn, const uint64_t *obs,
                      uint64_t n_shots, const bpm_decode_opts *opts,
                      const bpm_decode_out *out, void *workspace, size_t workspace_bytes,
                      void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * bpm_decode with its workspace taken from a fixed scratch array of
 * BPM_NOALLOC_SCRATCH_BYTES that the library keeps on every device it runs
 * on (from the first call on that device until the process ends), instead
 * of a workspace argument.  Calls no allocating routine.  Arguments, outputs
 * and results as bpm_decode, bit for bit.  Returns BPM_EINVAL, with the
 * bytes needed in bpm_last_error(), when bpm_decode_workspace_size exceeds
 * the array (about 460 bytes per shot at s_cap = 192 in the FP32 modes, so
 * ~1.4e5 shots per call; s_cap above 192 needs more than the array holds),
 * and BPM_EUNSUPPORTED for class_streams > 1.  Every call on one device
 * shares that device's array: calls that overlap on one device (on
 * different streams or threads) race and must be serialised by the
 * caller. */
#define BPM_NOALLOC_SCRATCH_BYTES (64u << 20)
bpm_status bpm_decode_noalloc(const bpm_graph *g, const uint64_t *syn, const uint64_t *obs,
                              uint64_t n_shots, const bpm_decode_opts *opts,
                              const bpm_decode_out *out, void *stream);

/* ---- Kernel configurations and autotuning ----
 * A message-passing stage may have several kernel configurations (lanes per
 * factor row, resident workgroups per CU); every configuration computes the
 * same results, bit for bit, and only their speed differs.  The choice is
 * process-wide, one index per stage (0 = default), and applies to every
 * bpm_decode issued after it is made. */
enum { BPM_MAX_CONFIGS = 4 };

/* Number of configurations of stage k of bpm_stage_table (1 if there is
 * nothing to choose; 0 if k is not a stage). */
int32_t bpm_stage_configs(int32_t stage);

/* cfg: host [BPM_MAX_STAGES].  Set fails with BPM_EINVAL (changing nothing)
 * if an entry is outside [0, bpm_stage_configs(k)), entries past the stage
 * count must be 0. */
bpm_status bpm_get_stage_config(int32_t *cfg);
bpm_status bpm_set_stage_config(const int32_t *cfg);

/* Time every configuration of every stage on n_shots shots sampled from g
 * with this seed, decoded with these options, and keep the fastest per
 * stage.  Synchronous: allocates its own device buffers, runs on `stream`,
 * waits for it, and frees them.  stage_ms (host [BPM_MAX_CONFIGS]
 * [BPM_MAX_STAGES] or NULL) receives the measured milliseconds of
 * configuration c of stage k at [c][k], -1 where none was measured.  In
 * BPM_FP64_SPEC there is one kernel and nothing is timed. */
bpm_status bpm_autotune(const bpm_graph *g, const bpm_decode_opts *opts, uint64_t n_shots, uint64_t seed,
                        float *stage_ms, void *stream);

/* ---- Several graphs in one call ----
 * bpm_decode_multi decodes the shots of up to BPM_MAX_INSTANCES instances,
 * each with its own graph, in one sequence of launches: the instances'
 * shots share the per-size-class work queues, so one launch per size class
 * covers every instance (Sec. III.E workloads at several distances).  The
 * options are common to all instances.  Results per instance are those
 * bpm_decode gives for that instance alone, bit for bit. */
enum { BPM_MAX_INSTANCES = 8 };

typedef struct {
    const bpm_graph *graph;
    /* Input, device memory.  rows_words == 0: detector bit planes
     * syn[n_det][W] and obs[W], as bpm_sample writes them.  rows_words > 0:
     * shot-major syndromes, syn[n_shots][rows_words] with bit (k mod 64) of
     * word (k div 64) set iff detector k fired (rows_words >=
     * ceil(n_det / 64)); obs may then be NULL, and failures are counted
     * against an observable flip of 0. */
    const uint64_t *syn;
    const uint64_t *obs;
    uint64_t n_shots;
    int32_t rows_words;
    bpm_decode_out out;         /* outputs of this instance; stage_events unused */
} bpm_decode_item;

bpm_status bpm_decode_multi_workspace_size(const bpm_decode_item *items, int32_t n_items,
                                           const bpm_decode_opts *opts, size_t *bytes);

/* stage_events: NULL or [2 * BPM_MAX_STAGES] hipEvent_t, as in
 * bpm_decode_out.  Total shots over the items must stay below 2^32; s_cap 0
 * means min(largest n_det, 512).  Argument errors are reported before
 * anything is enqueued. */
bpm_status bpm_decode_multi(const bpm_decode_item *items, int32_t n_items, const bpm_decode_opts *opts,
                            void *const *stage_events, void *workspace, size_t workspace_bytes,
                            void *stream);

/* ---- Decode server: continuous batching of small requests ----
 * Requests of 1..64 shots of one resident graph are queued with
 * bpm_server_submit and decoded by a worker thread in batches: whenever
 * one of `slots` in-flight slots is free, every pending request (up to
 * max_batch_shots per graph) is packed into that slot and decoded with one
 * bpm_decode_multi launch sequence on the slot's own stream, so requests
 * that arrive while others are on the GPU are admitted as slots free up and
 * their work overlaps on the device.  A shot's result depends only on its
 * own syndrome: it is the same alone and in any mix.  Admission is bounded
 * by max_pending_shots (queued, not yet in a slot) and, if mem_budget is
 * set, by device memory: beyond either submit returns BPM_EAGAIN.  Device
 * memory per slot is fixed at creation.  The server
 * holds pointers to the graphs, which must outlive it.  Calls are
 * thread-safe. */
typedef struct bpm_server bpm_server;

typedef struct {
    int32_t max_batch_shots;    /* shots per graph per batch: a multiple of 64 in [64, 65536] */
    int32_t max_pending_shots;  /* admission budget, >= 64                                    */
    int32_t slots;              /* batches in flight at once, 1..8                            */
    int32_t use_graphs;         /* 1: replay a captured HIP graph of the launch sequence,
                                   one per slot and shot bucket (batches padded with empty
                                   shots to a power of 4 >= 64)                              */
    bpm_decode_opts decode;
    int32_t one_graph_per_batch; /* 1: a batch takes only requests of the graph of the oldest
                                   pending request, so requests of small graphs are not held
                                   to the pace of large ones; 0: every graph in one batch    */
    uint64_t mem_budget;        /* 0: admission by max_pending_shots only.  Otherwise device
                                   bytes the server may account for: the slots' buffers
                                   (fixed at creation; BPM_ENOMEM if they exceed it) plus,
                                   for every queued request, the device bytes its shots take
                                   once in a slot (syndrome rows, flags and decode workspace
                                   per shot of its graph); submit returns BPM_EAGAIN when a
                                   request would not fit, so large graphs weigh more       */
} bpm_server_opts;

typedef struct {
    uint64_t req_id;
    int32_t graph;
    uint32_t n_shots;
    uint64_t pred;              /* bit i: predicted observable flip of shot i                */
    uint64_t fc_chosen;         /* bit i: shot i's output came from forced convergence       */
    uint64_t overflow;          /* bit i: shot i had more than s_cap defects (not decoded)   */
    double latency_us;          /* submit to result, server clock                            */
} bpm_server_result;

typedef struct {
    uint64_t requests_done, shots_done, batches, pending_shots;
} bpm_server_stats;

/* graphs: n_graphs (1..BPM_MAX_INSTANCES) device-resident graphs, indexed by
 * graph_idx in submit.  Allocates the slots' pinned host and device buffers
 * and starts the worker. */
bpm_status bpm_server_create(const bpm_graph *const *graphs, int32_t n_graphs, const bpm_server_opts *opts,
                             bpm_server **out);
/* rows: host [n_shots][ceil(n_det / 64)] shot-major syndromes (bit k of a
 * row: detector k fired), copied before the call returns. */
bpm_status bpm_server_submit(bpm_server *srv, int32_t graph_idx, const uint64_t *rows, uint32_t n_shots,
                             uint64_t req_id);
/* Moves up to max_results finished requests into res; returns how many. */
int32_t bpm_server_poll(bpm_server *srv, bpm_server_result *res, int32_t max_results);
/* Counters; returns BPM_EDEVICE if the worker stopped on a device error. */
bpm_status bpm_server_stats_get(bpm_server *srv, bpm_server_stats *stats);
/* Finishes the batches in flight, drops requests not yet admitted, frees. */
void bpm_server_destroy(bpm_server *srv);

/* Message of the last failed call on this thread ("" if none). */
const char *bpm_last_error(void);

/* ---- B-BP4MF: quaternary BP, then BP4MF on re-weighted paths ----
 * (Sec. III.D "Belief-BP4MF"; correlated decoding, Sec. II.E.)  For graphs
 * built with BPM_CODE_CAPACITY_DEPOL (either code), whose noise is
 * depolarizing of strength p on every data qubit. */

/* Sample depolarizing noise on every data qubit, with both syndromes:
 * per qubit v and shot sigma, u = word 0 of Philox4x32-10(counter (v,
 * sigma mod 2^32, sigma div 2^32, 0x44455031), key (seed mod 2^32,
 * seed div 2^32)) gives X if u < t1, Y if u < t2, Z if u < t3, else I, with
 * t_k = round(k p/3 2^32) (k = 1, 2) and t3 = round(p 2^32).
 * syn_x: device [n_det][W] planes of the X checks (the graph's detectors);
 * syn_z: device [n_det][W] planes of the Z checks (the same count for these
 * codes); obs: device [W], the Z part on the observable's qubits.
 * BPM_EUNSUPPORTED for other graphs. */
bpm_status bpm_sample_depolarizing(const bpm_graph *g, uint64_t seed, uint64_t shot0, uint64_t n_shots,
                                   uint64_t *syn_x, uint64_t *syn_z, uint64_t *obs, void *stream);

/* Bytes of device workspace bpm_decode_bbp4mf needs. */
bpm_status bpm_bbp4mf_workspace_size(const bpm_graph *g, uint64_t n_shots, const bpm_decode_opts *opts,
                                     size_t *bytes);

/* B-BP4MF of every shot: (1) quaternary BP on the code's Tanner graph (both
 * check types, depolarizing prior, opts->max_iters iterations); a shot whose
 * hard decision reproduces both syndromes at some iteration takes it as the
 * output (flag BPM_SHOT_QBP_CONVERGED); (2) otherwise each qubit's posterior
 * probability P of a Z component re-weights its decoding-graph edge
 * (ln((1-P)/P), at least 2^-32), the shortest paths between the shot's X
 * defects are recomputed, and (3) opts->variant (BPM_BP4MF as in the paper;
 * BPM_BP4M also allowed) runs for max_iters iterations on their priors.
 * Precision must be BPM_FP64_SPEC: every step runs in FP64 in a fixed order,
 * reproducible bit for bit.  Outputs as bpm_decode (obs_pred, fail, flags, s
 * = X defects, match for shots decoded by stage 3, counters); corr and
 * lambda_out must be NULL (BPM_EUNSUPPORTED).  s_cap: 0 = min(n_det, 256).
 * Codes of up to 1024 qubits whose decoding graph has at most 512 detectors
 * of at most 8 edges each (every rotated or unrotated code-capacity graph
 * within the qubit limit); otherwise BPM_EUNSUPPORTED. */
bpm_status bpm_decode_bbp4mf(const bpm_graph *g, const uint64_t *syn_x, const uint64_t *syn_z,
                             const uint64_t *obs, uint64_t n_shots, const bpm_decode_opts *opts,
                             const bpm_decode_out *out, void *workspace, size_t workspace_bytes,
                             void *stream);

#ifdef __cplusplus
}
#endif
#endif
