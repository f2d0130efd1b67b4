#!/usr/bin/env python3
"""Throughput benchmark: decoded shots per second of BP4M on one MI355X.

Workload (default): rotated surface code, circuit-level memory-Z experiment,
d = 13, 13 rounds, depolarizing p = 0.005 (1176 detectors, 6085 mechanisms),
BP4M with T = 50 iterations (the paper's circuit-level budget, Sec. III.E),
FP32 messages.  One step samples 10^6 fresh shots on the GPU (counter-based,
shot indices continue from step to step) and decodes them; syndromes stay in
HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--shots N] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from tests.inputs import seed_for  # noqa: E402  (seed recipe; no decoding arithmetic)

# Work model of one message update (one (factor, variable) pair in one
# iteration): 2 transcendental operations (one exp2, one log2) and 8 other
# FP32 operations, 10 in all.  roofline.peak is the published FP32 vector
# rate of MI355X, 157.3 TFLOP/s (256 CUs x 128 lanes x 2 (FMA) x 2.4 GHz).
# An issue-slot model is reported beside it as a diagnostic: FP32 VALU
# instructions without packed math issue at most 128 lanes/clock/CU (a wave64
# instruction every 2 cycles per SIMD), exp2/log2 at a quarter of that, so a
# message update of 8 plain + 2 transcendental operations costs 8 + 2 x 4 =
# 16 issue slots: 256 x 128 x 2.4e9 / 16 = 4.9e12 updates/s at most.
OPS_PER_MSG = 10
PEAK_FP32_TFLOPS = 157.3
SLOTS_PER_MSG = 16
LANE_SLOTS_PER_S = 256 * 128 * 2.4e9
PEAK_MSG_PER_S = LANE_SLOTS_PER_S / SLOTS_PER_MSG


# Sources of the FP32 group kernels: HBM traffic measured with rocprofv3
# counters is recorded in profiles/ together with their hash, and reported
# only while the sources are unchanged.
KERNEL_SOURCES = ("paper_2603_05381_amd/csrc/bp_group_impl.hpp", "paper_2603_05381_amd/csrc/bp_group_f32.hip",
                  "paper_2603_05381_amd/csrc/device_common.hpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(stage, shots):
    """HBM bytes per launch of `stage` from a 'traffic-record:' line in
    profiles/*.md, if it was measured on the current kernel sources at this
    batch size; else None."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    want = kernel_source_hash()
    for name in sorted(os.listdir(d)):
        if not name.endswith(".md"):
            continue
        for ln in open(os.path.join(d, name)):
            if ln.startswith("traffic-record:"):
                try:
                    rec = json.loads(ln[len("traffic-record:"):])
                except ValueError:
                    continue
                if rec.get("source_sha256") == want and rec.get("shots_per_launch") == shots:
                    per = rec.get("bytes_per_launch", {})
                    if stage in per:
                        return per[stage]
    return None


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(d, rounds, p, iters, seed, target_s=15.0):
    """The FP64 oracle on a bounded sample of the same workload: on every
    host thread this process may use, then on one thread."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    dem = oracle.memory_z(d, rounds, p)
    tab = oracle.tables(dem)

    def run(nthreads, budget, n):
        spent, shots = 0.0, 0
        while spent < budget:
            syn, obs = oracle.sample(dem, seed, shots, n)
            t0 = time.perf_counter()
            oracle.decode(dem, tab, syn, obs, n, iters, threads=nthreads)
            dt = time.perf_counter() - t0
            spent += dt
            shots += n
            if dt < budget / 4:
                n *= 2
        return shots, spent

    # the oracle spreads a batch over threads by 64-shot words: 64 shots per thread
    shots, spent = run(threads, target_s, 64 * threads)
    shots1, spent1 = run(1, max(2.0, target_s / 3), 4)
    return {"value": shots / spent, "unit": "shots/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "single_thread_shots_per_s": shots1 / spent1,
            "sample": "%d shots of the same workload on %d threads (%.1f s), then %d shots on 1 thread (%.1f s); "
                      "FP64 oracle" % (shots, threads, spent, shots1, spent1)}


def storage_variants(bpm, g, syn, obs, stream, seed, args, T, c32):
    """Reduced-precision message storage (BF16 / FP16, FP32 arithmetic) and
    the BP4MF variant (FP32) on the same kind of shots: throughput of one
    untimed-by-the-contract pass each, and the logical error rate against the
    FP32 BP4M run's.  The kernel configurations are restored afterwards."""
    import torch
    n = args.storage_shots
    W = (n + 63) // 64
    out = {}
    ler32 = c32["failures"] / max(c32["shots"], 1)
    saved_cfg = bpm.bpm_get_stage_config()
    for name, prec, variant in (("bf16", bpm.BPM_BF16_STORE, bpm.BPM_BP4M), ("fp16", bpm.BPM_FP16_STORE, bpm.BPM_BP4M),
                                ("bp4mf", bpm.BPM_FP32, bpm.BPM_BP4MF)):
        opts = bpm.bpm_decode_opts(T, variant, prec, 0, 1.0)
        if not args.no_autotune:
            bpm.bpm_autotune(g.handle, opts, args.autotune_shots, seed ^ 0x5A5A, stream.cuda_stream)
        ws_bytes = bpm.bpm_decode_workspace_size(g.handle, n, opts)
        ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
        ws_ptr = (ws.data_ptr() + 255) & ~255
        counters = torch.zeros(6, dtype=torch.int64, device="cuda")
        obs_pred = torch.empty(W, dtype=torch.int64, device="cuda")
        fail = torch.empty(W, dtype=torch.int64, device="cuda")
        times = []
        for rep in range(2):                     # the first pass warms up
            bpm.bpm_sample(g.handle, seed, (1000 + rep) * n, n, syn.data_ptr(), obs.data_ptr(), None, stream.cuda_stream)
            o = bpm.bpm_decode_out()
            o.obs_pred, o.fail, o.counters = obs_pred.data_ptr(), fail.data_ptr(), counters.data_ptr()
            if rep:
                counters.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bpm.bpm_decode(g.handle, syn.data_ptr(), obs.data_ptr(), n, opts, o, ws_ptr, ws_bytes, stream.cuda_stream)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        cc = bpm.counters_dict(counters)
        ler = cc["failures"] / max(cc["shots"], 1)
        sd = (max(ler32 * (1 - ler32), 1e-12) / max(cc["shots"], 1)) ** 0.5
        out[name] = {"decode_shots_per_s": n / times[1], "ler": ler, "ler_fp32": ler32,
                     "ler_diff_in_sd": (ler - ler32) / sd, "r_nc": cc["never_converged"] / max(cc["shots"], 1)}
        del ws
    bpm.bpm_set_stage_config(saved_cfg)
    return out


def threshold_sweep(bpm, n):
    """Logical error rates of the unrotated code under code-capacity noise
    (the layout of the paper's code-capacity experiments, T = 25), FP32."""
    import torch
    out = {"workload": "unrotated surface code, code capacity, T=25, FP32, %d shots per point" % n}
    for vname, variant in (("bp4m", bpm.BPM_BP4M), ("bp4mf", bpm.BPM_BP4MF)):
        tab = {}
        for d in (5, 9, 13):
            for p in (0.10, 0.11, 0.12, 0.13, 0.14, 0.15):
                g = bpm.Graph("code_capacity_unrotated", d, p)
                syn, obs = g.sample(seed_for(1, d, p), 0, n)
                r = g.decode(syn, obs, n, 25, precision=bpm.BPM_FP32, variant=variant)
                torch.cuda.synchronize()
                c = bpm.counters_dict(r["counters"])
                tab["d%d_p%.2f" % (d, p)] = {"ler": c["failures"] / n, "r_nc": c["never_converged"] / n}
                g.close()
        out[vname] = tab
    return out


def capacity_sweep(bpm, n):
    """The rotated code-capacity grid: d in {5, 7, 9, 11, 15}, p = 0.02 ...
    0.18, T = 25, FP32, one decode call per (d, p) on n sampled shots:
    logical error rate, mean defects per shot and decode rate."""
    import torch
    out = {"workload": "rotated surface code, code capacity, T=25, FP32, BP4M, %d shots per point" % n}
    # kernel configurations of the small classes (lanes per row, which sets the
    # unrolled entries per lane and the shots per workgroup) timed on a point
    # where they carry the work, then kept for the sweep
    ga = bpm.Graph("code_capacity", 15, 0.14)
    opts = bpm.bpm_decode_opts(25, bpm.BPM_BP4M, bpm.BPM_FP32, 0, 1.0)
    t_ms = bpm.bpm_autotune(ga.handle, opts, min(n, 1_000_000), 0xCC15, torch.cuda.current_stream().cuda_stream)
    cfg = bpm.bpm_get_stage_config()
    out["autotune_d15_p0.14"] = {bpm.STAGES[k]: {"chosen": cfg[k], "ms": [round(t_ms[c][k], 3) for c in range(4)
                                                                       if t_ms[c][k] >= 0]}
                                 for k in range(len(bpm.STAGES)) if bpm.bpm_stage_configs(k) > 1
                                 and bpm.STAGE_MAX_S[k] <= 64}
    ga.close()
    tab = {}
    for d in (5, 7, 9, 11, 15):
        for k in range(1, 10):
            p = 0.02 * k
            g = bpm.Graph("code_capacity", d, p)
            syn, obs = g.sample(seed_for(2, d, p), 0, n)
            g.decode(syn, obs, min(n, 4096), 25, precision=bpm.BPM_FP32)     # kernel loading
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = g.decode(syn, obs, n, 25, precision=bpm.BPM_FP32)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c = bpm.counters_dict(r["counters"])
            tab["d%d_p%.2f" % (d, p)] = {"ler": c["failures"] / n, "mean_s": c["sum_s"] / n,
                                         "shots_per_s": n / dt}
            g.close()
        print("capacity sweep: d=%d done" % d, file=sys.stderr, flush=True)
    out["points"] = tab
    return out


def runtime_table(bpm, n):
    """Decode time per 10^6 shots on the workloads of the paper's only timing
    (its runtime figure): unrotated surface code, code-capacity depolarizing
    noise (the Z part), T = 25, p in {0.03, 0.06}, d = 3 ... 11, BP4M and
    BP4MF, FP32, syndromes resident on the GPU; one decode call of n shots per
    point, its small-class kernel configurations first timed on d = 11,
    p = 0.06."""
    import torch
    out = {"workload": "unrotated surface code, code capacity (Z part), T=25, FP32, %d shots per call" % n}
    ga = bpm.Graph("code_capacity_unrotated", 11, 0.06)
    opts = bpm.bpm_decode_opts(25, bpm.BPM_BP4M, bpm.BPM_FP32, 0, 1.0)
    bpm.bpm_autotune(ga.handle, opts, min(n, 1_000_000), 0x5E11, torch.cuda.current_stream().cuda_stream)
    ga.close()
    for vname, variant in (("bp4m", bpm.BPM_BP4M), ("bp4mf", bpm.BPM_BP4MF)):
        tab = {}
        for p in (0.03, 0.06):
            for d in (3, 5, 7, 9, 11):
                g = bpm.Graph("code_capacity_unrotated", d, p)
                syn, obs = g.sample(seed_for(5, d, p), 0, n)
                g.decode(syn, obs, min(n, 4096), 25, precision=bpm.BPM_FP32, variant=variant)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = g.decode(syn, obs, n, 25, precision=bpm.BPM_FP32, variant=variant)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                c = bpm.counters_dict(r["counters"])
                tab["d%d_p%.2f" % (d, p)] = {"s_per_1e6_shots": dt * 1e6 / n, "shots_per_s": n / dt,
                                             "ler": c["failures"] / n, "mean_s": c["sum_s"] / n}
                g.close()
        out[vname] = tab
        print("runtime table: %s done" % vname, file=sys.stderr, flush=True)
    return out


def memory_sweep(bpm, n):
    """The rotated memory-Z grid: d in {5, 7, 9, 11, 13} with d rounds, p =
    0.002 ... 0.012, BP4M T = 50, FP32, one decode call per (d, p) on n
    sampled shots: logical error rate, never-converged rate, mean defects per
    shot and decode rate."""
    import torch
    out = {"workload": "rotated memory-Z, d rounds, BP4M T=50, FP32, %d shots per point" % n}
    tab = {}
    for d in (5, 7, 9, 11, 13):
        for k in range(2, 13):
            p = 0.001 * k
            g = bpm.Graph("memory_z", d, p, d)
            syn, obs = g.sample(seed_for(3, d, p), 0, n)
            g.decode(syn, obs, min(n, 4096), 50, precision=bpm.BPM_FP32)     # kernel loading
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = g.decode(syn, obs, n, 50, precision=bpm.BPM_FP32)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c = bpm.counters_dict(r["counters"])
            tab["d%d_p%.3f" % (d, p)] = {"ler": c["failures"] / n, "r_nc": c["never_converged"] / n,
                                         "mean_s": c["sum_s"] / n, "overflow": c["overflow"], "shots_per_s": n / dt}
            g.close()
        print("memory sweep: d=%d done" % d, file=sys.stderr, flush=True)
    out["points"] = tab
    return out


def circuit_sweep(bpm, n):
    """Logical error rates of memory-Z experiments (d rounds) on the unrotated
    and the rotated code, T = 50, FP32, BP4M and BP4MF: the circuit-level
    counterpart of threshold_sweep."""
    import torch
    out = {"workload": "memory-Z, d rounds, T=50, FP32, %d shots per point" % n}
    for kind in ("memory_z_unrotated", "memory_z"):
        for vname, variant in (("bp4m", bpm.BPM_BP4M), ("bp4mf", bpm.BPM_BP4MF)):
            tab = {}
            for d in (5, 9, 13):
                for p in (0.004, 0.0045, 0.005, 0.0055, 0.006, 0.0065, 0.007):
                    g = bpm.Graph(kind, d, p, d)
                    syn, obs = g.sample(seed_for(6, d, p), 0, n)
                    r = g.decode(syn, obs, n, 50, precision=bpm.BPM_FP32, variant=variant)
                    torch.cuda.synchronize()
                    c = bpm.counters_dict(r["counters"])
                    tab["d%d_p%.4f" % (d, p)] = {"ler": c["failures"] / n, "r_nc": c["never_converged"] / n,
                                                 "overflow": c["overflow"]}
                    g.close()
                print("circuit sweep: %s %s d=%d done" % (kind, vname, d), file=sys.stderr, flush=True)
            out["%s_%s" % (kind, vname)] = tab
    return out


def alpha_sweep(bpm, n):
    """Memory-BP4MF (Sec. III.E, "BP Improvements"): the paper's grid
    alpha = 0.6 + 0.05 k, k = 0..20, for BP4MF on the rotated memory-Z
    circuit (d rounds, T = 50, FP32) at d in {5, 9, 13} and p in {0.004,
    0.005, 0.006}; the same n sampled shots for every alpha of a (d, p)
    point, so differences between alphas are paired.  Logical error rate,
    95% Wilson interval and never-converged rate per point, and the alpha of
    the lowest rate per (d, p)."""
    import torch
    alphas = [round(0.6 + 0.05 * k, 2) for k in range(21)]
    out = {"workload": "rotated memory-Z, d rounds, BP4MF T=50, FP32, %d shots per point" % n, "alphas": alphas}
    tab = {}
    for d in (5, 9, 13):
        for p in (0.004, 0.005, 0.006):
            g = bpm.Graph("memory_z", d, p, d)
            syn, obs = g.sample(seed_for(8, d, p), 0, n)
            row = {}
            for a in alphas:
                r = g.decode(syn, obs, n, 50, precision=bpm.BPM_FP32, variant=bpm.BPM_BP4MF, alpha=a)
                torch.cuda.synchronize()
                c = bpm.counters_dict(r["counters"])
                row["%.2f" % a] = {"ler": c["failures"] / n, "wilson95": wilson(c["failures"], n),
                                   "r_nc": c["never_converged"] / n, "overflow": c["overflow"]}
            best = min(row, key=lambda k: row[k]["ler"])
            tab["d%d_p%.3f" % (d, p)] = {"by_alpha": row, "best_alpha": float(best),
                                         "ler_alpha1": row["1.00"]["ler"], "ler_best": row[best]["ler"]}
            g.close()
        print("alpha sweep: d=%d done" % d, file=sys.stderr, flush=True)
    out["points"] = tab
    return out


def fig4_sweep(bpm, n, kind="memory_z", variant_name="BP4MF",
               golden="paper_circuit_bp4mf_rotated.txt"):
    """One printed panel of the paper's circuit-level threshold figure: T = 50,
    FP32, memory-Z with d rounds, d in {3, 5, 7, 9, 11}, p = 0.002 ... 0.012;
    logical error rate with its 95% Wilson interval next to the printed value
    (tests/golden/<golden>, whose d labels are an inference).  The rotated
    BP4MF panel by default; the unrotated BP4M panel with
    kind="memory_z_unrotated", variant_name="BP4M",
    golden="paper_circuit_bp4m_unrotated.txt"."""
    import torch
    variant = {"BP4M": bpm.BPM_BP4M, "BP4MF": bpm.BPM_BP4MF}[variant_name]
    paper = {}
    for ln in open(os.path.join(ROOT, "tests", "golden", golden)):
        if ln.startswith("#") or not ln.strip():
            continue
        d, p, v = ln.split()
        paper[(int(d), round(float(p), 3))] = float(v)
    code = "unrotated" if kind.endswith("_unrotated") else "rotated"
    out = {"workload": "%s memory-Z, d rounds, %s T=50, FP32, %d shots per point" % (code, variant_name, n)}
    tab = {}
    for d in (3, 5, 7, 9, 11):
        for k in range(2, 13):
            p = round(0.001 * k, 3)
            g = bpm.Graph(kind, d, p, d)
            syn, obs = g.sample(seed_for(10, d, p), 0, n)
            r = g.decode(syn, obs, n, 50, precision=bpm.BPM_FP32, variant=variant)
            torch.cuda.synchronize()
            c = bpm.counters_dict(r["counters"])
            tab["d%d_p%.3f" % (d, p)] = {"ler": c["failures"] / n, "wilson95": wilson(c["failures"], n),
                                         "paper": paper.get((d, p)), "overflow": c["overflow"]}
            g.close()
        print("fig4 sweep (%s %s): d=%d done" % (code, variant_name, d), file=sys.stderr, flush=True)
    out["points"] = tab
    return out


def bbp4mf_bench(bpm, n):
    """B-BP4MF (quaternary BP, then BP4MF on re-weighted paths; FP64 fixed
    order) on the unrotated code under depolarizing code-capacity noise, the
    paper's B-BP4MF configuration (T = 25 + 25): logical error rates over a
    (d, p) grid next to BP4MF on the same X syndromes, and the decode rate."""
    import torch
    out = {"workload": "unrotated surface code, depolarizing code capacity, T=25+25, FP64, %d shots per point" % n}
    tab = {}
    for d in (5, 9, 13):
        for p in (0.13, 0.14, 0.15, 0.16):
            g = bpm.Graph("code_capacity_unrotated", d, p)
            sx, sz, ob = g.sample_depolarizing(seed_for(9, d, p), 0, n)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = g.decode_bbp4mf(sx, sz, ob, n, 25)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            r2 = g.decode(sx, ob, n, 25, precision=bpm.BPM_FP32, variant=bpm.BPM_BP4MF)
            torch.cuda.synchronize()
            c, c2 = bpm.counters_dict(r["counters"]), bpm.counters_dict(r2["counters"])
            fl = r["flags"].cpu().numpy()[:n]
            tab["d%d_p%.2f" % (d, p)] = {"ler_bbp4mf": c["failures"] / n, "ler_bp4mf": c2["failures"] / n,
                                         "stage1_frac": float(((fl & bpm.SHOT_QBP_CONVERGED) != 0).mean()),
                                         "shots_per_s": n / dt}
            g.close()
        print("bbp4mf: d=%d done" % d, file=sys.stderr, flush=True)
    out["points"] = tab
    return out


def ler_reference(bpm, g, syn, obs, n, T, m):
    """The headline's LER reference: the first m shots of the last timed step
    (still in the syndrome buffers) decoded again in FP32 and in the FP64
    fixed-order mode (bit-exact against the oracle in the tests), logical
    error rates with 95% Wilson intervals and the shots on which the two
    modes' predictions differ."""
    import numpy as np
    import torch
    m = min(m, n)
    Wm = (m + 63) // 64
    sub_syn, sub_obs = syn[:, :Wm].contiguous(), obs[:Wm].contiguous()
    fails = {}
    for name, prec in (("fp32", bpm.BPM_FP32), ("fp64_spec", bpm.BPM_FP64_SPEC)):
        r = g.decode(sub_syn, sub_obs, m, T, precision=prec)
        torch.cuda.synchronize()
        fails[name] = np.unpackbits(r["fail"][:Wm].cpu().numpy().view(np.uint8), bitorder="little")[:m].astype(bool)
    out = {"shots": m}
    for name, f in fails.items():
        out[name] = {"ler": float(f.mean()), "wilson95": wilson(int(f.sum()), m)}
    out["fp32"]["disagreements"] = int((fails["fp32"] != fails["fp64_spec"]).sum())
    return out


def wilson(k, n, z=1.96):
    """95% Wilson score interval of a binomial proportion k / n."""
    if n <= 0:
        return [0.0, 1.0]
    ph = k / n
    den = 1.0 + z * z / n
    c = (ph + z * z / (2 * n)) / den
    h = z * ((ph * (1 - ph) / n + z * z / (4.0 * n * n)) ** 0.5) / den
    return [max(0.0, c - h), min(1.0, c + h)]


def batched_bench(bpm, args, T):
    """Several distances in one call: memory-Z, d rounds, p = 0.005, n shots
    per distance.  BF16 and FP16 message storage (FP32 arithmetic): one
    bpm_decode_multi call vs one bpm_decode call per distance on the same
    shots, shots/s.  Logical error rates per distance with 95% Wilson
    intervals for BF16, FP16 and FP32 on all n shots, and for the FP64
    fixed-order mode (the reference the FP32 and 16-bit modes are held
    against; bit-exact against the oracle in the tests) on the first
    args.batched_spec_shots shots of each distance, with the 16-bit and FP32
    rates on that same subset beside it."""
    import numpy as np
    import torch
    ds = [int(x) for x in args.batched_distances.split(",")]
    n = args.batched_shots
    W = (n + 63) // 64
    stream = torch.cuda.current_stream()
    parts = []
    for d in ds:
        g = bpm.Graph("memory_z", d, 0.005, d)
        syn, obs = g.sample(seed_for(3, d, 0.005), 0, n)
        parts.append((g, syn, obs, n))
    out = {"workload": "memory-Z p=0.005, d in %s (d rounds), %d shots each, BP4M T=%d" % (ds, n, T)}
    fails = {}
    for name, prec in (("bf16", bpm.BPM_BF16_STORE), ("fp16", bpm.BPM_FP16_STORE), ("fp32", bpm.BPM_FP32)):
        opts = bpm.bpm_decode_opts(T, bpm.BPM_BP4M, prec, 0, 1.0)
        if not args.no_autotune:
            bpm.bpm_autotune(parts[-2][0].handle, opts, min(n, 100_000), 77, stream.cuda_stream)
        bpm.decode_multi(parts, T, precision=prec)          # warm-up (kernels, allocator)
        for g, syn, obs, k in parts:
            g.decode(syn, obs, k, T, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = bpm.decode_multi(parts, T, precision=prec)
        torch.cuda.synchronize()
        t_multi = time.perf_counter() - t0
        t0 = time.perf_counter()
        sep = [g.decode(syn, obs, k, T, precision=prec) for g, syn, obs, k in parts]
        torch.cuda.synchronize()
        t_sep = time.perf_counter() - t0
        ler, ovf = {}, {}
        fails[name] = {}
        for (g, syn, obs, k), r, r2 in zip(parts, res, sep):
            c = bpm.counters_dict(r["counters"])
            assert torch.equal(r["fail"][:W], r2["fail"][:W])
            fb = np.unpackbits(r["fail"][:W].cpu().numpy().view(np.uint8), bitorder="little")[:n].astype(bool)
            fails[name][g.d] = fb
            ler["d%d" % g.d] = {"ler": c["failures"] / max(c["shots"], 1),
                                "wilson95": wilson(c["failures"], c["shots"])}
            ovf["d%d" % g.d] = c["overflow"]
        out[name] = {"one_call_shots_per_s": len(ds) * n / t_multi, "separate_calls_shots_per_s": len(ds) * n / t_sep,
                     "ler": ler, "overflow": ovf}
    m = min(n, args.batched_spec_shots)
    if m > 0:
        Wm = (m + 63) // 64
        # the first m shots as planes of their own width (ceil(m / 64) words)
        sub = [(g, syn[:, :Wm].contiguous(), obs[:Wm].contiguous(), m) for g, syn, obs, k in parts]
        t0 = time.perf_counter()
        res = bpm.decode_multi(sub, T, precision=bpm.BPM_FP64_SPEC)
        torch.cuda.synchronize()
        t_spec = time.perf_counter() - t0
        ref = {"shots_per_distance": m, "shots_per_s": len(ds) * m / t_spec, "ler": {}}
        for (g, syn, obs, k), r in zip(sub, res):
            fb = np.unpackbits(r["fail"][:Wm].cpu().numpy().view(np.uint8), bitorder="little")[:m].astype(bool)
            kf = int(fb.sum())
            row = {"fp64_spec": {"ler": kf / m, "wilson95": wilson(kf, m)}}
            for name in fails:
                f2 = fails[name][g.d][:m]
                row[name] = {"ler": float(f2.mean()), "wilson95": wilson(int(f2.sum()), m),
                             "paired_disagreements": int((f2 != fb).sum())}
            ref["ler"]["d%d" % g.d] = row
        out["reference_subset"] = ref
    return out


def _pct(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def serving_bench(bpm, args, T):
    """Requests of 1..64 shots (uniform), graphs of distance d uniform over
    the given set (memory-Z, d rounds, p = 0.005), Poisson arrivals at 0.5,
    0.8 and 0.95 of the measured saturated request rate; latency percentiles
    from the server's clock (submit to result).  Compared with the plain
    path: one request at a time, copied in, decoded alone, copied out."""
    import numpy as np
    import torch
    ds = [int(x) for x in args.serve_distances.split(",")]
    pool_n = 8192
    P = []
    for d in ds:
        g = bpm.Graph("memory_z", d, 0.005, d)
        syn, obs = g.sample(seed_for(4, d, 0.005), 0, pool_n)
        P.append((g, bpm.planes_to_rows(syn, pool_n, g.n_det)))
    rng = np.random.default_rng(20260305)

    def request(i):
        gi = int(rng.integers(len(ds)))
        k = int(rng.integers(1, 65))
        a = int(rng.integers(0, pool_n - k))
        return gi, P[gi][1][a:a + k]

    srv = bpm.Server([p[0] for p in P], T, max_batch_shots=args.serve_batch, max_pending_shots=1 << 18,
                     slots=args.serve_slots, use_graphs=bool(args.serve_graphs),
                     one_graph_per_batch=args.serve_one_graph,
                     mem_budget=args.serve_mem_budget << 20)
    out = {"workload": "memory-Z p=0.005, d uniform over %s (d rounds), 1-64 shots per request, BP4M T=%d FP32"
                       % (ds, T), "slots": args.serve_slots, "max_batch_shots": args.serve_batch,
           "one_graph_per_batch": bool(args.serve_one_graph), "mem_budget_mib": args.serve_mem_budget,
           "hip_graphs": bool(args.serve_graphs)}
    try:
        # warm-up (kernel loading), then the saturated rate: a closed loop
        # that keeps the admission queue full
        for i in range(200):
            gi, rows = request(i)
            while not srv.submit(gi, rows, i):
                srv.poll()
        t_end = time.time() + 30
        done = 0
        while done < 200 and time.time() < t_end:
            done += len(srv.poll())
        n_sat, shots_sat, done, rid = 0, 0, 0, 10_000
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.serve_seconds:
            gi, rows = request(rid)
            if srv.submit(gi, rows, rid):
                rid += 1
                n_sat += 1
                shots_sat += rows.shape[0]
            done += len(srv.poll())
        while done < n_sat:
            done += len(srv.poll())
        t_sat = time.perf_counter() - t0
        sat = n_sat / t_sat
        out["saturated"] = {"requests_per_s": sat, "shots_per_s": shots_sat / t_sat}
        levels = {}
        for frac in (0.5, 0.8, 0.95):
            rate = frac * sat
            n_req = args.serve_requests if args.serve_requests > 0 else max(200, int(rate * args.serve_seconds))
            gaps = rng.exponential(1.0 / rate, n_req)
            due = np.cumsum(gaps)
            reqs = [request(i) for i in range(n_req)]
            lat, shots = [], 0
            lat_g = [[] for _ in ds]                 # per graph (distance)
            t0 = time.perf_counter()
            i = 0
            while i < n_req or len(lat) < n_req:
                now = time.perf_counter() - t0
                while i < n_req and due[i] <= now:
                    gi, rows = reqs[i]
                    if not srv.submit(gi, rows, 1_000_000 + i):
                        break
                    shots += rows.shape[0]
                    i += 1
                for r in srv.poll():
                    lat.append(r[6])
                    lat_g[r[1]].append(r[6])
            wall = time.perf_counter() - t0
            print("serving: load %.2f done (%d requests)" % (frac, n_req), file=sys.stderr, flush=True)
            levels["%.2f" % frac] = {"offered_requests_per_s": rate, "requests": n_req,
                                     "requests_per_s": n_req / wall, "shots_per_s": shots / wall,
                                     "p50_us": _pct(lat, 50), "p99_us": _pct(lat, 99), "p999_us": _pct(lat, 99.9),
                                     "by_distance": {"d%d" % ds[gi]: {"p50_us": _pct(lat_g[gi], 50),
                                                                      "p99_us": _pct(lat_g[gi], 99)}
                                                     for gi in range(len(ds)) if lat_g[gi]}}
        out["poisson"] = levels
        out["server_stats"] = srv.stats()
    finally:
        srv.close()
    # plain path: each request alone, synchronously (copy in, decode, copy out)
    stream = torch.cuda.current_stream()
    opts = bpm.bpm_decode_opts(T, bpm.BPM_BP4M, bpm.BPM_FP32, 0, 1.0)
    lat = []
    n_plain = args.serve_plain_requests
    dev_rows = [torch.empty((64, p[1].shape[1]), dtype=torch.int64, device="cuda") for p in P]
    flags = torch.empty(64, dtype=torch.uint8, device="cuda")
    host_flags = torch.empty(64, dtype=torch.uint8).pin_memory()
    pinned = [torch.empty((64, p[1].shape[1]), dtype=torch.int64).pin_memory() for p in P]
    ws = {}
    t0 = time.perf_counter()
    for i in range(n_plain):
        gi, rows = request(i)
        k = rows.shape[0]
        ts = time.perf_counter()
        pinned[gi][:k].numpy()[:] = rows.view(np.int64)
        dev_rows[gi][:k].copy_(pinned[gi][:k], non_blocking=True)
        it = bpm.bpm_decode_item()
        it.graph, it.syn, it.obs, it.n_shots, it.rows_words = (P[gi][0].handle, dev_rows[gi].data_ptr(), None, k,
                                                              dev_rows[gi].shape[1])
        it.out.shot_flags = flags.data_ptr()
        if gi not in ws:
            it.n_shots = 64                      # room for the largest request
            nb = bpm.bpm_decode_multi_workspace_size([it], opts)
            it.n_shots = k
            ws[gi] = (torch.empty(nb + 256, dtype=torch.uint8, device="cuda"), nb)
        buf, nb = ws[gi]
        bpm.bpm_decode_multi([it], opts, None, (buf.data_ptr() + 255) & ~255, nb, stream.cuda_stream)
        host_flags[:k].copy_(flags[:k], non_blocking=True)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ts) * 1e6)
    wall = time.perf_counter() - t0
    out["plain"] = {"requests": n_plain, "requests_per_s": n_plain / wall, "p50_us": _pct(lat, 50),
                    "p99_us": _pct(lat, 99), "p999_us": _pct(lat, 99.9)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--shots", type=int, default=1_000_000)
    ap.add_argument("--d", type=int, default=13)
    ap.add_argument("--p", type=float, default=0.005)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default kernel configuration of every stage")
    ap.add_argument("--autotune-shots", type=int, default=200_000)
    ap.add_argument("--serve-requests", type=int, default=0,
                    help="requests per load level in the serving measurement (0 = --serve-seconds of arrivals)")
    ap.add_argument("--serve-plain-requests", type=int, default=2000,
                    help="requests decoded one at a time on the plain path")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="seconds of Poisson arrivals per load level in the serving measurement (0 = skip)")
    ap.add_argument("--serve-distances", type=str, default="5,9,13,17")
    ap.add_argument("--serve-slots", type=int, default=3, help="server: batches in flight at once (1..8)")
    ap.add_argument("--serve-batch", type=int, default=4096,
                    help="server: most shots of one graph in a batch (a multiple of 64)")
    ap.add_argument("--serve-mem-budget", type=int, default=4096, metavar="MIB",
                    help="server: device-memory admission budget in MiB (slots plus queued shots; 0 = none)")
    ap.add_argument("--serve-graphs", type=int, default=0,
                    help="server: 1 = replay each batch's launch sequence as a captured HIP graph "
                         "(shot counts padded to 64*4^k)")
    ap.add_argument("--serve-one-graph", type=int, default=1,
                    help="server: 1 = each batch takes one graph's requests (that of the oldest request)")
    ap.add_argument("--threshold-sweep", type=int, default=0, metavar="SHOTS",
                    help="also decode SHOTS shots per point of a code-capacity sweep of the unrotated code "
                         "(d in 5,9,13; p in 0.10..0.15; BP4M and BP4MF, T=25) and report the logical error rates")
    ap.add_argument("--capacity-sweep", type=int, default=0, metavar="SHOTS",
                    help="also decode SHOTS shots per point of the rotated code-capacity grid "
                         "(d in 5..15, p in 0.02..0.18)")
    ap.add_argument("--runtime-table", type=int, default=0, metavar="SHOTS",
                    help="also time SHOTS-shot decodes on the workloads of the paper's runtime figure "
                         "(unrotated code capacity, T=25, p in 0.03/0.06, d in 3..11, BP4M and BP4MF)")
    ap.add_argument("--memory-sweep", type=int, default=0, metavar="SHOTS",
                    help="also decode SHOTS shots per point of the rotated memory-Z grid "
                         "(d in 5..13, d rounds, p in 0.002..0.012)")
    ap.add_argument("--circuit-sweep", type=int, default=0, metavar="SHOTS",
                    help="diagnostic: memory-Z logical error rates, unrotated and rotated code (0 = skip)")
    ap.add_argument("--fig4-sweep", type=int, default=0, metavar="SHOTS",
                    help="also run BP4MF on rotated memory-Z at the paper's printed circuit-level points "
                         "(d in 3..11, p in 0.002..0.012), SHOTS shots per point (0 = skip)")
    ap.add_argument("--fig4-unrotated-sweep", type=int, default=0, metavar="SHOTS",
                    help="also run BP4M on unrotated memory-Z at the paper's printed circuit-level points "
                         "(d in 3..11, p in 0.002..0.012), SHOTS shots per point (0 = skip)")
    ap.add_argument("--alpha-sweep", type=int, default=0, metavar="SHOTS",
                    help="also run the memory-factor grid alpha = 0.6..1.6 for BP4MF on memory-Z "
                         "(d in 5, 9, 13; p in 0.004..0.006), SHOTS shots per point (0 = skip)")
    ap.add_argument("--bbp4mf-shots", type=int, default=10_000, metavar="SHOTS",
                    help="B-BP4MF code-capacity sweep and rate, SHOTS per point (0 = skip)")
    ap.add_argument("--batched-shots", type=int, default=100_000,
                    help="shots per distance in the mixed-distance batched measurement (0 = skip)")
    ap.add_argument("--batched-distances", type=str, default="7,11,15,21")
    ap.add_argument("--ler-ref-shots", type=int, default=20_000,
                    help="shots of the last timed step also decoded in FP64 fixed order, the headline's LER "
                         "reference (0 = skip)")
    ap.add_argument("--batched-spec-shots", type=int, default=20_000,
                    help="shots per distance of the mixed batch also decoded in FP64 fixed order (0 = skip)")
    ap.add_argument("--storage-shots", type=int, default=1_000_000,
                    help="shots of the same workload decoded once with BF16 and once with FP16 "
                         "message storage after the timed region (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--class-streams", type=int, default=0,
                    help="run the size-class kernels concurrently on this many streams (0/1 = one stream)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="before the steps, copy MIB MiB device to device once (a plain copy kernel "
                         "of known size, to calibrate HBM byte counters in the same profiled run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(shots are independent and shard across GPUs trivially). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2603_05381_amd as bpm

    d, rounds, p, T, n = args.d, args.d, args.p, args.iters, args.shots
    seed = seed_for(2, d, p)
    g = bpm.Graph("memory_z", d, p, rounds)
    N = g.n_det
    W = (n + 63) // 64
    stream = torch.cuda.current_stream()
    syn = torch.empty((N, W), dtype=torch.int64, device="cuda")
    obs = torch.empty(W, dtype=torch.int64, device="cuda")
    opts = bpm.bpm_decode_opts(T, bpm.BPM_BP4M, bpm.BPM_FP32, 0, 1.0, args.class_streams)
    ws_bytes = bpm.bpm_decode_workspace_size(g.handle, n, opts)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
    ws_ptr = (ws.data_ptr() + 255) & ~255
    obs_pred = torch.empty(W, dtype=torch.int64, device="cuda")
    fail = torch.empty(W, dtype=torch.int64, device="cuda")
    counters = torch.zeros(6, dtype=torch.int64, device="cuda")
    K, Wm = args.steps, args.warmup
    s_out = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(K)]
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(2 * len(bpm.STAGES))] for _ in range(K)]
    for evs in events:
        for ev in evs:
            ev.record(stream)

    def step(i, evs=None, s_t=None):
        bpm.bpm_sample(g.handle, seed, i * n, n, syn.data_ptr(), obs.data_ptr(), None, stream.cuda_stream)
        out = bpm.bpm_decode_out()
        out.obs_pred = obs_pred.data_ptr()
        out.fail = fail.data_ptr()
        out.counters = counters.data_ptr()
        if s_t is not None:
            out.shot_s = s_t.data_ptr()
        if evs is not None:
            for k, ev in enumerate(evs):
                out.stage_events[k] = ev.cuda_event
        bpm.bpm_decode(g.handle, syn.data_ptr(), obs.data_ptr(), n, opts, out, ws_ptr, ws_bytes,
                       stream.cuda_stream)

    tuned = None
    if not args.no_autotune:
        # setup, before the timed region: time each kernel configuration of
        # every size class on shots of the same workload (other seed)
        t_ms = bpm.bpm_autotune(g.handle, opts, args.autotune_shots, seed ^ 0x5A5A, stream.cuda_stream)
        cfg = bpm.bpm_get_stage_config()
        tuned = {bpm.STAGES[k]: {"config": cfg[k], "ms": [round(t_ms[c][k], 3) for c in range(bpm.BPM_MAX_CONFIGS)
                                                           if t_ms[c][k] >= 0]}
                 for k in range(len(bpm.STAGES)) if bpm.bpm_stage_configs(k) > 1}
    if args.copy_probe > 0:
        nf = (args.copy_probe << 20) // 4
        src = torch.ones(nf, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)                  # reads and writes MIB MiB
        torch.cuda.synchronize()
        del src, dst
    for i in range(Wm):
        step(i)
    torch.cuda.synchronize()
    counters.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        step(Wm + i, events[i], s_out[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # stage times (ms, mean over steps) and per-class message-update counts
    n_st = len(bpm.STAGES)
    stage_ms = np.zeros(n_st)
    for evs in events:
        for k in range(n_st):
            stage_ms[k] += evs[2 * k].elapsed_time(evs[2 * k + 1]) / K
    tops = bpm.STAGE_MAX_S[1:-1]                 # largest s of each message-passing stage
    bounds = [(lo + 1 if c else 2, hi) for c, (lo, hi) in enumerate(zip([0] + tops[:-1], tops))]
    msgs = np.zeros(len(bounds))
    shots_in = np.zeros(len(bounds))
    for s_t in s_out:
        s = s_t.cpu().numpy().astype(np.int64)
        for c, (lo, hi) in enumerate(bounds):
            sel = s[(s >= lo) & (s <= hi)]
            msgs[c] += float(T * (sel * sel).sum()) / K
            shots_in[c] += sel.size / K
    c = bpm.counters_dict(counters)
    bp = stage_ms[1:n_st - 1]                    # message-passing stages
    dom = int(np.argmax(bp))                     # dominant message-passing kernel
    t_dom = bp[dom] / 1e3
    achieved = msgs[dom] * OPS_PER_MSG / t_dom / 1e12 if t_dom > 0 else 0.0
    total_bp_s = bp.sum() / 1e3
    all_tflops = msgs.sum() * OPS_PER_MSG / total_bp_s / 1e12 if total_bp_s else 0.0
    value = K * n / elapsed
    line = {
        "metric": "decoded shots/s (circuit-level d=13, d rounds) at fixed LER; p50/p99 latency",
        "value": value,
        "unit": "shots/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: shots sampled on the GPU from the project's own memory-Z circuit model",
        "config": {
            "workload": "rotated surface code memory-Z, circuit-level depolarizing p=%g, d=%d, %d rounds, "
                        "BP4M T=%d, FP32 messages, %d shots per step" % (p, d, rounds, T, n),
            "shots_per_step": n, "d": d, "rounds": rounds, "p": p, "max_iters": T,
            "n_det": N, "n_mech": g.info.n_mech, "seed": seed, "class_streams": args.class_streams,
        },
        "roofline": {
            "bound": "alu",
            "kernel": bpm.STAGES[1 + dom],
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": recorded_traffic(bpm.STAGES[1 + dom], n),
            "work_per_unit": "%d FP32 ops (2 of them exp2/log2) per message update" % OPS_PER_MSG,
            "units_per_launch": msgs[dom],
            "kernel_ms": stage_ms[1 + dom],
            "issue_model": {
                "peak_updates_per_s": PEAK_MSG_PER_S,
                "slots_per_update": SLOTS_PER_MSG,
                "frac": msgs[dom] / t_dom / PEAK_MSG_PER_S if t_dom > 0 else 0.0,
            },
            "all_message_passing": {"achieved": all_tflops, "frac": all_tflops / PEAK_FP32_TFLOPS,
                                    "issue_model_frac": float(msgs.sum() / total_bp_s / PEAK_MSG_PER_S)
                                    if total_bp_s else 0.0},
        },
        "stages_ms": {bpm.STAGES[k]: round(float(stage_ms[k]), 4) for k in range(n_st)},
        "stage_shots": {bpm.STAGES[1 + c]: float(shots_in[c]) for c in range(len(bounds))},
        "stage_updates": {bpm.STAGES[1 + c]: float(msgs[c]) for c in range(len(bounds))},
        "autotune": tuned,
        "ler": c["failures"] / max(c["shots"], 1),
        "r_nc": c["never_converged"] / max(c["shots"], 1),
        "mean_s": c["sum_s"] / max(c["shots"], 1),
        "overflow": c["overflow"],
    }
    if c["overflow"]:
        print("bench.py: %d shots exceeded s_cap and were counted as failures" % c["overflow"], file=sys.stderr)
    if args.ler_ref_shots > 0:
        line["ler_reference"] = ler_reference(bpm, g, syn, obs, n, T, args.ler_ref_shots)
    if args.storage_shots > 0:
        line["storage"] = storage_variants(bpm, g, syn, obs, stream, seed, args, T, c)
    if args.threshold_sweep > 0:
        line["threshold_sweep"] = threshold_sweep(bpm, args.threshold_sweep)
    if args.circuit_sweep > 0:
        line["circuit_sweep"] = circuit_sweep(bpm, args.circuit_sweep)
    if args.capacity_sweep > 0:
        line["capacity_sweep"] = capacity_sweep(bpm, args.capacity_sweep)
    if args.memory_sweep > 0:
        line["memory_sweep"] = memory_sweep(bpm, args.memory_sweep)
    if args.runtime_table > 0:
        line["runtime_table"] = runtime_table(bpm, args.runtime_table)
    if args.fig4_sweep > 0:
        line["fig4_sweep"] = fig4_sweep(bpm, args.fig4_sweep)
    if args.fig4_unrotated_sweep > 0:
        line["fig4_unrotated_sweep"] = fig4_sweep(bpm, args.fig4_unrotated_sweep, "memory_z_unrotated", "BP4M",
                                                  "paper_circuit_bp4m_unrotated.txt")
    if args.alpha_sweep > 0:
        line["alpha_sweep"] = alpha_sweep(bpm, args.alpha_sweep)
    if args.bbp4mf_shots > 0:
        line["bbp4mf"] = bbp4mf_bench(bpm, args.bbp4mf_shots)
    if args.batched_shots > 0:
        line["batched"] = batched_bench(bpm, args, T)
    if args.serve_seconds > 0:
        line["serving"] = serving_bench(bpm, args, T)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(d, rounds, p, T, seed, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
