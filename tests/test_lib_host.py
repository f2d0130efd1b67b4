"""CPU tests of libbpm's host side: it loads, exports every entry point that
include/bpm.h declares, rejects bad arguments, and builds detector graphs and
path tables identical, bit for bit, to the oracle's.

The library builds the memory-Z model by propagating detectors backward
through the circuit and its tables with its own Dijkstra; the oracle
propagates faults forward and uses a different search, so agreement pins
both.  No GPU is needed: without a device the library keeps host tables.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2603_05381_amd as bpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bpm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bpm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "bpm_decode" in names and "bpm_sample" in names and "bpm_build_graph" in names
    lib = bpm.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(bpm.EXPORTS) == names


def test_bad_arguments_are_rejected():
    for args in [(4, 1, bpm.BPM_CODE_CAPACITY_DEPOL, 0.1), (3, 1, bpm.BPM_CODE_CAPACITY_DEPOL, 0.0),
                 (5, 0, bpm.BPM_CIRCUIT_MEMORY_Z, 0.01), (5, 5, bpm.BPM_CIRCUIT_MEMORY_Z, 0.7),
                 (5, 5, 7, 0.01)]:
        d, r, kind, p = args
        with pytest.raises(bpm.BpmError):
            bpm.bpm_build_graph(bpm.BPM_ROTATED_SURFACE, d, r, kind, p)
    with pytest.raises(bpm.BpmError, match="rounds"):
        bpm.bpm_build_graph(bpm.BPM_UNROTATED_SURFACE, 3, 0, bpm.BPM_CIRCUIT_MEMORY_Z, 0.01)
    with pytest.raises(bpm.BpmError, match="unknown code"):
        bpm.bpm_build_graph(7, 3, 1, bpm.BPM_CODE_CAPACITY_DEPOL, 0.1)
    g = bpm.Graph("code_capacity", 3, 0.05)
    for opts in [bpm.bpm_decode_opts(0, 0, 1, 0, 1.0), bpm.bpm_decode_opts(5, 3, 1, 0, 1.0),
                 bpm.bpm_decode_opts(5, 0, 9, 0, 1.0), bpm.bpm_decode_opts(5, 0, 1, 0, -1.0),
                 bpm.bpm_decode_opts(5, 0, 1, 5000, 1.0), bpm.bpm_decode_opts(5, 0, 1, 0, 1.0, 9)]:
        with pytest.raises(bpm.BpmError):
            bpm.bpm_decode_workspace_size(g.handle, 100, opts)
    assert bpm.bpm_decode_workspace_size(g.handle, 100, bpm.bpm_decode_opts(5, 0, 1, 0, 1.0)) > 0


CASES = [("code_capacity", 3, 1, 0.05), ("code_capacity", 5, 1, 0.1), ("code_capacity", 9, 1, 0.17),
         ("code_capacity_unrotated", 2, 1, 0.1), ("code_capacity_unrotated", 5, 1, 0.1),
         ("code_capacity_unrotated", 11, 1, 0.12),
         ("memory_z", 3, 3, 0.01), ("memory_z", 5, 5, 0.005), ("memory_z", 7, 3, 0.002),
         ("memory_z", 9, 9, 0.008),
         ("memory_z_unrotated", 2, 2, 0.01), ("memory_z_unrotated", 3, 3, 0.01),
         ("memory_z_unrotated", 5, 5, 0.005), ("memory_z_unrotated", 7, 4, 0.003)]


@pytest.mark.parametrize("kind,d,rounds,p", CASES)
def test_graph_and_tables_match_oracle_bitwise(kind, d, rounds, p):
    g = bpm.Graph(kind, d, p, rounds)
    if kind.startswith("memory_z"):
        ref = oracle.memory_z(d, rounds, p, unrotated=kind.endswith("_unrotated"))
    else:
        ref = oracle.code_capacity(d, p, unrotated=kind.endswith("_unrotated"))
    m = g.mechanisms()
    assert g.n_det == ref.n_det and m.n_mech == ref.n_mech
    assert np.array_equal(m.off, ref.off) and np.array_equal(m.dets, ref.dets)
    assert np.array_equal(m.obs, ref.obs)
    assert np.array_equal(m.q.view(np.uint64), ref.q.view(np.uint64))
    tab = oracle.tables(ref)
    dist, hops, par, pred, llr = g.tables()
    assert np.array_equal(dist, tab.dist)
    assert np.array_equal(hops, tab.hops)
    assert np.array_equal(par, tab.par)
    assert np.array_equal(pred, tab.pred)
    assert np.array_equal(llr.view(np.uint64), tab.llr.view(np.uint64))


def test_d13_headline_graph_matches_oracle():
    g = bpm.Graph("memory_z", 13, 0.005, 13)
    ref = oracle.memory_z(13, 13, 0.005)
    m = g.mechanisms()
    assert g.n_det == 1176 == ref.n_det
    assert np.array_equal(m.dets, ref.dets) and np.array_equal(m.q.view(np.uint64), ref.q.view(np.uint64))
    dist, hops, par, pred, llr = g.tables()
    tab = oracle.tables(ref)
    assert np.array_equal(dist, tab.dist) and np.array_equal(pred, tab.pred) and np.array_equal(par, tab.par)
    assert np.array_equal(llr.view(np.uint64), tab.llr.view(np.uint64))


def test_d21_largest_batched_graph_matches_oracle():
    # the largest graph the mixed-distance batch uses (4840 detectors): the
    # library's detector error model and N x N tables bit-identical to the
    # oracle's
    g = bpm.Graph("memory_z", 21, 0.005, 21)
    ref = oracle.memory_z(21, 21, 0.005)
    m = g.mechanisms()
    assert g.n_det == 4840 == ref.n_det
    assert np.array_equal(m.dets, ref.dets) and np.array_equal(m.q.view(np.uint64), ref.q.view(np.uint64))
    dist, hops, par, pred, llr = g.tables()
    tab = oracle.tables(ref)
    assert np.array_equal(dist, tab.dist) and np.array_equal(pred, tab.pred) and np.array_equal(par, tab.par)
    assert np.array_equal(llr.view(np.uint64), tab.llr.view(np.uint64))
    g.close()


def test_device_calls_refuse_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    g = bpm.Graph("code_capacity", 3, 0.05)
    with pytest.raises(bpm.BpmError, match="without a device"):
        bpm.bpm_sample(g.handle, 1, 0, 64, 1 << 20, 1 << 21, None, 0)


def test_stage_table_and_configurations():
    ms = bpm.STAGE_MAX_S
    n = len(ms)
    assert n == len(bpm.STAGES) and n <= bpm.BPM_MAX_STAGES
    assert ms[0] == 0 and ms[-1] == 0 and ms[-2] == 2**31 - 1
    tops = ms[1:-1]
    assert all(a < b for a, b in zip(tops, tops[1:])) and tops[0] >= 2
    counts = [bpm.bpm_stage_configs(k) for k in range(n)]
    assert all(1 <= c <= bpm.BPM_MAX_CONFIGS for c in counts)
    assert counts[0] == counts[-1] == 1 and max(counts) > 1
    assert bpm.bpm_stage_configs(n) == 0 and bpm.bpm_stage_configs(-1) == 0
    old = bpm.bpm_get_stage_config()
    try:
        want = [c - 1 for c in counts]
        bpm.bpm_set_stage_config(want)
        assert bpm.bpm_get_stage_config()[:n] == want
        bad = list(want)
        bad[counts.index(1)] = 1                      # a stage with one configuration
        with pytest.raises(bpm.BpmError, match="out of range"):
            bpm.bpm_set_stage_config(bad)
        assert bpm.bpm_get_stage_config()[:n] == want  # unchanged by the failed call
    finally:
        bpm.bpm_set_stage_config(old)


def test_autotune_refuses_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    g = bpm.Graph("code_capacity", 3, 0.05)
    with pytest.raises(bpm.BpmError, match="without a device"):
        bpm.bpm_autotune(g.handle, bpm.bpm_decode_opts(5, 0, 1, 0, 1.0), 1000, 1, 0)


def test_multi_call_arguments_checked_without_device():
    g5 = bpm.Graph("memory_z", 5, 0.005, 5)
    g3 = bpm.Graph("code_capacity", 3, 0.05)
    opts = bpm.bpm_decode_opts(5, 0, 1, 0, 1.0)

    def item(g, n, rows=0):
        it = bpm.bpm_decode_item()
        it.graph = g.handle
        it.n_shots = n
        it.rows_words = rows
        return it

    one = bpm.bpm_decode_workspace_size(g5.handle, 1000, opts)
    both = bpm.bpm_decode_multi_workspace_size([item(g5, 1000), item(g3, 500)], opts)
    assert both > one
    assert bpm.bpm_decode_multi_workspace_size([item(g5, 1000)], opts) == one
    with pytest.raises(bpm.BpmError, match="n_items"):
        bpm.bpm_decode_multi_workspace_size([item(g3, 10)] * (bpm.BPM_MAX_INSTANCES + 1), opts)
    with pytest.raises(bpm.BpmError, match="rows_words"):
        bpm.bpm_decode_multi([item(g5, 10, rows=1)], opts, None, 1 << 20, both, 0)
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(bpm.BpmError, match="without a device"):
            it = item(g5, 10)
            it.syn, it.obs = 1 << 20, 1 << 21
            bpm.bpm_decode_multi([it], opts, None, 1 << 22, both, 0)
    # nothing to decode: accepted without touching a device
    bpm.bpm_decode_multi([item(g5, 0), item(g3, 0)], opts, None, None, 0, 0)


def test_server_options_checked():
    g = bpm.Graph("code_capacity", 3, 0.05)
    with pytest.raises(bpm.BpmError, match="max_batch_shots"):
        bpm.Server([g], 10, max_batch_shots=100)
    with pytest.raises(bpm.BpmError, match="slots"):
        bpm.Server([g], 10, slots=0)
    # the flags are 0 or 1 (the Python wrapper passes bools; the C ABI checks)
    import ctypes
    arr = (ctypes.c_void_p * 1)(g.handle)
    h = ctypes.c_void_p()
    for fields, msg in [(dict(use_graphs=2), "use_graphs"), (dict(one_graph_per_batch=-1), "one_graph_per_batch")]:
        o = bpm.bpm_server_opts(4096, 1 << 16, 3, 0, bpm.bpm_decode_opts(10, 0, bpm.BPM_FP32, 0, 1.0, 0), 0)
        for k, v in fields.items():
            setattr(o, k, v)
        assert bpm._lib.bpm_server_create(arr, 1, ctypes.byref(o), ctypes.byref(h)) == -1
        assert msg in bpm._lib.bpm_last_error().decode()
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(bpm.BpmError, match="without a device"):
            bpm.Server([g], 10)


def test_bbp4mf_argument_checks():
    # B-BP4MF: code-capacity graphs only, FP64 fixed order only
    g = bpm.Graph("code_capacity_unrotated", 5, 0.1)
    ok = bpm.bpm_decode_opts(25, bpm.BPM_BP4MF, bpm.BPM_FP64_SPEC, 0, 1.0)
    assert bpm.bpm_bbp4mf_workspace_size(g.handle, 100, ok) > bpm.bpm_bbp4mf_workspace_size(g.handle, 10, ok)
    for opts, msg in [(bpm.bpm_decode_opts(25, 1, bpm.BPM_FP32, 0, 1.0), "FP64"),
                      (bpm.bpm_decode_opts(0, 1, bpm.BPM_FP64_SPEC, 0, 1.0), "max_iters"),
                      (bpm.bpm_decode_opts(25, 1, bpm.BPM_FP64_SPEC, 0, -1.0), "alpha")]:
        with pytest.raises(bpm.BpmError, match=msg):
            bpm.bpm_bbp4mf_workspace_size(g.handle, 100, opts)
    gz = bpm.Graph("memory_z", 3, 0.01, 3)
    with pytest.raises(bpm.BpmError, match="code-capacity"):
        bpm.bpm_bbp4mf_workspace_size(gz.handle, 100, ok)
    with pytest.raises(bpm.BpmError, match="code-capacity"):
        bpm.bpm_sample_depolarizing(gz.handle, 1, 0, 10, 0, 0, 0, 0)
    # both code-capacity layouts qualify
    g2 = bpm.Graph("code_capacity", 7, 0.1)
    assert bpm.bpm_bbp4mf_workspace_size(g2.handle, 100, ok) > 0
