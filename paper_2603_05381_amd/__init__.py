"""Python binding of libbpm (BP4M decoding on MI355X, see include/bpm.h).

Argument marshalling only: every step of sampling and decoding runs in the
library's HIP kernels.  Device buffers are torch tensors on the current HIP
device; streams are torch streams.  The library must be built
(``python paper_2603_05381_amd/build.py``); importing this module fails
loudly when it is not.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BPM_LIBRARY") or os.path.join(_HERE, "libbpm.so")

BPM_OK = 0
BPM_ROTATED_SURFACE = 0
BPM_UNROTATED_SURFACE = 1
BPM_CODE_CAPACITY_DEPOL = 0
BPM_CIRCUIT_MEMORY_Z = 1
BPM_BP4M = 0
BPM_BP4MF = 1
BPM_FP64_SPEC = 0
BPM_FP32 = 1
BPM_BF16_STORE = 2
BPM_FP16_STORE = 3
BPM_EAGAIN = -5

SHOT_CONVERGED_ANY = 1
SHOT_FC_RAN = 2
SHOT_FC_CHOSEN = 4
SHOT_PRED = 8
SHOT_FAIL = 16
SHOT_OVERFLOW = 32
SHOT_QBP_CONVERGED = 64


class bpm_noise(C.Structure):
    _fields_ = [("kind", C.c_int), ("p", C.c_double)]


class bpm_graph_info(C.Structure):
    _fields_ = [("n_det", C.c_int32), ("n_mech", C.c_int32), ("n_edges", C.c_int32),
                ("d", C.c_int32), ("rounds", C.c_int32), ("max_degree", C.c_int32),
                ("p", C.c_double), ("device_bytes", C.c_uint64)]


class bpm_decode_opts(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("variant", C.c_int32), ("precision", C.c_int32),
                ("s_cap", C.c_int32), ("alpha", C.c_double), ("class_streams", C.c_int32)]


class bpm_counters(C.Structure):
    _fields_ = [("shots", C.c_uint64), ("failures", C.c_uint64), ("never_converged", C.c_uint64),
                ("fc_chosen", C.c_uint64), ("sum_s", C.c_uint64), ("overflow", C.c_uint64)]


class bpm_decode_out(C.Structure):
    _fields_ = [("obs_pred", C.c_void_p), ("fail", C.c_void_p), ("corr", C.c_void_p),
                ("shot_flags", C.c_void_p), ("shot_s", C.c_void_p), ("match", C.c_void_p),
                ("match_stride", C.c_int32), ("lambda_out", C.c_void_p), ("lambda_stride", C.c_int32),
                ("counters", C.c_void_p), ("stage_events", C.c_void_p * 64)]


BPM_MAX_STAGES = 32
BPM_MAX_INSTANCES = 8


class bpm_decode_item(C.Structure):
    _fields_ = [("graph", C.c_void_p), ("syn", C.c_void_p), ("obs", C.c_void_p), ("n_shots", C.c_uint64),
                ("rows_words", C.c_int32), ("out", bpm_decode_out)]


class bpm_server_opts(C.Structure):
    _fields_ = [("max_batch_shots", C.c_int32), ("max_pending_shots", C.c_int32), ("slots", C.c_int32),
                ("use_graphs", C.c_int32), ("decode", bpm_decode_opts), ("one_graph_per_batch", C.c_int32),
                ("mem_budget", C.c_uint64)]


class bpm_server_result(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("graph", C.c_int32), ("n_shots", C.c_uint32), ("pred", C.c_uint64),
                ("fc_chosen", C.c_uint64), ("overflow", C.c_uint64), ("latency_us", C.c_double)]


class bpm_server_stats(C.Structure):
    _fields_ = [("requests_done", C.c_uint64), ("shots_done", C.c_uint64), ("batches", C.c_uint64),
                ("pending_shots", C.c_uint64)]


# names exported by libbpm.so, as declared in include/bpm.h
EXPORTS = ("bpm_build_graph", "bpm_graph_info_get", "bpm_graph_free", "bpm_graph_copy_mechanisms",
           "bpm_graph_copy_tables", "bpm_sample", "bpm_decode_workspace_size", "bpm_decode",
           "bpm_last_error", "bpm_stage_table", "bpm_stage_configs", "bpm_get_stage_config",
           "bpm_set_stage_config", "bpm_autotune", "bpm_decode_multi_workspace_size", "bpm_decode_multi",
           "bpm_server_create", "bpm_server_submit", "bpm_server_poll", "bpm_server_stats_get",
           "bpm_server_destroy", "bpm_sample_depolarizing", "bpm_bbp4mf_workspace_size", "bpm_decode_bbp4mf",
           "bpm_decode_noalloc")

BPM_NOALLOC_SCRATCH_BYTES = 64 << 20


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbpm.so is not built: run `python paper_2603_05381_amd/build.py`")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.bpm_build_graph.argtypes = [C.c_int, C.c_int32, C.c_int32, C.POINTER(bpm_noise), C.POINTER(C.c_void_p)]
    L.bpm_build_graph.restype = C.c_int
    L.bpm_graph_info_get.argtypes = [P, C.POINTER(bpm_graph_info)]
    L.bpm_graph_info_get.restype = C.c_int
    L.bpm_graph_free.argtypes = [P]
    L.bpm_graph_free.restype = None
    L.bpm_graph_copy_mechanisms.argtypes = [P, P, P, P, P]
    L.bpm_graph_copy_mechanisms.restype = C.c_int
    L.bpm_graph_copy_tables.argtypes = [P, P, P, P, P, P]
    L.bpm_graph_copy_tables.restype = C.c_int
    L.bpm_sample.argtypes = [P, C.c_uint64, C.c_uint64, C.c_uint64, P, P, P, P]
    L.bpm_sample.restype = C.c_int
    L.bpm_decode_workspace_size.argtypes = [P, C.c_uint64, C.POINTER(bpm_decode_opts), C.POINTER(C.c_size_t)]
    L.bpm_decode_workspace_size.restype = C.c_int
    L.bpm_decode.argtypes = [P, P, P, C.c_uint64, C.POINTER(bpm_decode_opts), C.POINTER(bpm_decode_out),
                             P, C.c_size_t, P]
    L.bpm_decode.restype = C.c_int
    L.bpm_decode_noalloc.argtypes = [P, P, P, C.c_uint64, C.POINTER(bpm_decode_opts), C.POINTER(bpm_decode_out), P]
    L.bpm_decode_noalloc.restype = C.c_int
    L.bpm_last_error.argtypes = []
    L.bpm_last_error.restype = C.c_char_p
    L.bpm_stage_table.argtypes = [P]
    L.bpm_stage_table.restype = C.c_int32
    L.bpm_stage_configs.argtypes = [C.c_int32]
    L.bpm_stage_configs.restype = C.c_int32
    L.bpm_get_stage_config.argtypes = [P]
    L.bpm_get_stage_config.restype = C.c_int
    L.bpm_set_stage_config.argtypes = [P]
    L.bpm_set_stage_config.restype = C.c_int
    L.bpm_autotune.argtypes = [P, C.POINTER(bpm_decode_opts), C.c_uint64, C.c_uint64, P, P]
    L.bpm_autotune.restype = C.c_int
    L.bpm_decode_multi_workspace_size.argtypes = [C.POINTER(bpm_decode_item), C.c_int32,
                                                  C.POINTER(bpm_decode_opts), C.POINTER(C.c_size_t)]
    L.bpm_decode_multi_workspace_size.restype = C.c_int
    L.bpm_decode_multi.argtypes = [C.POINTER(bpm_decode_item), C.c_int32, C.POINTER(bpm_decode_opts), P, P,
                                   C.c_size_t, P]
    L.bpm_decode_multi.restype = C.c_int
    L.bpm_server_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(bpm_server_opts), C.POINTER(C.c_void_p)]
    L.bpm_server_create.restype = C.c_int
    L.bpm_server_submit.argtypes = [P, C.c_int32, P, C.c_uint32, C.c_uint64]
    L.bpm_server_submit.restype = C.c_int
    L.bpm_server_poll.argtypes = [P, C.POINTER(bpm_server_result), C.c_int32]
    L.bpm_server_poll.restype = C.c_int32
    L.bpm_server_stats_get.argtypes = [P, C.POINTER(bpm_server_stats)]
    L.bpm_server_stats_get.restype = C.c_int
    L.bpm_server_destroy.argtypes = [P]
    L.bpm_server_destroy.restype = None
    L.bpm_sample_depolarizing.argtypes = [P, C.c_uint64, C.c_uint64, C.c_uint64, P, P, P, P]
    L.bpm_sample_depolarizing.restype = C.c_int
    L.bpm_bbp4mf_workspace_size.argtypes = [P, C.c_uint64, C.POINTER(bpm_decode_opts), C.POINTER(C.c_size_t)]
    L.bpm_bbp4mf_workspace_size.restype = C.c_int
    L.bpm_decode_bbp4mf.argtypes = [P, P, P, P, C.c_uint64, C.POINTER(bpm_decode_opts), C.POINTER(bpm_decode_out),
                                    P, C.c_size_t, P]
    L.bpm_decode_bbp4mf.restype = C.c_int
    return L


_lib = _load()


def bpm_stage_table():
    """Stage table of bpm_decode: list of max_s per stage (0 for extraction
    and packing, 2**31 - 1 for the stage that takes every larger shot)."""
    buf = (C.c_int32 * BPM_MAX_STAGES)()
    n = _lib.bpm_stage_table(buf)
    return [int(buf[k]) for k in range(n)]


BPM_MAX_CONFIGS = 4
STAGE_MAX_S = bpm_stage_table()
STAGES = tuple(["extract"] + ["bp_s%d" % m if m < 2**31 - 1 else "bp_large" for m in STAGE_MAX_S[1:-1]]
               + ["finalize"])


class BpmError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != BPM_OK:
        raise BpmError("%s failed (%d): %s" % (what, rc, _lib.bpm_last_error().decode()))


def lib():
    return _lib


# ------------------------------------------------------------ C-ABI names --

def bpm_build_graph(code: int, d: int, rounds: int, noise_kind: int, p: float) -> int:
    out = C.c_void_p()
    nz = bpm_noise(noise_kind, p)
    _check(_lib.bpm_build_graph(code, d, rounds, C.byref(nz), C.byref(out)), "bpm_build_graph")
    return out.value


def bpm_graph_info_get(g: int) -> bpm_graph_info:
    info = bpm_graph_info()
    _check(_lib.bpm_graph_info_get(g, C.byref(info)), "bpm_graph_info_get")
    return info


def bpm_graph_free(g: int) -> None:
    _lib.bpm_graph_free(g)


def bpm_graph_copy_mechanisms(g: int, off, dets, obs, q) -> None:
    _check(_lib.bpm_graph_copy_mechanisms(g, *(None if a is None else a.ctypes.data for a in (off, dets, obs, q))),
           "bpm_graph_copy_mechanisms")


def bpm_graph_copy_tables(g: int, dist, hops, par, pred, llr) -> None:
    _check(_lib.bpm_graph_copy_tables(g, *(None if a is None else a.ctypes.data
                                           for a in (dist, hops, par, pred, llr))), "bpm_graph_copy_tables")


def bpm_sample(g: int, seed: int, shot0: int, n_shots: int, syn_ptr: int, obs_ptr: int, err_ptr, stream: int) -> None:
    _check(_lib.bpm_sample(g, seed, shot0, n_shots, syn_ptr, obs_ptr, err_ptr, stream), "bpm_sample")


def bpm_decode_workspace_size(g: int, n_shots: int, opts: bpm_decode_opts) -> int:
    n = C.c_size_t(0)
    _check(_lib.bpm_decode_workspace_size(g, n_shots, C.byref(opts), C.byref(n)), "bpm_decode_workspace_size")
    return n.value


def bpm_decode_multi_workspace_size(items, opts: bpm_decode_opts) -> int:
    arr = (bpm_decode_item * len(items))(*items)
    n = C.c_size_t()
    _check(_lib.bpm_decode_multi_workspace_size(arr, len(items), C.byref(opts), C.byref(n)),
           "bpm_decode_multi_workspace_size")
    return n.value


def bpm_decode_multi(items, opts: bpm_decode_opts, stage_events, workspace_ptr: int, workspace_bytes: int,
                     stream: int) -> None:
    arr = (bpm_decode_item * len(items))(*items)
    ev = None
    if stage_events is not None:
        ev = (C.c_void_p * (2 * BPM_MAX_STAGES))(*stage_events)
    _check(_lib.bpm_decode_multi(arr, len(items), C.byref(opts), ev, workspace_ptr, workspace_bytes, stream),
           "bpm_decode_multi")


def bpm_stage_configs(stage: int) -> int:
    return int(_lib.bpm_stage_configs(stage))


def bpm_get_stage_config() -> list:
    buf = (C.c_int32 * BPM_MAX_STAGES)()
    _check(_lib.bpm_get_stage_config(buf), "bpm_get_stage_config")
    return list(buf)


def bpm_set_stage_config(cfg) -> None:
    buf = (C.c_int32 * BPM_MAX_STAGES)(*([int(x) for x in cfg] + [0] * (BPM_MAX_STAGES - len(cfg))))
    _check(_lib.bpm_set_stage_config(buf), "bpm_set_stage_config")


def bpm_autotune(g: int, opts: bpm_decode_opts, n_shots: int, seed: int, stream: int):
    """Returns the measured stage times, [BPM_MAX_CONFIGS][BPM_MAX_STAGES] ms (-1 = not measured)."""
    buf = (C.c_float * (BPM_MAX_CONFIGS * BPM_MAX_STAGES))()
    _check(_lib.bpm_autotune(g, C.byref(opts), n_shots, seed, buf, stream), "bpm_autotune")
    return [[float(buf[c * BPM_MAX_STAGES + k]) for k in range(BPM_MAX_STAGES)] for c in range(BPM_MAX_CONFIGS)]


def bpm_decode(g: int, syn_ptr: int, obs_ptr: int, n_shots: int, opts: bpm_decode_opts,
               out: bpm_decode_out, workspace_ptr: int, workspace_bytes: int, stream: int) -> None:
    _check(_lib.bpm_decode(g, syn_ptr, obs_ptr, n_shots, C.byref(opts), C.byref(out), workspace_ptr,
                           workspace_bytes, stream), "bpm_decode")


def bpm_decode_noalloc(g: int, syn_ptr: int, obs_ptr: int, n_shots: int, opts: bpm_decode_opts,
                       out: bpm_decode_out, stream: int) -> None:
    _check(_lib.bpm_decode_noalloc(g, syn_ptr, obs_ptr, n_shots, C.byref(opts), C.byref(out), stream),
           "bpm_decode_noalloc")


def bpm_sample_depolarizing(g: int, seed: int, shot0: int, n_shots: int, synx_ptr: int, synz_ptr: int,
                            obs_ptr: int, stream: int) -> None:
    _check(_lib.bpm_sample_depolarizing(g, seed, shot0, n_shots, synx_ptr, synz_ptr, obs_ptr, stream),
           "bpm_sample_depolarizing")


def bpm_bbp4mf_workspace_size(g: int, n_shots: int, opts: bpm_decode_opts) -> int:
    n = C.c_size_t(0)
    _check(_lib.bpm_bbp4mf_workspace_size(g, n_shots, C.byref(opts), C.byref(n)), "bpm_bbp4mf_workspace_size")
    return n.value


def bpm_decode_bbp4mf(g: int, synx_ptr: int, synz_ptr: int, obs_ptr: int, n_shots: int, opts: bpm_decode_opts,
                      out: bpm_decode_out, workspace_ptr: int, workspace_bytes: int, stream: int) -> None:
    _check(_lib.bpm_decode_bbp4mf(g, synx_ptr, synz_ptr, obs_ptr, n_shots, C.byref(opts), C.byref(out),
                                  workspace_ptr, workspace_bytes, stream), "bpm_decode_bbp4mf")


# ------------------------------------------------------------ convenience --

@dataclass
class Mechanisms:
    n_det: int
    off: np.ndarray
    dets: np.ndarray
    obs: np.ndarray
    q: np.ndarray

    @property
    def n_mech(self):
        return int(self.q.size)


class Graph:
    """A detector graph resident on the current device (owns its tables)."""

    def __init__(self, kind: str, d: int, p: float, rounds: int = 1):
        """kind: "code_capacity", "memory_z" (rotated code),
        "code_capacity_unrotated" or "memory_z_unrotated"."""
        nk = {"code_capacity": BPM_CODE_CAPACITY_DEPOL, "memory_z": BPM_CIRCUIT_MEMORY_Z,
              "code_capacity_unrotated": BPM_CODE_CAPACITY_DEPOL,
              "memory_z_unrotated": BPM_CIRCUIT_MEMORY_Z}[kind]
        code = BPM_UNROTATED_SURFACE if kind.endswith("_unrotated") else BPM_ROTATED_SURFACE
        self.kind, self.d, self.p, self.rounds = kind, d, p, rounds
        self.handle = bpm_build_graph(code, d, rounds, nk, p)
        self.info = bpm_graph_info_get(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            bpm_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_det(self):
        return self.info.n_det

    def mechanisms(self) -> Mechanisms:
        n = self.info.n_mech
        off = np.zeros(n + 1, dtype=np.int32)
        bpm_graph_copy_mechanisms(self.handle, off, None, None, None)
        dets = np.zeros(max(int(off[-1]), 1), dtype=np.int32)
        obs = np.zeros(n, dtype=np.uint8)
        q = np.zeros(n, dtype=np.float64)
        bpm_graph_copy_mechanisms(self.handle, off, dets, obs, q)
        return Mechanisms(self.n_det, off, dets[: off[-1]], obs, q)

    def tables(self):
        N = self.n_det
        dist = np.zeros((N, N), dtype=np.int64)
        hops = np.zeros((N, N), dtype=np.int32)
        par = np.zeros((N, N), dtype=np.uint8)
        pred = np.zeros((N, N), dtype=np.int32)
        llr = np.zeros((N, N), dtype=np.float64)
        bpm_graph_copy_tables(self.handle, dist, hops, par, pred, llr)
        return dist, hops, par, pred, llr

    # -- device work (torch tensors) --------------------------------------
    def sample(self, seed: int, shot0: int, n: int, stream=None, want_err: bool = False):
        """(syn [n_det, W], obs [W]) device tensors, plus err [n_mech, W]
        (the sampled error's mechanism planes) with want_err."""
        import torch
        W = (n + 63) // 64
        syn = torch.empty((self.n_det, max(W, 1)), dtype=torch.int64, device="cuda")
        obs = torch.empty(max(W, 1), dtype=torch.int64, device="cuda")
        err = torch.empty((self.info.n_mech, max(W, 1)), dtype=torch.int64, device="cuda") if want_err else None
        st = stream or torch.cuda.current_stream()
        bpm_sample(self.handle, seed, shot0, n, syn.data_ptr(), obs.data_ptr(),
                   err.data_ptr() if want_err else None, st.cuda_stream)
        return (syn, obs, err) if want_err else (syn, obs)

    def sample_depolarizing(self, seed: int, shot0: int, n: int, stream=None):
        """Depolarizing noise with both syndromes (code-capacity graphs):
        (syn_x [n_det, W], syn_z [n_det, W], obs [W]) device tensors."""
        import torch
        W = (n + 63) // 64
        sx = torch.empty((self.n_det, max(W, 1)), dtype=torch.int64, device="cuda")
        sz = torch.empty((self.n_det, max(W, 1)), dtype=torch.int64, device="cuda")
        obs = torch.empty(max(W, 1), dtype=torch.int64, device="cuda")
        st = stream or torch.cuda.current_stream()
        bpm_sample_depolarizing(self.handle, seed, shot0, n, sx.data_ptr(), sz.data_ptr(), obs.data_ptr(),
                                st.cuda_stream)
        return sx, sz, obs

    def decode_bbp4mf(self, syn_x, syn_z, obs, n: int, max_iters: int, variant: int = BPM_BP4MF,
                      alpha: float = 1.0, s_cap: int = 0, want_match: bool = False, stream=None):
        """B-BP4MF (FP64 fixed order) of n shots; returns a dict of device tensors."""
        import torch
        st = stream or torch.cuda.current_stream()
        opts = bpm_decode_opts(max_iters, variant, BPM_FP64_SPEC, s_cap, alpha)
        s_eff = s_cap if s_cap > 0 else min(self.n_det, 256)
        res, out = self.outputs(n, syn_x.device, s_cap, False, want_match, 0, s_eff=s_eff)
        nbytes = bpm_bbp4mf_workspace_size(self.handle, n, opts)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=syn_x.device)
        aligned = (ws.data_ptr() + 255) & ~255
        bpm_decode_bbp4mf(self.handle, syn_x.data_ptr(), syn_z.data_ptr(),
                          obs.data_ptr() if obs is not None else None, n, opts, out, aligned, nbytes, st.cuda_stream)
        res["_workspace"] = ws
        return res

    def outputs(self, n: int, dev, s_cap: int = 0, want_corr: bool = False, want_match: bool = False,
                lambda_stride: int = 0, s_eff: int = 0):
        """Allocate the output tensors of a decode of n shots and the
        bpm_decode_out pointing at them."""
        import torch
        W = (n + 63) // 64
        res = {
            "obs_pred": torch.zeros(max(W, 1), dtype=torch.int64, device=dev),
            "fail": torch.zeros(max(W, 1), dtype=torch.int64, device=dev),
            "flags": torch.zeros(max(n, 1), dtype=torch.uint8, device=dev),
            "s": torch.zeros(max(n, 1), dtype=torch.int32, device=dev),
            "counters": torch.zeros(6, dtype=torch.int64, device=dev),
        }
        s_eff = s_eff or (s_cap if s_cap > 0 else min(self.n_det, 512))
        out = bpm_decode_out()
        out.obs_pred = res["obs_pred"].data_ptr()
        out.fail = res["fail"].data_ptr()
        out.shot_flags = res["flags"].data_ptr()
        out.shot_s = res["s"].data_ptr()
        out.counters = res["counters"].data_ptr()
        if want_corr:
            res["corr"] = torch.zeros((self.info.n_edges, max(W, 1)), dtype=torch.int64, device=dev)
            out.corr = res["corr"].data_ptr()
        if want_match:
            res["match"] = torch.full((max(n, 1), s_eff), -1, dtype=torch.int32, device=dev)
            out.match = res["match"].data_ptr()
            out.match_stride = s_eff
        if lambda_stride:
            res["lambda"] = torch.full((max(n, 1), lambda_stride, lambda_stride), float("nan"),
                                       dtype=torch.float64, device=dev)
            out.lambda_out = res["lambda"].data_ptr()
            out.lambda_stride = lambda_stride
        return res, out

    def decode(self, syn, obs, n: int, max_iters: int, precision: int = BPM_FP32, variant: int = BPM_BP4M,
               alpha: float = 1.0, s_cap: int = 0, want_corr: bool = False, want_match: bool = False,
               lambda_stride: int = 0, workspace=None, stream=None, events=None, class_streams: int = 0):
        """Decode n shots; returns a dict of device tensors."""
        import torch
        st = stream or torch.cuda.current_stream()
        opts = bpm_decode_opts(max_iters, variant, precision, s_cap, alpha, class_streams)
        dev = syn.device
        res, out = self.outputs(n, dev, s_cap, want_corr, want_match, lambda_stride)
        if events is not None:
            # events: 2 * len(STAGES) torch.cuda.Event(enable_timing=True), two per stage
            for k, ev in enumerate(events):
                if not ev.cuda_event:          # torch creates events lazily
                    ev.record(st)
                out.stage_events[k] = ev.cuda_event
        nbytes = bpm_decode_workspace_size(self.handle, n, opts)
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        ptr = workspace.data_ptr()
        aligned = (ptr + 255) & ~255
        avail = workspace.numel() - (aligned - ptr)
        bpm_decode(self.handle, syn.data_ptr(), obs.data_ptr(), n, opts, out, aligned, avail, st.cuda_stream)
        res["_workspace"] = workspace
        return res


def decode_multi(parts, max_iters: int, precision: int = BPM_FP32, variant: int = BPM_BP4M, alpha: float = 1.0,
                 s_cap: int = 0, want_match: bool = False, stream=None, events=None):
    """Decode several graphs' shots in one call.  parts: list of
    (graph, syn, obs, n) for bit planes, or (graph, rows, None, n) for
    shot-major rows (rows: [n][words] int64 tensor).  Returns one result dict
    per part."""
    import torch
    st = stream or torch.cuda.current_stream()
    opts = bpm_decode_opts(max_iters, variant, precision, s_cap, alpha)
    s_eff = s_cap if s_cap > 0 else min(max(p[0].n_det for p in parts), 512)
    items, results = [], []
    for g, syn, obs, n in parts:
        res, out = g.outputs(n, syn.device, s_cap, False, want_match, 0, s_eff=s_eff)
        it = bpm_decode_item()
        it.graph = g.handle
        it.syn = syn.data_ptr()
        it.obs = obs.data_ptr() if obs is not None else None
        it.n_shots = n
        it.rows_words = 0 if obs is not None else int(syn.shape[1])
        it.out = out
        items.append(it)
        results.append(res)
    nbytes = bpm_decode_multi_workspace_size(items, opts)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    aligned = (ws.data_ptr() + 255) & ~255
    ev = None
    if events is not None:
        ev = []
        for e in events:
            if not e.cuda_event:
                e.record(st)
            ev.append(e.cuda_event)
        ev += [None] * (2 * BPM_MAX_STAGES - len(ev))
    bpm_decode_multi(items, opts, ev, aligned, nbytes, st.cuda_stream)
    for r in results:
        r["_workspace"] = ws
    return results


class Server:
    """Continuous-batching decode server over resident graphs (C ABI
    bpm_server_*).  submit() takes shot-major rows: a uint64 array
    [n_shots][ceil(n_det / 64)], n_shots in 1..64."""

    def __init__(self, graphs, max_iters: int, precision: int = BPM_FP32, variant: int = BPM_BP4M,
                 alpha: float = 1.0, max_batch_shots: int = 4096, max_pending_shots: int = 1 << 16,
                 slots: int = 3, use_graphs: bool = False, class_streams: int = 4,
                 one_graph_per_batch: bool = False, mem_budget: int = 0):
        self.graphs = list(graphs)                 # kept alive: the server points at them
        arr = (C.c_void_p * len(self.graphs))(*[g.handle for g in self.graphs])
        o = bpm_server_opts(max_batch_shots, max_pending_shots, slots, int(bool(use_graphs)),
                            bpm_decode_opts(max_iters, variant, precision, 0, alpha, class_streams),
                            int(bool(one_graph_per_batch)), int(mem_budget))
        h = C.c_void_p()
        _check(_lib.bpm_server_create(arr, len(self.graphs), C.byref(o), C.byref(h)), "bpm_server_create")
        self.handle = h.value
        self._buf = (bpm_server_result * 4096)()

    def submit(self, graph_idx: int, rows, req_id: int) -> bool:
        """False if the admission budget is full (BPM_EAGAIN)."""
        import numpy as np
        rows = np.ascontiguousarray(rows, dtype=np.uint64)
        rc = _lib.bpm_server_submit(self.handle, graph_idx, rows.ctypes.data, rows.shape[0], req_id)
        if rc == BPM_EAGAIN:
            return False
        _check(rc, "bpm_server_submit")
        return True

    def poll(self):
        """Finished requests: list of (req_id, graph, n_shots, pred, fc_chosen, overflow, latency_us)."""
        out = []
        while True:
            k = _lib.bpm_server_poll(self.handle, self._buf, len(self._buf))
            for i in range(k):
                r = self._buf[i]
                out.append((r.req_id, r.graph, r.n_shots, r.pred, r.fc_chosen, r.overflow, r.latency_us))
            if k < len(self._buf):
                return out

    def stats(self) -> dict:
        st = bpm_server_stats()
        _check(_lib.bpm_server_stats_get(self.handle, C.byref(st)), "bpm_server_stats_get")
        return {"requests_done": st.requests_done, "shots_done": st.shots_done, "batches": st.batches,
                "pending_shots": st.pending_shots}

    def close(self):
        if getattr(self, "handle", None):
            _lib.bpm_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


def planes_to_rows(syn, n: int, n_det: int):
    """Detector bit planes [n_det][W] (device int64 tensor) -> shot-major
    rows [n][ceil(n_det/64)] uint64 numpy array (host)."""
    import numpy as np
    planes = syn.cpu().numpy().view(np.uint64)[:n_det]
    bits = np.unpackbits(planes.view(np.uint8), axis=1, bitorder="little")[:, :n]     # [n_det][n]
    words = (n_det + 63) // 64
    padded = np.zeros((n, words * 64), dtype=np.uint8)
    padded[:, :n_det] = bits.T
    return np.packbits(padded, axis=1, bitorder="little").view(np.uint64)


def counters_dict(t) -> dict:
    v = [int(x) for x in t.cpu().tolist()]
    return dict(zip(("shots", "failures", "never_converged", "fc_chosen", "sum_s", "overflow"), v))
