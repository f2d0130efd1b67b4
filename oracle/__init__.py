"""FP64 CPU oracle for the BP4M decoding pipeline -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C in
this directory, built with gcc) and shares no code with the GPU library.

Every routine follows a passage of "Achieving Thresholds via Standalone Belief
Propagation on Surface Codes" (arXiv 2603.05381); see the C sources.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["spec_math.c", "philox.c", "codes.c", "paths.c", "sample.c", "bp4m.c", "vec.c", "qbp.c"]

F_CONVERGED_ANY = 1
F_FC_RAN = 2
F_FC_CHOSEN = 4
F_PRED = 8
F_FAIL = 16


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, no contraction of a*b+c)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(p) for p in srcs + [os.path.join(HERE, "oracle.h")])
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-pthread", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Dem(C.Structure):
    _fields_ = [("n_det", C.c_int32), ("n_mech", C.c_int32),
                ("off", C.POINTER(C.c_int32)), ("dets", C.POINTER(C.c_int32)),
                ("obs", C.POINTER(C.c_uint8)), ("q", C.POINTER(C.c_double))]


class _Tables(C.Structure):
    _fields_ = [("n", C.c_int32), ("dist", C.POINTER(C.c_int64)),
                ("hops", C.POINTER(C.c_int32)), ("par", C.POINTER(C.c_uint8)),
                ("pred", C.POINTER(C.c_int32)), ("llr", C.POINTER(C.c_double))]


class _Opts(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("variant", C.c_int32), ("alpha", C.c_double),
                ("schedule", C.c_int32), ("fc_rule", C.c_int32), ("weight_rule", C.c_int32)]


class _Tanner(C.Structure):
    _fields_ = [("n_q", C.c_int32), ("n_xc", C.c_int32), ("n_zc", C.c_int32),
                ("qx", C.POINTER(C.c_int32)), ("qz", C.POINTER(C.c_int32)),
                ("qobs", C.POINTER(C.c_uint8)), ("qmech", C.POINTER(C.c_int32)),
                ("cq", C.POINTER(C.c_int32))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.or_exp.restype = C.c_double
        L.or_exp.argtypes = [C.c_double]
        L.or_log1p.restype = C.c_double
        L.or_log1p.argtypes = [C.c_double]
        L.or_maxstar.restype = C.c_double
        L.or_maxstar.argtypes = [C.c_double, C.c_double]
        for name in ("or_exp_v", "or_log1p_v"):
            getattr(L, name).argtypes = [P, P, C.c_int64]
        L.or_maxstar_v.argtypes = [P, P, P, C.c_int64]
        L.or_philox_v.argtypes = [P, P, P, C.c_int64]
        L.or_threshold_v.argtypes = [P, P, C.c_int64]
        L.or_prior_llr_v.argtypes = [P, P, C.c_int64]
        L.or_fixed_weight_v.argtypes = [P, P, C.c_int64]
        L.or_build_code_capacity.argtypes = [C.c_int, C.c_double, C.POINTER(_Dem)]
        L.or_build_code_capacity_unrotated.argtypes = [C.c_int, C.c_double, C.POINTER(_Dem)]
        L.or_build_memory_z.argtypes = [C.c_int, C.c_int, C.c_double, C.POINTER(_Dem),
                                        C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.or_build_memory_z_unrotated.argtypes = [C.c_int, C.c_int, C.c_double, C.POINTER(_Dem),
                                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.or_dem_free.argtypes = [C.POINTER(_Dem)]
        L.or_build_tables.argtypes = [C.POINTER(_Dem), C.POINTER(_Tables)]
        L.or_tables_free.argtypes = [C.POINTER(_Tables)]
        L.or_sample.argtypes = [C.POINTER(_Dem), C.c_uint64, C.c_uint64, C.c_uint64, P, P, P]
        L.or_factor_update.argtypes = [P, C.c_int, P]
        L.or_forced_convergence.argtypes = [P, C.c_int, P]
        L.or_marginal_decision.argtypes = [P, C.c_int, P]
        L.or_marginal_decision.restype = C.c_int
        L.or_bp4m_instance.argtypes = [P, P, C.c_int, C.POINTER(_Opts), P, P, P, P]
        L.or_bp4m_instance.restype = C.c_int
        L.or_select_sequence.argtypes = [P, C.c_int, C.c_int, P, C.c_int, P, P]
        L.or_select_sequence.restype = C.c_int
        L.or_forced_convergence_blocks.argtypes = [P, C.c_int, P]
        L.or_forced_convergence_blocks.restype = None
        L.or_decode.argtypes = [C.POINTER(_Dem), C.POINTER(_Tables), P, P, C.c_uint64,
                                C.POINTER(_Opts), C.c_int, P, P, P, C.c_int32, P]
        L.or_decode.restype = C.c_int
        L.or_build_tanner_code_capacity.argtypes = [C.c_int, C.c_int, C.POINTER(_Dem), C.POINTER(_Tanner)]
        L.or_tanner_free.argtypes = [C.POINTER(_Tanner)]
        L.or_build_tables_w.argtypes = [C.POINTER(_Dem), P, C.POINTER(_Tables)]
        L.or_spec_log.restype = C.c_double
        L.or_spec_log.argtypes = [C.c_double]
        L.or_spec_prior.restype = C.c_double
        L.or_spec_prior.argtypes = [C.c_int64]
        L.or_qbp_weight.restype = C.c_int64
        L.or_qbp_weight.argtypes = [C.c_double]
        L.or_qbp_zprob.restype = C.c_double
        L.or_qbp_zprob.argtypes = [P]
        L.or_sample_depolarizing.argtypes = [C.POINTER(_Tanner), C.c_double, C.c_uint64, C.c_uint64,
                                             C.c_uint64, P, P, P]
        L.or_qbp.argtypes = [C.POINTER(_Tanner), C.c_double, P, P, C.c_int, C.c_int, P, P, P]
        L.or_qbp.restype = C.c_int
        L.or_bbp4mf_decode.argtypes = [C.POINTER(_Dem), C.POINTER(_Tanner), C.c_double, P, P, P,
                                       C.c_uint64, C.POINTER(_Opts), C.c_int, P, P, P, C.c_int32]
        L.or_bbp4mf_decode.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- numerics --

def exp(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().or_exp_v(_p(x), _p(y), x.size)
    return y


def log1p(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().or_log1p_v(_p(x), _p(y), x.size)
    return y


def maxstar(a, b) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    y = np.empty_like(a)
    lib().or_maxstar_v(_p(a), _p(b), _p(y), a.size)
    return y


def philox(ctr, key) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    lib().or_philox_v(_p(ctr), _p(key), _p(out), ctr.shape[0])
    return out


def threshold(q) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    t = np.empty(q.shape, dtype=np.uint32)
    lib().or_threshold_v(_p(q), _p(t), q.size)
    return t


def prior_llr(dist_fixed) -> np.ndarray:
    d = np.ascontiguousarray(dist_fixed, dtype=np.int64)
    y = np.empty(d.shape, dtype=np.float64)
    lib().or_prior_llr_v(_p(d), _p(y), d.size)
    return y


def fixed_weight(q) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    w = np.empty(q.shape, dtype=np.int64)
    lib().or_fixed_weight_v(_p(q), _p(w), q.size)
    return w


# ------------------------------------------------------------------ graphs --

@dataclass
class Dem:
    """Detector error model: mechanism m flips dets[off[m]:off[m+1]], obs[m]."""
    n_det: int
    off: np.ndarray
    dets: np.ndarray
    obs: np.ndarray
    q: np.ndarray
    n_hyper: int = 0
    n_gauge_bad: int = 0

    @property
    def n_mech(self) -> int:
        return int(self.q.size)

    def mech(self, m: int):
        return tuple(int(x) for x in self.dets[self.off[m]:self.off[m + 1]]), int(self.obs[m])

    def _c(self) -> _Dem:
        self._keep = [np.ascontiguousarray(self.off, dtype=np.int32),
                      np.ascontiguousarray(self.dets, dtype=np.int32),
                      np.ascontiguousarray(self.obs, dtype=np.uint8),
                      np.ascontiguousarray(self.q, dtype=np.float64)]
        o, d, b, q = self._keep
        return _Dem(self.n_det, self.n_mech, o.ctypes.data_as(C.POINTER(C.c_int32)),
                    d.ctypes.data_as(C.POINTER(C.c_int32)),
                    b.ctypes.data_as(C.POINTER(C.c_uint8)),
                    q.ctypes.data_as(C.POINTER(C.c_double)))


def _take_dem(g: _Dem, **extra) -> Dem:
    n, nd = g.n_mech, g.n_det
    off = np.ctypeslib.as_array(g.off, shape=(n + 1,)).copy()
    dets = np.ctypeslib.as_array(g.dets, shape=(max(int(off[-1]), 1),))[: off[-1]].copy()
    obs = np.ctypeslib.as_array(g.obs, shape=(n,)).copy()
    q = np.ctypeslib.as_array(g.q, shape=(n,)).copy()
    lib().or_dem_free(C.byref(g))
    return Dem(nd, off, dets, obs, q, **extra)


def code_capacity(d: int, p: float, unrotated: bool = False) -> Dem:
    g = _Dem()
    f = lib().or_build_code_capacity_unrotated if unrotated else lib().or_build_code_capacity
    if f(d, p, C.byref(g)) != 0:
        raise ValueError("bad code-capacity parameters")
    return _take_dem(g)


def memory_z(d: int, rounds: int, p: float, unrotated: bool = False) -> Dem:
    g = _Dem()
    nh, ng = C.c_int32(0), C.c_int32(0)
    f = lib().or_build_memory_z_unrotated if unrotated else lib().or_build_memory_z
    if f(d, rounds, p, C.byref(g), C.byref(nh), C.byref(ng)) != 0:
        raise ValueError("bad memory-Z parameters")
    return _take_dem(g, n_hyper=nh.value, n_gauge_bad=ng.value)


@dataclass
class Tables:
    """N x N path tables; [u][u] holds u's boundary path."""
    dist: np.ndarray
    hops: np.ndarray
    par: np.ndarray
    pred: np.ndarray
    llr: np.ndarray

    def _c(self) -> _Tables:
        self._keep = [np.ascontiguousarray(a) for a in (self.dist, self.hops, self.par, self.pred, self.llr)]
        d, h, p, r, l = self._keep
        return _Tables(d.shape[0], d.ctypes.data_as(C.POINTER(C.c_int64)),
                       h.ctypes.data_as(C.POINTER(C.c_int32)),
                       p.ctypes.data_as(C.POINTER(C.c_uint8)),
                       r.ctypes.data_as(C.POINTER(C.c_int32)),
                       l.ctypes.data_as(C.POINTER(C.c_double)))


def tables(dem: Dem) -> Tables:
    t = _Tables()
    gd = dem._c()
    rc = lib().or_build_tables(C.byref(gd), C.byref(t))
    if rc != 0:
        raise ValueError("or_build_tables failed (%d)" % rc)
    N = t.n
    def take(ptr, dt):
        return np.ctypeslib.as_array(ptr, shape=(N, N)).astype(dt, copy=True)
    out = Tables(take(t.dist, np.int64), take(t.hops, np.int32), take(t.par, np.uint8),
                 take(t.pred, np.int32), take(t.llr, np.float64))
    lib().or_tables_free(C.byref(t))
    return out


# ---------------------------------------------------------------- sampling --

def sample(dem: Dem, seed: int, shot0: int, n: int, want_err: bool = False):
    """Bit planes syn[n_det, W] and obs[W] (uint64), W = ceil(n/64); with
    want_err also err[n_mech, W], the mechanisms that fired."""
    W = (n + 63) // 64
    syn = np.zeros((dem.n_det, max(W, 1)), dtype=np.uint64)
    obs = np.zeros(max(W, 1), dtype=np.uint64)
    err = np.zeros((dem.n_mech, max(W, 1)), dtype=np.uint64) if want_err else None
    gd = dem._c()
    lib().or_sample(C.byref(gd), seed, shot0, n, _p(syn), _p(obs), _p(err) if want_err else None)
    if want_err:
        return syn[:, :W], obs[:W], err[:, :W]
    return syn[:, :W], obs[:W]


# ---------------------------------------------------------------- decoding --

def factor_update(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().or_factor_update(_p(x), x.size, _p(out))
    return out


def forced_convergence_blocks(lam) -> np.ndarray:
    """Block-maxima forced convergence, conflicts to the boundary (a
    diagnostic reading of Sec. II.D)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    s = lam.shape[0]
    part = np.empty(s, dtype=np.int32)
    lib().or_forced_convergence_blocks(_p(lam), s, _p(part))
    return part


def forced_convergence(lam) -> np.ndarray:
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    s = lam.shape[0]
    part = np.empty(s, dtype=np.int32)
    lib().or_forced_convergence(_p(lam), s, _p(part))
    return part


def marginal_decision(lam):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    s = lam.shape[0]
    part = np.empty(s, dtype=np.int32)
    conv = lib().or_marginal_decision(_p(lam), s, _p(part))
    return bool(conv), part


def bp4m_instance(L, W, max_iters: int, alpha: float = 1.0, variant: int = 0, schedule: int = 0,
                  fc_rule: int = 0):
    """Run BP4M (variant 0) / BP4MF (1) on one s x s instance.  schedule /
    fc_rule: diagnostic readings (see oracle.h), 0 = the default reading.

    Returns (flags, partner, weight, M, lam) after the last iteration."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.int64)
    s = L.shape[0]
    part = np.empty(max(s, 1), dtype=np.int32)
    w = np.zeros(1, dtype=np.int64)
    M = np.zeros((s, s), dtype=np.float64)
    lam = np.zeros((s, s), dtype=np.float64)
    o = _Opts(max_iters, variant, alpha, schedule, fc_rule, 0)
    fl = lib().or_bp4m_instance(_p(L), _p(W), s, C.byref(o), _p(part), _p(w),
                                _p(M) if s else None, _p(lam) if s else None)
    return fl, part[:s], int(w[0]), M, lam


def select_sequence(lam_seq, W, variant: int = 0):
    """Candidate rules of BP4M (variant 0) / BP4MF (1), Sec. III.A-B, applied
    to given posteriors lam_seq[T, s, s] of iterations 1..T (symmetric,
    diagonal = boundary) with integer weights W[s, s].  Returns (flags,
    partner, weight)."""
    lam_seq = np.ascontiguousarray(lam_seq, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.int64)
    T, s = lam_seq.shape[0], lam_seq.shape[1]
    assert T >= 1 and lam_seq.shape == (T, s, s) and W.shape == (s, s)
    part = np.empty(max(s, 1), dtype=np.int32)
    w = np.zeros(1, dtype=np.int64)
    fl = lib().or_select_sequence(_p(lam_seq), T, s, _p(W), variant, _p(part), _p(w))
    return fl, part[:s], int(w[0])


@dataclass
class DecodeResult:
    flags: np.ndarray     # uint8 per shot (F_* bits)
    s: np.ndarray         # defects per shot
    partner: np.ndarray | None
    corr: np.ndarray | None

    @property
    def pred(self):
        return (self.flags & F_PRED) != 0

    @property
    def fail(self):
        return (self.flags & F_FAIL) != 0


def decode(dem: Dem, tab: Tables, syn: np.ndarray, obs: np.ndarray, n: int,
           max_iters: int, alpha: float = 1.0, variant: int = 0, threads: int | None = None,
           s_cap: int = 0, want_corr: bool = False,
           schedule: int = 0, fc_rule: int = 0, weight_rule: int = 0) -> DecodeResult:
    syn = np.ascontiguousarray(syn, dtype=np.uint64)
    obs = np.ascontiguousarray(obs, dtype=np.uint64)
    W = (n + 63) // 64
    assert syn.shape == (dem.n_det, W) and obs.shape == (W,)
    flags = np.zeros(max(n, 1), dtype=np.uint8)
    s_out = np.zeros(max(n, 1), dtype=np.int32)
    partner = np.full((max(n, 1), max(s_cap, 1)), -1, dtype=np.int32) if s_cap else None
    corr = np.zeros((dem.n_mech, max(W, 1)), dtype=np.uint64) if want_corr else None
    if threads is None:
        threads = os.cpu_count() or 1
    gd, gt = dem._c(), tab._c()
    o = _Opts(max_iters, variant, alpha, schedule, fc_rule, weight_rule)
    rc = lib().or_decode(C.byref(gd), C.byref(gt), _p(syn), _p(obs), n, C.byref(o), threads,
                         _p(flags), _p(s_out), _p(partner) if partner is not None else None,
                         s_cap, _p(corr) if corr is not None else None)
    if rc != 0:
        raise ValueError("or_decode failed")
    return DecodeResult(flags[:n], s_out[:n], partner[:n] if partner is not None else None,
                        corr[:, :W] if corr is not None else None)


# ------------------------------------- quaternary BP and B-BP4MF (Sec. II.E, III.D) --

F_OVERFLOW = 32
F_QBP = 64


@dataclass
class Tanner:
    """Both check types of a code-capacity code: qubit v's X checks qx[v],
    Z checks qz[v] (ascending, -1 = none), check c's qubits cq[c] (X checks
    first), qobs[v] (a Z error flips the observable) and qmech[v] (the
    code-capacity DEM mechanism that is v's Z error)."""
    n_xc: int
    n_zc: int
    qx: np.ndarray
    qz: np.ndarray
    qobs: np.ndarray
    qmech: np.ndarray
    cq: np.ndarray

    @property
    def n_q(self) -> int:
        return int(self.qobs.size)

    def _c(self) -> _Tanner:
        self._keep = [np.ascontiguousarray(a) for a in (self.qx, self.qz, self.qobs, self.qmech, self.cq)]
        qx, qz, qo, qm, cq = self._keep
        i32 = C.POINTER(C.c_int32)
        return _Tanner(self.n_q, self.n_xc, self.n_zc, qx.ctypes.data_as(i32), qz.ctypes.data_as(i32),
                       qo.ctypes.data_as(C.POINTER(C.c_uint8)), qm.ctypes.data_as(i32), cq.ctypes.data_as(i32))


def tanner(d: int, dem: Dem, unrotated: bool = False) -> Tanner:
    t = _Tanner()
    gd = dem._c()
    rc = lib().or_build_tanner_code_capacity(d, int(unrotated), C.byref(gd), C.byref(t))
    if rc != 0:
        raise ValueError("or_build_tanner_code_capacity failed (%d)" % rc)
    nq, nc = t.n_q, t.n_xc + t.n_zc
    def take(ptr, shape, dt):
        return np.ctypeslib.as_array(ptr, shape=shape).astype(dt, copy=True)
    out = Tanner(t.n_xc, t.n_zc, take(t.qx, (nq, 2), np.int32), take(t.qz, (nq, 2), np.int32),
                 take(t.qobs, (nq,), np.uint8), take(t.qmech, (nq,), np.int32), take(t.cq, (nc, 4), np.int32))
    lib().or_tanner_free(C.byref(t))
    return out


def tables_w(dem: Dem, w) -> Tables:
    """Path tables with the given fixed-point mechanism weights."""
    w = np.ascontiguousarray(w, dtype=np.int64)
    assert w.shape == (dem.n_mech,)
    t = _Tables()
    gd = dem._c()
    rc = lib().or_build_tables_w(C.byref(gd), _p(w), C.byref(t))
    if rc != 0:
        raise ValueError("or_build_tables_w failed (%d)" % rc)
    N = t.n
    def take(ptr, dt):
        return np.ctypeslib.as_array(ptr, shape=(N, N)).astype(dt, copy=True)
    out = Tables(take(t.dist, np.int64), take(t.hops, np.int32), take(t.par, np.uint8),
                 take(t.pred, np.int32), take(t.llr, np.float64))
    lib().or_tables_free(C.byref(t))
    return out


def spec_log(x: float) -> float:
    return lib().or_spec_log(float(x))


def spec_prior(dist_fixed: int) -> float:
    return lib().or_spec_prior(int(dist_fixed))


def qbp_weight(P: float) -> int:
    return lib().or_qbp_weight(float(P))


def qbp_zprob(L) -> float:
    L = np.ascontiguousarray(L, dtype=np.float64)
    assert L.shape == (4,)
    return lib().or_qbp_zprob(_p(L))


def sample_depolarizing(T: Tanner, p: float, seed: int, shot0: int, n: int):
    """Bit planes synx[n_xc, W], synz[n_zc, W] and obs[W] (Z part on the
    observable qubits) of depolarizing noise on every qubit."""
    W = (n + 63) // 64
    sx = np.zeros((T.n_xc, max(W, 1)), dtype=np.uint64)
    sz = np.zeros((T.n_zc, max(W, 1)), dtype=np.uint64)
    ob = np.zeros(max(W, 1), dtype=np.uint64)
    gt = T._c()
    lib().or_sample_depolarizing(C.byref(gt), p, seed, shot0, n, _p(sx), _p(sz), _p(ob))
    return sx[:, :W], sz[:, :W], ob[:W]


def qbp(T: Tanner, p: float, zx, zz, max_iters: int, stop: bool = True):
    """Quaternary BP on one shot: (converged, iterations, hard[n_q] in
    0..3 = I, X, Y, Z, log-posteriors[n_q, 4]); stop=False runs all
    max_iters iterations."""
    zx = np.ascontiguousarray(zx, dtype=np.uint8)
    zz = np.ascontiguousarray(zz, dtype=np.uint8)
    hard = np.zeros(T.n_q, dtype=np.uint8)
    post = np.zeros((T.n_q, 4), dtype=np.float64)
    it = C.c_int(0)
    gt = T._c()
    conv = lib().or_qbp(C.byref(gt), p, _p(zx), _p(zz), max_iters, int(stop), C.byref(it), _p(hard), _p(post))
    return bool(conv), it.value, hard, post


def bbp4mf_decode(dem: Dem, T: Tanner, p: float, synx, synz, obs, n: int, max_iters: int,
                  alpha: float = 1.0, s_cap: int = 0, threads: int | None = None, variant: int = 1) -> DecodeResult:
    """B-BP4MF (quaternary BP, then BP4MF on re-weighted paths) of n shots."""
    synx = np.ascontiguousarray(synx, dtype=np.uint64)
    synz = np.ascontiguousarray(synz, dtype=np.uint64)
    obs = np.ascontiguousarray(obs, dtype=np.uint64)
    s_cap = s_cap or dem.n_det
    flags = np.zeros(max(n, 1), dtype=np.uint8)
    s_out = np.zeros(max(n, 1), dtype=np.int32)
    partner = np.full((max(n, 1), s_cap), -1, dtype=np.int32)
    if threads is None:
        threads = os.cpu_count() or 1
    gd, gt = dem._c(), T._c()
    o = _Opts(max_iters, variant, alpha)
    lib().or_bbp4mf_decode(C.byref(gd), C.byref(gt), p, _p(synx), _p(synz), _p(obs), n, C.byref(o),
                           threads, _p(flags), _p(s_out), _p(partner), s_cap)
    if (flags[:n] == 0xFF).any():
        raise ValueError("or_bbp4mf_decode failed")
    return DecodeResult(flags[:n], s_out[:n], partner[:n], None)
