"""GPU parity of libbpm against the FP64 oracle, through the C ABI.

 - Sampler: detector and observable bit planes bit-exact.
 - FP64 fixed-order decoding: per-shot flags, matchings, correction planes,
   predictions and failures bit-exact (BP4M and BP4MF, memory factor).
 - FP32 decoding: posteriors after t iterations within the stated tolerance,
   and whole-decoder agreement / logical error rate within the binomial
   interval of the oracle on the same syndromes.
 - Edge cases: empty and ragged batches, s = 0 / 1 shots, s above s_cap,
   the largest class sizes.
"""
import numpy as np
import pytest

import oracle
from tests.inputs import WORKLOADS, seed_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2603_05381_amd as bpm


def np64(t):
    return t.cpu().numpy().view(np.uint64)


def unpack(planes, n):
    bits = np.unpackbits(np.ascontiguousarray(planes).view(np.uint8), axis=-1, bitorder="little")
    return bits[..., :n].astype(bool)


_GRAPHS = {}


def graph_pair(kind, d, rounds, p):
    key = (kind, d, rounds, p)
    if key not in _GRAPHS:
        g = bpm.Graph(kind, d, p, rounds)
        if kind.startswith("memory_z"):
            ref = oracle.memory_z(d, rounds, p, unrotated=kind.endswith("_unrotated"))
        else:
            ref = oracle.code_capacity(d, p, unrotated=kind.endswith("_unrotated"))
        _GRAPHS[key] = (g, ref, oracle.tables(ref))
    return _GRAPHS[key]


# ------------------------------------------------------------------ sampler

@pytest.mark.parametrize("kind,d,rounds,p,seed,shot0,n", [
    ("code_capacity", 3, 1, 0.05, seed_for(0, 3, 0.05), 0, 10_000),
    ("code_capacity", 7, 1, 0.1, 7, 1000, 5_003),
    ("memory_z", 5, 5, 0.005, seed_for(2, 5, 0.005), 0, 3_001),
    ("memory_z", 13, 13, 0.005, seed_for(2, 13, 0.005), 123_456_789_000, 700),
    ("memory_z", 3, 3, 0.02, 5, 0, 1),
    ("memory_z_unrotated", 5, 5, 0.005, seed_for(2, 5, 0.005), 0, 2_001),
    ("memory_z_unrotated", 9, 9, 0.004, 3, 77, 500),
])
def test_sampler_bit_exact(kind, d, rounds, p, seed, shot0, n):
    g, ref, _ = graph_pair(kind, d, rounds, p)
    syn, obs = g.sample(seed, shot0, n)
    torch.cuda.synchronize()
    rs, ro = oracle.sample(ref, seed, shot0, n)
    assert np.array_equal(np64(syn)[:, :rs.shape[1]], rs)
    assert np.array_equal(np64(obs)[:ro.shape[0]], ro)


# ------------------------------------------------------- FP64 fixed order

def spec_compare(kind, d, rounds, p, seed, shot0, n, T, variant=0, alpha=1.0, syn_obs=None):
    g, ref, tab = graph_pair(kind, d, rounds, p)
    if syn_obs is None:
        syn, obs = g.sample(seed, shot0, n)
        rs, ro = oracle.sample(ref, seed, shot0, n)
    else:
        rs, ro = syn_obs
        syn = torch.from_numpy(rs.view(np.int64).copy()).cuda()
        obs = torch.from_numpy(ro.view(np.int64).copy()).cuda()
    res = g.decode(syn, obs, n, T, precision=bpm.BPM_FP64_SPEC, variant=variant, alpha=alpha,
                   s_cap=ref.n_det if ref.n_det <= 1024 else 1024, want_corr=True, want_match=True)
    torch.cuda.synchronize()
    s_cap = res["match"].shape[1]
    r = oracle.decode(ref, tab, rs, ro, n, T, alpha=alpha, variant=variant, s_cap=s_cap, want_corr=True)
    gs = res["s"].cpu().numpy()[:n]
    assert np.array_equal(gs, r.s)
    gf = res["flags"].cpu().numpy()[:n]
    bad = np.nonzero(gf != r.flags)[0]
    assert bad.size == 0, ("flags differ", bad[:10], gf[bad[:10]], r.flags[bad[:10]], r.s[bad[:10]])
    gm = res["match"].cpu().numpy()[:n]
    for b in range(n):
        s = r.s[b]
        assert np.array_equal(gm[b, :s], r.partner[b, :s]), (b, s)
    W = (n + 63) // 64
    assert np.array_equal(np64(res["corr"])[:, :W], r.corr)
    assert np.array_equal(unpack(np64(res["obs_pred"])[:W], n), r.pred)
    assert np.array_equal(unpack(np64(res["fail"])[:W], n), r.fail)
    c = bpm.counters_dict(res["counters"])
    assert c["shots"] == n and c["failures"] == int(r.fail.sum()) and c["sum_s"] == int(r.s.sum())
    assert c["fc_chosen"] == int(((r.flags & oracle.F_FC_CHOSEN) != 0).sum())
    nc = int(((r.s >= 2) & ((r.flags & oracle.F_CONVERGED_ANY) == 0)).sum())
    assert c["never_converged"] == nc and c["overflow"] == 0
    return r


def test_spec_c1_sampled_and_exhaustive():
    kind, d, rounds, p, T, n = WORKLOADS["cc_d3"]
    r = spec_compare(kind, d, rounds, p, seed_for(0, d, p), 0, n, T)
    assert r.fail.sum() > 0
    # all 16 syndromes of the d = 3 graph
    n = 16
    syn = np.zeros((4, 1), dtype=np.uint64)
    for b in range(16):
        for k in range(4):
            if (b >> k) & 1:
                syn[k, 0] |= np.uint64(1) << np.uint64(b)
    spec_compare(kind, d, rounds, p, 0, 0, n, T, syn_obs=(syn, np.zeros(1, dtype=np.uint64)))


@pytest.mark.parametrize("kind,d,rounds,p,n,T", [
    ("code_capacity", 5, 1, 0.1, 2000, 25),
    ("code_capacity", 11, 1, 0.12, 300, 25),
    ("code_capacity_unrotated", 5, 1, 0.1, 2000, 25),
    ("code_capacity_unrotated", 11, 1, 0.12, 300, 25),
    ("memory_z", 5, 5, 0.005, 1000, 50),
    ("memory_z", 7, 7, 0.008, 120, 50),
    ("memory_z_unrotated", 3, 3, 0.01, 2000, 50),
    ("memory_z_unrotated", 5, 5, 0.006, 300, 50),
])
def test_spec_bit_exact(kind, d, rounds, p, n, T):
    spec_compare(kind, d, rounds, p, seed_for(1, d, p), 0, n, T)


def test_spec_headline_d13_sample():
    # circuit-level d = 13, d rounds, p = 0.005: a few shots at full size
    spec_compare("memory_z", 13, 13, 0.005, seed_for(2, 13, 0.005), 0, 24, 50)


@pytest.mark.parametrize("variant,alpha", [(1, 1.0), (0, 0.85), (1, 0.85)])
def test_spec_bp4mf_and_memory(variant, alpha):
    spec_compare("code_capacity", 7, 1, 0.12, 11, 0, 400, 25, variant=variant, alpha=alpha)
    spec_compare("code_capacity_unrotated", 7, 1, 0.12, 11, 0, 300, 25, variant=variant, alpha=alpha)
    spec_compare("memory_z", 5, 5, 0.008, 12, 0, 150, 30, variant=variant, alpha=alpha)


def test_spec_edge_cases():
    # ragged batch sizes around a word boundary, and a single shot
    for n in (1, 63, 65):
        spec_compare("code_capacity", 5, 1, 0.08, 3, 17, n, 10)
    # empty batch: nothing is written
    g, ref, tab = graph_pair("code_capacity", 5, 1, 0.08)
    syn, obs = g.sample(3, 0, 64)
    res = g.decode(syn, obs, 0, 10, precision=bpm.BPM_FP64_SPEC)
    torch.cuda.synchronize()
    assert bpm.counters_dict(res["counters"])["shots"] == 0


def test_overflow_is_flagged_not_decoded():
    g, ref, tab = graph_pair("memory_z", 5, 5, 0.02)
    n = 500
    syn, obs = g.sample(9, 0, n)
    res = g.decode(syn, obs, n, 5, precision=bpm.BPM_FP32, s_cap=8)
    torch.cuda.synchronize()
    s = res["s"].cpu().numpy()[:n]
    f = res["flags"].cpu().numpy()[:n]
    assert (s > 8).any()
    assert np.all(((f & bpm.SHOT_OVERFLOW) != 0) == (s > 8))
    assert bpm.counters_dict(res["counters"])["overflow"] == int((s > 8).sum())


@pytest.mark.parametrize("s_cap", [10, 11, 12, 13])
def test_defect_rows_any_capacity(s_cap):
    # defect rows whose length is a multiple of four are written four
    # defects at a time, others one at a time: both give the oracle's lists
    # (seen through its matchings and verdicts) on the shots that fit
    g, ref, tab = graph_pair("memory_z", 5, 5, 0.012)
    n, T = 400, 8
    seed = seed_for(11, 5, 0.012)
    syn, obs = g.sample(seed, 0, n)
    res = g.decode(syn, obs, n, T, precision=bpm.BPM_FP64_SPEC, s_cap=s_cap, want_match=True)
    torch.cuda.synchronize()
    rs, ro = oracle.sample(ref, seed, 0, n)
    r = oracle.decode(ref, tab, rs, ro, n, T, s_cap=s_cap)
    gs = res["s"].cpu().numpy()[:n]
    gf = res["flags"].cpu().numpy()[:n]
    gm = res["match"].cpu().numpy()[:n]
    assert np.array_equal(gs, r.s)
    fit = r.s <= s_cap
    assert fit.any() and (~fit).any()
    assert np.all(((gf & bpm.SHOT_OVERFLOW) != 0) == ~fit)
    assert np.array_equal(gf[fit], r.flags[fit])
    for b in np.nonzero(fit)[0]:
        assert np.array_equal(gm[b, :r.s[b]], r.partner[b, :r.s[b]]), (b, r.s[b])


# ------------------------------------------------------------------ FP32

def fp32_posteriors(kind, d, rounds, p, seed, n, T, stride):
    g, ref, tab = graph_pair(kind, d, rounds, p)
    syn, obs = g.sample(seed, 0, n)
    res = g.decode(syn, obs, n, T, precision=bpm.BPM_FP32, lambda_stride=stride)
    torch.cuda.synchronize()
    rs, ro = oracle.sample(ref, seed, 0, n)
    lam = res["lambda"].cpu().numpy()
    s_all = res["s"].cpu().numpy()[:n]
    det = unpack(rs, n)
    worst = 0.0
    checked = 0
    for b in range(n):
        s = int(s_all[b])
        if s < 2 or s > stride:
            continue
        dd = np.nonzero(det[:, b])[0]
        L = tab.llr[np.ix_(dd, dd)]
        W = tab.dist[np.ix_(dd, dd)]
        _, _, _, _, lref = oracle.bp4m_instance(L, W, max_iters=T)
        got = lam[b, :s, :s]
        err = np.abs(got - lref) / (1.0 + np.abs(lref))
        worst = max(worst, float(err.max()))
        checked += 1
    return worst, checked, s_all


@pytest.mark.parametrize("kind,d,rounds,p,T,tol", [
    ("code_capacity", 9, 1, 0.1, 1, 2e-6),
    ("code_capacity", 9, 1, 0.1, 3, 1e-5),
    ("memory_z", 7, 7, 0.01, 2, 1e-5),
    ("memory_z", 9, 9, 0.008, 2, 1e-5),
    ("memory_z_unrotated", 7, 7, 0.006, 2, 1e-5),
])
def test_fp32_posteriors_within_tolerance(kind, d, rounds, p, T, tol):
    worst, checked, s_all = fp32_posteriors(kind, d, rounds, p, 21, 300, T, 200)
    assert checked > 50
    assert worst <= tol, worst


def test_fp32_classes_all_exercised():
    # shots spread over every size class (2..16, ..., 97..128, > 128)
    worst, checked, s_all = fp32_posteriors("memory_z", 13, 13, 0.008, 22, 160, 2, 256)
    assert (s_all > 128).any() and ((s_all > 96) & (s_all <= 128)).any()
    assert worst <= 1e-5, worst


def test_fp32_global_slot_classes_within_tolerance():
    # d=17: shots with 193..256 defects run in the classes whose tiles and
    # priors live in global memory
    worst, checked, s_all = fp32_posteriors("memory_z", 17, 17, 0.006, 24, 120, 2, 260)
    big = (s_all > 192) & (s_all <= 256)
    assert big.sum() > 20 and (s_all <= 224).any() and (s_all > 224).any()
    assert worst <= 1e-5, worst


def test_fp32_stream_class_within_tolerance():
    # d=15 at p=0.012: shots with 257..512 defects run in the streaming class
    worst, checked, s_all = fp32_posteriors("memory_z", 15, 15, 0.012, 25, 60, 2, 420)
    big = (s_all > 256) & (s_all <= 420)
    assert big.sum() > 20
    assert worst <= 1e-5, worst


def test_fp32_stream_class_at_d21_full_size():
    # the largest graph of the mixed-distance batch (d = 21, 21 rounds, 4840
    # detectors; mean s ~ 380): a sample of its shots, decoded in the
    # streaming class's launch configuration, against the oracle's messages
    worst, checked, s_all = fp32_posteriors("memory_z", 21, 21, 0.005, 5, 12, 2, 512)
    assert checked >= 10 and (s_all[:12] > 256).sum() >= 10
    assert worst <= 1e-5, worst


@pytest.mark.parametrize("kind,d,rounds,p,n,T", [
    ("code_capacity", 9, 1, 0.1, 4000, 25),
    ("code_capacity_unrotated", 9, 1, 0.1, 3000, 25),
    ("memory_z", 9, 9, 0.006, 600, 50),
    ("memory_z", 17, 17, 0.006, 200, 30),
    ("memory_z", 15, 15, 0.012, 150, 20),
    ("memory_z_unrotated", 7, 7, 0.005, 800, 50),
    ("memory_z_unrotated", 11, 11, 0.005, 150, 50),
])
def test_fp32_decoder_agrees_with_oracle(kind, d, rounds, p, n, T):
    g, ref, tab = graph_pair(kind, d, rounds, p)
    seed = seed_for(3, d, p)
    syn, obs = g.sample(seed, 0, n)
    res = g.decode(syn, obs, n, T, precision=bpm.BPM_FP32)
    torch.cuda.synchronize()
    rs, ro = oracle.sample(ref, seed, 0, n)
    r = oracle.decode(ref, tab, rs, ro, n, T)
    W = (n + 63) // 64
    gfail = unpack(np64(res["fail"])[:W], n)
    gpred = unpack(np64(res["obs_pred"])[:W], n)
    disc = int((gpred != r.pred).sum())
    assert disc <= max(3, 0.02 * n), disc
    # logical error rates within the binomial interval of the oracle's
    pf = r.fail.mean()
    sd = np.sqrt(max(pf * (1 - pf), 1.0 / n) / n)
    assert abs(gfail.mean() - pf) <= 4 * sd + 2.0 / n


# --------------------------------------------- reduced-precision storage

# unit roundoff of the storage formats (round to nearest even)
U_STORE = {2: 2.0 ** -8, 3: 2.0 ** -11}       # BPM_BF16_STORE, BPM_FP16_STORE


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("kind,d,rounds,p,n,stride,min_big", [
    ("code_capacity", 9, 1, 0.1, 200, 200, 0),
    ("memory_z", 9, 9, 0.008, 200, 200, 0),
    # shots with 257..420 defects: the streaming class
    ("memory_z", 15, 15, 0.012, 60, 420, 20),
])
def test_reduced_storage_posteriors_after_one_iteration(prec, kind, d, rounds, p, n, stride, min_big):
    # After iteration 1 each stored message is the FP32 message rounded once,
    # so |lambda_ij - lambda_ref| <= u (|M'ij| + |M'ji|) (u the format's unit
    # roundoff), plus the FP32 arithmetic's own error.
    assert prec in (bpm.BPM_BF16_STORE, bpm.BPM_FP16_STORE)
    u = U_STORE[prec]
    g, ref, tab = graph_pair(kind, d, rounds, p)
    syn, obs = g.sample(23, 0, n)
    res = g.decode(syn, obs, n, 1, precision=prec, lambda_stride=stride)
    torch.cuda.synchronize()
    rs, ro = oracle.sample(ref, 23, 0, n)
    lam = res["lambda"].cpu().numpy()
    s_all = res["s"].cpu().numpy()[:n]
    det = unpack(rs, n)
    checked, big, worst = 0, 0, 0.0
    for b in range(n):
        s = int(s_all[b])
        if s < 2 or s > stride:
            continue
        dd = np.nonzero(det[:, b])[0]
        _, _, _, M, lref = oracle.bp4m_instance(tab.llr[np.ix_(dd, dd)], tab.dist[np.ix_(dd, dd)], max_iters=1)
        aM = np.abs(M)
        mag = aM + aM.T
        np.fill_diagonal(mag, np.diag(aM))
        bound = u * mag + 4e-6 * mag + 2e-6 * (1.0 + np.abs(lref))
        err = np.abs(lam[b, :s, :s] - lref)
        worst = max(worst, float((err / bound).max()))
        checked += 1
        big += s > 256
    assert checked > min(50, n // 2)
    assert big >= min_big
    assert worst <= 1.0, worst


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("kind,d,rounds,p,n,T", [
    ("code_capacity", 9, 1, 0.1, 4000, 25),
    ("memory_z", 9, 9, 0.006, 600, 50),
    ("memory_z", 17, 17, 0.006, 200, 30),
    ("memory_z", 15, 15, 0.012, 150, 20),
])
def test_reduced_storage_decoder_agrees_with_oracle(prec, kind, d, rounds, p, n, T):
    # logical error rate within the binomial interval of the FP64 oracle's on
    # the same syndromes, and few paired disagreements
    g, ref, tab = graph_pair(kind, d, rounds, p)
    seed = seed_for(3, d, p)
    syn, obs = g.sample(seed, 0, n)
    res = g.decode(syn, obs, n, T, precision=prec)
    torch.cuda.synchronize()
    rs, ro = oracle.sample(ref, seed, 0, n)
    r = oracle.decode(ref, tab, rs, ro, n, T)
    W = (n + 63) // 64
    gfail = unpack(np64(res["fail"])[:W], n)
    gpred = unpack(np64(res["obs_pred"])[:W], n)
    disc = int((gpred != r.pred).sum())
    assert disc <= max(5, 0.05 * n), disc
    pf = r.fail.mean()
    sd = np.sqrt(max(pf * (1 - pf), 1.0 / n) / n)
    assert abs(gfail.mean() - pf) <= 4 * sd + 2.0 / n


def test_fp32_deterministic_and_batch_independent():
    g, ref, tab = graph_pair("memory_z", 7, 7, 0.008)
    n = 777
    syn, obs = g.sample(31, 0, n)
    a = g.decode(syn, obs, n, 20, precision=bpm.BPM_FP32, want_match=True)
    b = g.decode(syn, obs, n, 20, precision=bpm.BPM_FP32, want_match=True)
    # the same shots inside a larger batch (shifted by 100 shots)
    syn2, obs2 = g.sample(31, 0, n + 100)
    torch.cuda.synchronize()
    assert torch.equal(a["flags"], b["flags"]) and torch.equal(a["match"], b["match"])
    c = g.decode(syn2, obs2, n + 100, 20, precision=bpm.BPM_FP32, want_match=True)
    torch.cuda.synchronize()
    assert torch.equal(a["flags"][:n], c["flags"][:n]) and torch.equal(a["match"][:n], c["match"][:n])


# ------------------------------------------------- kernel configurations

def _with_config(cfg, fn):
    old = bpm.bpm_get_stage_config()
    try:
        bpm.bpm_set_stage_config(cfg)
        return fn()
    finally:
        bpm.bpm_set_stage_config(old)


@pytest.mark.parametrize("kind,d,rounds,p,n", [
    # d=13 at p=0.005: most shots have 65..128 defects
    ("memory_z", 13, 13, 0.005, 1500),
    # code capacity d=11 at p=0.1 and d=15 at p=0.14: shots of 2..48 defects
    # (the small classes, whose configurations also change the shots per
    # workgroup)
    ("code_capacity", 11, 1, 0.1, 6000),
    ("code_capacity", 15, 1, 0.14, 6000),
])
def test_fp32_every_kernel_configuration_gives_identical_results(kind, d, rounds, p, n):
    # Every configuration of a class with a choice of kernels must give the
    # default's flags and matchings on that class's shots; BP4M and BP4MF.
    g, ref, tab = graph_pair(kind, d, rounds, p)
    syn, obs = g.sample(seed_for(2, d, p), 10_000, n)
    counts = [bpm.bpm_stage_configs(k) for k in range(len(bpm.STAGES))]
    assert max(counts) > 1
    bad = []
    exercised = 0
    for variant, T, prec in ((bpm.BPM_BP4M, 30, bpm.BPM_FP32), (bpm.BPM_BP4MF, 8, bpm.BPM_FP32),
                             (bpm.BPM_BP4M, 30, bpm.BPM_BF16_STORE)):
        runs = []
        for c in range(max(counts)):
            cfg = [min(c, m - 1) for m in counts]
            r = _with_config(cfg, lambda: g.decode(syn, obs, n, T, precision=prec, variant=variant,
                                                   want_match=True))
            torch.cuda.synchronize()
            runs.append({k: v.cpu().numpy() for k, v in r.items()})
        again = _with_config([0] * bpm.BPM_MAX_STAGES,
                             lambda: g.decode(syn, obs, n, T, precision=prec, variant=variant,
                                              want_match=True))
        torch.cuda.synchronize()
        rerun = (again["flags"].cpu().numpy()[:n] != runs[0]["flags"][:n])
        if rerun.any():
            bad.append((variant, prec, "rerun of configuration 0", 0, int(rerun.sum()), n))
        s = runs[0]["s"][:n]
        for k in range(1, len(counts) - 1):
            lo, hi = (bpm.STAGE_MAX_S[k - 1] if k > 1 else 1) + 1, bpm.STAGE_MAX_S[k]
            sel = (s >= lo) & (s <= hi)
            if counts[k] > 1 and sel.sum() >= 20:
                exercised += 1
            for c in range(1, counts[k]):
                df = (runs[c]["flags"][:n] != runs[0]["flags"][:n]) | (runs[c]["match"][:n] != runs[0]["match"][:n]).any(axis=1)
                if (df & sel).any():
                    bad.append((variant, prec, bpm.STAGES[k], c, int((df & sel).sum()), int(sel.sum())))
    assert not bad, bad
    assert exercised >= 2 * 3, exercised       # two multi-configuration classes or more, each run
def test_autotune_measures_and_chooses_a_valid_configuration():
    g, ref, tab = graph_pair("memory_z", 9, 9, 0.008)
    old = bpm.bpm_get_stage_config()
    try:
        opts = bpm.bpm_decode_opts(20, bpm.BPM_BP4M, bpm.BPM_FP32, 0, 1.0)
        t = bpm.bpm_autotune(g.handle, opts, 20_000, 77, torch.cuda.current_stream().cuda_stream)
        cfg = bpm.bpm_get_stage_config()
        for k in range(len(bpm.STAGES)):
            m = bpm.bpm_stage_configs(k)
            assert 0 <= cfg[k] < m
            assert all(t[c][k] >= 0 for c in range(m)), (k, t)
            assert all(t[c][k] == -1 for c in range(m, bpm.BPM_MAX_CONFIGS))
            if m > 1:
                assert t[cfg[k]][k] == min(t[c][k] for c in range(m))
        # FP64 fixed order: a single kernel, nothing timed or changed
        t64 = bpm.bpm_autotune(g.handle, bpm.bpm_decode_opts(5, 0, bpm.BPM_FP64_SPEC, 0, 1.0), 1000, 1,
                               torch.cuda.current_stream().cuda_stream)
        assert all(x == -1 for row in t64 for x in row) and bpm.bpm_get_stage_config() == cfg
        # decoding still matches the oracle-agreeing default path
        n = 500
        syn, obs = g.sample(5, 0, n)
        a = g.decode(syn, obs, n, 20, precision=bpm.BPM_FP32, want_match=True)
        b = _with_config([0] * bpm.BPM_MAX_STAGES,
                         lambda: g.decode(syn, obs, n, 20, precision=bpm.BPM_FP32, want_match=True))
        torch.cuda.synchronize()
        assert torch.equal(a["flags"][:n], b["flags"][:n]) and torch.equal(a["match"][:n], b["match"][:n])
    finally:
        bpm.bpm_set_stage_config(old)


# ------------------------------------------------- several graphs per call

MULTI = [("code_capacity", 5, 1, 0.08, 700), ("memory_z", 5, 5, 0.006, 500), ("memory_z", 9, 9, 0.006, 400),
         ("memory_z", 13, 13, 0.005, 300)]


@pytest.mark.parametrize("precision,T", [(1, 30), (0, 20), (2, 30)])
def test_multi_instance_call_matches_separate_calls(precision, T):
    parts, singles = [], []
    for kind, d, rounds, p, n in MULTI:
        g, ref, tab = graph_pair(kind, d, rounds, p)
        syn, obs = g.sample(seed_for(4, d, p), 0, n)
        parts.append((g, syn, obs, n))
    s_cap = 512
    for g, syn, obs, n in parts:
        singles.append(g.decode(syn, obs, n, T, precision=precision, s_cap=s_cap, want_match=True))
    multi = bpm.decode_multi(parts, T, precision=precision, s_cap=s_cap, want_match=True)
    torch.cuda.synchronize()
    for (g, syn, obs, n), a, b in zip(parts, singles, multi):
        W = (n + 63) // 64
        assert torch.equal(a["flags"][:n], b["flags"][:n])
        assert torch.equal(a["match"][:n], b["match"][:n])
        assert torch.equal(a["obs_pred"][:W], b["obs_pred"][:W]) and torch.equal(a["fail"][:W], b["fail"][:W])
        assert torch.equal(a["counters"], b["counters"])


def test_shot_major_rows_input_matches_bit_planes():
    g, ref, tab = graph_pair("memory_z", 9, 9, 0.008)
    n = 333
    syn, obs = g.sample(41, 5, n)
    planes = g.decode(syn, obs, n, 25, want_match=True)
    # rows[b] = the shot's detector bits, from the planes on the host
    bits = unpack(np64(syn), n)                             # [N][n]
    words = (g.n_det + 63) // 64 + 1                        # one spare word
    packed = np.zeros((n, words * 64), dtype=bool)
    packed[:, :g.n_det] = bits.T
    rows = np.packbits(packed, axis=1, bitorder="little").view(np.int64)
    rows_t = torch.from_numpy(rows.copy()).cuda()
    (r,) = bpm.decode_multi([(g, rows_t, None, n)], 25, want_match=True)
    torch.cuda.synchronize()
    keep = ~np.uint8(bpm.SHOT_FAIL)                        # no sampled flips given
    fa = planes["flags"].cpu().numpy()[:n] & keep
    fb = r["flags"].cpu().numpy()[:n] & keep
    assert np.array_equal(fa, fb)
    assert torch.equal(planes["match"][:n], r["match"][:n])
    W = (n + 63) // 64
    assert torch.equal(planes["obs_pred"][:W], r["obs_pred"][:W])
    # failures are counted against an observable flip of 0: the predictions
    assert torch.equal(r["fail"][:W], r["obs_pred"][:W])


def test_concurrent_class_streams_give_identical_results():
    # size classes spread over 4 streams: same flags, matchings, counters
    g, ref, tab = graph_pair("memory_z", 17, 17, 0.005)
    n = 600
    syn, obs = g.sample(seed_for(4, 17, 0.005), 0, n)
    a = g.decode(syn, obs, n, 20, want_match=True)
    b = g.decode(syn, obs, n, 20, want_match=True, class_streams=4)
    c = g.decode(syn, obs, n, 20, want_match=True, class_streams=8, precision=bpm.BPM_BF16_STORE)
    d = g.decode(syn, obs, n, 20, want_match=True, precision=bpm.BPM_BF16_STORE)
    torch.cuda.synchronize()
    assert torch.equal(a["flags"][:n], b["flags"][:n]) and torch.equal(a["match"][:n], b["match"][:n])
    assert torch.equal(a["counters"], b["counters"])
    assert torch.equal(c["flags"][:n], d["flags"][:n]) and torch.equal(c["match"][:n], d["match"][:n])
