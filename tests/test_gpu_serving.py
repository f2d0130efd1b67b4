"""Decode server (continuous batching) on the GPU: every request's result is
the same alone, in a mix of concurrent requests of several graphs, and as
the plain batch decoder gives it for the same shots (FP32, bit for bit:
each shot's result depends only on its own syndrome)."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2603_05381_amd as bpm

T = 30
DISTANCES = (5, 9, 13)


def pools(n):
    out = []
    for d in DISTANCES:
        g = bpm.Graph("memory_z", d, 0.005, d)
        syn, obs = g.sample(1000 + d, 0, n)
        ref = g.decode(syn, obs, n, T, precision=bpm.BPM_FP32)
        torch.cuda.synchronize()
        flags = ref["flags"].cpu().numpy()[:n]
        pred = (flags & bpm.SHOT_PRED) != 0
        out.append((g, bpm.planes_to_rows(syn, n, g.n_det), pred))
    return out


def make_requests(n_req, pool_n, seed):
    rng = np.random.default_rng(seed)
    cursor = [0] * len(DISTANCES)
    reqs = []
    for r in range(n_req):
        gi = int(rng.integers(len(DISTANCES)))
        k = int(rng.integers(1, 65))
        if cursor[gi] + k > pool_n:
            cursor[gi] = 0
        reqs.append((r, gi, cursor[gi], k))
        cursor[gi] += k
    return reqs


def expected_bits(pred, a, k):
    return int(sum(1 << i for i in range(k) if pred[a + i]))


def run(server, P, reqs, one_at_a_time=False, deadline_s=120.0):
    got = {}
    t_end = time.time() + deadline_s
    i = 0
    while len(got) < len(reqs):
        assert time.time() < t_end, "server did not finish in time"
        if i < len(reqs) and (not one_at_a_time or len(got) == i):
            rid, gi, a, k = reqs[i]
            if server.submit(gi, P[gi][1][a:a + k], rid):
                i += 1
        for res in server.poll():
            got[res[0]] = res
        if one_at_a_time or i == len(reqs):
            time.sleep(0.0002)
    return got


@pytest.mark.parametrize("use_graphs,one_graph", [(False, False), (True, False), (False, True), (True, True)])
def test_server_results_same_alone_and_in_mix(use_graphs, one_graph):
    n = 3000
    P = pools(n)
    reqs = make_requests(500, n, 7)
    srv = bpm.Server([p[0] for p in P], T, max_batch_shots=1024, max_pending_shots=1 << 14, slots=3,
                     use_graphs=use_graphs, one_graph_per_batch=one_graph)
    try:
        mix = run(srv, P, reqs)
        st = srv.stats()
    finally:
        srv.close()
    assert st["requests_done"] == len(reqs) and st["batches"] >= 1
    for rid, gi, a, k in reqs:
        r = mix[rid]
        assert r[1] == gi and r[2] == k and r[5] == 0
        assert r[3] == expected_bits(P[gi][2], a, k), (rid, gi, a, k)
        assert r[6] > 0.0
    # the same requests alone, each one in its own batch
    alone_srv = bpm.Server([p[0] for p in P], T, max_batch_shots=256, slots=1, use_graphs=use_graphs)
    try:
        alone = run(alone_srv, P, reqs[:40], one_at_a_time=True)
        st = alone_srv.stats()
    finally:
        alone_srv.close()
    assert st["batches"] == 40
    for rid, gi, a, k in reqs[:40]:
        assert alone[rid][3] == mix[rid][3] and alone[rid][4] == mix[rid][4]


def test_server_rejects_bad_requests():
    g = bpm.Graph("memory_z", 5, 0.005, 5)
    srv = bpm.Server([g], T, max_batch_shots=128, slots=1)
    try:
        words = (g.n_det + 63) // 64
        with pytest.raises(bpm.BpmError, match="1 to 64"):
            srv.submit(0, np.zeros((65, words), dtype=np.uint64), 1)
        with pytest.raises(bpm.BpmError, match="graph index"):
            srv.submit(3, np.zeros((2, words), dtype=np.uint64), 1)
        # an empty syndrome decodes to "no flip"
        assert srv.submit(0, np.zeros((5, words), dtype=np.uint64), 9)
        t_end = time.time() + 30
        res = []
        while not res:
            assert time.time() < t_end
            res = srv.poll()
            time.sleep(0.001)
        assert res[0][0] == 9 and res[0][3] == 0
    finally:
        srv.close()


def test_server_admits_by_device_memory():
    # mem_budget: the slots' buffers plus the device bytes of every queued
    # request's shots must fit; a budget below the slots is refused at
    # creation, and a tight one turns a burst of requests partly away
    # (BPM_EAGAIN) while every admitted request still gets its own result
    import re
    n = 2000
    P = pools(n)
    gs = [p[0] for p in P]
    with pytest.raises(bpm.BpmError, match="mem_budget"):
        bpm.Server(gs, T, max_batch_shots=256, slots=1, mem_budget=1)
    need = int(re.search(r"the (\d+) bytes", bpm.lib().bpm_last_error().decode()).group(1))
    srv = bpm.Server(gs, T, max_batch_shots=256, slots=1, mem_budget=need + 300_000)
    reqs = make_requests(300, n, 11)
    admitted, refused = [], 0
    try:
        for rid, gi, a, k in reqs:
            if srv.submit(gi, P[gi][1][a:a + k], rid):
                admitted.append((rid, gi, a, k))
            else:
                refused += 1
        got = {}
        t_end = time.time() + 60
        while len(got) < len(admitted):
            assert time.time() < t_end, "server did not finish in time"
            for res in srv.poll():
                got[res[0]] = res
            time.sleep(0.0005)
    finally:
        srv.close()
    assert refused > 0 and len(admitted) > 0
    for rid, gi, a, k in admitted:
        assert got[rid][3] == expected_bits(P[gi][2], a, k)
