"""Serving loop (continuous batching) on the GPU: every request's answer is
the one pmlsh_ann gives it alone, bit for bit, whatever it was batched with;
admission under a tight HBM budget; argument errors."""

import math
import threading

import numpy as np
import pytest

import synth
from oracle import chi2
from parity import compare_ann, oracle_ann, oracle_r_min, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_05537_amd as pm
    pm.load_library()
    return pm


@pytest.fixture(scope="module")
def served():
    pm = _gpu()
    w = synth.parity()
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(w["D"]).to(dev), torch.from_numpy(w["A"]).to(dev))
    return pm, idx, w


def _requests(w, n_req, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    dev = torch.device("cuda", 0)
    Qall = w["Q"]
    out = []
    for _ in range(n_req):
        nq = int(rng.integers(1, 300))
        rows = rng.integers(0, Qall.shape[0], size=nq)
        noise = rng.standard_normal((nq, Qall.shape[1])).astype(np.float32) * 0.05
        Q = torch.from_numpy(Qall[rows] + noise).to(dev)
        k = int(rng.choice([1, 10, 50]))
        c = float(rng.choice([1.2, 1.5, 2.0]))
        out.append((Q, k, c))
    torch.cuda.synchronize()
    return out


def test_each_request_alone_equals_in_the_mix(served):
    pm, idx, w = served
    reqs = _requests(w, 48, 3)
    say("case: 48 mixed requests, 4 submitting threads, max_batch 128")
    srv = pm.Server(idx, max_batch=128, max_inflight=3)
    handles = [None] * len(reqs)

    def submitter(t):
        rng = np.random.Generator(np.random.PCG64(100 + t))
        for i in range(t, len(reqs), 4):
            Q, k, c = reqs[i]
            handles[i] = srv.submit(Q, k, c=c, confidence=0.9, beta=0.05)
            if rng.random() < 0.3:
                threading.Event().wait(0.001)

    threads = [threading.Thread(target=submitter, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    results = [h.wait() for h in handles]
    st = srv.stats()
    srv.close()
    assert st["requests"] == len(reqs)
    assert st["queries"] == sum(Q.shape[0] for Q, _, _ in reqs)
    assert st["latency_p50_ms"] > 0.0
    say("server stats", st)
    for (Q, k, c), (ids, dist) in zip(reqs, results):
        ids0, dist0 = idx.ann(Q, k, c=c, confidence=0.9, beta=0.05)
        torch.cuda.synchronize()
        assert torch.equal(ids, ids0)
        assert torch.equal(dist, dist0)
    # served answers against the oracle: the first three queries of every
    # eighth request (each request has its own k and c)
    D, A = w["D"], w["A"]
    for i in range(0, len(reqs), 8):
        Q, k, c = reqs[i]
        ids, dist = results[i]
        rows = slice(0, min(3, Q.shape[0]))
        Qn = Q[rows].cpu().numpy()
        B = chi2.ann_budget(0.05, D.shape[0], k)
        r0 = oracle_r_min(D, 0x5EED, B)
        res, _ = oracle_ann(D, A, Qn, k, c, 0.9, 0.05, r_min=r0)
        say(f"request {i}: k={k} c={c}, {Qn.shape[0]} queries against the oracle")
        compare_ann(D, Qn, res, ids[rows].cpu().numpy(), dist[rows].cpu().numpy(), fp64=True,
                    min_exact_frac=0.0)


def test_tight_hbm_budget_still_serves_one_launch_at_a_time(served):
    pm, idx, w = served
    reqs = _requests(w, 6, 4)
    say("case: hbm_budget 1 byte")
    srv = pm.Server(idx, max_batch=64, max_inflight=4, hbm_budget=1)
    hs = [srv.submit(Q, k, c=c, confidence=0.9, beta=0.05) for Q, k, c in reqs]
    res = [h.wait() for h in hs]
    st = srv.stats()
    srv.close()
    # one launch at a time, each of at most 64 queries (requests of any
    # parameters share launches)
    assert st["launches"] >= (sum(Q.shape[0] for Q, _, _ in reqs) + 63) // 64
    for (Q, k, c), (ids, dist) in zip(reqs, res):
        ids0, dist0 = idx.ann(Q, k, c=c, confidence=0.9, beta=0.05)
        torch.cuda.synchronize()
        assert torch.equal(ids, ids0) and torch.equal(dist, dist0)


def test_server_errors_and_empty_request(served):
    pm, idx, w = served
    dev = torch.device("cuda", 0)
    srv = pm.Server(idx)
    Q = torch.from_numpy(w["Q"][:4]).to(dev)
    with pytest.raises(pm.PmlshError) as e:
        srv.submit(Q, 0)
    assert e.value.code == pm.EINVAL
    with pytest.raises(pm.PmlshError) as e:
        srv.submit(Q, 5, c=0.5)
    assert e.value.code == pm.EINVAL
    with pytest.raises(pm.PmlshError) as e:
        srv.submit(Q, pm.MAX_K + 1)
    assert e.value.code in (pm.EINVAL, pm.EUNSUPPORTED)
    bad = (torch.empty((4, 4), dtype=torch.int64, device=dev),
           torch.empty((4, 5), dtype=torch.float32, device=dev))
    with pytest.raises(ValueError):
        srv.submit(Q, 5, out=bad)
    # answers into caller-owned tensors equal those of a lone call
    out = (torch.full((4, 5), -7, dtype=torch.int64, device=dev),
           torch.full((4, 5), -7.0, dtype=torch.float32, device=dev))
    ids_o, dist_o = srv.submit(Q, 5, out=out).wait()
    assert ids_o.data_ptr() == out[0].data_ptr() and dist_o.data_ptr() == out[1].data_ptr()
    ids_a, dist_a = idx.ann(Q, 5)
    assert torch.equal(ids_o, ids_a) and torch.equal(dist_o, dist_a)
    h = srv.submit(Q[:0], 5)
    assert h.done()
    ids, dist = h.wait()
    assert ids.shape == (0, 5)
    lib = pm.load_library()
    assert lib.pmlsh_server_wait(srv._h, 123456789) == pm.EINVAL
    srv.close()
    srv.close()   # idempotent
