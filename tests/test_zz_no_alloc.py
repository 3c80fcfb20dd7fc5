"""pmlsh_ann_noalloc (the ANN entry point whose workspace is the library's
fixed per-device array) against pmlsh_ann, through the C ABI.

Two calls in a row on one index, the second with fewer queries (so it runs
on the array the first call left behind): ids, distances and per-query
statistics must equal pmlsh_ann's bit for bit (the same kernels run on the
same inputs); the count of scanned points, a work statistic that depends
on the batch size, only has to be positive. The first call has more
queries than one pass over the array holds, so it runs as several batches.
"""

import math

import numpy as np
import pytest
import torch

import paper_2107_05537_amd as pm
import synth

pytestmark = pytest.mark.gpu

SCRATCH = 64 * 1024 * 1024


def _run_both(idx, Q, k, c, conf, beta):
    nq = Q.shape[0]
    dev = Q.device
    ref = idx.ann(Q, k, c=c, confidence=conf, beta=beta, stats=True)
    ids = torch.full((nq, k), -7, dtype=torch.int64, device=dev)
    dist = torch.full((nq, k), -7.0, dtype=torch.float32, device=dev)
    st = torch.full((nq, 4), -7, dtype=torch.int32, device=dev)
    idx.ann_noalloc(Q, k, c, conf, beta, 0.0, ids, dist, st)
    torch.cuda.synchronize()
    return ref, (ids, dist, st)


def _assert_same(ref, got, tag):
    # ids, distances, rounds, |C| and exit kind bit for bit. The fourth
    # statistic counts the points the filter scanned: it depends on the
    # launch shape (the scan grid follows the batch size, and a query whose
    # candidate stage fills is finished by the per-query kernel, which scans
    # differently), and the array holds smaller batches than pmlsh_ann's
    # workspace, so it is only checked to be positive.
    ref = (ref[0], ref[1], ref[2][:, :3], ref[2][:, 3] > 0)
    got = (got[0], got[1], got[2][:, :3], got[2][:, 3] > 0)
    for name, a, b in zip(("ids", "dist", "stats", "scanned > 0"), ref, got):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert a.shape == b.shape, (tag, name)
        assert np.array_equal(a, b), (tag, name, np.argwhere(a != b)[:5])


def test_noalloc_matches_ann_on_two_calls():
    print("noalloc: 200000 x 64, k=10, c=1.5, 1500 then 97 queries", flush=True)
    w = synth.mixture(synth.MixtureSpec(n=200_000, d=64, n_centres=400, centre_std=2.0,
                                        sigma_lo=0.2, sigma_hi=0.5, n_queries=1500), seed=77)
    dev = torch.device("cuda", 0)
    D = torch.from_numpy(w["D"]).to(dev)
    A = torch.from_numpy(w["A"]).to(dev)
    idx = pm.Index(D, A)
    Q = torch.from_numpy(w["Q"]).to(dev)
    k, c, conf, beta = 10, 1.5, 1 - 1 / math.e, 4e-3
    # one query's share of the array at this size (pool of 16,384 leaf
    # positions, chunk-distance row, C and its bounds): 1,500 queries need
    # more than one pass
    per_query = 16384 * 4 + (200_000 // 64) * 2 + 3 * (math.ceil(beta * 200_000) + k) * 4
    assert 1500 * per_query > SCRATCH
    ref, got = _run_both(idx, Q, k, c, conf, beta)
    _assert_same(ref, got, "first call (1500 queries)")
    ref2, got2 = _run_both(idx, Q[:97].contiguous(), k, c, conf, beta)
    _assert_same(ref2, got2, "second call (97 queries)")


def test_noalloc_per_query_path_and_other_k():
    # a budget above the batched path's limit: every query takes the
    # per-query kernel (tree walk), whose frontier lists also live in the array
    print("noalloc: 20000 x 32, k=50, budget > batched limit", flush=True)
    w = synth.mixture(synth.MixtureSpec(n=20_000, d=32, n_centres=40, centre_std=1.0,
                                        sigma_lo=0.3, sigma_hi=0.3, n_queries=300), seed=78)
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(w["D"]).to(dev), torch.from_numpy(w["A"]).to(dev))
    Q = torch.from_numpy(w["Q"]).to(dev)
    ref, got = _run_both(idx, Q, 50, 2.0, 0.9, 0.2)
    _assert_same(ref, got, "per-query path")
    ref2, got2 = _run_both(idx, Q[:5].contiguous(), 1, 1.2, 0.9, -1.0)
    _assert_same(ref2, got2, "k=1 after it")


def test_noalloc_rejects_like_ann():
    w = synth.mixture(synth.MixtureSpec(n=3000, d=16, n_centres=5, centre_std=1.0,
                                        sigma_lo=0.3, sigma_hi=0.3, n_queries=4), seed=79)
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(w["D"]).to(dev), torch.from_numpy(w["A"]).to(dev))
    Q = torch.from_numpy(w["Q"]).to(dev)
    ids = torch.empty((4, 10), dtype=torch.int64, device=dev)
    dist = torch.empty((4, 10), dtype=torch.float32, device=dev)
    with pytest.raises(pm.PmlshError) as e:
        idx.ann_noalloc(Q, 10, 0.9, 0.9, -1.0, 0.0, ids, dist)    # c <= 1
    assert e.value.code == pm.EINVAL
    with pytest.raises(pm.PmlshError) as e:
        idx.ann_noalloc(Q, 2000, 1.5, 0.9, -1.0, 0.0, ids, dist)  # k above the limit
    assert e.value.code == pm.EUNSUPPORTED
