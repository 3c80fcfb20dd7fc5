"""GPU parity of (c,k)-ANN through the C ABI against the FP64 oracle.

Every case runs the library (pmlsh_build + pmlsh_ann on the GPU) and the
oracle on the same seeded inputs and compares them with the rule in
tests/parity.py. Sizes span many leaves and tiles with ragged tails; edge
cases cover tiny and degenerate inputs, ties, multi-round searches and budgets
larger than one LDS sort.
"""

import math

import numpy as np
import pytest

import synth
from oracle import brute, chi2
from parity import TOL, compare_ann, oracle_ann, oracle_r_min, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_05537_amd as pm
    pm.load_library()
    return pm


def _run(pm, D, A, Q, k, c, conf, beta, r_min, **build_kw):
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev), **build_kw)
    ids, dist, st = idx.ann(torch.from_numpy(Q).to(dev), k, c=c, confidence=conf,
                            beta=beta, r_min=r_min, stats=True)
    torch.cuda.synchronize()
    return idx, ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy()


@pytest.fixture(scope="module")
def parity_wl():
    return synth.parity()


def test_parity_workload_full(parity_wl):
    """10,000 x 128, 100 queries, k=10, c=1.5, confidence 0.9, beta 0.1."""
    pm = _gpu()
    w = parity_wl
    D, A, Q = w["D"], w["A"], w["Q"]
    say("case: parity workload n=10000 d=128 nq=100")
    res, B = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.1, r_min=1.0)   # B only
    r0 = oracle_r_min(D, 0x5EED, B)
    res, B = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.1, r_min=r0)
    idx, ids, dist, st = _run(pm, D, A, Q, 10, 1.5, 0.9, 0.1, r0)
    # the library's own r_min rule reproduces the oracle's
    assert idx.default_r_min(B) == pytest.approx(r0, rel=1e-12)
    nf = compare_ann(D, Q, res, ids, dist, st, fp64=True)
    say("fragile queries:", nf)
    # default r_min (0) gives the same answers as passing it explicitly
    ids2, dist2 = idx.ann(torch.from_numpy(Q).cuda(), 10, c=1.5, confidence=0.9, beta=0.1)
    assert np.array_equal(ids2.cpu().numpy(), ids)


def test_exact_special_case(parity_wl):
    """B = n and an unbounded first radius: exact kNN, ties by id."""
    pm = _gpu()
    w = parity_wl
    D, A, Q = w["D"], w["A"], w["Q"][:40]
    say("case: exact special case")
    _, ids, dist, st = _run(pm, D, A, Q, 10, 1.5, 0.9, 1.0, 1e30)
    eid, ed = brute.knn(D, Q, 10)
    assert np.array_equal(ids, eid)
    np.testing.assert_allclose(dist, ed, rtol=1e-5)
    assert np.all(st[:, 2] == 2) and np.all(st[:, 1] == D.shape[0])


def test_projected_knn_special_case(parity_wl):
    """B = k and an unbounded first radius: C is the k projected-nearest
    points (the projection and the budget cut alone decide the answer)."""
    pm = _gpu()
    w = parity_wl
    D, A, Q = w["D"], w["A"], w["Q"][:50]
    say("case: projected kNN special case")
    res, B = oracle_ann(D, A, Q, 8, 1.5, 0.9, 0.0, r_min=1e30)
    assert B == 8
    _, ids, dist, st = _run(pm, D, A, Q, 8, 1.5, 0.9, 0.0, 1e30)
    compare_ann(D, Q, res, ids, dist, st, fp64=True)


@pytest.mark.parametrize("scale,beta,k,expect", [(0.05, 0.1, 10, "multi"),
                                                 (0.3, 0.02, 1, "multi"),
                                                 (0.5, 0.05, 100, "cr_stop")])
def test_multi_round_and_cr_stop(parity_wl, scale, beta, k, expect):
    """Small first radius: several range queries, c r stops and budget exits."""
    pm = _gpu()
    w = parity_wl
    D, A, Q = w["D"], w["A"], w["Q"][:60]
    say(f"case: multi-round scale={scale} beta={beta} k={k}")
    res, B = oracle_ann(D, A, Q, k, 1.5, 0.9, beta, r_min=1.0)
    r0 = scale * oracle_r_min(D, 7, B)
    res, _ = oracle_ann(D, A, Q, k, 1.5, 0.9, beta, r_min=r0)
    _, ids, dist, st = _run(pm, D, A, Q, k, 1.5, 0.9, beta, r0)
    compare_ann(D, Q, res, ids, dist, st, fp64=True)
    kinds = {r.exit_kind for r in res}
    rounds = max(r.rounds for r in res)
    say("exit kinds", kinds, "max rounds", rounds)
    if expect == "multi":
        assert rounds >= 2          # several range queries
    else:
        assert 1 in kinds           # Algorithm 2's c r stop


def test_topk_larger_than_one_workgroup(parity_wl):
    """k = 300: more top-k members than threads of a workgroup (the top-k is
    then selected and sorted rather than ranked in one step)."""
    pm = _gpu()
    w = parity_wl
    D, A, Q = w["D"], w["A"], w["Q"][:20]
    say("case: k=300")
    res, B = oracle_ann(D, A, Q, 300, 1.5, 0.9, 0.05, r_min=1e30)
    assert B == 800
    _, ids, dist, st = _run(pm, D, A, Q, 300, 1.5, 0.9, 0.05, 1e30)
    compare_ann(D, Q, res, ids, dist, st, fp64=True)


def test_budget_larger_than_one_sort(parity_wl):
    """B = 4010 > 2048: the radix-select refinement and the top-k selection
    over a candidate set larger than one LDS sort."""
    pm = _gpu()
    w = parity_wl
    D, A, Q = w["D"], w["A"], w["Q"][:30]
    say("case: B > CAP")
    res, B = oracle_ann(D, A, Q, 50, 1.5, 0.9, 0.4, r_min=1e30)
    assert B == 4050
    _, ids, dist, st = _run(pm, D, A, Q, 50, 1.5, 0.9, 0.4, 1e30)
    compare_ann(D, Q, res, ids, dist, st, fp64=True)


@pytest.mark.parametrize("n,d,m,leaf,fan,piv", [
    (3001, 130, 7, 16, 4, 0),      # ragged n and d, deep tree, no pivots
    (5000, 64, 15, 256, 64, 8),    # wide leaves and fanout, 8 pivots
    (777, 33, 16, 8, 2, 3),        # binary inner levels, d not a multiple of 4
    (50, 16, 15, 64, 16, 5),       # a single leaf
])
def test_shapes(n, d, m, leaf, fan, piv):
    pm = _gpu()
    say(f"case: shape n={n} d={d} m={m} L={leaf} F={fan} s={piv}")
    rng = np.random.Generator(np.random.PCG64(n + d))
    cen = rng.standard_normal((20, d)).astype(np.float32) * 2
    lab = rng.integers(0, 20, n)
    D = (cen[lab] + 0.4 * rng.standard_normal((n, d))).astype(np.float32)
    Q = (cen[rng.integers(0, 20, 25)] + 0.4 * rng.standard_normal((25, d))).astype(np.float32)
    A = rng.standard_normal((m, d)).astype(np.float32)
    k = min(10, n)
    res, B = oracle_ann(D, A, Q, k, 1.5, 0.9, 0.05, r_min=1.0)
    r0 = oracle_r_min(D, 3, B)
    res, _ = oracle_ann(D, A, Q, k, 1.5, 0.9, 0.05, r_min=r0)
    idx, ids, dist, st = _run(pm, D, A, Q, k, 1.5, 0.9, 0.05, r0, leaf_size=leaf,
                              fanout=fan, num_pivots=piv, sample_seed=3)
    info = idx.info()
    say("levels", info["levels"], "leaves", info["n_leaves"])
    compare_ann(D, Q, res, ids, dist, st, fp64=True)


@pytest.mark.parametrize("c", [1.2, 1.5, 2.0])
def test_heavy_tailed_d960(c):
    """The mixed-precision workload's shape and value distribution at a size
    the oracle finishes quickly: 20,000 x 960 non-negative heavy-tailed rows
    (|N(0,1)|^1.5, L2-normalised, x100), 32 queries, k = 10, every c of the
    workload. d = 960 gives FP16 rows of 120 words (a ragged last step of
    the verification) and FP32 rows of 240 words."""
    pm = _gpu()
    say(f"case: heavy-tailed n=20000 d=960 c={c}")
    w = synth.heavy_tailed(n=20_000, n_queries=32)
    D, A, Q = w["D"], w["A"], w["Q"]
    k, beta = 10, 0.05
    B = min(D.shape[0], math.ceil(beta * D.shape[0]) + k)
    r0 = oracle_r_min(D, 5, B)
    res, _ = oracle_ann(D, A, Q, k, c, 0.9, beta, r_min=r0)
    idx, ids, dist, st = _run(pm, D, A, Q, k, c, 0.9, beta, r0, sample_seed=5)
    compare_ann(D, Q, res, ids, dist, st, fp64=True)
    say("exit kinds", np.bincount(st[:, 2], minlength=3), "rounds", np.bincount(st[:, 0]))


def test_data_far_from_the_origin():
    """The parity mixture shifted by +30 in every coordinate (the projected
    points then sit far from the origin): the scan rows are centred on the
    mean projected point, and answers must match the oracle's."""
    pm = _gpu()
    say("case: data offset +30")
    w = synth.parity(n=6000, n_queries=40)
    D = (w["D"] + 30.0).astype(np.float32)
    Q = (w["Q"] + 30.0).astype(np.float32)
    A = w["A"]
    res, B = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.1, r_min=1.0)
    r0 = oracle_r_min(D, 3, B)
    res, _ = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.1, r_min=r0)
    _, ids, dist, st = _run(pm, D, A, Q, 10, 1.5, 0.9, 0.1, r0, sample_seed=3)
    compare_ann(D, Q, res, ids, dist, st, fp64=True)


@pytest.mark.parametrize("scale", [1e-4, 1e4])
def test_data_scale_extremes(scale):
    """The same mixture scaled by 1e-4 and 1e4: the FP16 scan rows, the bf16
    chunk distances and the FP16 verification rows all rescale (power-of-two
    factors per index and per row), so answers must match the oracle."""
    pm = _gpu()
    say(f"case: data scale {scale}")
    rng = np.random.Generator(np.random.PCG64(77))
    n, d = 4000, 96
    cen = rng.standard_normal((20, d)) * 2
    lab = rng.integers(0, 20, n)
    D = ((cen[lab] + 0.4 * rng.standard_normal((n, d))) * scale).astype(np.float32)
    Q = ((cen[rng.integers(0, 20, 40)] + 0.4 * rng.standard_normal((40, d))) * scale).astype(np.float32)
    A = rng.standard_normal((15, d)).astype(np.float32)
    res, B = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.05, r_min=1.0)
    r0 = oracle_r_min(D, 3, B)
    res, _ = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.05, r_min=r0)
    _, ids, dist, st = _run(pm, D, A, Q, 10, 1.5, 0.9, 0.05, r0, sample_seed=3)
    compare_ann(D, Q, res, ids, dist, st, fp64=True)


def test_ties_duplicates_and_self_queries():
    """Exact duplicate points (equal projected and exact distances: ties go to
    the smaller id) and queries that are data points (distance 0)."""
    pm = _gpu()
    say("case: duplicates")
    rng = np.random.Generator(np.random.PCG64(99))
    base = rng.standard_normal((300, 24)).astype(np.float32)
    D = np.concatenate([base, base[:150], base[:50]])     # ids 300.. duplicate 0..
    perm = rng.permutation(D.shape[0])
    D = D[perm]
    A = rng.standard_normal((15, 24)).astype(np.float32)
    Q = np.concatenate([D[:10], rng.standard_normal((10, 24)).astype(np.float32)])
    res, B = oracle_ann(D, A, Q, 7, 1.5, 0.9, 0.1, r_min=1e30)
    _, ids, dist, st = _run(pm, D, A, Q, 7, 1.5, 0.9, 0.1, 1e30, leaf_size=16)
    # duplicates tie exactly in FP32 as in FP64, so both sides break the tie
    # on the id: the answers must agree id for id (every query has margin 0
    # by construction, so none is held exactly by the margin rule)
    compare_ann(D, Q, res, ids, dist, st, fp64=True, min_exact_frac=0.0)
    assert np.array_equal(ids, np.stack([r.ids for r in res]))
    assert np.all(dist[:10, 0] == 0)


def test_fp64_decisions_fall_back_on_mass_ties():
    """700 exact copies of one point among 3,000 others, the query on top of
    them and B = 601 (beta = 0.1, k = 1 ... 20): the budget cut's band and the
    top-k's near-tie set both hold more than 512 entries, so both FP64
    decisions fall back to the FP32 order, which on exact ties is the id
    order as in the oracle. C is the 601 copies with the smallest ids and the
    answer the k smallest of them, at distance 0 from a query equal to the
    point; a query slightly off the point gets the same ids."""
    pm = _gpu()
    say("case: 700 copies of one point")
    rng = np.random.Generator(np.random.PCG64(7))
    d = 32
    others = (rng.standard_normal((3000, d)) * 3.0 + 10.0).astype(np.float32)
    p0 = rng.standard_normal(d).astype(np.float32)
    D = np.concatenate([others, np.repeat(p0[None, :], 700, axis=0)])
    order = rng.permutation(D.shape[0])
    D = D[order]
    copies = np.sort(np.flatnonzero(np.all(D == p0[None, :], axis=1)))
    assert copies.size == 700
    A = rng.standard_normal((15, d)).astype(np.float32)
    Q = np.stack([p0, p0 + np.float32(1e-3)])
    n = D.shape[0]
    beta = 600.0 / n
    for k in (1, 20):
        res, B = oracle_ann(D, A, Q, k, 1.5, 0.9, beta, r_min=1e30)
        assert B > 512 and B < 700
        _, ids, dist, st = _run(pm, D, A, Q, k, 1.5, 0.9, beta, 1e30)
        for qi in range(2):
            assert ids[qi].tolist() == copies[:k].tolist(), (k, qi, ids[qi])
            assert ids[qi].tolist() == res[qi].ids.tolist()
            assert st[qi, 1] == B and st[qi, 2] == res[qi].exit_kind
        assert np.all(dist[0] == 0)
        np.testing.assert_allclose(dist[1], res[1].dist, rtol=TOL, atol=1e-6)


def test_far_queries_take_the_per_query_path():
    """Queries far outside the data: their scan rows would leave the FP16
    range, so the batched path hands them to the per-query kernel; answers
    must still match the oracle. Near queries in the same launch stay on the
    batched path."""
    pm = _gpu()
    say("case: far queries")
    rng = np.random.Generator(np.random.PCG64(123))
    D = rng.standard_normal((4000, 32)).astype(np.float32)
    A = rng.standard_normal((15, 32)).astype(np.float32)
    Qn = rng.standard_normal((8, 32)).astype(np.float32)
    Qf = (rng.standard_normal((8, 32)) * 1e4).astype(np.float32)
    Q = np.concatenate([Qn, Qf])
    res, B = oracle_ann(D, A, Q, 5, 1.5, 0.9, 0.05, r_min=1.0)
    _, ids, dist, st = _run(pm, D, A, Q, 5, 1.5, 0.9, 0.05, 1.0)
    compare_ann(D, Q, res, ids, dist, st, fp64=True)


def test_stage_overflow_takes_the_per_query_path():
    """5,000 exact copies of one point and 64 queries next to it: every copy
    is a candidate of every query, more than a scan wave can stage for one
    chunk, so those queries are answered by the per-query kernel. The budget
    cuts through the tied copies, which go by id."""
    pm = _gpu()
    say("case: stage overflow")
    rng = np.random.Generator(np.random.PCG64(321))
    p = rng.standard_normal((1, 24)).astype(np.float32)
    D = np.concatenate([np.repeat(p, 5000, 0), rng.standard_normal((3000, 24)).astype(np.float32)])
    D = D[rng.permutation(D.shape[0])]
    A = rng.standard_normal((15, 24)).astype(np.float32)
    Q = (p + 1e-3 * rng.standard_normal((64, 24))).astype(np.float32)
    res, B = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.1, r_min=1.0)
    assert B < 5000
    _, ids, dist, st = _run(pm, D, A, Q, 10, 1.5, 0.9, 0.1, 1.0)
    # the copies tie exactly (margin 0 for every query), and ties go by id on
    # both sides: the answers must agree id for id
    compare_ann(D, Q, res, ids, dist, st, fp64=True, min_exact_frac=0.0)
    assert np.array_equal(ids, np.stack([r.ids for r in res]))


def test_tiny_inputs():
    pm = _gpu()
    say("case: tiny")
    rng = np.random.Generator(np.random.PCG64(5))
    D = rng.standard_normal((1, 8)).astype(np.float32)
    A = rng.standard_normal((15, 8)).astype(np.float32)
    Q = rng.standard_normal((3, 8)).astype(np.float32)
    _, ids, dist, st = _run(pm, D, A, Q, 1, 1.5, 0.9, -1.0, 0.0)
    assert np.all(ids == 0)
    np.testing.assert_allclose(dist[:, 0], np.sqrt(((Q - D[0]) ** 2).sum(1)), rtol=1e-5)
    # k = n, several rounds from a tiny radius
    D = rng.standard_normal((9, 8)).astype(np.float32)
    res, B = oracle_ann(D, A, Q, 9, 2.0, 0.9, 0.0, r_min=1e-3)
    _, ids, dist, st = _run(pm, D, A, Q, 9, 2.0, 0.9, 0.0, 1e-3)
    compare_ann(D, Q, res, ids, dist, st, fp64=True)


def test_empty_batch_and_errors(parity_wl):
    pm = _gpu()
    w = parity_wl
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(w["D"][:500]).to(dev), torch.from_numpy(w["A"]).to(dev))
    ids, dist = idx.ann(torch.empty((0, 128), device=dev), 5)
    assert ids.shape == (0, 5)
    with pytest.raises(pm.PmlshError) as e:
        idx.ann(torch.zeros((2, 128), device=dev), 501)
    assert e.value.code == pm.EINVAL
    with pytest.raises(pm.PmlshError) as e:
        idx.ann(torch.zeros((2, 128), device=dev), 5, c=0.5)
    assert e.value.code == pm.EINVAL


def test_deterministic(parity_wl):
    pm = _gpu()
    w = parity_wl
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(w["D"]).to(dev), torch.from_numpy(w["A"]).to(dev))
    Q = torch.from_numpy(w["Q"]).to(dev)
    a = idx.ann(Q, 10, confidence=0.9, beta=0.1, stats=True)
    b = idx.ann(Q, 10, confidence=0.9, beta=0.1, stats=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.fixture(scope="module")
def headline_wl():
    """1,000,000 x 256 headline workload with its 10,000 queries, the index
    built on the GPU and the FP64 projections of the oracle."""
    pm = _gpu()
    say("building the headline workload (1,000,000 x 256)")
    w = synth.headline()
    dev = torch.device("cuda", 0)
    w["idx"] = pm.Index(torch.from_numpy(w["D"]).to(dev), torch.from_numpy(w["A"]).to(dev))
    from oracle import ann as oann
    w["Dp"] = oann.project(w["D"], w["A"])
    yield w
    del w["idx"]


def _sample_both_kinds(st, n_even, n_kind=2):
    """n_even evenly spaced queries plus the first n_kind of each exit kind."""
    nq = st.shape[0]
    pick = set(np.linspace(0, nq - 1, n_even).astype(int).tolist())
    for kind in (1, 2):
        pick.update(np.nonzero(st[:, 2] == kind)[0][:n_kind].tolist())
    return np.array(sorted(pick))


# (k, beta): the operating points of the benchmark (smallest beta of its
# grid with recall@k >= 0.9) at the headline workload
HEADLINE_POINTS = [(1, 8.5e-4), (10, 9e-4), (50, 9e-4), (100, 8.5e-4)]


@pytest.mark.parametrize("k,beta", HEADLINE_POINTS)
def test_headline_scale_sampled(headline_wl, k, beta):
    """The headline workload at the benchmark's operating point for this k,
    one 1,024-query launch as the benchmark issues it (queries 0..1023);
    16 or more sampled queries, including both exit kinds where the launch
    has them, checked against the oracle."""
    w = headline_wl
    say(f"case: headline scale k={k} beta={beta}")
    D, A, Q, idx = w["D"], w["A"], w["Q"][:1024], w["idx"]
    dev = torch.device("cuda", 0)
    B = min(D.shape[0], math.ceil(beta * D.shape[0]) + k)
    r0 = oracle_r_min(D, 0x5EED, B)
    assert idx.default_r_min(B) == pytest.approx(r0, rel=1e-12)
    ids, dist, st = idx.ann(torch.from_numpy(Q).to(dev), k, c=1.5, beta=beta, r_min=r0,
                            stats=True)
    torch.cuda.synchronize()
    ids, dist, st = ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy()
    sample = _sample_both_kinds(st, 14)
    say("exit kinds", np.bincount(st[:, 2], minlength=3), "rounds", np.bincount(st[:, 0]),
        "sample", sample.tolist())
    res, _ = oracle_ann(D, A, Q[sample], k, 1.5, 1 - 1 / math.e, beta, r_min=r0, Dp=w["Dp"])
    compare_ann(D, Q[sample], res, ids[sample], dist[sample], st[sample], fp64=True)


def test_headline_tail_batch(headline_wl):
    """The benchmark's last batch: queries 9,216..9,999 (784 queries) in one
    launch, k = 10 at beta = 9e-4; 16 sampled queries against the oracle."""
    w = headline_wl
    say("case: headline tail batch of 784 queries")
    D, A, idx = w["D"], w["A"], w["idx"]
    Q = np.ascontiguousarray(w["Q"][9216:])
    assert Q.shape[0] == 784
    k, beta = 10, 9e-4
    B = min(D.shape[0], math.ceil(beta * D.shape[0]) + k)
    r0 = idx.default_r_min(B)
    dev = torch.device("cuda", 0)
    ids, dist, st = idx.ann(torch.from_numpy(Q).to(dev), k, c=1.5, beta=beta, r_min=r0,
                            stats=True)
    torch.cuda.synchronize()
    ids, dist, st = ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy()
    sample = _sample_both_kinds(st, 14)
    res, _ = oracle_ann(D, A, Q[sample], k, 1.5, 1 - 1 / math.e, beta, r_min=r0, Dp=w["Dp"])
    compare_ann(D, Q[sample], res, ids[sample], dist[sample], st[sample], fp64=True)


def test_serving_scale_sampled():
    """The serving index at full size, 10,000,000 x 128 FP16-valued points in
    [0, 255] around 10,000 centres, one 1,024-query launch at the serving
    beta (1e-4, B = 1,010): 8 sampled queries checked against the oracle
    for k = 10, c = 1.5 and 4 for k = 100, c = 2.0 (2,441 groups of 64
    chunks per distance row)."""
    pm = _gpu()
    say("case: serving scale, n=10M d=128")
    w = synth.serving(n_queries=1024)
    D, A, Q = w["D"], w["A"], w["Q"]
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev))
    from oracle import ann as oann
    Dp = oann.project(D, A)
    Qd = torch.from_numpy(Q).to(dev)
    beta = 1e-4
    for k, c, sample in ((10, 1.5, np.arange(0, 1024, 128)), (100, 2.0, np.arange(64, 1024, 256))):
        say(f"case: serving scale k={k} c={c}")
        B = min(D.shape[0], math.ceil(beta * D.shape[0]) + k)
        r0 = idx.default_r_min(B)
        ids, dist, st = idx.ann(Qd, k, c=c, beta=beta, r_min=r0, stats=True)
        torch.cuda.synchronize()
        ids, dist, st = ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy()
        res, _ = oracle_ann(D, A, Q[sample], k, c, 1 - 1 / math.e, beta, r_min=r0, Dp=Dp)
        compare_ann(D, Q[sample], res, ids[sample], dist[sample], st[sample], fp64=True)
        say("exit kinds", np.bincount(st[:, 2], minlength=3), "rounds", np.bincount(st[:, 0]))


GROUP_SETTINGS = [(2048, 0), (0, 1), (1, 1), (7, 0)]


def _with_tuning(pm, cap, lds, fn):
    pm.tune(pm.TUNE_GROUP_LIST, cap)
    pm.tune(pm.TUNE_GROUP_MINIMA_LDS, lds)
    try:
        return fn()
    finally:
        pm.tune(pm.TUNE_GROUP_LIST, -1)
        pm.tune(pm.TUNE_GROUP_MINIMA_LDS, -1)


def test_group_filter_settings_agree(parity_wl):
    """The bound kernel's group filter with its minima in HBM, with no group
    list (whole-row passes), and with lists too short for the qualifying
    groups: every answer equals the default run's, which the oracle pins."""
    pm = _gpu()
    D, A, Q = parity_wl["D"], parity_wl["A"], parity_wl["Q"]
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev))
    Qd = torch.from_numpy(Q).to(dev)
    for beta in (0.01, 0.1):
        ref = [t.cpu().numpy() for t in idx.ann(Qd, 10, c=1.5, beta=beta, stats=True)]
        for cap, lds in GROUP_SETTINGS:
            say(f"case: beta={beta} group list {cap} minima in LDS {lds}")
            out = _with_tuning(pm, cap, lds,
                               lambda: [t.cpu().numpy() for t in
                                        idx.ann(Qd, 10, c=1.5, beta=beta, stats=True)])
            np.testing.assert_array_equal(out[0], ref[0])
            np.testing.assert_array_equal(out[1], ref[1])
            np.testing.assert_array_equal(out[2][:, :3], ref[2][:, :3])
    with pytest.raises(pm.PmlshError):
        pm.tune(pm.TUNE_GROUP_LIST, 2049)
    with pytest.raises(pm.PmlshError):
        pm.tune(5, 0)


def test_scan_shapes_agree(parity_wl):
    """The range filter in both block shapes (512 and 1,024 queries per
    workgroup, pmlsh_tune) gives the same answers and statistics, and they
    match the oracle."""
    pm = _gpu()
    D, A, Q = parity_wl["D"], parity_wl["A"], parity_wl["Q"]
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev))
    Qd = torch.from_numpy(Q).to(dev)
    res, B = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.1, r_min=1.0)
    r0 = idx.default_r_min(B)
    res, _ = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.1, r_min=r0)
    outs = []
    try:
        for shape in (1, 2):
            say(f"case: scan shape {shape}")
            pm.tune(pm.TUNE_SCAN_SHAPE, shape)
            ids, dist, st = idx.ann(Qd, 10, c=1.5, confidence=0.9, beta=0.1, r_min=r0, stats=True)
            torch.cuda.synchronize()
            outs.append((ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy()))
    finally:
        pm.tune(pm.TUNE_SCAN_SHAPE, -1)
    for a_, b_ in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a_, b_)
    compare_ann(D, Q, res, *outs[1], fp64=True)


def test_large_n_sampled():
    """2,600,000 x 16 mixture (635 groups of 64 chunks per query row): 16
    sampled queries of one launch checked against the oracle, and the whole
    launch repeated under every setting of the group filter (minima in HBM,
    whole-row passes, short lists) with identical answers."""
    pm = _gpu()
    say("case: n=2.6M, d=16")
    spec = synth.MixtureSpec(n=2_600_000, d=16, n_centres=2_000, centre_std=2.0,
                             sigma_lo=0.2, sigma_hi=0.5, n_queries=512)
    w = synth.mixture(spec, 7)
    D, A, Q = w["D"], w["A"], w["Q"]
    beta, k = 2e-4, 10
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev))
    B = min(D.shape[0], math.ceil(beta * D.shape[0]) + k)
    r0 = oracle_r_min(D, 0x5EED, B)
    Qd = torch.from_numpy(Q).to(dev)
    ids, dist, st = idx.ann(Qd, k, c=1.5, beta=beta, r_min=r0, stats=True)
    torch.cuda.synchronize()
    ids, dist, st = ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy()
    from oracle import ann as oann
    Dp = oann.project(D, A)
    sample = np.arange(0, 512, 32)
    res, _ = oracle_ann(D, A, Q[sample], k, 1.5, 1 - 1 / math.e, beta, r_min=r0, Dp=Dp)
    compare_ann(D, Q[sample], res, ids[sample], dist[sample], st[sample], fp64=True)
    say("exit kinds", np.bincount(st[:, 2]), "rounds", np.bincount(st[:, 0]))
    for cap, lds in GROUP_SETTINGS:
        say(f"case: n=2.6M group list {cap} minima in LDS {lds}")
        o_ids, o_dist, o_st = _with_tuning(
            pm, cap, lds, lambda: [t.cpu().numpy() for t in
                                   idx.ann(Qd, k, c=1.5, beta=beta, r_min=r0, stats=True)])
        np.testing.assert_array_equal(o_ids, ids)
        np.testing.assert_array_equal(o_dist, dist)
        np.testing.assert_array_equal(o_st[:, :3], st[:, :3])


def test_mixed_parameters_in_one_launch(parity_wl):
    """pmlsh_ann_mixed: 150 queries with their own k, c, confidence and beta
    in one call. Every row equals the query answered alone by pmlsh_ann with
    its own parameters (bit for bit: Algorithm 2 runs per query), and a
    sample agrees with the oracle. A second call adds one query whose budget
    exceeds the batched path's limit, which sends the launch to the
    per-query kernel."""
    pm = _gpu()
    D, A, Q = parity_wl["D"], parity_wl["A"], parity_wl["Q"]
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev))
    rng = np.random.Generator(np.random.PCG64(31))
    nq = 150
    rows = rng.integers(0, Q.shape[0], size=nq)
    Qm = (Q[rows] + 0.05 * rng.standard_normal((nq, Q.shape[1]))).astype(np.float32)
    params = [{"k": int(rng.choice([1, 7, 10, 50, 300])), "c": float(rng.choice([1.2, 1.5, 2.0])),
               "confidence": float(rng.choice([0.9, 1 - 1 / math.e])),
               "beta": float(rng.choice([0.01, 0.05, 0.1]))} for _ in range(nq)]
    Qd = torch.from_numpy(Qm).to(dev)
    for extra in (False, True):
        say(f"case: mixed parameters, one launch (budget above the batched limit: {extra})")
        ps = list(params)
        if extra:
            ps[7] = {"k": 10, "c": 1.5, "confidence": 0.9, "beta": 0.3}
        ids, dist, st = idx.ann_mixed(Qd, ps, stats=True)
        torch.cuda.synchronize()
        ids, dist, st = ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy()
        for i, p in enumerate(ps):
            a_ids, a_dist, a_st = idx.ann(Qd[i:i + 1], p["k"], c=p["c"], confidence=p["confidence"],
                                          beta=p["beta"], stats=True)
            assert ids[i, :p["k"]].tolist() == a_ids.cpu().numpy()[0].tolist(), (i, p)
            assert np.array_equal(dist[i, :p["k"]], a_dist.cpu().numpy()[0]), (i, p)
            assert st[i, :3].tolist() == a_st.cpu().numpy()[0, :3].tolist(), (i, p)
    # the oracle on every tenth query
    for i in range(0, nq, 10):
        p = params[i]
        B = chi2.ann_budget(p["beta"], D.shape[0], p["k"])
        r0 = oracle_r_min(D, 0x5EED, B)
        res, _ = oracle_ann(D, A, Qm[i:i + 1], p["k"], p["c"], p["confidence"], p["beta"],
                            r_min=r0)
        compare_ann(D, Qm[i:i + 1], res, ids[i:i + 1, :p["k"]], dist[i:i + 1, :p["k"]],
                    st[i:i + 1], fp64=True, min_exact_frac=0.0)


def test_fp32_path_equals_batched_path(parity_wl):
    """The plain FP32 path (every query on the per-query kernel: PM-tree walk
    with Eq. 5, FP32 distances) gives the batched path's answers."""
    pm = _gpu()
    D, A, Q = parity_wl["D"], parity_wl["A"], parity_wl["Q"]
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev))
    Qd = torch.from_numpy(Q).to(dev)
    for k, beta in ((10, 0.1), (50, 0.02)):
        say(f"case: FP32 path k={k} beta={beta}")
        ref = [t.cpu().numpy() for t in idx.ann(Qd, k, c=1.5, confidence=0.9, beta=beta,
                                                stats=True)]
        pm.tune(pm.TUNE_FP32_PATH, 1)
        try:
            out = [t.cpu().numpy() for t in idx.ann(Qd, k, c=1.5, confidence=0.9, beta=beta,
                                                    stats=True)]
        finally:
            pm.tune(pm.TUNE_FP32_PATH, -1)
        np.testing.assert_array_equal(out[0], ref[0])
        np.testing.assert_array_equal(out[1], ref[1])
        np.testing.assert_array_equal(out[2][:, :3], ref[2][:, :3])
