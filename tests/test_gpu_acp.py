"""GPU parity of (c,k)-ACP through the C ABI against the FP64 oracle.

The oracle takes the index's leaf partition as data (pmlsh_index_export_leaves)
and finds candidates by brute force over all pairs, so a pair lost by the
Mindist tile pruning shows up as a mismatch.
"""

import gc
import math

import numpy as np
import pytest
from scipy.spatial.distance import pdist

import synth
from oracle import acp as oacp
from oracle import ann as oann
from oracle import chi2
from parity import TOL, acp_exact, compare_acp, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_05537_amd as pm
    pm.load_library()
    return pm


def _index(pm, D, A, **kw):
    dev = torch.device("cuda", 0)
    return pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev), **kw)


def _oracle(idx, D, A, k, c, conf, beta):
    """The oracle's canonical ACP on the index's leaves, and a closure that
    re-runs it with the pair filter's radius or the budget moved."""
    perm, offsets = idx.export_leaves()
    m = A.shape[0]
    t = chi2.radius_factor(1 - conf, m)
    if beta < 0:
        beta = chi2.default_beta(1 - conf, c, m)
    T = chi2.acp_budget(beta, D.shape[0], k)
    Dp = oann.project(D, A)

    def rerun(t_scale=1.0, dT=0):
        return oacp.run(D, Dp, perm, offsets, k=k, t=t * t_scale, T=T + dT)

    res = oacp.run(D, Dp, perm, offsets, k=k, t=t, T=T)
    res.rerun, res.D = rerun, D
    return res, T


def _compare(res, pairs, dist, st):
    kind = compare_acp(res.D, res, pairs.cpu().numpy(), dist.cpu().numpy(), st,
                       rerun=res.rerun)
    say("ACP comparison:", kind)


def test_planted_small():
    pm = _gpu()
    say("case: ACP planted n=3000 d=32")
    w = synth.planted_pairs(n=3000, d=32, n_centres=10)
    D, A = w["D"], w["A"]
    idx = _index(pm, D, A)
    for k in (1, 10, 30):
        pairs, dist, st = idx.acp(k, c=1.5)
        torch.cuda.synchronize()
        res, T = _oracle(idx, D, A, k, 1.5, 1 - 1 / math.e, -1.0)
        say("k", k, "stats", st)
        assert st["budget"] == T
        _compare(res, pairs, dist, st)


def test_uniform_many_leaf_pairs():
    """Structureless data: the radius filter admits many cross-leaf pairs."""
    pm = _gpu()
    say("case: ACP uniform n=2500 d=12")
    w = synth.uniform_cube(3, 2500, 12, 1)
    D, A = w["D"], w["A"]
    idx = _index(pm, D, A, leaf_size=32, fanout=4)
    pairs, dist, st = idx.acp(20, c=1.5)
    torch.cuda.synchronize()
    res, _ = _oracle(idx, D, A, 20, 1.5, 1 - 1 / math.e, -1.0)
    say("stats", st, "oracle raw", res.n_cand_raw)
    assert st["tiles_scanned"] < st["tiles_total"]
    _compare(res, pairs, dist, st)


def test_single_leaf_is_exact():
    pm = _gpu()
    say("case: ACP single leaf")
    rng = np.random.Generator(np.random.PCG64(8))
    D = rng.standard_normal((200, 40)).astype(np.float32)
    A = rng.standard_normal((15, 40)).astype(np.float32)
    idx = _index(pm, D, A, leaf_size=256)
    pairs, dist, st = idx.acp(50)
    dv = pdist(D.astype(np.float64))
    ii, jj = np.triu_indices(200, k=1)
    o = np.lexsort((jj, ii, dv))[:50]
    assert pairs.cpu().numpy().tolist() == np.stack([ii[o], jj[o]], 1).tolist()
    np.testing.assert_allclose(dist.cpu().numpy(), dv[o], rtol=TOL)
    assert st["n_cand_raw"] == 0 and st["tiles_total"] == 0


def test_single_leaf_near_ties_take_fp64_order():
    """100 planted pairs (a, a + v) with |v| = 1: the FP32 rounding of a + v
    spreads their distances over about 3e-6 relative, close to the FP32
    verify error at d = 64, so on this seed the FP32 top-k differs from the
    exact one even as a set. The library re-decides the band around the k-th
    distance in FP64 and must return the exact (dist, i, j) order."""
    pm = _gpu()
    say("case: ACP single leaf, near-tied planted pairs")
    rng = np.random.Generator(np.random.PCG64(21))
    a = (rng.standard_normal((100, 64)) * 50).astype(np.float32)
    v = rng.standard_normal(64)
    b = (a + v / np.linalg.norm(v)).astype(np.float32)
    D = np.concatenate([a, b])
    A = rng.standard_normal((15, 64)).astype(np.float32)
    k = 50
    dv = pdist(D.astype(np.float64))
    ii, jj = np.triu_indices(200, k=1)
    o = np.lexsort((jj, ii, dv))[:k + 1]
    gaps = np.diff(dv[o]) / dv[o][:-1]
    say("smallest relative gap in the top-k", gaps.min())
    assert 1e-11 < gaps.min() < 1e-6          # near ties for FP32, not for FP64
    idx = _index(pm, D, A, leaf_size=256)
    pairs, dist, st = idx.acp(k)
    assert pairs.cpu().numpy().tolist() == np.stack([ii[o[:k]], jj[o[:k]]], 1).tolist()
    np.testing.assert_allclose(dist.cpu().numpy(), dv[o[:k]], rtol=TOL)


def test_single_leaf_mass_ties_keep_fp32_order():
    """16 groups of 16 identical points: 1,920 pairs at distance 0, more than
    the FP64 top-k takes, so the FP32 order (exact here: every distance is 0
    or far from it) decides and ties go by (i, j)."""
    pm = _gpu()
    say("case: ACP single leaf, 1920 pairs at distance 0")
    rng = np.random.Generator(np.random.PCG64(22))
    centres = (rng.standard_normal((16, 32)) * 10).astype(np.float32)
    D = centres[rng.permutation(np.repeat(np.arange(16), 16))]
    A = rng.standard_normal((15, 32)).astype(np.float32)
    k = 30
    dv = pdist(D.astype(np.float64))
    ii, jj = np.triu_indices(256, k=1)
    assert int((dv == 0).sum()) == 1920
    o = np.lexsort((jj, ii, dv))[:k]
    idx = _index(pm, D, A, leaf_size=256)
    pairs, dist, st = idx.acp(k)
    assert pairs.cpu().numpy().tolist() == np.stack([ii[o], jj[o]], 1).tolist()
    assert np.all(dist.cpu().numpy() == 0)


@pytest.mark.parametrize("groups", [100, 1000])
def test_seed_bounds_mass_ties(groups):
    """Groups of 64 identical points in leaves of 64: every within-group seed
    is at distance 0, so ub = 0, no pair is a candidate, and the answer is
    the k smallest (i, j) among the zero-distance seeds. With 100 groups the
    band of seeds the Gram bounds cannot separate from the k-th (every zero
    pair, about 200,000) is verified exactly; with 1,000 groups it exceeds
    2^20 pairs and the direct self-join takes over."""
    pm = _gpu()
    say(f"case: ACP seed bounds, {groups} groups of 64 identical points")
    rng = np.random.Generator(np.random.PCG64(31))
    d, k = 24, 50
    centres = (rng.standard_normal((groups, d)) * 10).astype(np.float32)
    lab = rng.permutation(np.repeat(np.arange(groups), 64))
    D = centres[lab]
    A = rng.standard_normal((15, d)).astype(np.float32)
    idx = _index(pm, D, A, leaf_size=64)
    perm, offsets = idx.export_leaves()
    zi, zj = [], []
    for b in range(offsets.shape[0] - 1):
        ids = np.sort(perm[offsets[b]:offsets[b + 1]]).astype(np.int64)
        a, c = np.triu_indices(ids.shape[0], k=1)
        same = lab[ids[a]] == lab[ids[c]]
        zi.append(ids[a][same])
        zj.append(ids[c][same])
    zi, zj = np.concatenate(zi), np.concatenate(zj)
    say("zero-distance seeds", zi.shape[0])
    if groups == 1000:
        assert zi.shape[0] > 1 << 20
    o = np.lexsort((zj, zi))[:k]
    pairs, dist, st = idx.acp(k)
    torch.cuda.synchronize()
    say("stats", st)
    assert st["ub"] == 0.0
    assert st["n_cand_raw"] == 0
    assert pairs.cpu().numpy().tolist() == np.stack([zi[o], zj[o]], 1).tolist()
    assert np.all(dist.cpu().numpy() == 0)


def test_planted_far_from_the_origin():
    """The small planted workload shifted by +1000 in every coordinate: the
    Gram bounds of the seeds are taken relative to each leaf's first point,
    so ub and the answers must still match the oracle's."""
    pm = _gpu()
    say("case: ACP planted n=3000 d=32, offset +1000")
    w = synth.planted_pairs(n=3000, d=32, n_centres=10)
    D = (w["D"] + 1000.0).astype(np.float32)
    A = w["A"]
    idx = _index(pm, D, A)
    for k in (1, 10):
        pairs, dist, st = idx.acp(k, c=1.5)
        torch.cuda.synchronize()
        res, T = _oracle(idx, D, A, k, 1.5, 1 - 1 / math.e, -1.0)
        say("k", k, "stats", st)
        assert st["ub"] == pytest.approx(res.ub, rel=TOL)
        _compare(res, pairs, dist, st)


@pytest.mark.parametrize("d", [36, 2048, 2052])
def test_planted_row_widths(d):
    """Rows of 36 coordinates (the last 32-coordinate step of the Gram seeds
    is partly padding), 2,048 (the first point's row fills its LDS copy) and
    2,052 (past it: the first row is loaded with every step): ub and the
    answers match the oracle's."""
    pm = _gpu()
    say(f"case: ACP planted n=1500 d={d}")
    w = synth.planted_pairs(n=1500, d=d, n_centres=10)
    D, A = w["D"], w["A"]
    idx = _index(pm, D, A)
    for k in (1, 10):
        pairs, dist, st = idx.acp(k, c=1.5)
        torch.cuda.synchronize()
        res, T = _oracle(idx, D, A, k, 1.5, 1 - 1 / math.e, -1.0)
        say("k", k, "stats", st)
        assert st["budget"] == T
        _compare(res, pairs, dist, st)


def test_fewer_seeds_than_k_in_small_leaves():
    """k above the number of seeds with leaves of 8: ub = inf, every seed
    enters the pool and every cross-leaf pair is a candidate."""
    pm = _gpu()
    say("case: ACP ub = inf, leaves of 8")
    rng = np.random.Generator(np.random.PCG64(13))
    D = rng.standard_normal((100, 16)).astype(np.float32)
    A = rng.standard_normal((15, 16)).astype(np.float32)
    idx = _index(pm, D, A, leaf_size=8, fanout=2)
    _, _, st = idx.acp(1, beta=1.0)
    k = st["n_seed"] + 10
    assert k <= 1024
    pairs, dist, st = idx.acp(k, beta=1.0)
    torch.cuda.synchronize()
    res, _ = _oracle(idx, D, A, k, 1.5, 1 - 1 / math.e, 1.0)
    assert math.isinf(st["ub"])
    _compare(res, pairs, dist, st)


@pytest.mark.parametrize("first_cap", [1, 8])
def test_small_first_capacities_redo_at_full_count(first_cap):
    """ACP's first buffer capacities forced down (pmlsh_tune): the band of
    seeds verified exactly and the candidate list overflow, the band is
    gathered again at its size and the pair scan redone at the full count;
    the answers and the counts must equal the oracle's as with the
    defaults."""
    pm = _gpu()
    say(f"case: ACP first capacity {first_cap}")
    w = synth.uniform_cube(3, 2500, 12, 1)
    D, A = w["D"], w["A"]
    idx = _index(pm, D, A, leaf_size=32, fanout=4)
    base = idx.acp(20, c=1.5)
    pm.tune(pm.TUNE_ACP_FIRST_CAP, first_cap)
    try:
        pairs, dist, st = idx.acp(20, c=1.5)
        torch.cuda.synchronize()
    finally:
        pm.tune(pm.TUNE_ACP_FIRST_CAP, -1)
    res, _ = _oracle(idx, D, A, 20, 1.5, 1 - 1 / math.e, -1.0)
    say("stats", st, "oracle raw", res.n_cand_raw)
    assert st["n_cand_raw"] > first_cap
    _compare(res, pairs, dist, st)
    assert pairs.cpu().numpy().tolist() == base[0].cpu().numpy().tolist()
    assert st == base[2]


def test_budget_binding_and_unbounded_ub():
    pm = _gpu()
    say("case: ACP budget cut / ub = inf")
    rng = np.random.Generator(np.random.PCG64(12))
    D = rng.standard_normal((300, 16)).astype(np.float32)
    A = rng.standard_normal((15, 16)).astype(np.float32)
    idx = _index(pm, D, A, leaf_size=8, fanout=2)
    # tiny beta: T = k + ceil(beta n(n-1)/2) below the candidate count
    pairs, dist, st = idx.acp(5, beta=2e-3)
    res, T = _oracle(idx, D, A, 5, 1.5, 1 - 1 / math.e, 2e-3)
    say("budget", T, "stats", st, "oracle", res.n_seed, res.n_cand_raw, res.n_cand)
    assert res.n_seed + res.n_cand_raw > T
    _compare(res, pairs, dist, st)
    # k above the number of seed pairs: ub = inf, every cross pair is a candidate
    n_seed = st["n_seed"]
    k = n_seed + 10
    if k <= 1024:
        pairs, dist, st = idx.acp(k, beta=1.0)
        res, _ = _oracle(idx, D, A, k, 1.5, 1 - 1 / math.e, 1.0)
        assert math.isinf(st["ub"])
        _compare(res, pairs, dist, st)


def test_acp_scale_planted():
    """200,000 x 512 with 2,000 planted near-duplicates, k = 1, 10, 100.

    Against the oracle on the exported leaves: the seed count and ub (the
    oracle's self-join: FP64 distances of all 6.3 million within-leaf
    pairs), and the answer: the k closest pairs of the seeds and the
    candidates. Candidates are pairs in different leaves with projected
    distance below t ub; every planted copy is ~0.023 from its original
    and every other pair several units apart, so by construction the
    candidates are the planted pairs split across leaves whose FP64
    projected distance is below t ub (a non-planted pair would need a
    projected distance hundreds of times below its true one), and the
    filtered-pair count must equal that number."""
    pm = _gpu()
    say("case: ACP scale n=200000 d=512")
    w = synth.planted_pairs()
    D, A, planted = w["D"], w["A"], w["pairs"]
    idx = _index(pm, D, A)
    perm, offsets = idx.export_leaves()
    say("oracle self-join of the exported leaves")
    si, sj = oacp.seed_pairs(perm, offsets)
    sd = oacp.pair_dist(D, si, sj)
    so = np.lexsort((sj, si, sd))
    leaf_of = np.empty(D.shape[0], dtype=np.int64)
    for b in range(offsets.shape[0] - 1):
        leaf_of[perm[offsets[b]:offsets[b + 1]]] = b
    Dp = oann.project(D, A)
    cross = planted[leaf_of[planted[:, 0]] != leaf_of[planted[:, 1]]]
    cross_pd = oacp.pair_dist(Dp, cross[:, 0], cross[:, 1])
    cross_d = oacp.pair_dist(D, cross[:, 0], cross[:, 1])
    t = chi2.radius_factor(1 / math.e, A.shape[0])
    for k in (1, 10, 100):
        pairs, dist, st = idx.acp(k, c=1.5)
        torch.cuda.synchronize()
        say("k", k, "stats", st)
        assert st["n_seed"] == si.shape[0]
        ub = float(sd[so[k - 1]])
        assert st["ub"] == pytest.approx(ub, rel=TOL)
        thr = t * ub
        near = np.abs(cross_pd - thr) <= 1e-5 * thr
        assert not near.any(), "a planted pair lies on the filter threshold"
        cand = cross_pd < thr
        assert st["n_cand_raw"] == int(cand.sum())
        # the k closest pairs of seeds and candidates, by (dist, i, j)
        ai = np.concatenate([si, cross[cand, 0]])
        aj = np.concatenate([sj, cross[cand, 1]])
        ad = np.concatenate([sd, cross_d[cand]])
        o = np.lexsort((aj, ai, ad))[:k + 1]
        gaps = np.diff(ad[o]) / ad[o][:-1]
        got = pairs.cpu().numpy()
        if gaps.min() > 1e-11:
            assert got.tolist() == np.stack([ai[o[:k]], aj[o[:k]]], 1).tolist()
        np.testing.assert_allclose(dist.cpu().numpy(), ad[o[:k]], rtol=TOL)
        # and they are the k closest planted pairs
        pd_ = oacp.pair_dist(D, planted[:, 0], planted[:, 1])
        order = np.lexsort((planted[:, 1], planted[:, 0], pd_))
        assert got.tolist() == planted[order[:k]].tolist()


@pytest.mark.parametrize("beta", [1e-4, 0.05, 1.0])
def test_branch_and_bound_matches_oracle(beta):
    """Algorithm 3: the T projected-closest pairs verified. beta = 1e-4 puts
    T below the pairs inside leaves (d_T from their T-th projected distance),
    0.05 above them (d_T found by growing a radius), 1.0 takes every pair."""
    pm = _gpu()
    say(f"case: ACP branch and bound beta={beta}")
    w = synth.planted_pairs(n=3000, d=32, n_centres=10)
    D, A = w["D"], w["A"]
    idx = _index(pm, D, A)
    k = 10
    pairs, dist, st = idx.acp_bb(k, c=1.5, beta=beta)
    torch.cuda.synchronize()
    T = min(chi2.acp_budget(beta, D.shape[0], k), D.shape[0] * (D.shape[0] - 1) // 2)
    Dp = oann.project(D, A)
    res = oacp.branch_and_bound(D, Dp, k, T)
    say("stats", st, "T", T, "margin", res.margin, res.margin_kind)
    assert st["n_cand"] == T and st["n_seed"] == 0
    assert st["n_cand_raw"] >= T

    def rerun(dT=0):
        return oacp.branch_and_bound(D, Dp, k, T + dT)

    say("ACP comparison:", compare_acp(D, res, pairs.cpu().numpy(), dist.cpu().numpy(),
                                       rerun=rerun))


def test_every_tile_and_pair_on_long_rows():
    """20,000 points in leaves of 8 (2,500 leaves, rows of up to 2,500
    tiles: the tile filter flushes its LDS row buffer mid-row and the wave
    scan walks long contiguous runs) through branch and bound at beta = 1,
    so every tile and every pair is kept: the counts are the full triangle
    and the answer is the exact k closest pairs."""
    from oracle import brute
    pm = _gpu()
    say("case: ACP branch and bound, 2,500 leaves of 8, every pair")
    rng = np.random.Generator(np.random.PCG64(21))
    n, d, k = 20_000, 8, 10
    D = rng.standard_normal((n, d)).astype(np.float32)
    A = rng.standard_normal((15, d)).astype(np.float32)
    idx = _index(pm, D, A, leaf_size=8)
    NL = idx.info()["n_leaves"]
    assert NL == 2500
    pairs, dist, st = idx.acp_bb(k, c=1.5, beta=1.0)
    torch.cuda.synchronize()
    assert st["tiles_scanned"] == NL * (NL + 1) // 2
    assert st["n_cand_raw"] == n * (n - 1) // 2
    ep, ed = brute.closest_pairs(D, k + 1)
    got_d = dist.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got_d, ed[:k], rtol=TOL)
    gaps = np.diff(ed) / ed[1:]
    if gaps.min() > 1e-5:
        assert pairs.cpu().numpy().tolist() == ep[:k].tolist()


def test_branch_and_bound_budget_above_its_cap_fails_at_once():
    """T above the 2^28 pairs one branch-and-bound call collects is rejected
    before any scan: 24,000 points at beta = 1 give T = 287,988,000."""
    import time
    pm = _gpu()
    say("case: ACP branch and bound, T above 2^28")
    rng = np.random.Generator(np.random.PCG64(8))
    D = rng.standard_normal((24_000, 8)).astype(np.float32)
    A = rng.standard_normal((15, 8)).astype(np.float32)
    idx = _index(pm, D, A)
    t0 = time.perf_counter()
    with pytest.raises(pm.PmlshError) as e:
        idx.acp_bb(10, c=1.5, beta=1.0)
    assert e.value.code == pm.EUNSUPPORTED
    assert "2^28" in str(e.value)
    assert time.perf_counter() - t0 < 1.0


@pytest.mark.parametrize("scale,extra", [(1.0, None), (40.0, None), (40.0, 20)])
def test_radius_filtering_lca_matches_oracle(scale, extra):
    """Algorithms 4-5: FindLCA with gamma, live ub per node. gamma is the
    library's estimate (Pr = 0.85) times `scale` (40 makes FindLCA return
    nodes on this mixture, whose leaf pairs are then scanned); extra = 20
    sets T to the seed count plus 20, so the scan stops after the first node
    that passes T. The oracle gets the same gamma and the exported tree."""
    pm = _gpu()
    say(f"case: ACP FindLCA gamma x{scale} extra={extra}")
    w = synth.parity(n=3000, n_queries=1)
    D, A = w["D"], w["A"]
    idx = _index(pm, D, A, leaf_size=16, fanout=4)
    perm, offsets = idx.export_leaves()
    nodes = idx.export_nodes()
    n, k = D.shape[0], 10
    n_seed = int(sum((offsets[b + 1] - offsets[b]) * (offsets[b + 1] - offsets[b] - 1) // 2
                     for b in range(offsets.shape[0] - 1)))
    beta = 0.05 if extra is None else (n_seed + extra - k) / (n * (n - 1) / 2)
    say("estimating gamma")
    _, _, st0 = idx.acp_lca(k, c=1.5, beta=beta)
    gamma = st0["gamma"] * scale
    assert gamma > 0 and math.isfinite(gamma)
    say("running pmlsh_acp_lca with gamma", gamma)
    pairs, dist, st = idx.acp_lca(k, c=1.5, beta=beta, gamma=gamma)
    torch.cuda.synchronize()
    assert st["gamma"] == gamma
    t = chi2.radius_factor(1 / math.e, A.shape[0])
    T = chi2.acp_budget(beta, n, k)
    assert st["budget"] == T
    say("stats", st, "; running the oracle")
    Dp = oann.project(D, A)

    def rerun(t_scale=1.0, gamma_scale=1.0, dT=0):
        # t_scale moves the pair filter's radius t ub only (FindLCA's radius
        # gamma t ub is kept by dividing gamma by the same factor)
        return oacp.radius_filtering_lca(D, Dp, perm, offsets, nodes["level"],
                                         nodes["first_leaf"], nodes["end_leaf"],
                                         nodes["radius"], k, t * t_scale, T + dT,
                                         gamma * gamma_scale / t_scale)

    res = rerun()
    say("oracle n_cand", res.n_cand, "margin", res.margin, res.margin_kind)
    if scale > 1:
        assert st["tiles_scanned"] > 0
    if acp_exact(res):
        assert st["n_cand"] == res.n_cand
    say("ACP comparison:", compare_acp(D, res, pairs.cpu().numpy(), dist.cpu().numpy(), st,
                                       rerun=rerun, check_raw=False))


def test_lca_gamma_estimate_kept_with_the_index():
    """FindLCA's gamma estimate depends on the index alone: the first call
    without gamma computes it and later calls reuse it. Two such calls report
    the same gamma and answers, a call given that gamma answers the same, and
    a second index built from the same data (the build is deterministic)
    estimates the same gamma afresh."""
    pm = _gpu()
    say("case: ACP FindLCA gamma kept with the index")
    w = synth.parity(n=3000, n_queries=1)
    D, A = w["D"], w["A"]
    idx = _index(pm, D, A, leaf_size=16, fanout=4)
    k = 10
    p1, d1, s1 = idx.acp_lca(k, c=1.5, beta=0.05)
    p2, d2, s2 = idx.acp_lca(k, c=1.5, beta=0.05)
    p3, d3, s3 = idx.acp_lca(k, c=1.5, beta=0.05, gamma=s1["gamma"])
    torch.cuda.synchronize()
    say("gamma", s1["gamma"], s2["gamma"], s3["gamma"])
    assert s1["gamma"] > 0 and math.isfinite(s1["gamma"])
    assert s2["gamma"] == s1["gamma"] and s3["gamma"] == s1["gamma"]
    for p, d in ((p2, d2), (p3, d3)):
        assert torch.equal(p, p1) and torch.equal(d, d1)
    idx2 = _index(pm, D, A, leaf_size=16, fanout=4)
    _, _, s4 = idx2.acp_lca(k, c=1.5, beta=0.05)
    torch.cuda.synchronize()
    assert s4["gamma"] == s1["gamma"]


def test_free_releases_device_memory():
    """Building, using and freeing an index returns its device memory (the
    FP16 rows, chunk balls and the ACP buffers kept in the index included)."""
    pm = _gpu()
    say("case: build/free cycles")
    dev = torch.device("cuda", 0)
    w = synth.planted_pairs(n=100_000, d=256)
    D = torch.from_numpy(w["D"]).to(dev)
    A = torch.from_numpy(w["A"]).to(dev)
    torch.cuda.synchronize()

    def cycle():
        idx = pm.Index(D, A)
        idx.acp(5)
        torch.cuda.synchronize()
        del idx
        gc.collect()
        torch.cuda.synchronize()

    cycle()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(4):
        cycle()
    free1 = torch.cuda.mem_get_info()[0]
    say("free bytes before/after", free0, free1)
    assert free0 - free1 < 64 << 20
