"""Pins of the oracle's (c,k)-ACP by radius filtering (Section 6.3).

* One leaf holding every point: every pair is a self-join seed, so the
  answer is the exact k closest pairs (SciPy's pdist as the reference).
* Leaves of one point: no seeds, ub = inf, every pair is a candidate; with
  an unbounded budget the answer is again exact.
* The filter keeps exactly the cross-leaf pairs with projected distance
  strictly below t*ub (SciPy's pdist on projected points as the reference).
* Planted near-duplicates: the top-k are the k closest planted pairs.
"""

import math

import numpy as np
import pytest
from scipy.spatial.distance import pdist, squareform

import synth
from oracle import acp, ann, brute, chi2, metrics


def _exact_pairs(D, k):
    dv = pdist(D.astype(np.float64))
    n = D.shape[0]
    ii, jj = np.triu_indices(n, k=1)
    o = np.lexsort((jj, ii, dv))[:k]
    return np.stack([ii[o], jj[o]], axis=1), dv[o]


@pytest.fixture(scope="module")
def small():
    rng = np.random.Generator(np.random.PCG64(21))
    D = rng.standard_normal((300, 24)).astype(np.float32)
    A = rng.standard_normal((15, 24)).astype(np.float32)
    return D, A, ann.project(D, A)


def test_single_leaf_is_exact(small):
    D, A, Dp = small
    n, k = D.shape[0], 25
    perm = np.arange(n)
    offsets = np.array([0, n])
    res = acp.run(D, Dp, perm, offsets, k=k, t=3.0, T=10 ** 9)
    ep, ed = _exact_pairs(D, k)
    assert res.pairs.tolist() == ep.tolist()
    np.testing.assert_allclose(res.dist, ed, rtol=1e-12)
    assert res.n_cand_raw == 0


def test_topk_margin_is_the_smallest_relative_gap(small):
    """The per-kind margins: with one leaf the top-k margin is the smallest
    relative gap between consecutive exact distances of the k + 1 closest
    pairs (pdist as the reference), the reported margin is the smallest of
    all kinds, and a duplicated point (two pairs at one distance inside the
    top-k) gives a top-k margin of 0."""
    D, A, Dp = small
    n, k = D.shape[0], 25
    res = acp.run(D, Dp, np.arange(n), np.array([0, n]), k=k, t=3.0, T=10 ** 9)
    _, ed = _exact_pairs(D, k + 1)
    assert res.margins["topk_order"] == pytest.approx(float(np.min(np.diff(ed) / ed[:-1])),
                                                      rel=1e-9)
    assert res.margin == min(res.margins.values())
    ep, _ = _exact_pairs(D, 1)
    D2 = np.concatenate([D, D[ep[0, 0]][None]])
    Dp2 = ann.project(D2, A)
    res2 = acp.run(D2, Dp2, np.arange(n + 1), np.array([0, n + 1]), k=k, t=3.0, T=10 ** 9)
    assert res2.margins["topk_order"] == 0.0


def test_singleton_leaves_unbounded_budget_is_exact(small):
    D, A, Dp = small
    n, k = D.shape[0], 10
    res = acp.run(D, Dp, np.arange(n), np.arange(n + 1), k=k, t=3.0, T=10 ** 9)
    assert math.isinf(res.ub) and res.n_seed == 0
    assert res.n_cand_raw == n * (n - 1) // 2
    ep, ed = _exact_pairs(D, k)
    assert res.pairs.tolist() == ep.tolist()


def test_brute_closest_pairs_matches_pdist(small):
    D, _, _ = small
    bp, bd = brute.closest_pairs(D, 17)
    ep, ed = _exact_pairs(D, 17)
    assert bp.tolist() == ep.tolist()
    np.testing.assert_allclose(bd, ed, rtol=1e-12)


def test_filter_is_strict_threshold_on_projected_distance(small):
    D, A, Dp = small
    n, k = D.shape[0], 5
    rng = np.random.Generator(np.random.PCG64(4))
    perm = rng.permutation(n)
    L = 10
    offsets = np.arange(0, n + 1, L)
    t = chi2.radius_factor(1 / math.e, 15)
    res = acp.run(D, Dp, perm, offsets, k=k, t=t, T=10 ** 9)
    leaf_of = np.empty(n, dtype=np.int64)
    for b in range(len(offsets) - 1):
        leaf_of[perm[offsets[b]:offsets[b + 1]]] = b
    pv = pdist(Dp)
    ii, jj = np.triu_indices(n, k=1)
    expect = int(np.count_nonzero((pv < t * res.ub) & (leaf_of[ii] != leaf_of[jj])))
    assert res.n_cand_raw == expect
    assert res.n_seed == (n // L) * L * (L - 1) // 2
    # ub is the k-th smallest within-leaf distance
    dv = pdist(D.astype(np.float64))
    same = leaf_of[ii] == leaf_of[jj]
    assert res.ub == pytest.approx(np.sort(dv[same])[k - 1], rel=1e-12)


def test_budget_keeps_projected_nearest(small):
    D, A, Dp = small
    n, k = D.shape[0], 3
    perm = np.arange(n)
    offsets = np.arange(0, n + 1, 2)           # leaves of two points
    full = acp.run(D, Dp, perm, offsets, k=k, t=50.0, T=10 ** 9)
    T = full.n_seed + 40
    cut = acp.run(D, Dp, perm, offsets, k=k, t=50.0, T=T)
    assert cut.n_cand == 40 and cut.n_cand_raw == full.n_cand_raw
    assert T < full.n_seed + full.n_cand_raw
    # verified pairs of the cut run are a subset of the full run: the result
    # can only be worse or equal rank by rank
    assert np.all(cut.dist >= full.dist - 1e-12)


def test_planted_pairs_are_found():
    w = synth.planted_pairs(n=2000, d=32, n_centres=10)
    D, A, pairs = w["D"], w["A"], w["pairs"]
    Dp = ann.project(D, A)
    n, k = D.shape[0], 10
    rng = np.random.Generator(np.random.PCG64(9))
    perm = rng.permutation(n)                  # leaves unrelated to geometry
    offsets = np.arange(0, n + 1, 50)
    t = chi2.radius_factor(1 / math.e, 15)
    res = acp.run(D, Dp, perm, offsets, k=k, t=t, T=10 ** 9)
    pd_ = np.sqrt(((D[pairs[:, 0]].astype(np.float64) - D[pairs[:, 1]]) ** 2).sum(1))
    o = np.lexsort((pairs[:, 1], pairs[:, 0], pd_))[:k]
    assert metrics.pair_recall(res.pairs, pairs[o]) >= 0.8
    ep, ed = _exact_pairs(D, k)
    assert set(map(tuple, ep.tolist())) <= set(map(tuple, pairs.tolist()))
    assert np.all(res.dist >= ed - 1e-12)
    key = list(zip(res.dist.tolist(), res.pairs[:, 0].tolist(),
                   res.pairs[:, 1].tolist()))
    assert key == sorted(key)
    assert np.all(res.pairs[:, 0] < res.pairs[:, 1])


def _axis(points, scale):
    D = np.asarray(points, dtype=np.float32)
    A = np.array([[scale, 0.0]], dtype=np.float32)
    return D, ann.project(D, A)


def test_filter_threshold_is_strict():
    # leaves {0,1}, {2,3}, {4,5}; seed distances 2, 2, 1 -> ub (k=2) = 2 and
    # with t = 1 the filter radius is 2.  Every cross pair of the first two
    # leaves has projected distance exactly 2 (projection 2x), so none is a
    # candidate, although (0,2) and (1,3) are at exact distance 1.
    D, Dp = _axis([(0, 0), (0, 2), (1, 0), (1, 2), (50, 0), (50, 1)], 2.0)
    res = acp.run(D, Dp, np.arange(6), np.array([0, 2, 4, 6]), k=2, t=1.0,
                  T=10 ** 6)
    assert res.ub == 2.0 and res.n_cand_raw == 0
    assert res.pairs.tolist() == [[4, 5], [0, 1]]


def test_budget_cut_ranks_by_projected_distance():
    # singleton leaves: no seeds, ub = inf, all 3 pairs are candidates. T = 1
    # keeps the pair with the smallest projected distance, (0,1) (pd 1, exact
    # sqrt 26), not the exactly-closest pair (0,2) (pd 4, exact 4).
    D, Dp = _axis([(0, 0), (1, 5), (4, 0)], 1.0)
    res = acp.run(D, Dp, np.arange(3), np.arange(4), k=1, t=2.0, T=1)
    assert res.n_cand == 1 and res.n_cand_raw == 3
    assert res.pairs.tolist() == [[0, 1]]
    assert res.dist[0] == pytest.approx(math.sqrt(26.0))


# ---- branch and bound (Algorithm 3): the T projected-closest pairs, verified

def test_bb_trace_on_a_line():
    # projection onto the first coordinate: pd = |x_i - x_j|. Points
    # x = 0, 1, 3, 3.5 with y = 0, 5, 0, 0. Projected pair distances:
    # (2,3) 0.5, (0,1) 1, (1,2) 2, (1,3) 2.5, (0,2) 3, (0,3) 3.5. With T = 2
    # the candidates are (2,3) and (0,1), whose exact distances are 0.5 and
    # sqrt(26); k = 1 returns (2,3)
    D = np.array([[0, 0], [1, 5], [3, 0], [3.5, 0]], dtype=np.float32)
    A = np.array([[1.0, 0.0]], dtype=np.float32)
    res = acp.branch_and_bound(D, ann.project(D, A), k=2, T=2)
    assert res.pairs.tolist() == [[2, 3], [0, 1]]
    assert res.dist[0] == pytest.approx(0.5) and res.dist[1] == pytest.approx(math.sqrt(26))
    assert res.ub == pytest.approx(1.0)
    # T = 3 adds (1,2), exact sqrt(29): still ranked after (0,1)
    res = acp.branch_and_bound(D, ann.project(D, A), k=3, T=3)
    assert res.pairs.tolist() == [[2, 3], [0, 1], [1, 2]]


def test_bb_all_pairs_is_exact_closest_pairs():
    rng = np.random.Generator(np.random.PCG64(9))
    D = rng.standard_normal((120, 10)).astype(np.float32)
    A = rng.standard_normal((6, 10)).astype(np.float32)
    res = acp.branch_and_bound(D, ann.project(D, A), k=7, T=120 * 119 // 2)
    pairs, dist = brute.closest_pairs(D, 7)
    assert res.pairs.tolist() == pairs.tolist()
    np.testing.assert_allclose(res.dist, dist, rtol=1e-12)
    ref = np.sort(pdist(D.astype(np.float64)))[:7]
    np.testing.assert_allclose(res.dist, ref, rtol=1e-12)


def test_bb_candidates_are_the_projected_closest_pairs():
    rng = np.random.Generator(np.random.PCG64(10))
    D = rng.standard_normal((150, 12)).astype(np.float32)
    A = rng.standard_normal((5, 12)).astype(np.float32)
    Dp = ann.project(D, A)
    T = 40
    res = acp.branch_and_bound(D, Dp, k=40, T=T)
    # every pair returned is among the T smallest projected distances
    # (SciPy's pdist on the projections, an independent computation)
    pdp = squareform(pdist(Dp))
    thr = np.sort(pdist(Dp))[T - 1]
    for (i, j) in res.pairs:
        assert pdp[i, j] <= thr * (1 + 1e-12)
    assert res.n_cand == T
    # with an exact (orthonormal) projection the answer is the exact CP
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    res = acp.branch_and_bound(D, ann.project(D, Q.T.astype(np.float32)), k=5, T=5)
    pairs, _ = brute.closest_pairs(D, 5)
    assert res.pairs.tolist() == pairs.tolist()


# ---- radius filtering with FindLCA (Algorithms 4-5)

def _line_tree():
    """8 points on a line (y = 0), 4 leaves of 2, two inner nodes of two
    leaves each and a root; the projection is the first coordinate. All
    coordinates and differences are exact binary fractions."""
    x = [0, 0.125, 1, 1.125, 10, 10.125, 11, 11.125]
    D = np.array([[v, 0.0] for v in x], dtype=np.float32)
    Dp = ann.project(D, np.array([[1.0, 0.0]], dtype=np.float32))
    perm = np.arange(8, dtype=np.int32)
    offsets = np.array([0, 2, 4, 6, 8], dtype=np.int64)
    #            root  A    B    leaves
    level = np.array([0, 1, 1, 2, 2, 2, 2], dtype=np.int32)
    first = np.array([0, 0, 2, 0, 1, 2, 3], dtype=np.int32)
    end = np.array([4, 2, 4, 1, 2, 3, 4], dtype=np.int32)
    radius = np.array([6.0, 0.6, 0.6, 0.05, 0.05, 0.05, 0.05], dtype=np.float32)
    return D, Dp, perm, offsets, level, first, end, radius


def test_lca_trace_stops_after_the_node_that_passes_T():
    # seeds: four pairs at 0.125, ub (k = 2) = 0.125; t = 8, gamma = 1:
    # R = 1, FindLCA returns A and B (radius 0.6). In A the cross pairs have
    # projected distances 1, 1.125, 0.875, 1: only (1, 2) is below t ub = 1.
    # count = 5 > T = 4 after A, so B is never scanned.
    D, Dp, perm, off, lv, fl, el, rad = _line_tree()
    res = acp.radius_filtering_lca(D, Dp, perm, off, lv, fl, el, rad, k=2, t=8.0, T=4,
                                   gamma=1.0)
    assert res.n_seed == 4 and res.n_cand == 1
    assert res.pairs.tolist() == [[0, 1], [2, 3]]
    res = acp.radius_filtering_lca(D, Dp, perm, off, lv, fl, el, rad, k=2, t=8.0, T=100,
                                   gamma=1.0)
    assert res.n_cand == 2           # (1, 2) in A and (5, 6) in B


def test_lca_trace_findlca_descends_and_skips_leaves():
    # gamma = 0.5: R = 0.5 is below every inner radius, FindLCA descends to
    # the leaves, which it never returns: only the seeds are verified
    D, Dp, perm, off, lv, fl, el, rad = _line_tree()
    res = acp.radius_filtering_lca(D, Dp, perm, off, lv, fl, el, rad, k=2, t=8.0, T=100,
                                   gamma=0.5)
    assert res.n_cand == 0 and res.pairs.tolist() == [[0, 1], [2, 3]]


def test_lca_trace_unbounded_ub_scans_the_root():
    # k = 5 > 4 seeds: ub = +inf, R = +inf, FindLCA returns the root and all
    # 24 cross-leaf pairs are verified; the fifth nearest is (1, 2) at 0.875
    # (tied with (5, 6), which has the larger ids)
    D, Dp, perm, off, lv, fl, el, rad = _line_tree()
    res = acp.radius_filtering_lca(D, Dp, perm, off, lv, fl, el, rad, k=5, t=8.0, T=1000,
                                   gamma=1.0)
    assert res.n_cand == 24
    assert res.pairs.tolist() == [[0, 1], [2, 3], [4, 5], [6, 7], [1, 2]]
    assert res.dist[4] == 0.875


def test_lca_with_root_found_equals_canonical_filter():
    """With R above the root's radius the one node scanned is the root, with
    the self-join ub, so the candidates are those of the canonical filter."""
    w = synth.parity(n=600, n_queries=1)
    D, A = w["D"], w["A"]
    Dp = ann.project(D, A)
    L = 32
    perm = np.random.Generator(np.random.PCG64(1)).permutation(600).astype(np.int32)
    off = np.array([min(600, b * L) for b in range(600 // L + 2)], dtype=np.int64)
    off = np.unique(off)
    nl = off.shape[0] - 1
    level = np.concatenate([[0], np.ones(nl, dtype=np.int32)]).astype(np.int32)
    first = np.concatenate([[0], np.arange(nl)]).astype(np.int32)
    end = np.concatenate([[nl], np.arange(1, nl + 1)]).astype(np.int32)
    radius = np.concatenate([[1.0], np.zeros(nl)]).astype(np.float32)
    t = chi2.radius_factor(0.1, A.shape[0])
    T = 10 ** 9
    res = acp.radius_filtering_lca(D, Dp, perm, off, level, first, end, radius, k=5, t=t, T=T,
                                   gamma=1e9)
    ref = acp.run(D, Dp, perm, off, k=5, t=t, T=T)
    assert res.pairs.tolist() == ref.pairs.tolist()
    assert res.n_cand == ref.n_cand_raw
