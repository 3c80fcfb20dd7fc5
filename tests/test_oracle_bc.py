"""Pins of the oracle's (r,c)-BC query (Algorithm 1, Section 5.1).

* Hand-traced runs: points in the plane projected onto the first
  coordinate (m = 1) or scaled down by 10 (projected distances a tenth of
  the true ones), with t given directly, so every ball, candidate set and
  answer can be followed by hand: an empty ball, a ball below the budget
  with and without a point within c r, a ball that reaches the budget, and
  the (pd, id) order of the budget cut.
* Special cases: an unbounded radius with B = n returns the exact nearest
  neighbour (SciPy's k-d tree); an unbounded radius with any B gives the
  answer of the ANN oracle with k = 1 and the same budget (a separately
  pinned function); the answer of a ball below the budget is within c r.
* The definition of the (r,c)-BC query on a seeded mixture with the planner's
  t and beta: when B(q, r) holds a point, a point within c r is returned for
  most queries (the constant-probability guarantee of Theorem 1's setting).
"""

import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from oracle import ann, bc, chi2

ON_AXIS = [(1, 0), (2, 0), (4, 0), (8, 0), (16, 0)]


def _setup(points, A, qpt=(0.0, 0.0)):
    D = np.asarray(points, dtype=np.float32)
    A = np.asarray(A, dtype=np.float32)
    q = np.asarray(qpt, dtype=np.float32)
    return D, ann.project(D, A), q, ann.project(q[None, :], A)[0]


def test_trace_empty_ball_returns_nothing():
    D, Dp, q, qp = _setup(ON_AXIS, [[1.0, 0.0]])
    res = bc.query(D, Dp, q, qp, r=0.5, c=2.0, t=1.0, budget=3)
    assert res.id == -1 and math.isinf(res.dist)
    assert res.kind == bc.KIND_NONE and res.n_cand == 0


def test_trace_ball_below_budget_with_point_within_cr():
    # r = 2, t = 1: the closed ball of radius 2 holds ids 0, 1 (pd 1, 2);
    # 2 < B = 3; the nearest, id 0 at distance 1, is within c r = 4
    D, Dp, q, qp = _setup(ON_AXIS, [[1.0, 0.0]])
    res = bc.query(D, Dp, q, qp, r=2.0, c=2.0, t=1.0, budget=3)
    assert (res.id, res.dist, res.kind, res.n_cand) == (0, 1.0, bc.KIND_FOUND, 2)


def test_trace_ball_below_budget_without_point_within_cr():
    # projection scaled by 1/10: pd = dist / 10. r = 0.25, t = 1: the ball
    # (pd <= 0.25) holds ids 0 and 1 (dist 1 and 2); c r = 0.5 < 1, nothing
    D, Dp, q, qp = _setup(ON_AXIS, [[0.1, 0.0]])
    res = bc.query(D, Dp, q, qp, r=0.25, c=2.0, t=1.0, budget=3)
    assert res.id == -1 and math.isinf(res.dist)
    assert res.kind == bc.KIND_NONE and res.n_cand == 2


def test_trace_ball_reaching_budget_answers_without_cr_test():
    # projection scaled by 1/10, r = 0.45, t = 1: the ball pd <= 0.45 holds
    # ids 0, 1, 2 (dist 1, 2, 4) and reaches B = 3; c r = 0.675 < 1, yet the
    # budget exit returns the nearest candidate, id 0
    D, Dp, q, qp = _setup(ON_AXIS, [[0.1, 0.0]])
    res = bc.query(D, Dp, q, qp, r=0.45, c=1.5, t=1.0, budget=3)
    assert (res.id, res.dist, res.kind, res.n_cand) == (0, 1.0, bc.KIND_BUDGET, 3)


def test_trace_budget_cut_by_projected_distance_then_id():
    # points at equal projected distance 1 (x = 1) but different true
    # distances; B = 2 keeps the two smallest ids among the three tied
    # projected distances, so the true nearest (id 2, at (1, 0)) is cut
    pts = [(1, 3), (1, -2), (1, 0), (5, 0)]
    D, Dp, q, qp = _setup(pts, [[1.0, 0.0]])
    res = bc.query(D, Dp, q, qp, r=10.0, c=2.0, t=1.0, budget=2)
    assert res.kind == bc.KIND_BUDGET and res.n_cand == 2
    assert res.id == 1 and res.dist == pytest.approx(math.sqrt(5.0))


@pytest.fixture(scope="module")
def small_mixture():
    w = synth.parity(n=1500, n_queries=25)
    return w["D"], w["A"], w["Q"], ann.project(w["D"], w["A"])


def test_unbounded_radius_full_budget_is_exact_nn(small_mixture):
    D, A, Q, Dp = small_mixture
    tree = cKDTree(D.astype(np.float64))
    dd, ii = tree.query(Q.astype(np.float64), k=1)
    res = bc.run(D, A, Q, r=1e30, c=1.5, t=4.0, budget=D.shape[0], Dp=Dp)
    for r_, i_, d_ in zip(res, ii, dd):
        assert r_.kind == bc.KIND_BUDGET
        assert r_.id == int(i_) and r_.dist == pytest.approx(d_, rel=1e-12)


def test_unbounded_radius_matches_ann_with_k_1(small_mixture):
    D, A, Q, Dp = small_mixture
    B = 40
    res = bc.run(D, A, Q, r=1e30, c=1.5, t=4.0, budget=B, Dp=Dp)
    ref = ann.run(D, A, Q, 1, 1.5, 4.0, B, 1e30, Dp=Dp)
    for a, b in zip(res, ref):
        assert b.exit_kind == ann.EXIT_BUDGET
        assert a.id == int(b.ids[0]) and a.dist == b.dist[0]


def test_ball_below_budget_answers_within_cr(small_mixture):
    D, A, Q, Dp = small_mixture
    nn = cKDTree(D.astype(np.float64)).query(Q.astype(np.float64), k=1)[0]
    t = chi2.radius_factor(0.1, A.shape[0])
    for scale in (0.5, 1.0, 1.5):
        r = float(np.median(nn)) * scale
        for res in bc.run(D, A, Q, r=r, c=1.5, t=t, budget=D.shape[0], Dp=Dp):
            assert res.kind != bc.KIND_BUDGET
            if res.kind == bc.KIND_FOUND:
                assert res.dist <= 1.5 * r
            else:
                assert res.id == -1


def test_definition_holds_for_most_queries():
    """Queries whose B(q, r) holds a point get a point within c r back for at
    least the constant fraction the parameter setting promises (E1 and E2
    hold together with probability >= 1 - alpha1 - alpha2 / beta = 1/2 at
    beta = 2 alpha2; observed rates are far higher)."""
    w = synth.parity(n=4000, n_queries=80)
    D, A, Q = w["D"], w["A"], w["Q"]
    m, c, alpha1 = A.shape[0], 1.5, 0.1
    t = chi2.radius_factor(alpha1, m)
    budget = chi2.ann_budget(chi2.default_beta(alpha1, c, m), D.shape[0], 1)
    nn = cKDTree(D.astype(np.float64)).query(Q.astype(np.float64), k=1)[0]
    r = float(np.quantile(nn, 0.5))
    res = bc.run(D, A, Q, r=r, c=c, t=t, budget=budget)
    covered = nn <= r
    ok = [x.id >= 0 and x.dist <= c * r for x, cov in zip(res, covered) if cov]
    assert len(ok) >= 20
    assert np.mean(ok) >= 0.5
