"""Pins of the oracle's (c,k)-ANN (Algorithm 2, Section 5.2).

* Hand-traced runs on points on a line, where the projection is the first
  coordinate (m = 1, A = [1, 0]) and t is set to 1, so every projected
  distance, ball and round can be followed by hand. They fix the closed
  ball, the c r stopping test against c times the enlarged radius, the growth
  r <- c r, the budget exit and the (pd, id) order of the budget cut.
* Special cases that reduce to exact search: with B = n and an unbounded
  first radius the answer is the exact kNN (checked with SciPy's k-d tree);
  with B = k it is the k projected-nearest points re-ranked by exact
  distance (projected neighbours also found with SciPy's k-d tree).
* Invariants and the guarantee of Theorem 1 on a seeded mixture.
"""

import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from oracle import ann, chi2, metrics, rmin


def _line(points, qpt=(0.0, 0.0)):
    D = np.asarray(points, dtype=np.float32)
    A = np.array([[1.0, 0.0]], dtype=np.float32)
    q = np.asarray(qpt, dtype=np.float32)
    Dp = ann.project(D, A)
    qp = ann.project(q[None, :], A)[0]
    return D, Dp, q, qp


ON_AXIS = [(1, 0), (2, 0), (4, 0), (8, 0), (16, 0)]


def test_trace_closed_ball_and_cr_stop():
    # r = 0.5: ball empty.  r = 1: the point at projected distance exactly 1
    # is inside the closed ball, C = {0}.  r = 2: the c r stop with c r = 4 finds
    # 1 <= 4 and stops after two range queries.  An open ball would need a
    # third range query.
    D, Dp, q, qp = _line(ON_AXIS)
    res = ann.query(D, Dp, q, qp, k=1, c=2.0, t=1.0, budget=3, r_min=0.5)
    assert res.ids.tolist() == [0]
    assert res.dist.tolist() == [1.0]
    assert res.exit_kind == ann.EXIT_NEAR
    assert res.rounds == 2
    assert res.r_final == 2.0


def test_trace_cr_stop_needs_k_points():
    D, Dp, q, qp = _line(ON_AXIS)
    res = ann.query(D, Dp, q, qp, k=2, c=2.0, t=1.0, budget=3, r_min=0.5)
    # r=.5 {} ; r=1 {0} ; r=2: the c r stop (c r = 4) counts 1 < 2, ball {0,1} < 3 ;
    # r=4: the c r stop (c r = 8) counts 2 -> stop
    assert res.ids.tolist() == [0, 1]
    assert res.rounds == 3 and res.exit_kind == ann.EXIT_NEAR
    assert res.n_cand == 2


def test_trace_budget_exit():
    D, Dp, q, qp = _line(ON_AXIS)
    res = ann.query(D, Dp, q, qp, k=2, c=2.0, t=1.0, budget=2, r_min=0.5)
    # r=2: the c r stop counts 1 < 2, then the ball {0,1} reaches B = 2
    assert res.ids.tolist() == [0, 1]
    assert res.rounds == 3 and res.exit_kind == ann.EXIT_BUDGET


def test_trace_cr_stop_uses_enlarged_radius():
    # point 0 is nearest in projection (pd 1) but at exact distance sqrt(10).
    # After the first range query (r = 1, C = {0}), r becomes 2 and the c r stop
    # compares sqrt(10) with c r = 4: stop with point 0. Comparing with r or
    # with c times the old radius (2) would not stop and would return point 1.
    D, Dp, q, qp = _line([(1, 3), (2, 0), (4, 0), (8, 0), (16, 0)])
    res = ann.query(D, Dp, q, qp, k=1, c=2.0, t=1.0, budget=4, r_min=1.0)
    assert res.ids.tolist() == [0]
    assert res.dist[0] == pytest.approx(math.sqrt(10.0), rel=1e-7)
    assert res.rounds == 1


def test_trace_budget_cut_by_projected_distance_then_id():
    # projected distances 5, 3, 3, 3, 1 (ids 0..4); the ball at r = 3 holds
    # ids 1,2,3,4 >= B = 3, so C = the 3 smallest (pd, id): ids 4, 1, 2.
    # id 3 (exact distance 3.0017, the true nearest) loses the tie on id.
    pts = [(5, 0), (3, 1), (-3, 2), (3, 0.1), (1, 10)]
    D, Dp, q, qp = _line(pts)
    res = ann.query(D, Dp, q, qp, k=2, c=2.0, t=1.0, budget=3, r_min=3.0)
    assert res.exit_kind == ann.EXIT_BUDGET and res.rounds == 1
    assert res.ids.tolist() == [1, 2]
    assert res.dist[0] == pytest.approx(math.sqrt(10.0), rel=1e-7)
    assert res.dist[1] == pytest.approx(math.sqrt(13.0), rel=1e-7)


@pytest.fixture(scope="module")
def small_mixture():
    w = synth.parity(n=3000, n_queries=40)
    w["Dp"] = ann.project(w["D"], w["A"])
    return w


def test_exact_special_case_full_budget(small_mixture):
    w = small_mixture
    D, A, Q = w["D"], w["A"], w["Q"]
    n, k = D.shape[0], 10
    t = chi2.radius_factor(0.1, 15)
    res = ann.run(D, A, Q, k=k, c=1.5, t=t, budget=n, r_min=math.inf, Dp=w["Dp"])
    tree = cKDTree(D.astype(np.float64))
    dd, ii = tree.query(Q.astype(np.float64), k=k, eps=0.0)
    for r, di, ii_ in zip(res, dd, ii):
        assert r.ids.tolist() == ii_.tolist()
        np.testing.assert_allclose(r.dist, di, rtol=1e-12)


def test_special_case_budget_k_is_projected_knn(small_mixture):
    w = small_mixture
    D, A, Q = w["D"], w["A"], w["Q"]
    k = 5
    res = ann.run(D, A, Q, k=k, c=1.5, t=3.0, budget=k, r_min=math.inf,
                  Dp=w["Dp"])
    ptree = cKDTree(w["Dp"])
    Qp = Q.astype(np.float64) @ A.astype(np.float64).T
    _, pidx = ptree.query(Qp, k=k, eps=0.0)
    for qi, r in enumerate(res):
        assert sorted(r.ids.tolist()) == sorted(pidx[qi].tolist())
        ex = np.sqrt(((D[pidx[qi]].astype(np.float64) - Q[qi]) ** 2).sum(1))
        o = np.lexsort((pidx[qi], ex))
        assert r.ids.tolist() == pidx[qi][o].tolist()


def test_invariants_and_theorem1(small_mixture):
    w = small_mixture
    D, A, Q = w["D"], w["A"], w["Q"]
    n, k, c = D.shape[0], 10, 1.5
    alpha1 = 1 / math.e
    t = chi2.radius_factor(alpha1, 15)
    beta = 0.02
    B = chi2.ann_budget(beta, n, k)
    r0 = rmin.r_min(D, seed=5, budget=B)
    res = ann.run(D, A, Q, k=k, c=c, t=t, budget=B, r_min=r0, Dp=w["Dp"])
    tree = cKDTree(D.astype(np.float64))
    dd, ii = tree.query(Q.astype(np.float64), k=k)
    good = 0
    for r, dstar in zip(res, dd):
        assert len(set(r.ids.tolist())) == k
        assert r.ids.min() >= 0 and r.ids.max() < n
        key = list(zip(r.dist.tolist(), r.ids.tolist()))
        assert key == sorted(key)
        assert np.all(r.dist >= dstar - 1e-12)          # rank-wise >= exact
        assert r.n_cand <= B
        if r.exit_kind == ann.EXIT_NEAR:
            assert r.dist[-1] <= c * r.r_final
        assert metrics.overall_ratio(r.dist, dstar) >= 1.0
        good += r.dist[0] <= c * c * dstar[0]
    # Theorem 1: a c^2-approximate nearest neighbour with prob >= 1/2 - 1/e
    assert good / len(res) >= 0.5 - 1 / math.e


def test_parity_workload_quality():
    # the parity workload (k=10, c=1.5, confidence 0.9, beta=0.1) on a
    # 20-query slice: every query should find its exact 10 NN
    w = synth.parity(n_queries=20)
    D, A, Q = w["D"], w["A"], w["Q"]
    n, k = D.shape[0], 10
    t = chi2.radius_factor(0.1, 15)
    B = chi2.ann_budget(0.1, n, k)
    r0 = rmin.r_min(D, seed=1, budget=B)
    res = ann.run(D, A, Q, k=k, c=1.5, t=t, budget=B, r_min=r0)
    _, ii = cKDTree(D.astype(np.float64)).query(Q.astype(np.float64), k=k)
    rec = metrics.recall(np.stack([r.ids for r in res]), ii)
    assert rec >= 0.95


def test_trace_cr_stop_threshold_is_c_times_r():
    # point 0: projected distance 1, exact sqrt(26) = 5.10.  After r = 1
    # (C = {0}) the radius becomes 2 and the c r stop compares 5.10 with c r = 4:
    # no stop.  The ball at r = 2 adds point 1 (exact 2); r becomes 4 and
    # the c r stop (c r = 8) ends the loop; the answer is point 1.  A test against c^2 r
    # would stop one round early with point 0.
    D, Dp, q, qp = _line([(1, 5), (2, 0), (4, 0), (8, 0), (16, 0)])
    res = ann.query(D, Dp, q, qp, k=1, c=2.0, t=1.0, budget=4, r_min=1.0)
    assert res.ids.tolist() == [1]
    assert res.rounds == 2 and res.r_final == 4.0


def test_trace_radius_grows_by_c():
    # B = 5 is never reached before r = 8: r = 1 {0}, 2 {0,1}, 4 {0,1,2},
    # the c r stop never fires because k = 5 > |C|; at r = 16 the ball holds all
    # five points (>= B): 5 range queries with r = 1, 2, 4, 8, 16.
    D, Dp, q, qp = _line(ON_AXIS)
    res = ann.query(D, Dp, q, qp, k=5, c=2.0, t=1.0, budget=5, r_min=1.0)
    assert res.rounds == 5 and res.r_final == 16.0
    assert res.exit_kind == ann.EXIT_BUDGET
