"""Pins of the oracle's decision margins, and of the helpers the parity
checks rest on (brute-force kNN, the r_min pair sample).

The margins decide how strictly the GPU results are compared: a query whose
every margin clears the tolerance must match the oracle exactly, so a wrong
margin would quietly move real mismatches into the looser comparison. Each
kind is pinned on a hand-traced fixture whose gaps are worked out below, on
points in the plane projected onto the first coordinate (m = 1) with t = 1
(so the projected distance is |x| and every ball can be followed by hand):

  ANN (Algorithm 2, Section 5.2)  ball_count, ball_member, budget_cut,
                                  cr_stop, topk_order
  BC  (Algorithm 1, Section 5.1)  ball_count, ball_member, budget_cut,
                                  nearest_order, within_cr
  ACP (Section 6.3; Algorithm 3, Section 6.1; Algorithms 4-5)
                                  pair_filter, budget_cut, topk_order, find_lca

Each fixture is chosen so that the plausible mistakes give a different
number: the c r threshold taken against r, against c times the previous r or
against c^2 r; the ball-member gap taken over the members only or over the
non-members only; the budget gap one place off; the top-k gaps without the
(k+1)-th value; the pair-filter gap over the candidates only or the
non-candidates only, or with the (k+1)-th seed as ub.
"""

import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from oracle import acp, ann, bc, brute, rmin

GAMMA = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def _line(points, scale=1.0):
    D = np.asarray(points, dtype=np.float32)
    A = np.array([[scale, 0.0]], dtype=np.float32)
    q = np.zeros(2, dtype=np.float32)
    return D, ann.project(D, A), q, ann.project(q[None, :], A)[0]


# ------------------------------------------------------------------ ANN

def test_ann_margins_nearest_to_threshold_is_a_member():
    # projected distances 1, 3, 5, 9, 20; k = 1, c = 2, B = 3, r_min = 1.5.
    # Round 0: R = 1.5. The B-th projected distance is 5: ball_count =
    #   |5 - 1.5| / 1.5 = 7/3. The ball {pd 1} is short of B, so every
    #   point's membership counts: the closest pd to R is the member at 1,
    #   ball_member = 0.5 / 1.5 = 1/3 (over the non-members only: 1.5/1.5).
    # Round 1: r = 3, the c r stop compares the exact distance 1 with
    #   c r = 6: cr_stop = 5/6 (against r: 2/3; against c^2 r: 11/12), and
    #   stops with one point. One candidate: no top-k order gap.
    D, Dp, q, qp = _line([(1, 0), (3, 0), (5, 1), (9, 0), (20, 0)])
    res = ann.query(D, Dp, q, qp, k=1, c=2.0, t=1.0, budget=3, r_min=1.5)
    assert res.exit_kind == ann.EXIT_NEAR and res.rounds == 1
    assert set(res.margins) == {"ball_count", "ball_member", "cr_stop"}
    assert res.margins["ball_count"] == pytest.approx(7 / 3, rel=1e-12)
    assert res.margins["ball_member"] == pytest.approx(1 / 3, rel=1e-12)
    assert res.margins["cr_stop"] == pytest.approx(5 / 6, rel=1e-12)
    assert res.margin == pytest.approx(1 / 3, rel=1e-12)
    assert res.margin_kind == "ball_member"


def test_ann_margins_nearest_to_threshold_is_outside_the_ball():
    # the same points, r_min = 2.5: the ball {pd 1} is short of B = 3 and
    # the pd closest to R = 2.5 is the non-member at 3: ball_member =
    # 0.5 / 2.5 = 0.2 (over the members only: 1.5 / 2.5 = 0.6);
    # ball_count = |5 - 2.5| / 2.5 = 1; round 1 (r = 5): cr_stop =
    # |1 - 10| / 10 = 0.9
    D, Dp, q, qp = _line([(1, 0), (3, 0), (5, 1), (9, 0), (20, 0)])
    res = ann.query(D, Dp, q, qp, k=1, c=2.0, t=1.0, budget=3, r_min=2.5)
    assert res.margins["ball_member"] == pytest.approx(0.2, rel=1e-12)
    assert res.margins["ball_count"] == pytest.approx(1.0, rel=1e-12)
    assert res.margins["cr_stop"] == pytest.approx(0.9, rel=1e-12)


def test_ann_margins_budget_exit_and_topk_order():
    # points (pd, exact): id0 (1, sqrt 1.25), id1 (2, 2), id2 (2.5, 2.5),
    # id3 (4, 4), id4 (6, 6), id5 (8, 8); k = 2, B = 3, r_min = 5.
    # Round 0: R = 5 holds four points >= B: ball_count = |2.5 - 5| / 5 = 0.5
    #   (taking the (B+1)-th instead: |4 - 5| / 5 = 0.2);
    #   C = ids 0, 1, 2; budget_cut = (4 - 2.5) / 2.5 = 0.6 (one place lower:
    #   0.25; one higher: 0.5).
    # top-k order over the k + 1 = 3 nearest exact distances sqrt 1.25, 2,
    #   2.5: gaps 2 / sqrt 1.25 - 1 = 0.78885 and 0.25, so 0.25 (without the
    #   (k+1)-th: 0.78885)
    pts = [(1, 0.5), (2, 0), (2.5, 0), (4, 0), (6, 0), (8, 0)]
    D, Dp, q, qp = _line(pts)
    res = ann.query(D, Dp, q, qp, k=2, c=2.0, t=1.0, budget=3, r_min=5.0)
    assert res.exit_kind == ann.EXIT_BUDGET and res.rounds == 1
    assert res.ids.tolist() == [0, 1]
    assert set(res.margins) == {"ball_count", "budget_cut", "topk_order"}
    assert res.margins["ball_count"] == pytest.approx(0.5, rel=1e-12)
    assert res.margins["budget_cut"] == pytest.approx(0.6, rel=1e-12)
    assert res.margins["topk_order"] == pytest.approx(0.25, rel=1e-12)
    assert res.margin_kind == "topk_order"


def test_ann_cr_stop_margin_is_over_every_member():
    # id0 (pd 1, exact 1), id1 (pd 1.5, exact 2.5), id2 (pd 10); k = 1,
    # c = 2, B = 3, r_min = 2. Round 0: R = 2, ball {0, 1} < B:
    # ball_count = |10 - 2| / 2 = 4, ball_member = 0.5 / 2 = 0.25.
    # Round 1: r = 4, c r = 8: the member closest to 8 is id1 at 2.5, so
    # cr_stop = 5.5 / 8 = 0.6875 (the k-th member alone would give 7/8).
    # top-k over both candidates: 2.5 / 1 - 1 = 1.5
    D, Dp, q, qp = _line([(1, 0), (1.5, 2), (10, 0)])
    res = ann.query(D, Dp, q, qp, k=1, c=2.0, t=1.0, budget=3, r_min=2.0)
    assert res.exit_kind == ann.EXIT_NEAR and res.rounds == 1 and res.n_cand == 2
    assert res.margins["ball_count"] == pytest.approx(4.0, rel=1e-12)
    assert res.margins["ball_member"] == pytest.approx(0.25, rel=1e-12)
    assert res.margins["cr_stop"] == pytest.approx(0.6875, rel=1e-12)
    assert res.margins["topk_order"] == pytest.approx(1.5, rel=1e-12)


def test_ann_margins_are_minima_over_rounds():
    # id0 (pd 1, exact sqrt 26), then pd 2, 4, 8, 16 on the axis; k = 1,
    # c = 2, B = 4, r_min = 1.
    # Round 0: R = 1: the point at pd 1 sits on the closed ball's boundary,
    #   ball_member = 0; ball_count = |8 - 1| / 1 = 7.
    # Round 1: r = 2, c r = 4: |sqrt 26 - 4| / 4 = 0.27475 (no stop); R = 2,
    #   ball_count = 3, the point at pd 2 on the boundary again.
    # Round 2: r = 4, c r = 8: members at sqrt 26 and 2, the closer to 8 is
    #   sqrt 26: (8 - sqrt 26) / 8 = 0.36262; stop. cr_stop keeps the
    #   smaller, 0.27475; ball_count the smaller, 3.
    D, Dp, q, qp = _line([(1, 5), (2, 0), (4, 0), (8, 0), (16, 0)])
    res = ann.query(D, Dp, q, qp, k=1, c=2.0, t=1.0, budget=4, r_min=1.0)
    assert res.rounds == 2 and res.exit_kind == ann.EXIT_NEAR
    assert res.margins["ball_member"] == 0.0
    assert res.margins["ball_count"] == pytest.approx(3.0, rel=1e-12)
    assert res.margins["cr_stop"] == pytest.approx(abs(math.sqrt(26.0) - 4) / 4, rel=1e-12)
    assert res.margin == 0.0 and res.margin_kind == "ball_member"


# ------------------------------------------------------------------ BC

def test_bc_margins_ball_below_budget():
    # pd 1, 2, 4, 8, 16 on the axis; r = 2.8, c = 2, t = 1, B = 3:
    # R = 2.8, the B-th pd is 4: ball_count = 1.2 / 2.8; ball {1, 2}:
    # ball_member = 0.8 / 2.8 (the pd at 2); nearest order 2 / 1 - 1 = 1;
    # within_cr: |1 - c r| / (c r) = 4.6 / 5.6 (against r: 1.8 / 2.8)
    D, Dp, q, qp = _line([(1, 0), (2, 0), (4, 0), (8, 0), (16, 0)])
    res = bc.query(D, Dp, q, qp, r=2.8, c=2.0, t=1.0, budget=3)
    assert res.kind == bc.KIND_FOUND and res.id == 0
    assert set(res.margins) == {"ball_count", "ball_member", "nearest_order", "within_cr"}
    assert res.margins["ball_count"] == pytest.approx(1.2 / 2.8, rel=1e-12)
    assert res.margins["ball_member"] == pytest.approx(0.8 / 2.8, rel=1e-12)
    assert res.margins["nearest_order"] == pytest.approx(1.0, rel=1e-12)
    assert res.margins["within_cr"] == pytest.approx(4.6 / 5.6, rel=1e-12)
    assert res.margin == pytest.approx(0.8 / 2.8, rel=1e-12)


def test_bc_margins_budget_exit():
    # projection x / 8 (exact in binary): pd 0.125, 0.25, 0.5, 0.75, 2;
    # r = 0.625, B = 3: R = 0.625, the B-th pd 0.5: ball_count = 0.2; the
    # ball holds 3 >= B: budget_cut = (0.75 - 0.5) / 0.5 = 0.5 (one place
    # lower: 1; one higher: 5/3); the candidates' exact distances 1, 2, 4:
    # nearest_order = 1; no c r test
    D, Dp, q, qp = _line([(1, 0), (2, 0), (4, 0), (6, 0), (16, 0)], scale=0.125)
    res = bc.query(D, Dp, q, qp, r=0.625, c=1.5, t=1.0, budget=3)
    assert res.kind == bc.KIND_BUDGET and res.id == 0 and res.n_cand == 3
    assert set(res.margins) == {"ball_count", "budget_cut", "nearest_order"}
    assert res.margins["ball_count"] == pytest.approx(0.2, rel=1e-12)
    assert res.margins["budget_cut"] == pytest.approx(0.5, rel=1e-12)
    assert res.margins["nearest_order"] == pytest.approx(1.0, rel=1e-12)


# ------------------------------------------------------------------ ACP

def _acp_fixture():
    # leaves {0, 1}, {2, 3}, {4, 5}, the projection is the first coordinate:
    #   id0 (0, 0), id1 (0, 1)        seed distance 1
    #   id2 (3, 0), id3 (3.25, 1.5)   seed distance sqrt(0.0625 + 2.25)
    #   id4 (10, 0), id5 (10.5, 0)    seed distance 0.5
    pts = [(0, 0), (0, 1), (3, 0), (3.25, 1.5), (10, 0), (10.5, 0)]
    D = np.asarray(pts, dtype=np.float32)
    Dp = ann.project(D, np.array([[1.0, 0.0]], dtype=np.float32))
    return D, Dp, np.arange(6), np.array([0, 2, 4, 6])


def test_acp_margins_pair_filter_and_topk():
    # k = 2: seeds sorted 0.5, 1, 1.52069: ub = 1; t = 4, so R = 4.
    # Cross-leaf projected distances: first-second leaf 3, 3.25, 3, 3.25
    # (all candidates, gaps 0.25 and 0.1875); second-third 6.75 .. 7.5
    # (gap >= 0.6875); first-third 10, 10.5 (gap >= 1.5). pair_filter =
    # 0.1875 (over the non-candidates only: 0.6875; with the third seed as
    # ub, R = 6.08: a different gap). top-k over the three smallest: 0.5, 1,
    # 1.52069: gaps 1 and 0.52069
    D, Dp, perm, off = _acp_fixture()
    res = acp.run(D, Dp, perm, off, k=2, t=4.0, T=10 ** 6)
    assert res.ub == 1.0 and res.n_seed == 3 and res.n_cand_raw == 4
    assert res.pairs.tolist() == [[4, 5], [0, 1]]
    assert set(res.margins) == {"pair_filter", "topk_order"}
    assert res.margins["pair_filter"] == pytest.approx(0.1875, rel=1e-12)
    assert res.margins["topk_order"] == pytest.approx(math.sqrt(2.3125) - 1, rel=1e-12)


def test_acp_pair_filter_margin_counts_non_candidates():
    # t = 5.5: R = 5.5; the candidates' gaps are (5.5 - 3.25) / 5.5 and
    # more, the closest pair to R is the non-candidate (3, 4) at 6.75:
    # pair_filter = 1.25 / 5.5 (over the candidates only: 2.25 / 5.5)
    D, Dp, perm, off = _acp_fixture()
    res = acp.run(D, Dp, perm, off, k=2, t=5.5, T=10 ** 6)
    assert res.n_cand_raw == 4
    assert res.margins["pair_filter"] == pytest.approx(1.25 / 5.5, rel=1e-12)


def test_acp_margins_budget_cut():
    # T = 3 seeds + 2: the four candidates sorted by (pd, i, j) are (0,2) 3,
    # (1,2) 3, (0,3) 3.25, (1,3) 3.25; the cut keeps two, budget_cut =
    # (3.25 - 3) / 3 = 1/12 (one place later: 0; one earlier: 0)
    D, Dp, perm, off = _acp_fixture()
    res = acp.run(D, Dp, perm, off, k=2, t=4.0, T=5)
    assert res.n_cand == 2 and res.n_cand_raw == 4
    assert res.margins["budget_cut"] == pytest.approx(1 / 12, rel=1e-12)
    assert res.margins["pair_filter"] == pytest.approx(0.1875, rel=1e-12)


def test_bb_margins():
    # x = 0, 1, 3, 3.5 (y = 0, 5, 0, 0): projected pair distances (2,3) 0.5,
    # (0,1) 1, (1,2) 2, ...; T = 2: budget_cut = (2 - 1) / 1 = 1; the two
    # verified distances 0.5 and sqrt 26: topk_order = sqrt 26 / 0.5 - 1
    D = np.array([[0, 0], [1, 5], [3, 0], [3.5, 0]], dtype=np.float32)
    res = acp.branch_and_bound(D, ann.project(D, np.array([[1.0, 0.0]], dtype=np.float32)),
                               k=2, T=2)
    assert res.margins["budget_cut"] == pytest.approx(1.0, rel=1e-12)
    assert res.margins["topk_order"] == pytest.approx(math.sqrt(26.0) / 0.5 - 1, rel=1e-12)


def test_lca_margins():
    # the eight-point line tree (leaves of two points 0.125 apart, inner
    # nodes of radius 0.6, root 6): k = 2, t = 8, gamma = 1: ub = 0.125,
    # R = gamma t ub = 1. FindLCA tests the root (|6 - 1| / 1 = 5) and the
    # two inner nodes (|0.6 - 1| / 1 = 0.4): find_lca = 0.4 (in float32
    # 0.6 is 0.60000002384). In the first inner node the cross pairs'
    # projected distances 1, 1.125, 0.875, 1 against t ub = 1: two lie on
    # the threshold, pair_filter = 0
    x = [0, 0.125, 1, 1.125, 10, 10.125, 11, 11.125]
    D = np.array([[v, 0.0] for v in x], dtype=np.float32)
    Dp = ann.project(D, np.array([[1.0, 0.0]], dtype=np.float32))
    level = np.array([0, 1, 1, 2, 2, 2, 2], dtype=np.int32)
    first = np.array([0, 0, 2, 0, 1, 2, 3], dtype=np.int32)
    end = np.array([4, 2, 4, 1, 2, 3, 4], dtype=np.int32)
    radius = np.array([6.0, 0.6, 0.6, 0.05, 0.05, 0.05, 0.05], dtype=np.float32)
    res = acp.radius_filtering_lca(D, Dp, np.arange(8, dtype=np.int32),
                                   np.array([0, 2, 4, 6, 8]), level, first, end, radius,
                                   k=2, t=8.0, T=4, gamma=1.0)
    assert res.margins["find_lca"] == pytest.approx(1 - float(np.float32(0.6)), rel=1e-12)
    assert res.margins["pair_filter"] == 0.0


# ------------------------------------------------------------------ helpers

def test_brute_knn_matches_kdtree_on_a_mixture():
    w = synth.mixture(synth.MixtureSpec(n=3000, d=24, n_centres=12, centre_std=1.0,
                                        sigma_lo=0.2, sigma_hi=0.5, n_queries=40), seed=3)
    D, Q = w["D"], w["Q"]
    ids, dist = brute.knn(D, Q, 15)
    dd, ii = cKDTree(D.astype(np.float64)).query(Q.astype(np.float64), k=15, eps=0.0)
    assert ids.tolist() == ii.tolist()
    np.testing.assert_allclose(dist, dd, rtol=1e-12)


def test_brute_knn_duplicates_tie_by_id():
    # three copies of one point at ids 7, 2, 5 (inserted out of order) and a
    # query on it: the three zero distances come back as ids 2, 5, 7
    rng = np.random.Generator(np.random.PCG64(4))
    D = rng.standard_normal((20, 6)).astype(np.float32) + 5
    p = rng.standard_normal(6).astype(np.float32)
    D[[7, 2, 5]] = p
    ids, dist = brute.knn(D, p[None, :], 4)
    assert ids[0, :3].tolist() == [2, 5, 7]
    assert dist[0, :3].tolist() == [0.0, 0.0, 0.0]
    assert dist[0, 3] > 0


def test_splitmix64_published_sequence():
    # the generator started from state 0 gives 0xe220a8397b1dcdaf,
    # 0x6e789e6aa1b965f4, 0x06c45d188009454f, 0xf88bb8a8724c81ec (the
    # published test vector); the k-th output is the mix of k * gamma, so
    # the first output for the states gamma, 2 gamma, 3 gamma
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [rmin.splitmix64((j * GAMMA) & MASK) for j in range(4)] == expect


@pytest.mark.parametrize("j", [0, 1, 2, 3])
def test_sample_pairs_index_formula(j):
    """Pair 0 of the sample from the published outputs sm(j gamma):
    i_0 = sm(seed) mod n with seed = j gamma; and for seed = j gamma - S,
    l_0 = (i_0 + 1 + sm(j gamma) mod (n - 1)) mod n, so with n = 3 the step
    l_0 - i_0 (mod 3) is 1 for an even output and 2 for an odd one."""
    outs = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    for n in (3, 5, 7):
        ii, _ = rmin.sample_pairs(n, (j * GAMMA) & MASK)
        assert ii[0] == outs[j] % n
    n, S = 3, 3
    ii, ll = rmin.sample_pairs(n, (j * GAMMA - S) & MASK)
    assert (ll[0] - ii[0]) % 3 == 1 + outs[j] % 2
    n, S = 5, 10
    ii, ll = rmin.sample_pairs(n, (j * GAMMA - S) & MASK)
    assert (ll[0] - ii[0]) % 5 == 1 + outs[j] % 4
