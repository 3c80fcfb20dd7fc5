"""The comparison rule of the GPU parity tests, checked on the CPU with
answers built by hand: an answer explained by flipping a decision within
FRAGILE of its threshold passes, one that is not explained fails, and a
query held to the exact comparison fails on any difference.
"""

import math

import numpy as np
import pytest

from oracle import acp as oacp
from oracle import ann as oann
from parity import FRAGILE, OracleRuns, compare_acp, compare_ann

ON_AXIS = [(1, 0), (2, 0), (4, 0), (8, 0), (16, 0)]


def _runs(points, k, c, t, B, r_min, queries=((0.0, 0.0),)):
    D = np.asarray(points, dtype=np.float32)
    A = np.array([[1.0, 0.0]], dtype=np.float32)
    Q = np.asarray(queries, dtype=np.float32)
    Dp = oann.project(D, A)
    out = OracleRuns(oann.run(D, A, Q, k=k, c=c, t=t, budget=B, r_min=r_min, Dp=Dp))
    out.ctx = dict(D=D, A=A, Dp=Dp, Q=Q, k=k, c=c, t=t, B=B, r_min=r_min)
    return D, Q, out


def _lib(r, rounds=None):
    ids = r.ids[None, :].copy()
    dist = r.dist[None, :].astype(np.float32)
    st = np.array([[r.rounds if rounds is None else rounds, r.n_cand, r.exit_kind, 0]])
    return ids, dist, st


def test_boundary_point_flip_is_explained():
    # the point at projected distance 1 sits on the ball of round 1 (margin
    # 0). Closed ball (the oracle): found at r = 1, stop at r = 2 after two
    # range queries. A library that leaves it out (open ball) finds it at
    # r = 2 and stops after three: the same id, one more round.
    D, Q, res = _runs(ON_AXIS, k=1, c=2.0, t=1.0, B=3, r_min=0.5)
    assert res[0].margins["ball_member"] == 0.0 and res[0].rounds == 2
    ids, dist, st = _lib(res[0])
    assert compare_ann(D, Q, res, ids, dist, st, min_exact_frac=0.0) == (0, 1, 0)
    st_flip = st.copy()
    st_flip[0, 0] = 3
    assert compare_ann(D, Q, res, ids, dist, st_flip, min_exact_frac=0.0) == (0, 0, 1)
    st_bad = st.copy()
    st_bad[0, 0] = 4
    with pytest.raises(AssertionError):
        compare_ann(D, Q, res, ids, dist, st_bad, min_exact_frac=0.0)


def test_unexplained_id_fails():
    D, Q, res = _runs(ON_AXIS, k=2, c=2.0, t=1.0, B=3, r_min=0.5)
    ids, dist, st = _lib(res[0])
    ids[0, 1] = 3                                    # a point at distance 8
    dist[0, 1] = 8.0
    with pytest.raises(AssertionError):
        compare_ann(D, Q, res, ids, dist, st, min_exact_frac=0.0)


def test_exact_query_allows_no_difference():
    # margins well clear of FRAGILE (projected distances 1, 3, 5, 9, 20,
    # r_min = 1.5): a changed round count fails even with the right ids
    D, Q, res = _runs([(1, 0), (3, 0), (5, 1), (9, 0), (20, 0)], k=1, c=2.0, t=1.0, B=3,
                      r_min=1.5)
    assert res[0].margin > FRAGILE
    ids, dist, st = _lib(res[0])
    assert compare_ann(D, Q, res, ids, dist, st) == (1, 0, 0)
    st[0, 0] += 1
    with pytest.raises(AssertionError):
        compare_ann(D, Q, res, ids, dist, st)


def test_exact_fraction_floor():
    D, Q, res = _runs(ON_AXIS, k=1, c=2.0, t=1.0, B=3, r_min=0.5)
    ids, dist, st = _lib(res[0])
    with pytest.raises(AssertionError):
        compare_ann(D, Q, res, ids, dist, st)       # 0 of 1 held exactly < 75 %


def _acp_line(k):
    # leaves {0, 1}, {2, 3}: id0 (0, 0), id1 (0, 4), id2 (3, 0.5), id3 (3, 5);
    # seeds 4 and 4.5. With k = 1, ub = 4 and t = 0.75 put the filter radius
    # at 3, exactly the projected distance of all four cross pairs (margin
    # 0): the strict filter (the oracle) takes none and answers (0, 1) at 4;
    # a radius a hair larger takes all four and answers (0, 2) at
    # sqrt(9.25) = 3.041
    D = np.array([[0, 0], [0, 4], [3, 0.5], [3, 5]], dtype=np.float32)
    Dp = oann.project(D, np.array([[1.0, 0.0]], dtype=np.float32))
    perm, off = np.arange(4), np.array([0, 2, 4])

    def rerun(t_scale=1.0, dT=0):
        return oacp.run(D, Dp, perm, off, k=k, t=0.75 * t_scale, T=10 ** 6 + dT)

    return D, rerun


def test_acp_filter_flip_is_explained():
    D, rerun = _acp_line(1)
    res = rerun()
    assert res.margins["pair_filter"] == 0.0 and res.n_cand_raw == 0
    assert res.pairs.tolist() == [[0, 1]]
    up = rerun(t_scale=1 + FRAGILE)
    assert up.n_cand_raw == 4 and up.pairs.tolist() == [[0, 2]]
    st = dict(n_seed=2, ub=4.0, n_cand_raw=4, n_cand=4)
    assert compare_acp(D, res, up.pairs, up.dist.astype(np.float32), st,
                       rerun=rerun) == "flipped"
    with pytest.raises(AssertionError):          # more filtered pairs than any flip gives
        compare_acp(D, res, up.pairs, up.dist.astype(np.float32), dict(st, n_cand_raw=5),
                    rerun=rerun)
    with pytest.raises(AssertionError):          # a pair no flip returns
        compare_acp(D, res, np.array([[1, 3]]), np.array([math.sqrt(10.0)], np.float32), st,
                    rerun=rerun)


def test_acp_invalid_answers_fail():
    # k = 2: ub = 4.5, radius 3.375, the cross pairs are candidates with a
    # clear margin; the answer (0, 2), (1, 3) is held exactly
    D, rerun = _acp_line(2)
    res = rerun()
    assert res.margin > FRAGILE and res.pairs.tolist() == [[0, 2], [1, 3]]
    st = dict(n_seed=res.n_seed, ub=res.ub, n_cand_raw=res.n_cand_raw, n_cand=res.n_cand)
    pairs, dist = res.pairs.copy(), res.dist.astype(np.float32)
    assert compare_acp(D, res, pairs, dist, st, rerun=rerun) == "exact"
    bad = pairs.copy()
    bad[0] = bad[0][::-1]                              # i > j
    with pytest.raises(AssertionError):
        compare_acp(D, res, bad, dist, st, rerun=rerun)
    with pytest.raises(AssertionError):
        compare_acp(D, res, pairs, dist * np.float32(1.01), st, rerun=rerun)   # wrong distance
    dup = pairs.copy()
    dup[1] = dup[0]
    with pytest.raises(AssertionError):
        compare_acp(D, res, dup, dist[[0, 0]], st, rerun=rerun)
    with pytest.raises(AssertionError):
        compare_acp(D, res, pairs, dist, dict(st, n_cand_raw=3), rerun=rerun)
