"""Shared helpers of the GPU parity tests: run the oracle and the library on
the same seeded inputs and compare them under the tolerance rule.

Rule (ids bit-exact except near ties; distances to 1e-5 relative):
  * a query whose smallest oracle decision margin exceeds FRAGILE must come
    back with exactly the oracle's ids, in order, the same exit kind, number
    of range queries and candidate count, and distances within TOL;
  * a fragile query (some comparison within FRAGILE of its threshold, where
    FP32 and FP64 may decide differently) must return distinct ids, sorted by
    (distance, id), whose distances agree with their FP64 exact distances to
    TOL; if only the order of the top-k is near-tied, the distances must
    also agree rank by rank and ids may only be permuted within groups of
    near-equal distances; if a candidate-set decision is near-tied, all but
    at most one id must be the oracle's.
"""

from __future__ import annotations

import math
import sys

import numpy as np

from oracle import ann as oann
from oracle import chi2, rmin

TOL = 1e-5          # relative distance tolerance (FP32 vs FP64)
FRAGILE = 1e-5      # decision margin below which FP32 may legitimately differ


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_ann(D, A, Q, k, c, confidence, beta, r_min, Dp=None):
    n = D.shape[0]
    t = chi2.radius_factor(1 - confidence, A.shape[0])
    if beta < 0:
        beta = chi2.default_beta(1 - confidence, c, A.shape[0])
    B = chi2.ann_budget(beta, n, k)
    return oann.run(D, A, Q, k=k, c=c, t=t, budget=B, r_min=r_min, Dp=Dp), B


def _tie_groups(d, tol):
    """Split ascending distances into runs whose neighbours are within tol."""
    groups, start = [], 0
    for i in range(1, len(d) + 1):
        if i == len(d) or d[i] - d[i - 1] > tol * max(d[i - 1], 1e-30):
            groups.append((start, i))
            start = i
    return groups


# Decisions the library takes in the FP64 order (the budget cut and the
# top-k order): a query whose other margins are clear must match the oracle
# exactly when these two exceed FP64 resolution (the FP64 projections and
# distances of both sides differ by their summation order only).
FP64_DECIDED = ("topk_order", "budget_cut")
FP64_RESOLUTION = 1e-11


def _fp64_exact(r):
    return all(v > (FP64_RESOLUTION if kind in FP64_DECIDED else FRAGILE)
               for kind, v in r.margins.items())


ACP_FP64_DECIDED = ("topk_order",)


def acp_exact(r):
    """An ACP result the library must reproduce exactly: every decision it
    takes on FP32 has an oracle margin above FRAGILE, and the top-k order
    (taken in the FP64 order by the library) one above the FP64 resolution."""
    return all(v > (FP64_RESOLUTION if kind in ACP_FP64_DECIDED else FRAGILE)
               for kind, v in r.margins.items())


def compare_ann(D, Q, res, ids, dist, stats=None, fp64=False):
    """res: oracle results; ids/dist/stats: library outputs as NumPy arrays.
    With fp64, near ties of the budget cut and of the top-k order (decided in
    the FP64 order by both paths of the library) are held to exact agreement
    too.
    Returns (number of queries with a near-tie in the top-k order only,
    number with a near-tie at a candidate-set decision)."""
    n_order, n_set = 0, 0
    for qi, r in enumerate(res):
        gi = ids[qi].tolist()
        gd = dist[qi].astype(np.float64)
        oi = r.ids.tolist()
        if r.margin > FRAGILE or (fp64 and _fp64_exact(r)):
            assert gi == oi, (qi, gi, oi, r.margin_kind, r.margin)
            np.testing.assert_allclose(gd, r.dist, rtol=TOL, atol=1e-6,
                                       err_msg=f"query {qi}")
            if stats is not None:
                assert stats[qi, 0] == r.rounds, (qi, stats[qi], r.rounds)
                assert stats[qi, 1] == r.n_cand, (qi, stats[qi], r.n_cand)
                assert stats[qi, 2] == r.exit_kind, (qi, stats[qi], r.exit_kind)
            continue
        # a valid answer in every fragile case
        assert len(set(gi)) == len(gi)
        assert min(gi) >= 0 and max(gi) < D.shape[0]
        ex = oann.exact_dist(D, Q[qi], np.asarray(gi))
        np.testing.assert_allclose(gd, ex, rtol=TOL, atol=1e-6)
        # the library orders by (FP32 squared distance, id); the square root
        # can merge two squared distances, so only the distances are checked
        assert np.all(np.diff(gd) >= 0), (qi, gd)
        set_fragile = any(v <= FRAGILE for kind, v in r.margins.items()
                          if kind != "topk_order")
        if not set_fragile:
            # same candidate set: the same distances rank by rank, and ids may
            # only be permuted inside groups of near-equal distances
            n_order += 1
            np.testing.assert_allclose(gd, r.dist, rtol=TOL, atol=1e-6)
            for a, b in _tie_groups(r.dist, 2 * TOL):
                if b < len(oi):
                    assert set(gi[a:b]) == set(oi[a:b]), (qi, a, b, gi, oi)
            if stats is not None:
                assert stats[qi, 1] == r.n_cand and stats[qi, 2] == r.exit_kind
        else:
            # the candidate set itself may differ by near-threshold points
            n_set += 1
            assert len(set(gi) & set(oi)) >= len(gi) - 1, (qi, gi, oi, r.margins)
    return n_order, n_set


def oracle_r_min(D, seed, budget):
    return rmin.r_min(D, seed, budget)
