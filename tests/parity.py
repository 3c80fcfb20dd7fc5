"""Shared helpers of the GPU parity tests: run the oracle and the library on
the same seeded inputs and compare them under the tolerance rule.

Rule (ids bit-exact except near ties; distances to 1e-5 relative):
  * a query whose smallest oracle decision margin exceeds FRAGILE must come
    back with exactly the oracle's ids, in order, the same exit kind, number
    of range queries and candidate count, and distances within TOL;
  * a fragile query (some comparison within FRAGILE of its threshold, where
    FP32 and FP64 may decide differently) must return distinct ids, sorted by
    distance, whose distances agree with their FP64 exact distances to TOL,
    and its answer (ids up to permutations inside groups of near-equal
    distances, with rounds, |C| and exit kind) must be the oracle's, or the
    oracle's with the near-threshold decisions flipped: Algorithm 2 re-run
    with the ball radius and the c r threshold moved by FRAGILE. So every id
    that differs is explained by a comparison within FRAGILE of its
    threshold, including the later rounds such a flip causes;
  * each test holds at least a stated fraction of its queries (75 % unless
    the test says otherwise) to the exact comparison.
The same rule applies to ACP (`compare_acp`), where the flipped decisions
are the pair filter (t moved by FRAGILE), FindLCA (gamma moved) and the
budget cut (T moved by one pair).
"""

from __future__ import annotations

import math
import sys

import numpy as np

from oracle import acp as oacp
from oracle import ann as oann
from oracle import chi2, rmin

TOL = 1e-5          # relative distance tolerance (FP32 vs FP64)
FRAGILE = 1e-5      # decision margin below which FP32 may legitimately differ


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class OracleRuns(list):
    """Oracle results of one batch, with the inputs and parameters they came
    from (so a fragile query can be re-run with a decision flipped)."""
    ctx: dict


def oracle_ann(D, A, Q, k, c, confidence, beta, r_min, Dp=None):
    n = D.shape[0]
    t = chi2.radius_factor(1 - confidence, A.shape[0])
    if beta < 0:
        beta = chi2.default_beta(1 - confidence, c, A.shape[0])
    B = chi2.ann_budget(beta, n, k)
    if Dp is None:
        Dp = oann.project(D, A)
    out = OracleRuns(oann.run(D, A, Q, k=k, c=c, t=t, budget=B, r_min=r_min, Dp=Dp))
    out.ctx = dict(D=D, A=A, Dp=Dp, Q=Q, k=k, c=c, t=t, B=B, r_min=r_min)
    return out, B


def flipped_runs(ctx, qi):
    """The oracle's answers for query qi with its near-threshold decisions
    flipped: Algorithm 2 re-run with the ball radius t r and the c r stopping
    threshold each moved by FRAGILE relative, up or down (t scaled by
    (1 + e1 FRAGILE) / (1 + e2 FRAGILE) and r_min by (1 + e2 FRAGILE) moves
    every round's ball radius by (1 + e1 FRAGILE) and every stopping
    threshold by (1 + e2 FRAGILE)). A decision whose margin is at most
    FRAGILE goes the other way in one of these runs; decisions with larger
    margins stay as they are."""
    q = ctx["Q"][qi]
    qp = oann.project(q[None, :], ctx["A"])[0]
    out = []
    for e1 in (0, -1, 1):
        for e2 in (0, -1, 1):
            if e1 == 0 and e2 == 0:
                continue
            t2 = ctx["t"] * (1 + e1 * FRAGILE) / (1 + e2 * FRAGILE)
            r2 = ctx["r_min"] * (1 + e2 * FRAGILE)
            out.append(((e1, e2), oann.query(ctx["D"], ctx["Dp"], q, qp, ctx["k"], ctx["c"],
                                             t2, ctx["B"], r2)))
    return out


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


def _same_answer(gi, gd, oi, od):
    """ids equal in order, or equal as a set with the distances agreeing
    rank by rank and the ids permuted only inside groups of near-equal
    distances (an FP32 near tie of the top-k order)."""
    if gi == oi:
        return True
    if set(gi) != set(oi) or len(gi) != len(oi):
        return False
    if not np.allclose(gd, od, rtol=TOL, atol=1e-6):
        return False
    return all(set(gi[a:b]) == set(oi[a:b]) for a, b in _tie_groups(od, 2 * TOL))


def compare_ann(D, Q, res, ids, dist, stats=None, fp64=False, min_exact_frac=0.75):
    """res: oracle results (from oracle_ann); ids/dist/stats: library outputs
    as NumPy arrays.

    Queries whose oracle margins all clear FRAGILE (with fp64, the budget cut
    and top-k order only need to clear the FP64 resolution: the library
    decides them in the FP64 order) must match exactly: ids in order,
    distances to TOL, rounds, |C| and exit kind. Every other (fragile) query
    must return a valid answer (distinct ids, sorted, distances equal to
    their exact FP64 distances to TOL) that is either the oracle's own or the
    oracle's answer with its fragile decisions flipped (`flipped_runs`),
    with that run's rounds, |C| and exit kind. At least min_exact_frac of the
    queries must be held to the exact comparison.

    Returns (queries held exactly, fragile queries with the oracle's answer,
    fragile queries whose answer is a flipped run's)."""
    ctx = getattr(res, "ctx", None)
    n_exact, n_same, n_flip = 0, 0, 0
    for qi, r in enumerate(res):
        gi = ids[qi].tolist()
        gd = dist[qi].astype(np.float64)
        oi = r.ids.tolist()
        if r.margin > FRAGILE or (fp64 and _fp64_exact(r)):
            n_exact += 1
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

        def stats_match(o):
            return stats is None or (stats[qi, 0] == o.rounds and stats[qi, 1] == o.n_cand
                                     and stats[qi, 2] == o.exit_kind)

        if _same_answer(gi, gd, oi, r.dist) and stats_match(r):
            n_same += 1
            continue
        assert ctx is not None, "fragile query differs and the oracle run has no context"
        alts = flipped_runs(ctx, qi)
        hit = [flip for flip, o in alts
               if _same_answer(gi, gd, o.ids.tolist(), o.dist) and stats_match(o)]
        fragile = {kind: v for kind, v in r.margins.items() if v <= FRAGILE}
        assert hit, ("fragile query differs from the oracle and from every run with its "
                     "fragile decisions flipped", qi, gi, oi, fragile,
                     None if stats is None else stats[qi].tolist(),
                     (r.rounds, r.n_cand, r.exit_kind))
        n_flip += 1
    say(f"compare_ann: {len(res)} queries, {n_exact} held exactly, {n_same} fragile "
        f"with the oracle's answer, {n_flip} fragile with a flipped decision's answer")
    assert n_exact >= min_exact_frac * len(res), (n_exact, len(res))
    return n_exact, n_same, n_flip


def _same_pairs(gp, gd, op, od):
    """Pairs equal in order, or equal as a set with the distances agreeing
    rank by rank and the pairs permuted only inside groups of near-equal
    distances."""
    if gp == op:
        return True
    if set(gp) != set(op) or len(gp) != len(op):
        return False
    if not np.allclose(gd, od, rtol=TOL, atol=1e-7):
        return False
    return all(set(gp[a:b]) == set(op[a:b]) for a, b in _tie_groups(od, 2 * TOL))


def compare_acp(D, res, pairs, dist, st=None, rerun=None, check_raw=True):
    """ACP result of the library against the oracle's (same rule as ANN).

    Every answer must be valid: pairs i < j inside [0, n), no pair twice,
    distances equal to their FP64 exact distances to TOL and non-decreasing;
    the seed count and ub equal the oracle's. A result whose oracle margins
    all clear their bounds (`acp_exact`) must match exactly, candidate counts
    included. Otherwise the answer must be the oracle's (pairs permuted only
    inside near-equal distances) or the answer of the oracle re-run with a
    fragile decision flipped: rerun(t_scale=...) moves the pair filter's
    radius t ub by FRAGILE, rerun(gamma_scale=...) moves FindLCA's radius,
    rerun(dT=+-1) moves the budget cut by one pair. With check_raw, the
    library's count of filtered pairs must lie between the counts at t ub
    moved down and up by FRAGILE. Returns "exact", "same" or "flipped"."""
    pairs = np.asarray(pairs)
    dist = np.asarray(dist, dtype=np.float64)
    n, k = D.shape[0], pairs.shape[0]
    assert np.all(pairs[:, 0] < pairs[:, 1]), pairs
    assert pairs.min() >= 0 and pairs.max() < n
    gp = [tuple(p) for p in pairs.tolist()]
    assert len(set(gp)) == k, "a pair returned twice"
    ex = oacp.pair_dist(D, pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64))
    np.testing.assert_allclose(dist, ex, rtol=TOL, atol=1e-7)
    assert np.all(np.diff(dist) >= 0), dist
    if st is not None:
        assert st["n_seed"] == res.n_seed, (st, res.n_seed)
        if check_raw or acp_exact(res):     # the seed ub (FindLCA's ub is live)
            if math.isinf(res.ub):
                assert math.isinf(st["ub"])
            else:
                assert st["ub"] == pytest_approx(res.ub), (st["ub"], res.ub)
    if acp_exact(res):
        assert pairs.tolist() == res.pairs.tolist(), (pairs.tolist(), res.pairs.tolist())
        np.testing.assert_allclose(dist, res.dist, rtol=TOL, atol=1e-7)
        if st is not None:
            assert st["n_cand_raw"] == res.n_cand_raw, (st, res.n_cand_raw)
            assert st["n_cand"] == res.n_cand, (st, res.n_cand)
        return "exact"
    fragile = {kind: v for kind, v in res.margins.items() if v <= FRAGILE}
    say("fragile ACP case:", fragile)
    flips = []
    if rerun is not None:
        if "pair_filter" in fragile:
            flips += [dict(t_scale=1 - FRAGILE), dict(t_scale=1 + FRAGILE)]
        if "find_lca" in fragile:
            flips += [dict(gamma_scale=1 - FRAGILE), dict(gamma_scale=1 + FRAGILE)]
        if "budget_cut" in fragile:
            flips += [dict(dT=-1), dict(dT=1)]
    alts = {}

    def alt(f):
        key = tuple(sorted(f.items()))
        if key not in alts:
            alts[key] = rerun(**f)
        return alts[key]

    if check_raw and st is not None and "pair_filter" in fragile and rerun is not None:
        lo = alt(dict(t_scale=1 - FRAGILE)).n_cand_raw
        hi = alt(dict(t_scale=1 + FRAGILE)).n_cand_raw
        assert lo <= st["n_cand_raw"] <= hi, (lo, st["n_cand_raw"], hi)
    if _same_pairs(gp, dist, [tuple(p) for p in res.pairs.tolist()], res.dist):
        return "same"
    for f in flips:
        o = alt(f)
        if _same_pairs(gp, dist, [tuple(p) for p in o.pairs.tolist()], o.dist):
            say("  answer of the run with", f)
            return "flipped"
    raise AssertionError(("ACP answer differs from the oracle and from every run with its "
                          "fragile decisions flipped", gp, res.pairs.tolist(), fragile))


def pytest_approx(v):
    import pytest
    return pytest.approx(v, rel=TOL)


def oracle_r_min(D, seed, budget):
    return rmin.r_min(D, seed, budget)
