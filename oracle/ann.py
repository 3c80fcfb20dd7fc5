"""(c,k)-ANN by PM-LSH, Algorithm 2, one query at a time (oracle, FP64).

Steps (Section 5.2, Algorithm 2; projection of Section 3.2, Eq. 3):
  1. project: o' = (a_1.o, ..., a_m.o) for every data point and q' for the
     query, summed in FP64 from the FP32 inputs;
  2. r <- r_min, C <- {} ; repeat:
     a. (round > 0) if at least k points of C lie within c*r of q, stop;
     b. the ball is every point whose projected distance to q' is <= t*r
        (a closed ball: a range query returns the points inside B(q', t r));
     c. if the ball holds at least B = beta*n + k points, C becomes the B
        ball points nearest to q' in the projected space (ties by id), stop;
     d. otherwise C <- ball; r <- c*r. (B is capped at n, so a ball that
        covers the whole dataset always meets the budget in step c.)
  3. return the k points of C nearest to q by exact distance (ties by id).

Reading of step 2c. Algorithm 2 grows C node by node in tree order until it
holds beta*n + k points, so the paper's C depends on the tree and on the
traversal. Here C is the B points of the ball that are nearest to q' in the
projected space. This makes the result independent of the index (the tree
then only decides how fast the ball is found), and it is the nesting that
the proof of Theorem 1 relies on (the smaller-radius ball is contained in
the candidate set). Section 3.2 ranks candidates by projected distance for
the same reason (the estimator of Lemma 2).

Reading of step 2a. The test at the top of Algorithm 2's loop runs after the
radius has been multiplied by c, so it compares exact distances with c*r of
the *new* r; on the first pass C is empty and the test cannot succeed.

The function also reports the decision margins: the relative gap between a
value and the threshold it was compared with, for every comparison whose
outcome shaped the result. A query is "fragile" when the smallest margin is
at most 1e-5; FP32 and FP64 may then legitimately decide differently.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

EXIT_NEAR = 1     # enough verified points within c*r
EXIT_BUDGET = 2    # the ball reached the budget B


@dataclasses.dataclass
class AnnResult:
    ids: np.ndarray        # (k,) int64, ascending (dist, id)
    dist: np.ndarray       # (k,) float64, Euclidean
    exit_kind: int
    rounds: int            # number of range queries issued
    n_cand: int            # |C| at the end
    margin: float          # smallest relative decision margin
    margin_kind: str       # which comparison produced it
    r_final: float
    margins: dict          # smallest margin of each kind of comparison


def project(X: np.ndarray, A: np.ndarray) -> np.ndarray:
    """o' = A o for every row o of X (Eq. 3): (n, d) x (m, d) -> (n, m), FP64."""
    return X.astype(np.float64) @ A.astype(np.float64).T


def _rel(a: float, b: float) -> float:
    if math.isinf(b):
        return math.inf if math.isfinite(a) else 0.0
    den = max(abs(b), 1e-300)
    return abs(a - b) / den


def exact_dist(D: np.ndarray, q: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Euclidean distance from q to rows idx of D, FP64, direct differences."""
    diff = D[idx].astype(np.float64) - q.astype(np.float64)[None, :]
    return np.sqrt(np.sum(diff * diff, axis=1))


def query(D: np.ndarray, Dp: np.ndarray, q: np.ndarray, qp: np.ndarray,
          k: int, c: float, t: float, budget: int, r_min: float) -> AnnResult:
    """Algorithm 2 for one query. D: (n,d) FP32 data, Dp = project(D, A),
    q: (d,) query, qp = A q (FP64). budget = B (already capped at n)."""
    n = D.shape[0]
    ids = np.arange(n, dtype=np.int64)
    pd = np.sqrt(np.sum((Dp - qp[None, :]) ** 2, axis=1))
    order = np.lexsort((ids, pd))          # ascending (pd, id)
    pd_sorted = pd[order]

    margins = []                          # (value, kind)
    cand = np.empty(0, dtype=np.int64)     # C, as data ids
    cand_dist = np.empty(0, dtype=np.float64)
    r = float(r_min)
    rounds = 0
    exit_kind = None
    while True:
        if rounds > 0:
            thr = c * r
            margins.append((float(np.min(np.abs(cand_dist - thr))) / thr
                            if cand.size else math.inf, "cr_stop"))
            if int(np.count_nonzero(cand_dist <= thr)) >= k:
                exit_kind = EXIT_NEAR
                break
        R = t * r
        rounds += 1
        n_ball = int(np.searchsorted(pd_sorted, R, side="right"))
        # the decision "ball holds >= B points" turns on the B-th projected
        # distance against R
        margins.append((_rel(pd_sorted[budget - 1], R), "ball_count"))
        if n_ball >= budget:
            cand = order[:budget]
            if budget < n:
                margins.append((_rel(pd_sorted[budget], pd_sorted[budget - 1]),
                                "budget_cut"))
            exit_kind = EXIT_BUDGET
        else:
            # every point's membership in the ball matters
            margins.append((float(np.min(np.abs(pd - R))) / R, "ball_member"))
            cand = order[:n_ball]
        new = cand[cand_dist.size:]        # C only ever grows by a suffix
        cand_dist = np.concatenate([cand_dist, exact_dist(D, q, new)])
        if exit_kind is not None:
            break
        r = c * r

    # top-k of C by (exact distance, id)
    o = np.lexsort((cand, cand_dist))
    kk = min(k, cand.size)
    top = o[:kk]
    top_ids = cand[top]
    top_dist = cand_dist[top]
    # ordering margins among the first k+1 exact distances
    srt = cand_dist[o[:kk + 1]]
    for a, b in zip(srt[:-1], srt[1:]):
        margins.append((_rel(b, a) if a > 0 else (math.inf if b > 0 else 0.0),
                        "topk_order"))
    mval, mkind = min(margins, key=lambda x: x[0]) if margins else (math.inf, "")
    by_kind = {}
    for v, kind in margins:
        by_kind[kind] = min(v, by_kind.get(kind, math.inf))
    return AnnResult(ids=top_ids, dist=top_dist, exit_kind=exit_kind,
                     rounds=rounds, n_cand=int(cand.size), margin=mval,
                     margin_kind=mkind, r_final=r, margins=by_kind)


def run(D: np.ndarray, A: np.ndarray, Q: np.ndarray, k: int, c: float,
        t: float, budget: int, r_min: float, Dp: np.ndarray | None = None):
    """Algorithm 2 for every query in Q; returns a list of AnnResult."""
    if Dp is None:
        Dp = project(D, A)
    Qp = project(Q, A)
    return [query(D, Dp, Q[i], Qp[i], k, c, t, budget, r_min)
            for i in range(Q.shape[0])]
