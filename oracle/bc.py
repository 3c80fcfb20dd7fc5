"""(r,c)-BC query by PM-LSH, Algorithm 1, one query at a time (oracle, FP64).

Test infrastructure only: nothing in the library imports this module.

Steps (Section 5.1, Algorithm 1; projection of Section 3.2, Eq. 3):
  1. q' = A q, and o' = A o for every data point, in FP64;
  2. the range query of radius t*r around q' returns the candidate set C;
  3. if C holds at least B = beta*n + 1 points, the answer is the point of C
     nearest to q; otherwise it is the point of C nearest to q if that point
     lies within c*r of q, and nothing if no point of C does.

Reading of step 2 (the same as the ANN oracle's reading of the budget): the
range query stops collecting at B points, and the B points it keeps are the
ones nearest to q' in the projected space (ties by id); a ball with fewer
than B points is taken whole. Ties of the exact distance go to the smaller
id.

Like the ANN oracle, the function reports the smallest relative margin of
the comparisons that shaped the answer (ball membership against t*r, the
B-th against the (B+1)-th projected distance, the answer's distance against
c*r, the first against the second exact distance).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from .ann import _rel, exact_dist, project

KIND_NONE = 0      # the ball fell short of B and no candidate is within c*r
KIND_FOUND = 1     # the ball fell short of B; the nearest candidate is within c*r
KIND_BUDGET = 2    # the ball reached B points


@dataclasses.dataclass
class BcResult:
    id: int            # -1 for nothing
    dist: float        # +inf for nothing
    kind: int
    n_cand: int        # |C|
    margin: float
    margin_kind: str
    margins: dict = dataclasses.field(default_factory=dict)   # smallest margin per kind


def _by_kind(margins) -> dict:
    out = {}
    for v, kind in margins:
        out[kind] = min(v, out.get(kind, math.inf))
    return out


def query(D: np.ndarray, Dp: np.ndarray, q: np.ndarray, qp: np.ndarray, r: float,
          c: float, t: float, budget: int) -> BcResult:
    """Algorithm 1 for one query; budget = B = beta*n + 1, capped at n."""
    n = D.shape[0]
    ids = np.arange(n, dtype=np.int64)
    pd = np.sqrt(np.sum((Dp - qp[None, :]) ** 2, axis=1))
    order = np.lexsort((ids, pd))
    pd_sorted = pd[order]
    R = t * r
    margins = [(_rel(pd_sorted[budget - 1], R), "ball_count")]
    n_ball = int(np.searchsorted(pd_sorted, R, side="right"))
    if n_ball >= budget:
        cand = order[:budget]
        if budget < n:
            margins.append((_rel(pd_sorted[budget], pd_sorted[budget - 1]), "budget_cut"))
        kind = KIND_BUDGET
    else:
        margins.append((float(np.min(np.abs(pd - R))) / R, "ball_member"))
        cand = order[:n_ball]
        kind = None
    if cand.size == 0:
        return BcResult(-1, math.inf, KIND_NONE, 0, *min(margins, key=lambda x: x[0]),
                        margins=_by_kind(margins))
    dist = exact_dist(D, q, cand)
    o = np.lexsort((cand, dist))
    best, best_d = int(cand[o[0]]), float(dist[o[0]])
    if cand.size > 1:
        d2 = float(dist[o[1]])
        margins.append((_rel(d2, best_d) if best_d > 0 else (math.inf if d2 > 0 else 0.0),
                        "nearest_order"))
    if kind is None:
        margins.append((_rel(best_d, c * r), "within_cr"))
        kind = KIND_FOUND if best_d <= c * r else KIND_NONE
    mval, mkind = min(margins, key=lambda x: x[0])
    if kind == KIND_NONE:
        return BcResult(-1, math.inf, kind, int(cand.size), mval, mkind, _by_kind(margins))
    return BcResult(best, best_d, kind, int(cand.size), mval, mkind, _by_kind(margins))


def run(D: np.ndarray, A: np.ndarray, Q: np.ndarray, r: float, c: float, t: float,
        budget: int, Dp: np.ndarray | None = None):
    """Algorithm 1 for every query in Q; returns a list of BcResult."""
    if Dp is None:
        Dp = project(D, A)
    Qp = project(Q, A)
    return [query(D, Dp, Q[i], Qp[i], r, c, t, budget) for i in range(Q.shape[0])]
