"""(c,k)-ACP by radius filtering, Section 6.3 (oracle, FP64).

Steps (Section 6.3, Algorithm 4, in canonical form):
  1. self-join: every pair of points stored in the same leaf of the index is
     verified (exact distance); ub is the k-th smallest of those distances
     (+inf when the leaves hold fewer than k pairs);
  2. filter: every other pair whose projected distance is strictly below
     t * ub becomes a candidate (Lemma 4 with the roles of r and ub swapped);
  3. budget: at most T = beta * n(n-1)/2 + k pairs are verified in total;
     if the seeds and candidates exceed T, the candidates kept are the
     T - |seeds| with the smallest projected distance (ties by (i, j));
  4. the k verified pairs with the smallest exact distance, ties by (i, j),
     are returned.

Readings. Algorithm 4 lowers ub while it verifies, restricts the scan to the
subtrees returned by FindLCA (Algorithm 5) with the factor gamma, and stops
after T pairs in a traversal-dependent order. Here ub stays at its
self-join value, every cross-leaf pair is tested against t * ub, and the
T-cut keeps the projected-nearest candidates. This verifies a superset of
the pairs the paper verifies (so recall can only be higher) and makes the
result independent of traversal order. The self-join seeds still depend on
which points share a leaf, so the leaf partition is an input: the oracle
takes it as data (a permutation and leaf offsets), never as code.

Candidates are found by brute force over all pairs: no tree is used here, so
a pruned pair scan elsewhere is checked for losing nothing.

``branch_and_bound`` is the branch-and-bound algorithm of Section 6.1
(Algorithm 3) in the same brute-force form: the T projected-closest pairs,
verified. ``radius_filtering_lca`` is Algorithm 4 as printed (FindLCA with
gamma, a live ub, the count > T stop), with the tree as data.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class AcpResult:
    pairs: np.ndarray      # (k, 2) int64, i < j, ascending (dist, i, j)
    dist: np.ndarray       # (k,) float64
    ub: float              # k-th smallest seed distance
    n_seed: int
    n_cand: int            # candidates kept after the T cut
    n_cand_raw: int        # candidates before the T cut
    margin: float
    margin_kind: str
    margins: dict = dataclasses.field(default_factory=dict)   # smallest margin per kind


def _by_kind(margins) -> dict:
    out = {}
    for v, kind in margins:
        out[kind] = min(v, out.get(kind, math.inf))
    return out


def _pair_key_order(dist: np.ndarray, pi: np.ndarray, pj: np.ndarray):
    return np.lexsort((pj, pi, dist))


def seed_pairs(perm: np.ndarray, offsets: np.ndarray):
    """All within-leaf pairs as (i, j) with i < j (original ids)."""
    out_i, out_j = [], []
    for b in range(offsets.shape[0] - 1):
        members = np.sort(perm[offsets[b]:offsets[b + 1]].astype(np.int64))
        L = members.shape[0]
        if L < 2:
            continue
        a, c = np.triu_indices(L, k=1)
        out_i.append(members[a])
        out_j.append(members[c])
    if not out_i:
        e = np.empty(0, dtype=np.int64)
        return e, e.copy()
    return np.concatenate(out_i), np.concatenate(out_j)


def pair_dist(X: np.ndarray, pi: np.ndarray, pj: np.ndarray,
              block: int = 1 << 15) -> np.ndarray:
    """Euclidean distances of pairs of rows of X, FP64 direct differences."""
    out = np.empty(pi.shape[0], dtype=np.float64)
    for s in range(0, pi.shape[0], block):
        e = min(pi.shape[0], s + block)
        diff = X[pi[s:e]].astype(np.float64) - X[pj[s:e]].astype(np.float64)
        out[s:e] = np.sqrt(np.sum(diff * diff, axis=1))
    return out


def _cross_pairs_below(Dp: np.ndarray, leaf_of: np.ndarray, radius: float,
                       block: int = 256):
    """All pairs i < j in different leaves with ||o_i' - o_j'|| < radius.

    Brute force over row blocks; also returns the pair closest to the
    threshold (its relative gap) for the margin report."""
    n = Dp.shape[0]
    out_i, out_j, out_pd = [], [], []
    best_gap = math.inf
    for s in range(0, n, block):
        e = min(n, s + block)
        acc = np.zeros((e - s, n), dtype=np.float64)
        for dim in range(Dp.shape[1]):
            diff = Dp[s:e, dim][:, None] - Dp[None, :, dim]
            acc += diff * diff
        pd = np.sqrt(acc)
        rows = np.arange(s, e)[:, None]
        cols = np.arange(n)[None, :]
        valid = (cols > rows) & (leaf_of[s:e][:, None] != leaf_of[None, :])
        if math.isfinite(radius) and radius > 0:
            gaps = np.abs(pd[valid] - radius) / radius
            if gaps.size:
                best_gap = min(best_gap, float(gaps.min()))
        hit = valid & (pd < radius)
        r_idx, c_idx = np.nonzero(hit)
        out_i.append(r_idx + s)
        out_j.append(c_idx)
        out_pd.append(pd[r_idx, c_idx])
    return (np.concatenate(out_i).astype(np.int64),
            np.concatenate(out_j).astype(np.int64),
            np.concatenate(out_pd), best_gap)


def run(D: np.ndarray, Dp: np.ndarray, perm: np.ndarray, offsets: np.ndarray,
        k: int, t: float, T: int) -> AcpResult:
    """Radius-filtering ACP. D: (n,d) FP32 data; Dp: FP64 projections (n,m);
    perm/offsets: leaf partition (leaf b holds ids perm[offsets[b]:offsets[b+1]])."""
    n = D.shape[0]
    leaf_of = np.empty(n, dtype=np.int64)
    for b in range(offsets.shape[0] - 1):
        leaf_of[perm[offsets[b]:offsets[b + 1]]] = b
    margins = []

    # 1. self-join of every leaf, all seed pairs verified
    si, sj = seed_pairs(perm, offsets)
    sd = pair_dist(D, si, sj)
    so = _pair_key_order(sd, si, sj)
    ub = float(sd[so[k - 1]]) if sd.shape[0] >= k else math.inf

    # 2. every cross-leaf pair with projected distance < t * ub
    R = t * ub
    ci, cj, cpd, gap = _cross_pairs_below(Dp, leaf_of, R)
    margins.append((gap, "pair_filter"))
    n_raw = ci.shape[0]

    # 3. the budget T on verified pairs, nearest-by-projection kept
    keep = max(0, T - si.shape[0])
    if n_raw > keep:
        co = np.lexsort((cj, ci, cpd))
        if keep > 0:
            margins.append((abs(cpd[co[keep]] - cpd[co[keep - 1]])
                            / max(cpd[co[keep - 1]], 1e-300), "budget_cut"))
        sel = co[:keep]
        ci, cj, cpd = ci[sel], cj[sel], cpd[sel]

    # 4. verify candidates; top-k over seeds and candidates by (dist, i, j)
    cd = pair_dist(D, ci, cj)
    ai = np.concatenate([si, ci])
    aj = np.concatenate([sj, cj])
    ad = np.concatenate([sd, cd])
    o = _pair_key_order(ad, ai, aj)
    kk = min(k, o.shape[0])
    top = o[:kk]
    srt = ad[o[:kk + 1]]
    for a, b in zip(srt[:-1], srt[1:]):
        margins.append(((b - a) / a if a > 0 else (math.inf if b > 0 else 0.0),
                        "topk_order"))
    mval, mkind = min(margins, key=lambda x: x[0])
    return AcpResult(pairs=np.stack([ai[top], aj[top]], axis=1),
                     dist=ad[top], ub=ub, n_seed=int(si.shape[0]),
                     n_cand=int(ci.shape[0]), n_cand_raw=int(n_raw),
                     margin=mval, margin_kind=mkind,
                     margins=_by_kind(margins))


def _all_pairs_pd(Dp: np.ndarray, block: int = 256):
    """Projected distances of all pairs i < j (brute force, FP64)."""
    n = Dp.shape[0]
    out_i, out_j, out_pd = [], [], []
    for s in range(0, n, block):
        e = min(n, s + block)
        acc = np.zeros((e - s, n), dtype=np.float64)
        for dim in range(Dp.shape[1]):
            diff = Dp[s:e, dim][:, None] - Dp[None, :, dim]
            acc += diff * diff
        r_idx, c_idx = np.nonzero(np.arange(n)[None, :] > np.arange(s, e)[:, None])
        out_i.append(r_idx + s)
        out_j.append(c_idx)
        out_pd.append(np.sqrt(acc[r_idx, c_idx]))
    return (np.concatenate(out_i).astype(np.int64), np.concatenate(out_j).astype(np.int64),
            np.concatenate(out_pd))


def branch_and_bound(D: np.ndarray, Dp: np.ndarray, k: int, T: int) -> AcpResult:
    """(c,k)-ACP by branch and bound, Section 6.1 (Algorithm 3).

    The best-first search over node pairs with the Mindist bound stops once
    no unexamined node pair can hold a pair closer (in the projected space)
    than the T-th closest pair found, so its candidate set is the T pairs
    with the smallest projected distance over all pairs. Reading: ties of the
    projected distance go to the smaller (i, j), like every cut here. The T
    pairs are verified and the k with the smallest exact distance, ties by
    (i, j), returned. Computed by brute force over all pairs (no tree)."""
    n = D.shape[0]
    T = min(T, n * (n - 1) // 2)
    pi, pj, pd = _all_pairs_pd(Dp)
    o = np.lexsort((pj, pi, pd))
    margins = []
    if T < o.shape[0]:
        margins.append((abs(pd[o[T]] - pd[o[T - 1]]) / max(pd[o[T - 1]], 1e-300),
                        "budget_cut"))
    sel = o[:T]
    ci, cj = pi[sel], pj[sel]
    cd = pair_dist(D, ci, cj)
    oo = _pair_key_order(cd, ci, cj)
    kk = min(k, oo.shape[0])
    srt = cd[oo[:kk + 1]]
    for a, b in zip(srt[:-1], srt[1:]):
        margins.append(((b - a) / a if a > 0 else (math.inf if b > 0 else 0.0),
                        "topk_order"))
    mval, mkind = min(margins, key=lambda x: x[0]) if margins else (math.inf, "")
    top = oo[:kk]
    return AcpResult(pairs=np.stack([ci[top], cj[top]], axis=1), dist=cd[top],
                     ub=float(pd[o[T - 1]]), n_seed=0, n_cand=int(T),
                     n_cand_raw=int(T), margin=mval, margin_kind=mkind,
                     margins=_by_kind(margins))


def radius_filtering_lca(D: np.ndarray, Dp: np.ndarray, perm: np.ndarray, offsets: np.ndarray,
                         level: np.ndarray, first_leaf: np.ndarray, end_leaf: np.ndarray,
                         radius: np.ndarray, k: int, t: float, T: int,
                         gamma: float) -> AcpResult:
    """(c,k)-ACP by radius filtering with FindLCA, Section 6.3 (Algorithms 4-5).

    1. self-join of every leaf, all seed pairs verified; ub = the k-th
       smallest exact distance; count = number of verified pairs;
    2. FindLCA from the root with R = gamma * t * ub: an inner node with
       radius below R is returned (its subtree is not searched further),
       otherwise its children are searched; leaves are never returned;
    3. the returned nodes in ascending radius (ties by node index): every
       pair of points in different leaves under the node whose projected
       distance is below t * ub is verified, then ub becomes the k-th
       smallest verified distance and count grows by those pairs; the scan
       stops after the first node that leaves count > T;
    4. the k verified pairs with the smallest (distance, i, j).
    Reading: ub and count are updated node by node (Algorithm 4 updates them
    after every verified pair, in an order inside the node it leaves open).
    The tree is data (node levels, leaf ranges and radii of the index under
    test); pairs are found by brute force inside each node."""
    n = D.shape[0]
    leaf_of = np.empty(n, dtype=np.int64)
    for b in range(offsets.shape[0] - 1):
        leaf_of[perm[offsets[b]:offsets[b + 1]]] = b
    margins = []
    si, sj = seed_pairs(perm, offsets)
    sd = pair_dist(D, si, sj)
    pi, pj, pdv = [si], [sj], [sd]

    def kth():
        allv = np.concatenate(pdv)
        return float(np.partition(allv, k - 1)[k - 1]) if allv.shape[0] >= k else math.inf

    ub = kth()
    count = int(si.shape[0])
    n_levels = int(level.max()) + 1
    R = gamma * t * ub
    found, stack = [], [int(e) for e in np.nonzero(level == 0)[0]]
    while stack:
        e = stack.pop()
        if level[e] == n_levels - 1:
            continue
        if math.isfinite(R):
            margins.append((abs(float(radius[e]) - R) / R if R > 0 else math.inf, "find_lca"))
        if float(radius[e]) < R:
            found.append(e)
        else:
            kids = np.nonzero((level == level[e] + 1) & (first_leaf >= first_leaf[e])
                              & (end_leaf <= end_leaf[e]))[0]
            stack.extend(int(x) for x in kids)
    found.sort(key=lambda e: (float(radius[e]), e))
    n_cand = 0
    for e in found:
        if count > T:
            break
        members = np.nonzero((leaf_of >= first_leaf[e]) & (leaf_of < end_leaf[e]))[0]
        thr = t * ub
        a, b = np.triu_indices(members.shape[0], k=1)
        ia, ib = members[a], members[b]
        cross = leaf_of[ia] != leaf_of[ib]
        ia, ib = ia[cross], ib[cross]
        pd = pair_dist(Dp, ia, ib)
        if math.isfinite(thr) and thr > 0 and pd.shape[0]:
            margins.append((float(np.min(np.abs(pd - thr))) / thr, "pair_filter"))
        hit = pd < thr
        ci, cj = np.minimum(ia[hit], ib[hit]), np.maximum(ia[hit], ib[hit])
        cd = pair_dist(D, ci, cj)
        pi.append(ci)
        pj.append(cj)
        pdv.append(cd)
        count += int(ci.shape[0])
        n_cand += int(ci.shape[0])
        ub = kth()
    ai, aj, ad = np.concatenate(pi), np.concatenate(pj), np.concatenate(pdv)
    o = _pair_key_order(ad, ai, aj)
    kk = min(k, o.shape[0])
    srt = ad[o[:kk + 1]]
    for x, y in zip(srt[:-1], srt[1:]):
        margins.append(((y - x) / x if x > 0 else (math.inf if y > 0 else 0.0), "topk_order"))
    mval, mkind = min(margins, key=lambda z: z[0]) if margins else (math.inf, "")
    top = o[:kk]
    return AcpResult(pairs=np.stack([ai[top], aj[top]], axis=1), dist=ad[top], ub=ub,
                     n_seed=int(si.shape[0]), n_cand=n_cand, n_cand_raw=n_cand,
                     margin=mval, margin_kind=mkind,
                     margins=_by_kind(margins))
