"""Result-quality metrics of Section 7.1 (Eqs. 12-14), FP64."""

from __future__ import annotations

import numpy as np


def overall_ratio(dist: np.ndarray, exact_dist: np.ndarray) -> float:
    """Eq. 12 / Eq. 14: mean over ranks i of returned_i / exact_i.

    ``dist`` and ``exact_dist`` are (k,) or (nq, k); the mean is taken over
    ranks and, for 2-D input, over rows too. Ranks whose exact distance is
    zero count as 1 when the returned distance is also zero.
    """
    a = np.asarray(dist, dtype=np.float64)
    b = np.asarray(exact_dist, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(b > 0, a / np.where(b > 0, b, 1.0),
                     np.where(a > 0, np.inf, 1.0))
    return float(np.mean(r))


def recall(ids: np.ndarray, exact_ids: np.ndarray) -> float:
    """Eq. 13: |R intersect R*| / |R*|, averaged over rows for 2-D input."""
    ids = np.atleast_2d(np.asarray(ids))
    ex = np.atleast_2d(np.asarray(exact_ids))
    vals = []
    for r, e in zip(ids, ex):
        vals.append(len(set(map(int, r)) & set(map(int, e))) / float(len(e)))
    return float(np.mean(vals))


def pair_recall(pairs: np.ndarray, exact_pairs: np.ndarray) -> float:
    """Eq. 13 for closest pairs: pairs are compared as unordered (i, j)."""
    got = {(int(min(a, b)), int(max(a, b))) for a, b in pairs}
    ex = {(int(min(a, b)), int(max(a, b))) for a, b in exact_pairs}
    return len(got & ex) / float(len(ex))
