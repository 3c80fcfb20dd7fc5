"""Exact answers straight from the problem definitions (oracle, FP64).

Defs. 1-2 (Section 2.1): the exact k nearest neighbours of q are the k data
points with the smallest Euclidean distance to q. Defs. 3-4: the exact k
closest pairs are the k pairs (i < j) with the smallest distance. Ties are
broken by id, then by (i, j), so the answers are unique.
"""

from __future__ import annotations

import numpy as np


def knn(D: np.ndarray, Q: np.ndarray, k: int, block: int = 64):
    """Exact kNN of every row of Q: ids (nq,k) int64 and dist (nq,k) FP64."""
    n = D.shape[0]
    D64 = D.astype(np.float64)
    ids = np.empty((Q.shape[0], k), dtype=np.int64)
    dist = np.empty((Q.shape[0], k), dtype=np.float64)
    all_ids = np.arange(n, dtype=np.int64)
    for s in range(0, Q.shape[0], block):
        e = min(Q.shape[0], s + block)
        for qi in range(s, e):
            diff = D64 - Q[qi].astype(np.float64)[None, :]
            d = np.sqrt(np.sum(diff * diff, axis=1))
            o = np.lexsort((all_ids, d))[:k]
            ids[qi] = o
            dist[qi] = d[o]
    return ids, dist


def closest_pairs(D: np.ndarray, k: int):
    """Exact k closest pairs: pairs (k,2) int64 with i<j, dist (k,) FP64."""
    n = D.shape[0]
    D64 = D.astype(np.float64)
    pi, pj, pdist = [], [], []
    for i in range(n - 1):
        diff = D64[i + 1:] - D64[i][None, :]
        d = np.sqrt(np.sum(diff * diff, axis=1))
        # keep only what can still make the top k of the rows seen so far
        take = np.argsort(d, kind="stable")[:k]
        pi.append(np.full(take.shape[0], i, dtype=np.int64))
        pj.append(take.astype(np.int64) + i + 1)
        pdist.append(d[take])
    pi = np.concatenate(pi)
    pj = np.concatenate(pj)
    pdist = np.concatenate(pdist)
    o = np.lexsort((pj, pi, pdist))[:k]
    return np.stack([pi[o], pj[o]], axis=1), pdist[o]
