"""Initial radius r_min (oracle). Section 5.2, "Selecting the Radius r".

The paper picks r with n * F(r) = beta*n + k, where F is the distribution of
pairwise distances in the dataset (Section 4.2), and then takes r_min
"slightly smaller" than that r. It fixes neither how F is estimated nor the
margin. Reading used here:
  * F is estimated from S = min(n(n-1)/2, 100000) random pairs, pair j being
        i_j = sm(seed + j) mod n
        l_j = (i_j + 1 + sm(seed + S + j) mod (n - 1)) mod n
    (so i_j != l_j), where sm(x) is the first output of the SplitMix64
    generator started at state x (Steele, Lea and Flood, OOPSLA 2014):
        z = x + 0x9E3779B97F4A7C15
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
        z = (z ^ (z >> 27)) * 0x94D049BB133111EB
        sm(x) = z ^ (z >> 31)          (all arithmetic mod 2^64);
  * the pair distances (Euclidean, FP64) are sorted ascending and the
    element at index ceil(q*S) - 1 is taken, q = min(1, B/n) with B the
    candidate budget; r_min = kappa * that element, kappa = 0.9;
  * a zero element (duplicate points) would make r <- c r stall at 0, so the
    smallest positive sample distance replaces it (1 if there is none).
"""

from __future__ import annotations

import math

import numpy as np

SAMPLE_PAIRS = 100_000
KAPPA = 0.9

_MASK = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """First SplitMix64 output for state x (pure-Python, exact mod 2^64)."""
    z = (x + 0x9E3779B97F4A7C15) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def sample_size(n: int) -> int:
    return int(min(n * (n - 1) // 2, SAMPLE_PAIRS))


def sample_pairs(n: int, seed: int):
    """The S sampled pairs (i_j, l_j) as two int64 arrays."""
    if n < 2:
        raise ValueError("need n >= 2 for a pair sample")
    S = sample_size(n)
    ii = np.empty(S, dtype=np.int64)
    ll = np.empty(S, dtype=np.int64)
    for j in range(S):
        i = splitmix64((seed + j) & _MASK) % n
        ll[j] = (i + 1 + splitmix64((seed + S + j) & _MASK) % (n - 1)) % n
        ii[j] = i
    return ii, ll


def sorted_sample_distances(D: np.ndarray, seed: int) -> np.ndarray:
    """Ascending FP64 distances of the sampled pairs (the estimate of F)."""
    ii, ll = sample_pairs(D.shape[0], seed)
    diff = D[ii].astype(np.float64) - D[ll].astype(np.float64)
    dist = np.sqrt(np.sum(diff * diff, axis=1))
    return np.sort(dist)


def r_min_from_sample(sorted_dist: np.ndarray, n: int, budget: int,
                      kappa: float = KAPPA) -> float:
    """kappa * F^-1(B/n) read off the sorted sample (Section 5.2)."""
    S = sorted_dist.shape[0]
    if S == 0:
        return 1.0
    q = min(1.0, budget / n)
    idx = max(0, int(math.ceil(q * S)) - 1)
    v = float(sorted_dist[idx])
    if not v > 0.0:
        pos = sorted_dist[sorted_dist > 0.0]
        v = float(pos[0]) if pos.size else 1.0 / kappa
    return kappa * v


def r_min(D: np.ndarray, seed: int, budget: int, kappa: float = KAPPA) -> float:
    return r_min_from_sample(sorted_sample_distances(D, seed), D.shape[0],
                             budget, kappa)
