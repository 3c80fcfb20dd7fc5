"""Seeded synthetic workloads shaped like the PM-LSH evaluation data.

This module only draws random numbers. It holds none of the method's
arithmetic (no projection, no distance, no parameter setting), so that the
CPU oracle and the GPU library can both be fed from it without sharing any
part of the computation they are compared on.

Every workload comes from one 64-bit seed feeding NumPy's PCG64. The draw
order is fixed: cluster centres, per-centre spread, point labels, point
noise, query labels, query noise, then the hash matrix A (m x d, i.i.d.
N(0,1), the 2-stable entries of the projection of Section 3.2). Workloads
that plant near-duplicate pairs draw the copied originals and the copy noise
after the points and before A.

The paper evaluates on real datasets (Table 3) that are not available here;
these mixtures stand in for them by shape only:
  * ``parity``   - 10,000 x 128, 50 centres N(0,1), sigma 0.3, 100 queries.
  * ``headline`` - 1,000,000 x 256, 1,000 centres N(0, var 4), sigma
    U[0.2, 0.5], 10,000 queries (the shape of the Deep dataset).
  * ``acp``      - 200,000 x 512, 500 centres N(0, var 4), sigma
    U[0.2, 0.5]; 198,000 originals plus 2,000 copies of distinct originals
    perturbed by N(0, 1e-3^2) (a 1 % planted near-duplicate fraction).
  * ``serving``  - 10,000,000 x 128 FP16 values in [0, 255], 10,000 centres
    uniform in the cube, sigma 8; plus Poisson request streams.
"""

from __future__ import annotations

import dataclasses

import numpy as np

M_DEFAULT = 15

_CHUNK = 1 << 16  # rows of noise drawn per call, bounds peak host memory


@dataclasses.dataclass(frozen=True)
class MixtureSpec:
    n: int
    d: int
    n_centres: int
    centre_std: float
    sigma_lo: float
    sigma_hi: float
    n_queries: int
    m: int = M_DEFAULT


SPECS = {
    "parity": MixtureSpec(n=10_000, d=128, n_centres=50, centre_std=1.0,
                          sigma_lo=0.3, sigma_hi=0.3, n_queries=100),
    "headline": MixtureSpec(n=1_000_000, d=256, n_centres=1_000, centre_std=2.0,
                            sigma_lo=0.2, sigma_hi=0.5, n_queries=10_000),
}

SEEDS = {"parity": 20210712, "headline": 20210713, "acp": 20210714, "serving": 20210715,
         "heavy": 20210716}


def _draw_points(rng, labels, centres, sigmas, d):
    """centre[label] + sigma[label] * N(0,1)^d, drawn in row chunks (float32)."""
    n = labels.shape[0]
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        noise = rng.standard_normal((e - s, d), dtype=np.float32)
        lab = labels[s:e]
        out[s:e] = centres[lab] + sigmas[lab, None] * noise
    return out


def _centres_and_sigmas(rng, spec: MixtureSpec):
    centres = (rng.standard_normal((spec.n_centres, spec.d), dtype=np.float32)
               * np.float32(spec.centre_std))
    if spec.sigma_lo == spec.sigma_hi:
        sigmas = np.full(spec.n_centres, spec.sigma_lo, dtype=np.float32)
    else:
        sigmas = rng.uniform(spec.sigma_lo, spec.sigma_hi,
                             spec.n_centres).astype(np.float32)
    return centres, sigmas


def hash_matrix(rng, m: int, d: int) -> np.ndarray:
    """A: m x d, i.i.d. standard normal (2-stable), float32, row-major."""
    return rng.standard_normal((m, d), dtype=np.float32)


def mixture(spec: MixtureSpec, seed: int, n: int | None = None,
            n_queries: int | None = None):
    """Points, fresh queries and hash matrix of a Gaussian mixture.

    ``n`` and ``n_queries`` override the spec's sizes (same recipe, smaller
    draw) so tests can run scaled copies of a workload.
    Returns dict(D=(n,d) f32, Q=(nq,d) f32, A=(m,d) f32, labels, qlabels).
    """
    n = spec.n if n is None else int(n)
    nq = spec.n_queries if n_queries is None else int(n_queries)
    rng = np.random.Generator(np.random.PCG64(seed))
    centres, sigmas = _centres_and_sigmas(rng, spec)
    labels = rng.integers(0, spec.n_centres, size=n)
    D = _draw_points(rng, labels, centres, sigmas, spec.d)
    qlabels = rng.integers(0, spec.n_centres, size=nq)
    Q = _draw_points(rng, qlabels, centres, sigmas, spec.d)
    A = hash_matrix(rng, spec.m, spec.d)
    return {"D": D, "Q": Q, "A": A, "labels": labels, "qlabels": qlabels}


def parity(seed: int = SEEDS["parity"], n=None, n_queries=None):
    """10,000 x 128 parity workload (50 centres, sigma 0.3, 100 queries)."""
    return mixture(SPECS["parity"], seed, n, n_queries)


def headline(seed: int = SEEDS["headline"], n=None, n_queries=None):
    """1M x 256 workload (1,000 centres, var-4 centres, sigma U[0.2,0.5])."""
    return mixture(SPECS["headline"], seed, n, n_queries)


def planted_pairs(seed: int = SEEDS["acp"], n: int = 200_000, d: int = 512,
                  n_centres: int = 500, copy_frac: float = 0.01,
                  copy_std: float = 1e-3, m: int = M_DEFAULT):
    """Closest-pair workload: a mixture plus planted near-duplicate pairs.

    ``n_orig = n - n_copies`` originals are drawn from the mixture; then
    ``n_copies = round(copy_frac * n)`` distinct originals are copied and each
    copy gets N(0, copy_std^2) noise. Copies are appended after the
    originals. Returns dict(D, A, pairs=(n_copies, 2) int64 with
    pairs[:,0] < pairs[:,1]).
    """
    n_copies = int(round(copy_frac * n))
    n_orig = n - n_copies
    spec = MixtureSpec(n=n_orig, d=d, n_centres=n_centres, centre_std=2.0,
                       sigma_lo=0.2, sigma_hi=0.5, n_queries=0, m=m)
    rng = np.random.Generator(np.random.PCG64(seed))
    centres, sigmas = _centres_and_sigmas(rng, spec)
    labels = rng.integers(0, n_centres, size=n_orig)
    X = _draw_points(rng, labels, centres, sigmas, d)
    src = rng.choice(n_orig, size=n_copies, replace=False)
    noise = rng.standard_normal((n_copies, d), dtype=np.float32)
    copies = X[src] + np.float32(copy_std) * noise
    A = hash_matrix(rng, m, d)
    D = np.concatenate([X, copies], axis=0)
    pairs = np.stack([src.astype(np.int64),
                      np.arange(n_orig, n, dtype=np.int64)], axis=1)
    return {"D": D, "A": A, "pairs": pairs, "labels": labels}


def uniform_cube(seed: int, n: int, d: int, n_queries: int, m: int = M_DEFAULT,
                 lo: float = -1.0, hi: float = 1.0):
    """Structureless control workload: points and queries uniform in a cube."""
    rng = np.random.Generator(np.random.PCG64(seed))
    D = rng.uniform(lo, hi, size=(n, d)).astype(np.float32)
    Q = rng.uniform(lo, hi, size=(n_queries, d)).astype(np.float32)
    A = hash_matrix(rng, m, d)
    return {"D": D, "Q": Q, "A": A}


def heavy_tailed(seed: int = SEEDS["heavy"], n: int = 1_000_000, d: int = 960,
                 n_queries: int = 10_000, m: int = M_DEFAULT):
    """Mixed-precision workload: non-negative heavy-tailed features, every
    coordinate |N(0,1)|^1.5, rows L2-normalised and scaled by 100; queries
    drawn the same way."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def rows(count, block=65_536):
        # drawn in row blocks (the same numbers as one draw) to bound memory
        out = np.empty((count, d), dtype=np.float32)
        for s in range(0, count, block):
            x = np.abs(rng.standard_normal((min(block, count - s), d))) ** 1.5
            x *= 100.0 / np.linalg.norm(x, axis=1, keepdims=True)
            out[s:s + x.shape[0]] = x
        return out

    D = rows(n)
    Q = rows(n_queries)
    A = hash_matrix(rng, m, d)
    return {"D": D, "Q": Q, "A": A}


def serving(seed: int = SEEDS["serving"], n: int = 10_000_000, d: int = 128,
            n_centres: int = 10_000, sigma=None, n_queries: int = 20_000,
            m: int = M_DEFAULT):
    """Serving workload: a resident index of FP16-valued points in [0, 255].

    Centres uniform in [0, 255]^d, each with its own spread sigma_c drawn
    uniform in [4, 16] (or the fixed `sigma` when given); each point is a
    centre plus N(0, sigma_c^2) noise, clipped to [0, 255] and rounded to the
    nearest FP16 value (held as float32); queries drawn the same way. The
    request stream is drawn separately (``requests``).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.0, 255.0, size=(n_centres, d)).astype(np.float32)
    if sigma is None:
        sig = rng.uniform(4.0, 16.0, size=n_centres).astype(np.float32)
    else:
        sig = np.full(n_centres, sigma, dtype=np.float32)

    def draw(count):
        lab = rng.integers(0, n_centres, size=count)
        X = _draw_points(rng, lab, centres, sig, d)
        np.clip(X, 0.0, 255.0, out=X)
        return X.astype(np.float16).astype(np.float32)

    D = draw(n)
    Q = draw(n_queries)
    A = hash_matrix(rng, m, d)
    return {"D": D, "Q": Q, "A": A}


def requests(seed: int, rate_qps: float, duration_s: float, max_batch: int = 4096,
             ks=(1, 10, 50, 100), cs=(1.2, 1.5, 2.0)):
    """A Poisson stream of requests: arrival times (s), batch sizes
    (log-uniform in [1, max_batch]), k and c drawn uniformly from ks and cs.
    The request rate is rate_qps divided by the mean batch size."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mean_b = (max_batch - 1) / np.log(max_batch)     # mean of the log-uniform size
    lam = rate_qps / mean_b
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / lam)
        if t >= duration_s:
            break
        size = int(min(max_batch, max(1, np.floor(np.exp(rng.uniform(0.0, np.log(max_batch + 1)))))))
        out.append((t, size, int(rng.choice(ks)), float(rng.choice(cs))))
    return out
