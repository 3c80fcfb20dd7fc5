"""Index build on the GPU: the device bulk-load of the leaf order.

Properties that any correct run of the recursive gap-aware splits has,
checked through the exported structure:
* the leaf order is a permutation of the ids, every leaf holds leaf_size
  points but the last;
* two clusters far apart, each a whole number of leaves, never share a leaf
  (once a node's middle 60 % of leaves reaches the gap between them, the
  node is cut there);
* every node's covering radius (about its centre) holds all its points
  (checked in FP64 on the host against the FP32 projection);
* two builds of the same data give the same leaf order (fixed reduction
  order on the device).
"""

import numpy as np
import pytest

import synth
from oracle import ann as oann
from parity import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_05537_amd as pm
    pm.load_library()
    return pm


def _check_partition(perm, offsets, n, leaf):
    assert np.array_equal(np.sort(perm), np.arange(n, dtype=np.int32))
    sizes = np.diff(offsets)
    assert np.all(sizes[:-1] == leaf)
    assert 0 < sizes[-1] <= leaf


@pytest.mark.parametrize("na_leaves,nb_leaves", [(50, 30), (7, 121), (3, 3)])
def test_separated_clusters_never_share_a_leaf(na_leaves, nb_leaves):
    pm = _gpu()
    leaf, d = 64, 24
    rng = np.random.default_rng(11)
    na, nb = na_leaves * leaf, nb_leaves * leaf
    say(f"case: clusters of {na} and {nb} points")
    A = rng.normal(size=(na, d)).astype(np.float32)
    B = (rng.normal(size=(nb, d)) + 1000.0).astype(np.float32)
    D = np.concatenate([A, B])
    H = synth.hash_matrix(rng, 15, d)
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(H).to(dev))
    perm, offsets = idx.export_leaves()
    _check_partition(perm, offsets, na + nb, leaf)
    for b in range(len(offsets) - 1):
        ids = perm[offsets[b]:offsets[b + 1]]
        assert np.all(ids < na) or np.all(ids >= na), b


def test_radii_cover_points_and_build_is_deterministic():
    pm = _gpu()
    spec = synth.MixtureSpec(n=200_000, d=32, n_centres=300, centre_std=3.0,
                             sigma_lo=0.3, sigma_hi=0.6, n_queries=1)
    w = synth.mixture(spec, 5)
    D, H = w["D"], w["A"]
    say("case: n=200000 d=32 mixture, two builds")
    dev = torch.device("cuda", 0)
    Dd, Hd = torch.from_numpy(D).to(dev), torch.from_numpy(H).to(dev)
    idx = pm.Index(Dd, Hd)
    perm, offsets = idx.export_leaves()
    _check_partition(perm, offsets, D.shape[0], 64)
    P = oann.project(D, H)
    nodes = idx.export_nodes()
    # every node at the top two levels and 2,000 sampled leaves; the centre
    # is the mean of the node's points rounded to FP32, which the FP64 mean
    # here matches up to that rounding and the FP32 rounding of the
    # projection (relative 1e-5 covers both)
    sel = np.flatnonzero(nodes["level"] <= 1)
    leaves = np.flatnonzero(nodes["level"] == nodes["level"].max())
    sel = np.concatenate([sel, np.random.default_rng(1).choice(leaves, 2000, replace=False)])
    for i in sel:
        pts = P[perm[offsets[nodes["first_leaf"][i]]:offsets[nodes["end_leaf"][i]]]]
        c = pts.mean(axis=0)
        far = np.sqrt(((pts - c) ** 2).sum(axis=1)).max()
        r = float(nodes["radius"][i])
        assert far <= r + 1e-5 * (np.linalg.norm(c) + r), (i, far, r)
    idx2 = pm.Index(Dd, Hd)
    perm2, offsets2 = idx2.export_leaves()
    assert np.array_equal(perm, perm2) and np.array_equal(offsets, offsets2)
