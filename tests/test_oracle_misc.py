"""Pins of the oracle's helpers: SplitMix64, the r_min rule, metrics."""

import math

import numpy as np
import pytest

import synth
from oracle import brute, metrics, rmin


def test_splitmix64_reference_output():
    # first output of SplitMix64 started from state 0 (published generator)
    assert rmin.splitmix64(0) == 0xE220A8397B1DCDAF


def test_sample_pairs_valid():
    ii, ll = rmin.sample_pairs(37, seed=123)
    assert ii.shape[0] == 37 * 36 // 2
    assert np.all(ii != ll)
    assert ii.min() >= 0 and ll.max() < 37


def test_r_min_is_kappa_times_sample_quantile():
    w = synth.parity(n=500, n_queries=1)
    D = w["D"]
    srt = rmin.sorted_sample_distances(D, seed=9)
    S = srt.shape[0]
    assert S == min(500 * 499 // 2, rmin.SAMPLE_PAIRS)
    B = 60
    r = rmin.r_min_from_sample(srt, 500, B)
    base = r / rmin.KAPPA
    # at least a fraction B/n of the sample lies at or below base, and fewer
    # than that lie strictly below it
    assert np.count_nonzero(srt <= base) >= math.ceil(B / 500 * S)
    assert np.count_nonzero(srt < base) < math.ceil(B / 500 * S)
    assert rmin.r_min_from_sample(srt, 500, 10 ** 6) == pytest.approx(
        rmin.KAPPA * srt[-1])


def test_metrics_eq12_to_14():
    assert metrics.overall_ratio([2.0, 3.0], [1.0, 3.0]) == pytest.approx(1.5)
    assert metrics.overall_ratio([0.0], [0.0]) == 1.0
    assert metrics.recall([[1, 2, 3]], [[3, 4, 1]]) == pytest.approx(2 / 3)
    assert metrics.pair_recall([(1, 2), (5, 3)], [(3, 5), (0, 9)]) == 0.5


def test_brute_knn_tie_break_by_id():
    D = np.array([[1, 0], [0, 1], [-1, 0], [0, -1], [2, 2]], dtype=np.float32)
    ids, dist = brute.knn(D, np.zeros((1, 2), dtype=np.float32), 3)
    assert ids[0].tolist() == [0, 1, 2]
    np.testing.assert_allclose(dist[0], [1, 1, 1])


def test_generators_are_deterministic():
    a = synth.parity(n=200, n_queries=3)
    b = synth.parity(n=200, n_queries=3)
    for key in ("D", "Q", "A"):
        assert a[key].dtype == np.float32
        assert np.array_equal(a[key], b[key])
    assert a["D"].shape == (200, 128) and a["A"].shape == (15, 128)
    p = synth.planted_pairs(n=1000, d=16, n_centres=5)
    assert p["pairs"].shape == (10, 2)
    dd = np.sqrt(((p["D"][p["pairs"][:, 0]] - p["D"][p["pairs"][:, 1]]) ** 2).sum(1))
    assert np.all(dd < 0.01)
