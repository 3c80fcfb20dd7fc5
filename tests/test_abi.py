"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, the host-only planner agrees with the oracle, and invalid
arguments are rejected with the documented codes before any HIP call."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2107_05537_amd as pm
from oracle import chi2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pmlsh.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pm.library_path):
        pytest.skip("libpmlsh.so not built")
    return pm.load_library()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pmlsh_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert set(names) == set(pm.SIGNATURES)


@pytest.mark.parametrize("m", [1, 2, 7, 15, 16])
@pytest.mark.parametrize("c", [1.2, 1.5, 2.0, 4.0])
@pytest.mark.parametrize("conf", [0.5, 1 - 1 / math.e, 0.9, 0.99])
def test_planner_matches_oracle(lib, m, c, conf):
    p = pm.plan_params(1_000_000, m, 10, c, conf, -1.0)
    alpha1 = 1 - conf
    assert p["t"] == pytest.approx(chi2.radius_factor(alpha1, m), rel=1e-11)
    a2 = chi2.alpha2(alpha1, c, m)
    assert p["alpha2"] == pytest.approx(a2, rel=1e-9, abs=1e-15)
    assert p["beta"] == pytest.approx(2 * a2, rel=1e-9, abs=1e-15)
    assert p["budget"] == chi2.ann_budget(p["beta"], 1_000_000, 10)
    assert p["acp_budget"] == chi2.acp_budget(p["beta"], 1_000_000, 10)


def test_planner_budgets_explicit_beta(lib):
    for n, k, beta in [(10_000, 10, 0.1), (1001, 1, 0.0015), (100, 10, 1.0), (7, 7, 0.0),
                       (200_000, 100, 0.0967)]:
        p = pm.plan_params(n, 15, k, 1.5, 0.9, beta)
        assert p["beta"] == beta
        assert p["budget"] == chi2.ann_budget(beta, n, k)
        assert p["acp_budget"] == chi2.acp_budget(beta, n, k)


@pytest.mark.parametrize("args", [
    (0, 15, 10, 1.5, 0.9, 0.1),        # n < 1
    (100, 0, 10, 1.5, 0.9, 0.1),       # m < 1
    (100, 17, 10, 1.5, 0.9, 0.1),      # m > 16
    (100, 15, 0, 1.5, 0.9, 0.1),       # k < 1
    (100, 15, 10, 1.0, 0.9, 0.1),      # c <= 1
    (100, 15, 10, math.inf, 0.9, 0.1),
    (100, 15, 10, 1.5, 0.0, 0.1),      # confidence outside (0,1)
    (100, 15, 10, 1.5, 1.0, 0.1),
    (100, 15, 10, 1.5, 0.9, 1.5),      # beta > 1
    (100, 15, 10, 1.5, 0.9, math.nan),
])
def test_planner_rejects(lib, args):
    with pytest.raises(pm.PmlshError) as e:
        pm.plan_params(*args)
    assert e.value.code == pm.EINVAL
    assert lib.pmlsh_last_error()


def _build_args(**kw):
    a = pm._BuildArgs()
    D = np.zeros((10, 4), dtype=np.float32)
    H = np.ones((3, 4), dtype=np.float32)
    a.data, a.hash = D.ctypes.data, H.ctypes.data
    a.n, a.d, a.m = 10, 4, 3
    a.data_on_device = 0
    a.num_pivots, a.leaf_size, a.fanout = 5, 0, 0
    a.r_min_kappa = 0.0
    for k, v in kw.items():
        setattr(a, k, v)
    return a, (D, H)


@pytest.mark.parametrize("kw", [
    {"n": 0}, {"d": 0}, {"m": 0}, {"m": 17}, {"num_pivots": 9}, {"num_pivots": -1},
    {"leaf_size": 4}, {"leaf_size": 300}, {"fanout": 3}, {"fanout": 128},
    {"filter_gemm": 3}, {"filter_gemm": -1},
    {"r_min_kappa": 1.5}, {"data": None}, {"hash": None},
])
def test_build_rejects_before_touching_gpu(lib, kw):
    a, keep = _build_args(**kw)
    out = ctypes.c_void_p()
    assert lib.pmlsh_build(ctypes.byref(a), ctypes.byref(out)) == pm.EINVAL
    assert out.value is None
    assert lib.pmlsh_last_error()


def test_build_rejects_non_finite_host_data(lib):
    a, (D, H) = _build_args()
    D[3, 2] = np.nan
    out = ctypes.c_void_p()
    assert lib.pmlsh_build(ctypes.byref(a), ctypes.byref(out)) == pm.EINVAL
    assert b"non-finite" in lib.pmlsh_last_error()
    D[3, 2] = 0
    H[0, 0] = np.inf
    assert lib.pmlsh_build(ctypes.byref(a), ctypes.byref(out)) == pm.EINVAL


def test_null_handles_rejected(lib):
    assert lib.pmlsh_build(None, None) == pm.EINVAL
    ids = ctypes.c_void_p(1)
    assert lib.pmlsh_ann(None, ids, 1, 1, 1.5, 0.9, 0.1, 0.0, ids, ids, None, None) == pm.EINVAL
    assert lib.pmlsh_acp(None, 1, 1.5, 0.9, 0.1, ids, ids, None, None) == pm.EINVAL
    assert lib.pmlsh_bc(None, ids, 1, 1.0, 1.5, 0.9, 0.1, ids, ids, None, None) == pm.EINVAL
    assert lib.pmlsh_acp_bb(None, 1, 1.5, 0.9, 0.1, ids, ids, None, None) == pm.EINVAL
    assert lib.pmlsh_acp_lca(None, 1, 1.5, 0.9, 0.1, 0.0, ids, ids, None, None, None) == pm.EINVAL
    assert lib.pmlsh_index_export_nodes(None, None, None, None, None) == pm.EINVAL
    assert lib.pmlsh_get_index_info(None, None) == pm.EINVAL
    assert lib.pmlsh_index_export_leaves(None, None, None) == pm.EINVAL
    assert lib.pmlsh_default_r_min(None, 1, None) == pm.EINVAL
    lib.pmlsh_free(None)   # no-op


def test_binding_refuses_cpu_tensors(lib):
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        pm.Index(torch.zeros(10, 4), np.ones((3, 4), dtype=np.float32))


def test_timing_stage_mask(lib):
    """The timing switch takes a mask of stages; bits past the last stage are
    rejected, and reading with nothing timed returns zeros."""
    assert lib.pmlsh_ann_timing_enable(1 << len(pm.STAGES)) == pm.EINVAL
    assert lib.pmlsh_ann_timing_enable(-1) == pm.EINVAL
    assert lib.pmlsh_ann_timing_enable((1 << len(pm.STAGES)) - 1) == pm.OK
    assert lib.pmlsh_ann_timing_enable(0) == pm.OK
    t = pm.ann_timing_read(reset=True)
    assert set(t) == set(pm.STAGES)
    assert all(v["ms"] == 0 and v["launches"] == 0 for v in t.values())
    pm.ann_timing_enable(True, stages=["finish"])
    pm.ann_timing_enable(False)


def test_server_null_handles_rejected(lib):
    """The serving-loop entry points check their arguments before any HIP call."""
    t = ctypes.c_uint64(0)
    done = ctypes.c_int(0)
    out = ctypes.c_void_p()
    assert lib.pmlsh_server_create(None, None, ctypes.byref(out)) == pm.EINVAL
    assert lib.pmlsh_server_submit(None, None, 0, 1, 1.5, 0.9, 0.1, 0.0, None, None, None,
                                   ctypes.byref(t)) == pm.EINVAL
    assert lib.pmlsh_server_test(None, 1, ctypes.byref(done)) == pm.EINVAL
    assert lib.pmlsh_server_wait(None, 1) == pm.EINVAL
    assert lib.pmlsh_server_get_stats(None, None) == pm.EINVAL
    lib.pmlsh_server_destroy(None)   # no-op


def test_tune_switches(lib):
    """pmlsh_tune takes the two switches of the bound kernel's group filter,
    the FP32-path switch, the scan shape and ACP's first capacity within
    their ranges (-1
    restores the default) and rejects anything else; it touches no GPU."""
    for key, good in ((pm.TUNE_GROUP_LIST, (0, 1, 2048, -1)), (pm.TUNE_GROUP_MINIMA_LDS, (0, 1, -1)),
                      (pm.TUNE_FP32_PATH, (1, 0, -1)), (pm.TUNE_ACP_FIRST_CAP, (1, 1 << 20, 0, -1)),
                      (pm.TUNE_SCAN_SHAPE, (1, 2, 0, -1))):
        for v in good:
            assert lib.pmlsh_tune(key, v) == 0
    for key, bad in ((pm.TUNE_GROUP_LIST, (2049, -2)), (pm.TUNE_GROUP_MINIMA_LDS, (2, -5)),
                     (pm.TUNE_FP32_PATH, (2, -3)), (pm.TUNE_ACP_FIRST_CAP, ((1 << 20) + 1, -2)),
                     (pm.TUNE_SCAN_SHAPE, (3, -2))):
        for v in bad:
            assert lib.pmlsh_tune(key, v) == pm.EINVAL
    for key in (-1, 5, 99):
        assert lib.pmlsh_tune(key, 0) == pm.EINVAL
    with pytest.raises(pm.PmlshError):
        pm.tune(pm.TUNE_GROUP_LIST, 5000)
    pm.tune(pm.TUNE_GROUP_LIST, -1)
    pm.tune(pm.TUNE_GROUP_MINIMA_LDS, -1)
