"""Mixed-precision filter projection (filter_gemm): the FP16 / BF16
matrix-core projection behind the filter rows stays within its stated bound
of the exact projection (Eq. 3, Section 3.2), and since the filter widens
its radius by that bound while every later decision uses the FP64-accurate
projection, answers equal the oracle's (and the default index's) exactly."""

import math

import numpy as np
import pytest

import synth
from oracle.ann import project
from parity import compare_ann, oracle_ann, oracle_r_min, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_05537_amd as pm
    pm.load_library()
    return pm


MODES = {"fp16": 1, "bf16": 2}


@pytest.fixture(scope="module")
def heavy():
    return synth.heavy_tailed(n=20_000, n_queries=32)


@pytest.mark.parametrize("mode", ["fp16", "bf16"])
@pytest.mark.parametrize("wl", ["heavy", "parity"])
def test_projection_within_its_bound(mode, wl, heavy):
    """|o'_lp - o'| <= eps(o) for every point, o' the exact (FP64) projection
    of the FP32 row; eps_max of the index is the largest eps."""
    pm = _gpu()
    w = heavy if wl == "heavy" else synth.parity()
    D, A = w["D"], w["A"]
    say(f"case: filter projection bound, {mode}, {wl} {D.shape}")
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev),
                   filter_gemm=MODES[mode])
    lp, eps = idx.filter_projection()
    exact = project(D, A)
    err = np.sqrt(((lp.astype(np.float64) - exact) ** 2).sum(1))
    assert np.all(np.isfinite(eps)) and np.all(eps > 0)
    assert np.all(err <= eps), f"{int((err > eps).sum())} points outside their bound"
    info = idx.info()
    assert info["filter_gemm"] == MODES[mode]
    assert info["eps_max"] == pytest.approx(float(eps.max()), rel=0, abs=0)
    # the bound is the stated one, c1 S_i + eta' (A_i + X) per coordinate
    # (S_i = sum_j |a_ij| |o_j|), evaluated here in FP64: not looser
    u = 2.0 ** -11 if mode == "fp16" else 2.0 ** -8
    eta = 1.02 * (2.0 ** -14 if mode == "fp16" else 2.0 ** -126)
    d = D.shape[1]
    gd = d * 2.0 ** -23 / (1 - d * 2.0 ** -23)
    c1 = ((2 * u + u * u) / (1 - u) ** 2 + gd) / (1 - gd)
    S = np.abs(D).astype(np.float64) @ np.abs(A).astype(np.float64).T
    Ai = np.abs(A).astype(np.float64).sum(1)
    X = np.abs(D).astype(np.float64).sum(1)
    stated = np.sqrt(((c1 * S + eta * (Ai[None, :] + X[:, None])) ** 2).sum(1))
    assert np.all(eps <= stated * 1.001 + 1e-6)
    # the kernel sums |a~| |o~| of the rounded inputs, up to 2u below S
    assert np.all(eps >= stated * (1 - 2 * u - 2 * gd) - 1e-6)
    say(f"err/eps median {np.median(err / eps):.3g} max {np.max(err / eps):.3g}, "
        f"eps median {np.median(eps):.3g}, |o'| median {np.median(np.linalg.norm(exact, axis=1)):.3g}")


@pytest.mark.parametrize("mode", ["fp16", "bf16"])
@pytest.mark.parametrize("c", [1.2, 1.5, 2.0])
def test_mixed_precision_answers_match_oracle(mode, c, heavy):
    """20,000 x 960 heavy-tailed rows, 32 queries, k = 10: the widened filter
    misses no point the exact filter keeps, so answers equal the oracle's
    under the parity rule and the default index's bit for bit."""
    pm = _gpu()
    say(f"case: mixed precision {mode} heavy-tailed n=20000 d=960 c={c}")
    D, A, Q = heavy["D"], heavy["A"], heavy["Q"]
    k, beta = 10, 0.05
    B = min(D.shape[0], math.ceil(beta * D.shape[0]) + k)
    r0 = oracle_r_min(D, 5, B)
    res, _ = oracle_ann(D, A, Q, k, c, 0.9, beta, r_min=r0)
    dev = torch.device("cuda", 0)
    Dt, At, Qt = (torch.from_numpy(x).to(dev) for x in (D, A, Q))
    out = {}
    for name, fg in (("exact", 0), (mode, MODES[mode])):
        idx = pm.Index(Dt, At, sample_seed=5, filter_gemm=fg)
        ids, dist, st = idx.ann(Qt, k, c=c, confidence=0.9, beta=beta, r_min=r0, stats=True)
        torch.cuda.synchronize()
        out[name] = (ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy())
        del idx
    ids, dist, st = out[mode]
    compare_ann(D, Q, res, ids, dist, st, fp64=True)
    assert np.array_equal(ids, out["exact"][0])
    assert np.array_equal(dist, out["exact"][1])


def test_mixed_precision_parity_workload_batched():
    """10,000 x 128 parity workload, 100 queries, FP16 filter projection, on
    the batched path (B <= 2,048)."""
    pm = _gpu()
    w = synth.parity()
    D, A, Q = w["D"], w["A"], w["Q"]
    say("case: mixed precision fp16, parity workload")
    res, B = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.1, r_min=1.0)
    r0 = oracle_r_min(D, 0x5EED, B)
    res, B = oracle_ann(D, A, Q, 10, 1.5, 0.9, 0.1, r_min=r0)
    assert B <= 2048
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev), filter_gemm=1)
    ids, dist, st = idx.ann(torch.from_numpy(Q).to(dev), 10, c=1.5, confidence=0.9, beta=0.1,
                            r_min=r0, stats=True)
    torch.cuda.synchronize()
    compare_ann(D, Q, res, ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy(), fp64=True)


def test_filter_projection_needs_the_mode():
    pm = _gpu()
    dev = torch.device("cuda", 0)
    w = synth.parity(n=2000, n_queries=4)
    idx = pm.Index(torch.from_numpy(w["D"]).to(dev), torch.from_numpy(w["A"]).to(dev))
    with pytest.raises(pm.PmlshError) as e:
        idx.filter_projection()
    assert e.value.code == pm.EINVAL
