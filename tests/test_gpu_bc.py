"""(r,c)-BC query (Algorithm 1) on the GPU against the oracle.

The parity workload (10,000 x 128) at radii from far below the nearest-
neighbour distances (every ball empty: nothing) through the typical scale
(balls below the budget, answers found or not within c r) to radii whose
balls reach the budget. A query whose oracle decisions all have margins
above 1e-5 must match the oracle exactly (id, distance to 1e-5, whether the
budget was reached, |C|); a fragile one must return nothing or a real point
whose distance is its FP64 distance to 1e-5.
"""

import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import synth
from oracle import ann as oann
from oracle import bc as obc
from oracle import chi2
from parity import FRAGILE, TOL, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2107_05537_amd as pm
    pm.load_library()
    return pm


@pytest.fixture(scope="module")
def bc_setup():
    pm = _gpu()
    w = synth.parity()
    D, A, Q = w["D"], w["A"], w["Q"]
    dev = torch.device("cuda", 0)
    idx = pm.Index(torch.from_numpy(D).to(dev), torch.from_numpy(A).to(dev))
    nn = cKDTree(D.astype(np.float64)).query(Q.astype(np.float64), k=1)[0]
    return pm, idx, D, A, Q, oann.project(D, A), float(np.median(nn))


@pytest.mark.parametrize("scale,beta", [(1e-3, 0.05), (0.6, 0.05), (1.0, 0.05), (1.6, 0.05),
                                        (1.0, 0.0005), (50.0, 0.05)])
def test_bc_matches_oracle(bc_setup, scale, beta):
    pm, idx, D, A, Q, Dp, med = bc_setup
    c, conf = 1.5, 0.9
    r = med * scale
    say(f"case: (r,c)-BC r={r:.4g} (scale {scale}) beta={beta}")
    t = chi2.radius_factor(1 - conf, A.shape[0])
    B = chi2.ann_budget(beta, D.shape[0], 1)
    res = obc.run(D, A, Q, r=r, c=c, t=t, budget=B, Dp=Dp)
    dev = torch.device("cuda", 0)
    ids, dist, st = idx.bc(torch.from_numpy(Q).to(dev), r, c=c, confidence=conf, beta=beta,
                           stats=True)
    torch.cuda.synchronize()
    ids, dist, st = ids.cpu().numpy(), dist.cpu().numpy(), st.cpu().numpy()
    kinds = {obc.KIND_NONE: 0, obc.KIND_FOUND: 0, obc.KIND_BUDGET: 0}
    fragile = 0
    for qi, o in enumerate(res):
        kinds[o.kind] += 1
        assert st[qi, 0] == 1                      # one range query
        if o.margin > FRAGILE:
            assert ids[qi] == o.id, (qi, ids[qi], o)
            if o.id < 0:
                assert math.isinf(dist[qi])
            else:
                assert dist[qi] == pytest.approx(o.dist, rel=TOL)
            assert (st[qi, 2] == 2) == (o.kind == obc.KIND_BUDGET)
            assert st[qi, 1] == o.n_cand
        else:
            fragile += 1
            if ids[qi] >= 0:
                ex = float(np.sqrt(((D[ids[qi]].astype(np.float64)
                                     - Q[qi].astype(np.float64)) ** 2).sum()))
                assert dist[qi] == pytest.approx(ex, rel=TOL)
            else:
                assert math.isinf(dist[qi])
    say("oracle kinds", kinds, "fragile", fragile)
    if scale == 1e-3:
        assert kinds[obc.KIND_NONE] == len(res)
    if scale == 50.0:
        assert kinds[obc.KIND_BUDGET] == len(res)


def test_bc_empty_batch_and_errors(bc_setup):
    pm, idx, D, A, Q, Dp, med = bc_setup
    dev = torch.device("cuda", 0)
    ids, dist = idx.bc(torch.empty((0, D.shape[1]), device=dev), 1.0)
    assert ids.shape == (0,)
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(pm.PmlshError) as e:
            idx.bc(torch.from_numpy(Q[:2]).to(dev), bad)
        assert e.value.code == pm.EINVAL
    with pytest.raises(pm.PmlshError) as e:
        idx.bc(torch.from_numpy(Q[:2]).to(dev), 1.0, c=1.0)
    assert e.value.code == pm.EINVAL
