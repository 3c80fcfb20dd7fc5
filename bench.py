"""Benchmark of the PM-LSH (c,k)-ANN query path on one MI355X.

Workload: 1,000,000 x 256 Gaussian mixture (1,000 centres of variance 4,
per-centre sigma U[0.2, 0.5]), m = 15 projections, 10,000 fresh queries in
batches of 1,024 per launch, k = 10, c = 1.5, confidence 1 - 1/e. Inputs are
synthetic (seeded) and resident in HBM before timing starts.

Metric: queries/s at recall@10 >= 0.9. The candidate fraction beta is swept
({5e-4, 6e-4, 7e-4, then steps of 2.5e-5 or 5e-5 up to 1e-3, then 1.5e-3,
2e-3, 5e-3}); the smallest beta whose recall@10 over all 10,000 queries reaches
0.9 is the operating point, and only that point is timed. A step is one pmlsh_ann call on one batch of 1,024 queries
(projection, chunk distances, bound and Eq. 5 chunk test, range filter on
the matrix cores, budget selection, bounded verification, top-k); the calls
are asynchronous, back to back on one stream (--streams S issues them
round-robin on S streams instead). The same loop gives the operating points
for k = 1, 50 and 100 ("other_k").

Also reported: p50/p99 latency of one batch alone on one stream; per-stage
GPU time (HIP events around each stage, from the warm-up); the roofline of
the dominant stage (algorithmic work per launch / its launch time measured
with HIP events in the timed region, where only that stage of every eighth
batch is timed: flops
against the FP16 matrix peak for the filter, bytes against 8 TB/s for the
HBM-bound stages), with the HBM traffic that rocprofv3 counters measured for
that kernel when profiles/ holds them for the current kernel sources; the
FP64 CPU oracle timed on this host on a bounded sample of the same queries;
(c,k)-ACP time per call on the planted-pair workload for k = 1, 10, 100;
the serving loop on the 10,000,000 x 128 index (Poisson request streams of
mixed k and c at several rates: queries/s and p50/p99 request latency of
the server and of plain per-request calls, and both at saturation).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP16_MFMA_PEAK_TFLOPS = 2500.0    # MI355X published dense FP16 matrix peak
BETAS = [5e-4, 6e-4, 7e-4, 7.5e-4, 8e-4, 8.25e-4, 8.5e-4, 8.75e-4, 9e-4, 9.25e-4, 9.5e-4,
         9.75e-4, 1e-3, 1.5e-3, 2e-3, 5e-3]
K = 10
KS = (1, 10, 50, 100)        # k of the operating points (K is the headline)
C = 1.5
CONF = 1 - 1 / math.e
BATCH = 1024
PROBE_EVERY = 8              # batches per timed launch of the dominant stage
PMC_FILE = os.path.join(ROOT, "profiles", "ann_headline_pmc.json")
CALIB_BYTES = 256 << 20     # copy kernel of known size for counter calibration


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def exact_knn_gpu(torch, D, Q, k, chunk=128):
    """Ground-truth exact kNN: ids sorted by (distance, id) and their FP64
    distances, for recall and overall ratio.

    Measurement only, not part of the timed path: FP64 distances by the
    norm expansion on the GPU pick 4k candidates, which are re-ranked by FP64
    direct differences."""
    Dd = D.double()
    dn = (Dd * Dd).sum(1)
    out, outd = [], []
    for s in range(0, Q.shape[0], chunk):
        q = Q[s:s + chunk].double()
        d2 = (q * q).sum(1, keepdim=True) + dn[None, :] - 2.0 * (q @ Dd.T)
        cand = torch.topk(d2, 4 * k, dim=1, largest=False).indices
        diff = Dd[cand] - q[:, None, :]
        ex = (diff * diff).sum(2)
        # order by (exact distance, id)
        key_id = cand.double()
        o = torch.argsort(key_id, dim=1)
        ex, cand = torch.gather(ex, 1, o), torch.gather(cand, 1, o)
        o = torch.argsort(ex, dim=1, stable=True)
        out.append(torch.gather(cand, 1, o)[:, :k])
        outd.append(torch.gather(ex, 1, o)[:, :k].sqrt())
    return torch.cat(out), torch.cat(outd)


def overall_ratio(torch, D, Q, ids, truth_dist, chunk=256):
    """Overall ratio of Eqs. 12 and 14 (Section 7.1): the mean over queries
    and ranks of the returned point's distance over the exact i-th nearest
    neighbour's distance, both in FP64 (ranks at exact distance 0 count 1
    when the returned distance is 0 too)."""
    k = ids.shape[1]
    tot, cnt = 0.0, 0
    for s in range(0, Q.shape[0], chunk):
        e = min(Q.shape[0], s + chunk)
        q = Q[s:e].double()
        dd = D[ids[s:e].reshape(-1)].double().reshape(e - s, k, -1) - q[:, None, :]
        got = (dd * dd).sum(2).sqrt()
        ex = truth_dist[s:e, :k]
        r = torch.where(ex > 0, got / torch.where(ex > 0, ex, torch.ones_like(ex)),
                        torch.where(got > 0, torch.full_like(got, float("inf")),
                                    torch.ones_like(got)))
        tot += float(r.sum())
        cnt += r.numel()
    return tot / max(1, cnt)


def recall_at_k(ids, truth):
    hit = (ids[:, :, None] == truth[:, None, :]).any(2).sum(1).double()
    return float((hit / truth.shape[1]).mean())


def kernel_source_hash(files=("ann.hip", "project.hip", "internal.hpp")):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2107_05537_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(kernel, sha_key, files):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter summary in
    profiles/, when it was taken on the current kernel sources."""
    if not os.path.exists(PMC_FILE):
        return None
    with open(PMC_FILE) as fh:
        pmc = json.load(fh)
    if pmc.get(sha_key) != kernel_source_hash(files):
        return None
    return pmc.get("kernels", {}).get(kernel, {}).get("hbm_bytes_per_launch")


_CPU = {}     # workload and oracle projection, inherited by the forked CPU workers


def _cpu_worker(task):
    """One CPU-baseline worker: the oracle's Algorithm 2 for the queries
    [q0, q1) of the headline workload, as long as the time budget lasts."""
    from oracle import ann as oann
    q0, q1, t, budget, r_min, budget_s = task
    D, Dp, Q, A = _CPU["D"], _CPU["Dp"], _CPU["Q"], _CPU["A"]
    t0 = time.perf_counter()
    done = 0
    for qi in range(q0, q1):
        if done and time.perf_counter() - t0 > budget_s:
            break
        qp = oann.project(Q[qi:qi + 1], A)[0]
        oann.query(D, Dp, Q[qi], qp, K, C, t, budget, r_min)
        done += 1
    return done, time.perf_counter() - t0


def start_cpu_pool(w, workers):
    """Forks the CPU-baseline workers before anything touches the GPU, so the
    children hold no GPU handle; they inherit the workload and the oracle's
    FP64 projection of the data (index construction, not timed)."""
    import multiprocessing as mp
    from oracle import ann as oann
    _CPU.update(D=w["D"], Q=w["Q"], A=w["A"], Dp=oann.project(w["D"], w["A"]))
    return mp.get_context("fork").Pool(workers)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pool, workers, n, beta, r_min):
    """The FP64 oracle (Algorithm 2 as in oracle/ann.py, NumPy) on this host:
    one worker alone on the first queries (about 8 s), then every worker at
    once on its own slice of the next queries (about 1.5 s each)."""
    from oracle import chi2
    t = chi2.radius_factor(1 - CONF, 15)
    B = chi2.ann_budget(beta, n, K)
    done1, dt1 = pool.apply(_cpu_worker, ((0, 64, t, B, r_min, 8.0),))
    per = 16
    tasks = [(64 + i * per, 64 + (i + 1) * per, t, B, r_min, 1.5) for i in range(workers)]
    t0 = time.perf_counter()
    res = pool.map(_cpu_worker, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    cpu_s = dt1 + sum(r[1] for r in res)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"value": round(done / wall, 2), "unit": "queries/s", "cores": workers,
            "kind": "oracle",
            "sample": (f"{done} queries (numbers 64..{64 + workers * per - 1} of the 10,000, "
                       f"each worker taking its own slice) at beta={beta}, {workers} worker "
                       f"processes at once, {wall:.1f} s wall; FP64 NumPy oracle, projection "
                       f"of D precomputed; {cpu_s:.0f} s of CPU work in all"),
            "one_core": {"value": round(done1 / dt1, 2), "unit": "queries/s",
                         "sample": f"first {done1} of the 10,000 queries, {dt1:.1f} s"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity": avail}


FP32_PEAK_TFLOPS = 157.3     # MI355X published FP32 vector peak


def config3_bench(pm, torch, dev, cs=(1.2, 1.5, 2.0),
                  betas=(0.001, 0.002, 0.005, 0.02, 0.05), nq_eval=1024, k=10,
                  conf=1 - 1 / math.e, point_limit_s=20.0):
    """Low-contrast 1,000,000 x 960 workload (every coordinate |N(0,1)|^1.5,
    rows L2-normalised and scaled by 100): for every c, recall@10 and overall
    ratio (Eqs. 12-14) against exact FP64 kNN over the first nq_eval queries,
    and queries/s of the calls, as beta grows. Budgets above the batched
    path's limit go to the per-query path. A c stops at the first beta whose
    call takes longer than point_limit_s."""
    import synth
    t0 = time.perf_counter()
    w = synth.heavy_tailed()
    D = torch.from_numpy(w["D"]).to(dev)
    A = torch.from_numpy(w["A"]).to(dev)
    Q = torch.from_numpy(w["Q"][:nq_eval]).to(dev)
    n = D.shape[0]
    del w
    t1 = time.perf_counter()
    idx = pm.Index(D, A)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t1
    truth, truth_dist = exact_knn_gpu(torch, D, Q, k, chunk=64)
    torch.cuda.synchronize()
    log(f"config 3: data {t1 - t0:.1f} s, index {build_s:.1f} s, exact kNN done")
    rows = []
    for c in cs:
        for beta in betas:
            plan = pm.plan_params(n, A.shape[0], k, c, conf, beta)
            idx.ann(Q[:64], k, c=c, confidence=conf, beta=beta)
            torch.cuda.synchronize()
            t_0 = time.perf_counter()
            ids, _, st = idx.ann(Q, k, c=c, confidence=conf, beta=beta, stats=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t_0
            rec = recall_at_k(ids, truth)
            rat = overall_ratio(torch, D, Q, ids, truth_dist)
            stn = st.cpu().numpy().astype(np.int64)
            row = {"c": c, "beta": beta, "budget_B": int(plan["budget"]),
                   "path": "batched" if plan["budget"] <= 2048 else "per-query",
                   "recall@10": round(rec, 4), "overall_ratio": round(rat, 6),
                   "queries_per_s": round(Q.shape[0] / el, 1),
                   "mean_C": round(float(stn[:, 1].mean()), 1),
                   "mean_rounds": round(float(stn[:, 0].mean()), 3)}
            log(f"config 3: {row}")
            rows.append(row)
            if el > point_limit_s:
                break
    # the mixed-precision filter projection at one point of the sweep
    mixed = []
    for name, mode in (("fp16", pm.FILTER_GEMM_FP16), ("bf16", pm.FILTER_GEMM_BF16)):
        c, beta = 1.5, 0.002
        idx_m = pm.Index(D, A, filter_gemm=mode)
        ids0, dist0 = idx.ann(Q, k, c=c, confidence=conf, beta=beta)
        idx_m.ann(Q[:64], k, c=c, confidence=conf, beta=beta)
        torch.cuda.synchronize()
        t_0 = time.perf_counter()
        ids_m, dist_m = idx_m.ann(Q, k, c=c, confidence=conf, beta=beta)
        torch.cuda.synchronize()
        el = time.perf_counter() - t_0
        row = {"filter_gemm": name, "c": c, "beta": beta,
               "eps_max": round(float(idx_m.info()["eps_max"]), 4),
               "recall@10": round(recall_at_k(ids_m, truth), 4),
               "overall_ratio": round(overall_ratio(torch, D, Q, ids_m, truth_dist), 6),
               "answers_equal_exact_index": bool(torch.equal(ids_m, ids0) and torch.equal(dist_m, dist0)),
               "queries_per_s": round(Q.shape[0] / el, 1)}
        log(f"config 3: {row}")
        mixed.append(row)
        del idx_m
    del idx
    return {"workload": "heavy-tailed 1,000,000 x 960 (|N(0,1)|^1.5, rows L2-normalised x 100), "
                        f"first {nq_eval} of 10,000 queries, k={k}",
            "truth": "exact kNN in FP64 on the GPU (norm-expansion shortlist of 4k, "
                     "re-ranked by FP64 direct differences)",
            "build_s": round(build_s, 2), "points": rows, "mixed_precision": mixed}


def copy_rate_gbs(torch, dev, nbytes=256 << 20, reps=10):
    """HBM rate of a plain device copy (torch's copy kernel) of `nbytes`,
    counting the bytes read and written, timed with events over `reps`
    copies after a warm-up: what a streaming kernel reaches on this GPU, as
    context for the roofline fractions (which stay against the published
    peak)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return round(2.0 * nbytes / (ms * 1e-3) / 1e9, 1)


def with_copy_context(r, copy_gbs):
    """Adds the plain-copy rate and, where the counters give the kernel's HBM
    bytes per launch, the rate those bytes move at and its fraction of the
    copy rate."""
    r["copy_rate_gbs"] = copy_gbs
    if r.get("traffic") and r.get("per_launch_ms"):
        tr = r["traffic"] / (r["per_launch_ms"] * 1e-3) / 1e9
        r["traffic_rate_gbs"] = round(tr, 1)
        r["traffic_frac_of_copy"] = round(tr / copy_gbs, 4) if copy_gbs else None
    return r


def acp_bench(pm, torch, dev, ks=(1, 10, 100), c=1.5, calls=10, with_variants=True):
    """(c,k)-ACP on 200,000 x 512 with 2,000 planted near-duplicate pairs:
    time per call for each k (index built beforehand, data resident in HBM),
    recall and overall ratio (Eqs. 12-14) against the exact k closest pairs
    (the k closest planted pairs: each copy is ~0.023 from its original,
    every other pair several units apart), and the roofline of the two
    largest kernels from the library's per-stage HIP events: the self-join
    against HBM (4 n d_pad bytes, every row read once, Section 8(d)'s seed
    term) and the pair scan against the FP32 peak (3 x 16 flops per pair of
    every leaf pair that survives the Mindist test)."""
    import synth
    w = synth.planted_pairs()
    n, d = w["D"].shape
    D = torch.from_numpy(w["D"]).to(dev)
    A = torch.from_numpy(w["A"]).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx = pm.Index(D, A)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    copy_gbs = copy_rate_gbs(torch, dev)
    L = idx.info()["leaf_size"]
    d_pad = (d + 3) // 4 * 4
    Dn = w["D"].astype(np.float64)
    pl = w["pairs"]
    pd_ = np.sqrt(((Dn[pl[:, 0]] - Dn[pl[:, 1]]) ** 2).sum(1))
    order = np.lexsort((pl[:, 1], pl[:, 0], pd_))
    acp_stages = ["acp_selfjoin", "acp_select", "acp_tiles", "acp_scan", "acp_verify",
                  "acp_topk"]
    per_k = []
    for k in ks:
        pairs, dist, st = idx.acp(k, c=c)                     # warm-up
        torch.cuda.synchronize()
        # the calls are timed without stage events; the stage split comes
        # from as many further calls with the events on
        t0 = time.perf_counter()
        for _ in range(calls):
            pairs, dist, st = idx.acp(k, c=c)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / calls
        pm.ann_timing_read(reset=True)
        pm.ann_timing_enable(True, stages=acp_stages)
        for _ in range(3):
            idx.acp(k, c=c)
        torch.cuda.synchronize()
        pm.ann_timing_enable(False)
        tm = pm.ann_timing_read(reset=True)
        stage_ms = {s_: round(tm[s_]["ms"] / max(1, tm[s_]["launches"]), 4) for s_ in acp_stages
                    if tm[s_]["launches"]}
        got = pairs.cpu().numpy()
        exact = pl[order[:k]]
        correct = got.tolist() == exact.tolist()
        gd = np.sqrt(((Dn[got[:, 0]] - Dn[got[:, 1]]) ** 2).sum(1))
        ratio = float(np.mean(gd / pd_[order[:k]]))
        rec = len(set(map(tuple, got.tolist())) & set(map(tuple, exact.tolist()))) / k
        sj_bytes = 4.0 * n * d_pad
        sj_ms = stage_ms.get("acp_selfjoin")
        scan_flops = 48.0 * st["tiles_scanned"] * L * L
        sc_ms = stage_ms.get("acp_scan")
        roof = {
            "selfjoin": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                         "work": sj_bytes, "per_launch_ms": sj_ms,
                         "achieved": round(sj_bytes / (sj_ms * 1e-3) / 1e9, 1) if sj_ms else None},
            "scan": {"bound": "alu", "unit": "TFLOP/s", "peak": FP32_PEAK_TFLOPS,
                     "work": scan_flops, "per_launch_ms": sc_ms,
                     "achieved": round(scan_flops / (sc_ms * 1e-3) / 1e12, 2) if sc_ms else None,
                     "model": ("Section 8(d): 48 flops for every point pair of every scanned tile; "
                               "the parent-distance interval (Section 4.1) skips most pairs "
                               "without that work, so the rate can exceed the peak")},
        }
        for r_ in roof.values():
            r_["frac"] = round(r_["achieved"] / r_["peak"], 4) if r_["achieved"] else None
        roof["selfjoin"]["flops"] = 3.0 * d * st["n_seed"]
        roof["selfjoin"]["flops_achieved_tflops"] = (
            round(roof["selfjoin"]["flops"] / (sj_ms * 1e-3) / 1e12, 2) if sj_ms else None)
        acp_files = ("acp.hip", "internal.hpp")
        roof["selfjoin"]["model"] = "Section 8(d): 4 d_pad bytes per point (each row read once)"
        roof["selfjoin"]["traffic"] = pmc_traffic("acp_seed_gram_kernel", "acp_source_sha",
                                                  acp_files)
        roof["scan"]["traffic"] = pmc_traffic("acp_tile_scan_wave_kernel", "acp_source_sha",
                                              acp_files)
        with_copy_context(roof["selfjoin"], copy_gbs)
        log(f"ACP k={k}: {ms:.3f} ms per call, stages {stage_ms}, recall {rec:.3f}, "
            f"ratio {ratio:.6f}, roofline {roof}")
        per_k.append({"k": k, "ms_per_call": round(ms, 3), "calls": calls,
                      "k_closest_planted_pairs_returned": bool(correct),
                      "recall": rec, "overall_ratio": round(ratio, 6),
                      "stages_ms": stage_ms, "roofline": roof,
                      "n_seed": int(st["n_seed"]), "ub": st["ub"],
                      "tiles_scanned": int(st["tiles_scanned"]),
                      "tiles_total": int(st["tiles_total"]), "candidates": int(st["n_cand"]),
                      "budget_T": int(st["budget"])})
    # the paper-faithful variants beside the canonical one, k = 10, c = 1.5:
    # branch and bound (Algorithm 3) and radius filtering with FindLCA and
    # gamma estimated for Pr(gamma) = 0.85 (Algorithms 4-5), at the default
    # beta = 2 alpha2 (T ~ 1.9e9 pairs, beyond what the branch-and-bound scan
    # holds) and at beta = 1e-4 (T ~ 2e6, below the 6.3e6 seeds)
    variants = []
    k_v = 10
    exact = pl[order[:k_v]]
    for beta_v in ((-1.0, 1e-4) if with_variants else ()):
        for name, fn in (("canonical", lambda: idx.acp(k_v, c=c, beta=beta_v)),
                         ("branch_and_bound", lambda: idx.acp_bb(k_v, c=c, beta=beta_v)),
                         ("radius_filtering_lca", lambda: idx.acp_lca(k_v, c=c, beta=beta_v))):
            try:
                fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pairs, dist, st = fn()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
            except pm.PmlshError as e:
                variants.append({"algorithm": name, "beta": beta_v, "error": str(e)})
                log(f"ACP variant {name} beta={beta_v}: {e}")
                continue
            got = pairs.cpu().numpy()
            gd = np.sqrt(((Dn[got[:, 0]] - Dn[got[:, 1]]) ** 2).sum(1))
            row = {"algorithm": name, "k": k_v, "c": c, "beta": beta_v,
                   "ms_per_call": round(ms, 3),
                   "recall": len(set(map(tuple, got.tolist()))
                                 & set(map(tuple, exact.tolist()))) / k_v,
                   "overall_ratio": round(float(np.mean(gd / pd_[order[:k_v]])), 6),
                   "verified_candidates": int(st["n_cand"]), "n_seed": int(st["n_seed"]),
                   "budget_T": int(st["budget"])}
            if "gamma" in st:
                row["gamma"] = st["gamma"]
            log(f"ACP variant: {row}")
            variants.append(row)
    return {"workload": "200,000 x 512 Gaussian mixture with 2,000 planted near-duplicate pairs",
            "c": c, "build_s": round(build_s, 2), "per_k": per_k, "variants": variants}


def exact_knn_gpu32(torch, D, Q, k, chunk=32):
    """Exact kNN (ids by (distance, id), FP64 distances) for a large index:
    FP32 norm expansion picks 4k candidates per query, re-ranked by FP64
    direct differences (measurement only)."""
    dn = (D * D).sum(1)
    out, outd = [], []
    for s in range(0, Q.shape[0], chunk):
        q = Q[s:s + chunk]
        d2 = (q * q).sum(1, keepdim=True) + dn[None, :] - 2.0 * (q @ D.T)
        cand = torch.topk(d2, 4 * k, dim=1, largest=False).indices
        del d2
        diff = D[cand].double() - q.double()[:, None, :]
        ex = (diff * diff).sum(2)
        o = torch.argsort(cand.double(), dim=1)
        ex, cand = torch.gather(ex, 1, o), torch.gather(cand, 1, o)
        o = torch.argsort(ex, dim=1, stable=True)
        out.append(torch.gather(cand, 1, o)[:, :k])
        outd.append(torch.gather(ex, 1, o)[:, :k].sqrt())
    return torch.cat(out), torch.cat(outd)


def serving_bench(pm, torch, dev, rates=(5000, 20000, 50000, 400000, 800000), duration_s=2.0,
                  betas=(5e-5, 7.5e-5, 1e-4, 1.25e-4, 1.5e-4, 1.9e-4), conf=1 - 1 / math.e):
    """Serving loop on a resident 10,000,000 x 128 index: Poisson request
    streams (sizes log-uniform in 1..4,096, k in {1,10,50,100}, c in
    {1.2,1.5,2.0}) answered by the continuous-batching server (requests of
    any k and c share launches) and, for comparison, by one synchronous call
    per request in arrival order on the plain FP32 path (every query on the
    per-query kernel: PM-tree walk with Eq. 5, FP32 projected and exact
    distances) and on the batched path. beta is the smallest of `betas` whose
    recall over a sample of mixed requests reaches 0.9. Latency is arrival
    to completion."""
    import threading
    import synth
    t0 = time.perf_counter()
    w = synth.serving(n_queries=20_000)
    D = torch.from_numpy(w["D"]).to(dev)
    A = torch.from_numpy(w["A"]).to(dev)
    Q = torch.from_numpy(w["Q"]).to(dev)
    del w
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    idx = pm.Index(D, A)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t1
    log(f"serving index built in {build_s:.1f} s ({t1 - t0:.1f} s to draw the data)")
    nq_all = Q.shape[0]

    # beta: smallest with recall >= 0.9 on 256 queries of mixed k and c
    rng = np.random.Generator(np.random.PCG64(99))
    ns = 256
    ks = rng.choice([1, 10, 50, 100], size=ns)
    cs = rng.choice([1.2, 1.5, 2.0], size=ns)
    Qs = Q[nq_all - ns:].contiguous()
    t_ids, t_dist = exact_knn_gpu32(torch, D, Qs, 100)
    t_ids, t_dist = t_ids.cpu().numpy(), t_dist.cpu().numpy()
    beta, beta_sweep = betas[-1], []
    for bt in betas:
        params = [{"k": int(k_), "c": float(c_), "confidence": conf, "beta": bt}
                  for k_, c_ in zip(ks, cs)]
        ids, _ = idx.ann_mixed(Qs, params)
        ids = ids.cpu().numpy()
        rec = float(np.mean([len(set(ids[i, :ks[i]].tolist()) & set(t_ids[i, :ks[i]].tolist()))
                             / ks[i] for i in range(ns)]))
        beta_sweep.append({"beta": bt, "recall": round(rec, 4)})
        log(f"serving beta={bt:g}: sampled recall {rec:.4f}")
        if rec >= 0.9:
            beta = bt
            break

    def slices(reqs):
        out, pos = [], 0
        for (_, size, _, _) in reqs:
            if pos + size > nq_all - ns:
                pos = 0
            out.append((pos, pos + size))
            pos += size
        return out

    def pct(v, p):
        return round(float(np.percentile(np.asarray(v), p)), 3)

    def per_request(reqs, sl, fp32):
        """One synchronous call per request in arrival order."""
        if fp32:
            pm.tune(pm.TUNE_FP32_PATH, 1)
        gc.collect()
        gc.disable()
        try:
            lat, last = [], 0.0
            start = time.perf_counter() + 0.05
            for i, (t_arr, _, k, c) in enumerate(reqs):
                while time.perf_counter() < start + t_arr:
                    time.sleep(0.0001)
                s_, e_ = sl[i]
                idx.ann(Q[s_:e_], k, c=c, confidence=conf, beta=beta)
                torch.cuda.synchronize()
                last = time.perf_counter()
                lat.append((last - (start + t_arr)) * 1e3)
            return lat, last - start
        finally:
            gc.enable()
            if fp32:
                pm.tune(pm.TUNE_FP32_PATH, -1)

    # throughput of the plain FP32 path, all at once on the first requests
    # of the 50,000 queries/s stream (about 20,000 queries)
    reqs = synth.requests(50_000, 50_000, 0.4)
    sl = slices(reqs)
    nq_fp = sum(e - s for s, e in sl)
    pm.tune(pm.TUNE_FP32_PATH, 1)
    try:
        idx.ann(Q[:64], 10, c=1.5, confidence=conf, beta=beta)
        torch.cuda.synchronize()
        t_0 = time.perf_counter()
        for (s_, e_), (_, _, k, c) in zip(sl, reqs):
            idx.ann(Q[s_:e_], k, c=c, confidence=conf, beta=beta)
        torch.cuda.synchronize()
        fp32_qps = nq_fp / (time.perf_counter() - t_0)
    finally:
        pm.tune(pm.TUNE_FP32_PATH, -1)
    log(f"plain FP32 path: {fp32_qps:.0f} queries/s ({nq_fp} queries at once)")

    per_rate = []
    for rate in rates:
        reqs = synth.requests(int(rate), rate, duration_s)
        sl = slices(reqs)
        nq_tot = sum(e - s for s, e in sl)
        # server
        srv = pm.Server(idx, max_batch=1024, max_inflight=2)
        srv.submit(Q[:1024], 10, c=1.5, confidence=conf, beta=beta).wait()    # warm-up
        srv.close()
        srv = pm.Server(idx, max_batch=1024, max_inflight=2)
        handles = [None] * len(reqs)
        done_t = [0.0] * len(reqs)
        sub_t = [0.0] * len(reqs)
        # answers allocated before the stream starts; Python's collector off
        # while it runs (a collection pass stalls the submitting thread)
        outs = [(torch.empty((e_ - s_, r[2]), dtype=torch.int64, device=dev),
                 torch.empty((e_ - s_, r[2]), dtype=torch.float32, device=dev))
                for (s_, e_), r in zip(sl, reqs)]
        torch.cuda.synchronize()
        gc.collect()
        gc.disable()
        start = time.perf_counter() + 0.05

        def submitter():
            for i, (t_arr, _, k, c) in enumerate(reqs):
                while time.perf_counter() < start + t_arr:
                    time.sleep(0.0001)
                s_, e_ = sl[i]
                sub_t[i] = time.perf_counter()
                handles[i] = srv.submit(Q[s_:e_], k, c=c, confidence=conf, beta=beta,
                                        out=outs[i])

        try:
            th = threading.Thread(target=submitter)
            th.start()
            for i in range(len(reqs)):
                while handles[i] is None:
                    time.sleep(0.0001)
                handles[i].wait()
                done_t[i] = time.perf_counter()
            th.join()
        finally:
            gc.enable()
        st = srv.stats()
        srv.close()
        lat_srv = [(done_t[i] - (start + reqs[i][0])) * 1e3 for i in range(len(reqs))]
        lag = [(sub_t[i] - (start + reqs[i][0])) * 1e3 for i in range(len(reqs))]
        wall_srv = max(done_t) - start
        row = {"offered_qps": rate, "requests": len(reqs), "queries": nq_tot,
               "server": {"qps": round(nq_tot / wall_srv, 1), "p50_ms": pct(lat_srv, 50),
                          "p99_ms": pct(lat_srv, 99), "launches": int(st["launches"]),
                          "submit_to_done_p99_ms": round(float(st["latency_p99_ms"]), 3),
                          "submit_to_done_max_ms": round(float(st["latency_max_ms"]), 3),
                          "submit_lag_max_ms": round(max(lag), 3)}}
        slow = sorted(range(len(reqs)), key=lambda i: -lat_srv[i])[:3]
        log("  slowest server requests (index, arrival ms, size, k, c, latency ms, "
            "submit lag ms): "
            + str([(i, round(reqs[i][0] * 1e3, 2), reqs[i][1], reqs[i][2], reqs[i][3],
                    round(lat_srv[i], 2), round(lag[i], 2)) for i in slow]))
        # the plain FP32 path where it can keep up (offered rate below its
        # throughput), and per-request calls of the batched path
        if rate < 0.8 * fp32_qps:
            lat_pl, wall_pl = per_request(reqs, sl, True)
            row["plain_fp32"] = {"qps": round(nq_tot / wall_pl, 1), "p50_ms": pct(lat_pl, 50),
                                 "p99_ms": pct(lat_pl, 99)}
        else:
            row["plain_fp32"] = {"sustained": False,
                                 "note": f"offered rate above its throughput ({fp32_qps:.0f}/s)"}
        lat_pr, wall_pr = per_request(reqs, sl, False)
        row["per_request_batched"] = {"qps": round(nq_tot / wall_pr, 1),
                                      "p50_ms": pct(lat_pr, 50), "p99_ms": pct(lat_pr, 99)}
        log(f"serving at {rate} queries/s offered: {row}")
        per_rate.append(row)
    # saturation: every request of the heaviest stream submitted at once
    reqs = synth.requests(int(rates[-1]) + 1, rates[-1], duration_s)
    sl = slices(reqs)
    nq_tot = sum(e - s for s, e in sl)
    srv = pm.Server(idx, max_batch=1024, max_inflight=2)
    torch.cuda.synchronize()
    t_0 = time.perf_counter()
    hs = [srv.submit(Q[s_:e_], k, c=c, confidence=conf, beta=beta)
          for (s_, e_), (_, _, k, c) in zip(sl, reqs)]
    for h in hs:
        h.wait()
    sat_srv = nq_tot / (time.perf_counter() - t_0)
    srv.close()
    torch.cuda.synchronize()
    t_0 = time.perf_counter()
    for (s_, e_), (_, _, k, c) in zip(sl, reqs):
        idx.ann(Q[s_:e_], k, c=c, confidence=conf, beta=beta)
    torch.cuda.synchronize()
    sat_pl = nq_tot / (time.perf_counter() - t_0)
    log(f"saturation: server {sat_srv:.0f} queries/s, per-request batched {sat_pl:.0f} "
        f"queries/s, plain FP32 {fp32_qps:.0f} queries/s")
    # recall@k and overall ratio (Eqs. 12-14) of the server's answers on a
    # sample of the heaviest stream, against exact kNN
    rec, rat = [], []
    samp = list(range(0, len(hs), max(1, len(hs) // 32)))
    qrows, krow = [], []
    for i in samp:
        s_, e_ = sl[i]
        for j in range(0, e_ - s_, max(1, (e_ - s_) // 4)):
            qrows.append((i, j))
    Qx = torch.stack([Q[sl[i][0] + j] for i, j in qrows])
    x_ids, x_dist = exact_knn_gpu32(torch, D, Qx, 100)
    x_ids, x_dist = x_ids.cpu().numpy(), x_dist.cpu().numpy()
    Dd = None
    for r_, (i, j) in enumerate(qrows):
        ids, _ = hs[i].wait()
        k = reqs[i][2]
        got = ids[j].cpu()
        rec.append(len(set(got.tolist()) & set(x_ids[r_, :k].tolist())) / k)
        gd = ((D[got.to(dev)].double() - Q[sl[i][0] + j].double()) ** 2).sum(1).sqrt().cpu().numpy()
        ex = x_dist[r_, :k]
        rat.append(float(np.mean(np.where(ex > 0, gd / np.where(ex > 0, ex, 1.0), 1.0))))
    del Dd
    return {"workload": "10,000,000 x 128 FP16 values in [0, 255], 10,000 centres, sigma U[4, 16]; "
                        "Poisson requests of 1..4,096 queries, k in {1,10,50,100}, "
                        "c in {1.2,1.5,2.0}",
            "beta": beta, "beta_sweep": beta_sweep, "build_s": round(build_s, 1),
            "per_rate": per_rate,
            "saturation_qps": {"server": round(sat_srv, 1), "per_request_batched": round(sat_pl, 1),
                               "plain_fp32": round(fp32_qps, 1)},
            "recall_sampled": round(float(np.mean(rec)), 4),
            "overall_ratio_sampled": round(float(np.mean(rat)), 6), "recall_samples": len(rec)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--beta", type=float, default=None, help="skip the sweep")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-truth", action="store_true",
                    help="skip ground truth and recall (needs --beta; for profiler runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after timing, run a plain 256 MiB device copy (for counters)")
    ap.add_argument("--no-acp", action="store_true",
                    help="skip the (c,k)-ACP timing at 200,000 x 512")
    ap.add_argument("--streams", type=int, default=1,
                    help="HIP streams the batches are issued on, round-robin")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving-loop run on the 10,000,000 x 128 index")
    ap.add_argument("--no-ksweep", action="store_true",
                    help="skip the operating points for k = 1, 50, 100")
    ap.add_argument("--no-acp-variants", action="store_true",
                    help="skip the branch-and-bound and FindLCA ACP variants (profiler runs)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP16/BF16 filter-projection runs at the headline point")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip the 1,000,000 x 960 low-contrast sweep over c and beta")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                                   f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)

    import synth
    t0 = time.perf_counter()
    w = synth.headline()
    log(f"workload generated in {time.perf_counter() - t0:.1f} s")
    # the CPU-baseline workers are forked before anything touches the GPU
    cpu_workers = 16
    pool = None if args.no_cpu else start_cpu_pool(w, cpu_workers)

    import torch
    import paper_2107_05537_amd as pm

    pm.load_library()
    dev = torch.device("cuda", 0)
    D = torch.from_numpy(w["D"]).to(dev)
    A = torch.from_numpy(w["A"]).to(dev)
    Q = torch.from_numpy(w["Q"]).to(dev)
    n, d = D.shape
    nq = Q.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx = pm.Index(D, A)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log(f"index built in {build_s:.2f} s: {idx.info()}")

    if args.no_truth and args.beta is None:
        ap.error("--no-truth needs --beta")
    truth = None
    if not args.no_truth:
        t0 = time.perf_counter()
        truth_all, truth_dist = exact_knn_gpu(torch, D, Q, 10 if args.no_ksweep else max(KS))
        truth = truth_all[:, :K]
        torch.cuda.synchronize()
        log(f"ground truth in {time.perf_counter() - t0:.1f} s")

    batches = [(s, min(nq, s + BATCH)) for s in range(0, nq, BATCH)]
    ids = torch.empty((nq, K), dtype=torch.int64, device=dev)
    dist = torch.empty((nq, K), dtype=torch.float32, device=dev)
    stats = torch.empty((nq, 4), dtype=torch.int32, device=dev)

    def run_all(beta):
        for s, e in batches:
            idx.ann_into(Q[s:e], K, C, CONF, beta, 0.0, ids[s:e], dist[s:e], stats[s:e])
        torch.cuda.synchronize()

    sweep = []
    betas = BETAS if args.beta is None else [args.beta]
    chosen = None
    for beta in betas:
        run_all(beta)
        if truth is None:
            chosen = beta
            break
        rec = recall_at_k(ids, truth)
        sweep.append({"beta": beta, "recall@10": round(rec, 4)})
        log(f"beta={beta:g} recall@10={rec:.4f} exits={np.bincount(stats[:, 2].cpu().numpy(), minlength=3).tolist()}")
        if rec >= 0.9 and chosen is None:
            chosen = beta
            break
    if chosen is None:
        chosen = betas[-1]
    beta = chosen
    plan = pm.plan_params(n, A.shape[0], K, C, CONF, beta)
    B = plan["budget"]
    r_min = idx.default_r_min(B)

    # recall, overall ratio and the per-query work at the operating point
    run_all(beta)
    rec = recall_at_k(ids, truth) if truth is not None else None
    ratio = overall_ratio(torch, D, Q, ids, truth_dist) if truth is not None else None
    st = stats.cpu().numpy().astype(np.int64)
    batch_scan = [float(st[s:e, 3].sum()) for s, e in batches]
    batch_cand = [float(st[s:e, 1].sum()) for s, e in batches]

    # warm-up, with every stage timed once to find the dominant one; the
    # timed region then records events around that stage only
    pm.ann_timing_read(reset=True)
    pm.ann_timing_enable(True)
    for i in range(args.warmup):
        s, e = batches[i % len(batches)]
        idx.ann_into(Q[s:e], K, C, CONF, beta, r_min, ids[s:e], dist[s:e], stats[s:e])
    torch.cuda.synchronize()
    pm.ann_timing_enable(False)
    warm = pm.ann_timing_read(reset=True)
    dom = max(("dist", "tau", "filter", "finish", "per_query"), key=lambda k: warm[k]["ms"])
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream()
                                               for _ in range(max(1, args.streams) - 1)]

    def timed(k, beta_k, rmin_k, steps, out_ids, out_dist, out_stats, probe=None):
        """Wall time of `steps` batches issued round-robin on the streams.
        With probe = (stage, every), that stage of every `every`-th batch is
        bracketed by the library's HIP events (events on every batch would
        hold back the overlap of the streams)."""
        torch.cuda.synchronize()
        t_0 = time.perf_counter()
        nq_done = 0
        for i in range(steps):
            s_, e_ = batches[i % len(batches)]
            on = probe is not None and i % probe[1] == 0
            if on:
                pm.ann_timing_enable(True, stages=[probe[0]])
            with torch.cuda.stream(streams[i % len(streams)]):
                idx.ann_into(Q[s_:e_], k, C, CONF, beta_k, rmin_k, out_ids[s_:e_],
                             out_dist[s_:e_], out_stats[s_:e_])
            if on:
                pm.ann_timing_enable(False)
            nq_done += e_ - s_
        torch.cuda.synchronize()
        return time.perf_counter() - t_0, nq_done

    # queries of the timed steps; work of the probed ones (the launches whose
    # dominant stage is timed)
    queries = 0
    p_queries, scan_pts, cand_rows = 0, 0.0, 0.0
    for i in range(args.steps):
        b = i % len(batches)
        queries += batches[b][1] - batches[b][0]
        if i % PROBE_EVERY == 0:
            p_queries += batches[b][1] - batches[b][0]
            scan_pts += batch_scan[b]
            cand_rows += batch_cand[b]
    pm.ann_timing_read(reset=True)
    wall, _ = timed(K, beta, r_min, args.steps, ids, dist, stats, probe=(dom, PROBE_EVERY))
    stages = pm.ann_timing_read(reset=True)
    value = queries / wall

    # latency of one batch, alone on one stream (outside the timed region)
    lat = []
    for i in range(min(args.steps, 40)):
        s, e = batches[i % len(batches)]
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        idx.ann_into(Q[s:e], K, C, CONF, beta, r_min, ids[s:e], dist[s:e], stats[s:e])
        ev1.record()
        ev1.synchronize()
        lat.append(ev0.elapsed_time(ev1))
    lat = np.array(lat)

    # roofline of the dominant stage, from its live per-launch duration.
    # `achieved` follows the per-query algorithmic work of Section 8(d):
    #   bytes(q) = 4d + 64 N_scan + 116 N_node + 8 N_ball + (4d + 8) |C| + 12k
    # of which the finishing kernel (budget cut, verification, top-k) moves
    # 8 N_ball + (4d + 8) |C| + 4d + 12k (N_ball >= |C|: |C| is used, a lower
    # bound, as the pool size is not reported per query), the filter 64 N_scan
    # bytes, the chunk-distance stages the bf16 distance row. The finishing
    # kernel reads FP16 rows where the verification allows it, so its own
    # byte model is reported beside it ("fp16_rows").
    d_pad = (d + 3) // 4 * 4
    d16 = (d + 7) // 8 * 8
    launches = max(1, stages[dom]["launches"])
    per_launch_ms = stages[dom]["ms"] / launches
    q_l = p_queries / launches                       # queries per probed launch
    c_l = cand_rows / launches                       # members of C per launch
    s_l = scan_pts / launches                        # points scanned per launch

    def rate(work, unit):
        return work / (per_launch_ms * 1e-3) / (1e9 if unit == "GB/s" else 1e12)

    models = {}
    if dom == "filter":
        work = 64.0 * s_l
        models["mfma_flops"] = {"work": 32.0 * s_l, "unit": "TFLOP/s",
                                "peak": FP16_MFMA_PEAK_TFLOPS}
    elif dom in ("dist", "tau"):
        ldc = ((n + 63) // 64 + 15) // 16 * 16
        work = 2.0 * ldc * q_l
    else:
        work = (8.0 * c_l + (4.0 * d + 8.0) * c_l + (4.0 * d + 12.0 * K) * q_l)
        models["fp16_rows"] = {"work": (2.0 * d16 + 64.0) * c_l
                               + (4.0 * d_pad * K + 4 * d + 12 * K) * q_l,
                               "unit": "GB/s", "peak": HBM_PEAK_GBS}
    achieved = rate(work, "GB/s")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "model": "Section 8(d) algorithmic bytes"}
    for m_ in models.values():
        m_["achieved"] = round(rate(m_["work"], m_["unit"]), 2)
        m_["frac"] = round(m_["achieved"] / m_["peak"], 4)
    roof["other_models"] = models
    roof["kernel"] = {"dist": "dist_kernel", "tau": "tau_kernel", "filter": "scan_kernel",
                      "finish": "finish_kernel", "per_query": "ann_kernel"}[dom]
    roof["per_launch_ms"] = round(per_launch_ms, 4)
    roof["work_per_launch"] = work
    roof["queries_per_launch"] = q_l

    # the whole step under the same model (every query of a batch tests all
    # n/64 chunk balls in the chunk-distance pass: N_node = n/64 per query)
    n_chunk = (n + 63) // 64
    nq_all = st.shape[0]
    wq = {"N_scan": float(st[:, 3].mean()), "C": float(st[:, 1].mean()),
          "N_ball_lower_bound": float(st[:, 1].mean()), "N_node": n_chunk,
          "rounds": float(st[:, 0].mean()),
          "exit_kinds": np.bincount(st[:, 2], minlength=3)[1:].tolist()}
    terms = {"query": 4.0 * d, "scan": 64.0 * wq["N_scan"], "nodes": 116.0 * n_chunk,
             "ball": 8.0 * wq["C"], "verify": (4.0 * d + 8.0) * wq["C"], "out": 12.0 * K}
    wq["bytes_8d"] = {k_: round(v_, 1) for k_, v_ in terms.items()}
    wq["bytes_8d_total"] = round(sum(terms.values()), 1)
    wq["step_gbs_8d"] = round(sum(terms.values()) * queries / wall / 1e9, 1)
    wq["step_gbs_8d_without_nodes"] = round((sum(terms.values()) - terms["nodes"]) * queries
                                            / wall / 1e9, 1)
    log(f"work per query: {wq}")

    traffic = pmc_traffic(roof["kernel"], "kernel_source_sha",
                          ("ann.hip", "project.hip", "internal.hpp"))
    with open(PMC_FILE) as fh:
        if json.load(fh).get("beta") != beta:
            traffic = None
    roof["traffic"] = traffic
    with_copy_context(roof, copy_rate_gbs(torch, dev))

    if args.calib_copy:
        x = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev).uniform_()
        for _ in range(3):
            y = x.clone()
        torch.cuda.synchronize()
        del x, y

    # operating points for the other k of the workload: smallest beta with
    # recall@k >= 0.9, then the same timed loop
    ksweep = []
    if truth is not None and not args.no_ksweep:
        for k in KS:
            if k == K:
                continue
            ids_k = torch.empty((nq, k), dtype=torch.int64, device=dev)
            dist_k = torch.empty((nq, k), dtype=torch.float32, device=dev)
            b_k, rec_k = None, None
            for bt in BETAS:
                for s_, e_ in batches:
                    idx.ann_into(Q[s_:e_], k, C, CONF, bt, 0.0, ids_k[s_:e_], dist_k[s_:e_],
                                 stats[s_:e_])
                torch.cuda.synchronize()
                rec_k = recall_at_k(ids_k, truth_all[:, :k])
                if rec_k >= 0.9:
                    b_k = bt
                    break
            if b_k is None:
                b_k = BETAS[-1]
            B_k = pm.plan_params(n, A.shape[0], k, C, CONF, b_k)["budget"]
            rmin_k = idx.default_r_min(B_k)
            timed(k, b_k, rmin_k, 10, ids_k, dist_k, stats)          # warm-up
            wall_k, q_k = timed(k, b_k, rmin_k, args.steps, ids_k, dist_k, stats)
            log(f"k={k}: beta={b_k:g} recall@{k}={rec_k:.4f} {q_k / wall_k:.0f} queries/s")
            ratio_k = overall_ratio(torch, D, Q, ids_k, truth_dist[:, :k])
            ksweep.append({"k": k, "beta": b_k, "budget_B": B_k, f"recall@{k}": round(rec_k, 4),
                           "overall_ratio": round(ratio_k, 6),
                           "queries_per_s": round(q_k / wall_k, 1)})

    # mixed-precision filter projection at the same operating point: FP16 and
    # BF16 matrix-core projections behind the filter rows, radius widened by
    # their bound; answers must equal the exact index's
    mixed = []
    if not args.no_mixed:
        for name, mode in (("fp16", pm.FILTER_GEMM_FP16), ("bf16", pm.FILTER_GEMM_BF16)):
            idx_m = pm.Index(D, A, filter_gemm=mode)
            ids_m = torch.empty_like(ids)
            dist_m = torch.empty_like(dist)
            for s_, e_ in batches:
                idx_m.ann_into(Q[s_:e_], K, C, CONF, beta, r_min, ids_m[s_:e_], dist_m[s_:e_],
                               stats[s_:e_])
            torch.cuda.synchronize()
            same = bool(torch.equal(ids_m, ids) and torch.equal(dist_m, dist))
            pm.ann_timing_read(reset=True)
            pm.ann_timing_enable(True)
            for i in range(min(args.steps, 20)):
                s_, e_ = batches[i % len(batches)]
                idx_m.ann_into(Q[s_:e_], K, C, CONF, beta, r_min, ids_m[s_:e_], dist_m[s_:e_],
                               stats[s_:e_])
            torch.cuda.synchronize()
            pm.ann_timing_enable(False)
            tm_m = pm.ann_timing_read(reset=True)
            torch.cuda.synchronize()
            t_0 = time.perf_counter()
            q_m = 0
            for i in range(args.steps):
                s_, e_ = batches[i % len(batches)]
                idx_m.ann_into(Q[s_:e_], K, C, CONF, beta, r_min, ids_m[s_:e_], dist_m[s_:e_],
                               stats[s_:e_])
                q_m += e_ - s_
            torch.cuda.synchronize()
            qps_m = q_m / (time.perf_counter() - t_0)
            info_m = idx_m.info()
            row = {"filter_gemm": name, "eps_max": round(float(info_m["eps_max"]), 5),
                   "queries_per_s": round(qps_m, 1), "answers_equal_exact_index": same,
                   "stages_ms_per_batch": {k: round(v["ms"] / max(1, v["launches"]), 4)
                                           for k, v in tm_m.items()
                                           if v["launches"] and not k.startswith("acp")}}
            log(f"mixed precision: {row}")
            mixed.append(row)
            del idx_m
            torch.cuda.empty_cache()

    cpu = None
    if pool is not None:
        cpu = cpu_baseline(pool, cpu_workers, n, beta, r_min)
        pool.close()
        pool.join()
        log(f"cpu baseline: {cpu}")
    acp = None
    serving = None
    config3 = None
    if not (args.no_acp and args.no_serving and args.no_config3):
        del idx
        torch.cuda.empty_cache()
    if not args.no_config3:
        config3 = config3_bench(pm, torch, dev)
        torch.cuda.empty_cache()
    if not args.no_acp:
        acp = acp_bench(pm, torch, dev, with_variants=not args.no_acp_variants)
        torch.cuda.empty_cache()
    if not args.no_serving:
        serving = serving_bench(pm, torch, dev)

    out = {
        "metric": "c-ANN queries/s at recall@10>=0.9 (1M x 256)",
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(float(wall * 1e3 / args.steps), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "gaussian-mixture 1,000,000 x 256, 1,000 centres, "
                               "10,000 queries in batches of 1,024",
                   "k": K, "c": C, "confidence": round(CONF, 6), "m": 15,
                   "beta": beta, "budget_B": B, "r_min": r_min,
                   "batch": BATCH, "streams": len(streams), "parallelism": "single GPU"},
        "recall@10": round(rec, 4) if rec is not None else None,
        "overall_ratio": round(ratio, 6) if ratio is not None else None,
        "work_per_query": wq,
        "sweep": sweep,
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4),
                       "per": "batch of up to 1,024 queries, alone on one stream"},
        "other_k": ksweep,
        "mixed_precision": mixed,
        "roofline": roof,
        "stages_ms_per_batch": {k: round(v["ms"] / max(1, v["launches"]), 4)
                                for k, v in warm.items() if not k.startswith("acp")},
        "build_s": round(build_s, 2),
        "cpu_baseline": cpu,
        "acp": acp,
        "serving": serving,
        "config3": config3,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
