// extern "C" boundary of the PM-LSH library: argument validation (before any
// HIP call), error codes, the thread-local error message, and the host-side
// orchestration of the ANN batches.

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace pmlsh {

pmlsh_index* index_build(const pmlsh_build_args* a);
void index_release(pmlsh_index* x);
double index_default_r_min(const pmlsh_index* x, int64_t budget);
void run_acp(const pmlsh_index* x, int k, double c, double confidence, double beta,
             int64_t* out_pairs, float* out_dist, pmlsh_acp_stats* stats,
             hipStream_t stream);
void run_acp_bb(const pmlsh_index* x, int k, double c, double confidence, double beta,
                int64_t* out_pairs, float* out_dist, pmlsh_acp_stats* stats,
                hipStream_t stream);
void run_acp_lca(const pmlsh_index* x, int k, double c, double confidence, double beta,
                 double gamma, int64_t* out_pairs, float* out_dist, pmlsh_acp_stats* stats,
                 double* gamma_used, hipStream_t st);
void export_nodes(const pmlsh_index* x, int32_t* level, int32_t* first_leaf, int32_t* end_leaf,
                  float* radius);

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }
const char* error_cstr() { return g_error.c_str(); }
[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

// Per-query workspace bytes of the ANN kernel and the batch that fits a cap.
constexpr int64_t kWorkspaceCap = int64_t(4) << 30;

namespace {

// Workspace layout sizes of one ANN call: per query: projection, FP16 scan
// row, C, top-k scratch, and for the batched path three counters, a
// candidate region and the lower distance bounds of C; plus, for the batched
// path, the chunk distances, chosen chunks and the chunk x query mask (a
// 64-bit word per chunk and 64 queries, both layouts); plus the frontier
// lists of the per-query kernel's workgroups.
struct AnnWorkspace {
    int64_t B, pool_q, per_query, nchunk, batch, slots, bytes;
    bool fast;
};

// Workgroups of the per-query kernel, each with its own pair of frontier
// lists: few on the batched path (only the queries it hands over), more
// when every query takes the per-query path.
int64_t front_slots(const pmlsh_index* x, bool fast, int64_t batch) {
    const int64_t by_memory = std::max<int64_t>(1, (int64_t(1) << 30) / (8 * x->n_leaves));
    return std::min<int64_t>({batch, fast ? 256 : 2048, by_memory});
}

// Bytes of the workspace layout for batches of `batch` queries and `slots`
// frontier-list pairs (unrounded).
int64_t ann_layout_bytes(const pmlsh_index* x, const AnnWorkspace& w, int64_t batch,
                         int64_t slots) {
    const int64_t mask_bytes =
        w.fast ? batch * 8 + 2 * cdist_elems(batch, w.nchunk) +
                     (w.nchunk + 255) / 256 * 256 * ((batch + 63) / 64) * 8 + 64
               : 0;
    return batch * w.per_query + mask_bytes + slots * 2 * x->n_leaves * 4;
}

AnnWorkspace ann_workspace_base(const pmlsh_index* x, int k, int64_t B) {
    AnnWorkspace w{};
    w.B = B;
    // the batched path, unless the budget exceeds its limit or the plain
    // FP32 path is switched on (read once per call: layout and launch agree)
    w.fast = ann_fast_path(B) && tune_get(PMLSH_TUNE_FP32_PATH) == 0;
    w.pool_q = w.fast ? ann_pool_per_query(x->n) : 0;
    w.per_query = (int64_t)MP * 8 + 64 + B * 8 + 3 * (int64_t)k * 4 +
                  (w.fast ? 4 * 4 + w.pool_q * 4 + B * 4 : 0) +
                  (w.fast && x->filter_gemm ? (MP + 1) * 4 : 0);
    w.nchunk = x->n_pad16 / 64;
    return w;
}

AnnWorkspace ann_workspace(const pmlsh_index* x, int64_t nq, int k, int64_t B) {
    AnnWorkspace w = ann_workspace_base(x, k, B);
    // per query, with the distance blocks of a 64-query band spread over it
    const int64_t per_query_all =
        w.per_query + (w.fast ? 8 + 2 * (64 * cdist_groups(w.nchunk) + cdist_gmin_len(w.nchunk)) +
                                    (w.nchunk + 7) / 8
                              : 0);
    w.batch = std::max<int64_t>(1, std::min<int64_t>(nq, kWorkspaceCap / per_query_all));
    w.batch = std::min<int64_t>(w.batch, 65535);
    w.slots = front_slots(x, w.fast, w.batch);
    w.bytes = ann_layout_bytes(x, w, w.batch, w.slots);
    // sizes rounded up (to 1 MiB, or 64 MiB above 256 MiB) so that calls of
    // different batch sizes reuse the same pool blocks
    const int64_t q = w.bytes > (int64_t(256) << 20) ? int64_t(64) << 20 : int64_t(1) << 20;
    w.bytes = (w.bytes + q - 1) / q * q;
    return w;
}

// Layout that fits a fixed region of cap bytes: at most a quarter of it for
// the frontier lists, the largest batch that fits in the rest. batch = 0
// when not even one query fits.
AnnWorkspace ann_workspace_in(const pmlsh_index* x, int64_t nq, int k, int64_t B, int64_t cap) {
    AnnWorkspace w = ann_workspace_base(x, k, B);
    const int64_t per_slot = 2 * x->n_leaves * 4;
    int64_t slots = std::min<int64_t>(w.fast ? 256 : 2048, (cap / 4) / per_slot);
    slots = std::max<int64_t>(slots, 1);
    int64_t lo = 0, hi = std::min<int64_t>(nq, 65535);
    while (lo < hi) {   // largest batch with bytes <= cap
        const int64_t mid = (lo + hi + 1) / 2;
        if (ann_layout_bytes(x, w, mid, std::min(slots, mid)) <= cap) lo = mid;
        else hi = mid - 1;
    }
    w.batch = lo;
    w.slots = std::min(slots, std::max<int64_t>(lo, 1));
    w.bytes = lo > 0 ? ann_layout_bytes(x, w, w.batch, w.slots) : 0;
    return w;
}

}  // namespace

void validate_ann(const pmlsh_index* index, const float* queries, int64_t nq, int k,
                  const int64_t* out_ids, const float* out_dist, double r_min) {
    if (!index) fail(PMLSH_EINVAL, "index is NULL");
    if (nq < 0) fail(PMLSH_EINVAL, "nq must be >= 0");
    if (nq > 0 && (!queries || !out_ids || !out_dist))
        fail(PMLSH_EINVAL, "queries and outputs must not be NULL");
    if (k < 1) fail(PMLSH_EINVAL, "k must be >= 1");
    if (k > index->n) fail(PMLSH_EINVAL, "k must be <= n");
    if (k > PMLSH_MAX_K) fail(PMLSH_EUNSUPPORTED, "k above PMLSH_MAX_K");
    if (index->d_pad > 8192) fail(PMLSH_EUNSUPPORTED, "ANN supports d <= 8192");
    if (std::isnan(r_min)) fail(PMLSH_EINVAL, "r_min is NaN");
}

int64_t ann_workspace_bytes(const pmlsh_index* x, int64_t nq, int k, double c,
                            double confidence, double beta) {
    pmlsh_plan plan;
    plan_params(x->n, x->m, k, c, confidence, beta, &plan);
    return nq > 0 ? ann_workspace(x, nq, k, plan.budget).bytes : 0;
}

namespace {

// Parameters of one ANN call: the same for every query, or per query from
// the device array qpar (then k and budget are the largest of the call).
struct AnnCall {
    int k;
    int64_t budget;
    double c, t, r_min;
    const AnnQueryParams* qpar;
    int out_stride;
    int max_rounds;
};

// The batches of one ANN call over the workspace region ws laid out by w.
void run_ann_region(const pmlsh_index* x, const float* queries, int64_t nq, const AnnCall& call,
                    int64_t* out_ids, float* out_dist, int32_t* out_stats, hipStream_t st,
                    const AnnWorkspace& w, void* ws) {
    const int k = call.k;
    const int stride = call.out_stride > 0 ? call.out_stride : k;
    const int64_t B = w.B, pool_q = w.pool_q, nchunk = w.nchunk, batch = w.batch;
    const bool fast = w.fast;
    char* base = static_cast<char*>(ws);
    // projections and FP16 scan rows first: every row starts on a 64-byte
    // boundary
    float* qproj = reinterpret_cast<float*>(base);
    float* qproj_lo = qproj + batch * MP;
    uint16_t* qaug = reinterpret_cast<uint16_t*>(qproj_lo + batch * MP);
    uint16_t* cdist2 = qaug + batch * 32;
    uint16_t* cgmin = cdist2 + (fast ? cdist_block_elems(batch, nchunk) : 0);
    float2* qtest = reinterpret_cast<float2*>(cdist2 + (fast ? cdist_elems(batch, nchunk) : 0));
    uint64_t* cmask = reinterpret_cast<uint64_t*>(qtest + (fast ? batch : 0));
    uint32_t* list = reinterpret_cast<uint32_t*>(
        cmask + (fast ? (nchunk + 255) / 256 * 256 * ((batch + 63) / 64) : 0));
    int32_t* front = reinterpret_cast<int32_t*>(list + batch * pool_q);
    int32_t* cpos = front + w.slots * 2 * x->n_leaves;
    float* cdist = reinterpret_cast<float*>(cpos + batch * B);
    int32_t* topk = reinterpret_cast<int32_t*>(cdist + batch * B);
    float* clo = reinterpret_cast<float*>(topk + batch * 3 * (int64_t)k);
    int32_t* q_flag = reinterpret_cast<int32_t*>(clo + (fast ? batch * B : 0));
    uint32_t* l_count = reinterpret_cast<uint32_t*>(q_flag + batch);
    uint32_t* q_scanned = l_count + batch;
    // count, then the queries the batched path hands to the per-query kernel
    uint32_t* pq_list = q_scanned + batch;
    // low-precision query projections and their bounds (filter_gemm)
    float* qlp = reinterpret_cast<float*>(pq_list + batch + 1);
    float* qeps = qlp + batch * MP;
    const bool lp = fast && x->filter_gemm != 0;
    for (int64_t q0 = 0; q0 < nq; q0 += batch) {
        const int64_t nb = std::min(batch, nq - q0);
        const float* qb = queries + q0 * x->d;
        {
            StageTimer tm(PMLSH_STAGE_PROJECT, st);
            launch_project(qb, nb, x->d, x->d, x->hash, qproj, qproj_lo, st);
            if (lp) launch_project_lp(qb, nb, x->d, x->d, x->hash, x->filter_gemm, qlp, qeps, st);
        }
        AnnLaunch L{};
        L.idx = x;
        L.queries = qb;
        L.qproj = qproj;
        L.qproj_lo = qproj_lo;
        L.nq = nb;
        L.k = k;
        L.c = call.c;
        L.t = call.t;
        L.r_min = call.r_min;
        L.max_rounds = call.max_rounds;
        L.budget = B;
        L.qpar = call.qpar ? call.qpar + q0 : nullptr;
        L.out_stride = stride;
        L.fast = fast;
        L.ws_front = front;
        L.front_slots = std::min<int64_t>(w.slots, nb);
        L.ws_cpos = cpos;
        L.ws_cdist = cdist;
        L.ws_topk = topk;
        if (fast) {
            L.ws_qaug = qaug;
            L.ws_qtest = qtest;
            L.ws_clo = clo;
            L.ws_cmask = cmask;
            L.ws_cdist2 = cdist2;
            L.ws_cgmin = cgmin;
            L.q_flag = q_flag;
            L.l_count = l_count;
            L.q_scanned = q_scanned;
            L.pq_list = pq_list;
            L.ws_qlp = lp ? qlp : nullptr;
            L.ws_qeps = lp ? qeps : nullptr;
            L.l_list = list;
            L.pool_cap = pool_q;
        }
        L.out_ids = out_ids + q0 * stride;
        L.out_dist = out_dist + q0 * stride;
        L.out_stats = out_stats ? out_stats + q0 * 4 : nullptr;
        launch_ann(L, st);
    }
}

// Plan and first radius of one ANN call (host only).
double ann_plan(const pmlsh_index* x, int k, double c, double confidence, double beta,
                double r_min, pmlsh_plan* plan) {
    plan_params(x->n, x->m, k, c, confidence, beta, plan);
    if (!(r_min > 0.0)) r_min = index_default_r_min(x, plan->budget);
    if (!std::isfinite(r_min)) fail(PMLSH_EINVAL, "r_min must be finite");
    return r_min;
}

}  // namespace

void run_ann(const pmlsh_index* x, const float* queries, int64_t nq, int k, double c,
             double confidence, double beta, double r_min, int64_t* out_ids,
             float* out_dist, int32_t* out_stats, hipStream_t st, int max_rounds) {
    pmlsh_plan plan;
    r_min = ann_plan(x, k, c, confidence, beta, r_min, &plan);
    if (nq == 0) return;
    const AnnWorkspace w = ann_workspace(x, nq, k, plan.budget);
    const AnnCall call{k, plan.budget, c, plan.t, r_min, nullptr, k, max_rounds};
    void* ws = ws_alloc((size_t)w.bytes, st);
    try {
        run_ann_region(x, queries, nq, call, out_ids, out_dist, out_stats, st, w, ws);
    } catch (...) {
        ws_free(ws, st);
        throw;
    }
    ws_free(ws, st);
}

void run_ann_in(const pmlsh_index* x, const float* queries, int64_t nq, int k, double c,
                double confidence, double beta, double r_min, int64_t* out_ids,
                float* out_dist, int32_t* out_stats, hipStream_t st,
                const std::function<void*()>& region_of_device, int64_t region_bytes) {
    pmlsh_plan plan;
    r_min = ann_plan(x, k, c, confidence, beta, r_min, &plan);
    if (nq == 0) return;
    const AnnWorkspace w = ann_workspace_in(x, nq, k, plan.budget, region_bytes);
    if (w.batch < 1) {
        const AnnWorkspace one = ann_workspace_in(x, 1, k, plan.budget, int64_t(1) << 62);
        fail(PMLSH_EUNSUPPORTED,
             "one query of this index needs " + std::to_string(one.bytes) +
                 " bytes of workspace; the fixed region holds " + std::to_string(region_bytes));
    }
    const AnnCall call{k, plan.budget, c, plan.t, r_min, nullptr, k, 0};
    run_ann_region(x, queries, nq, call, out_ids, out_dist, out_stats, st, w, region_of_device());
}

void plan_queries(const pmlsh_index* x, const pmlsh_query_args* args, int64_t nq,
                  std::vector<AnnQueryParams>* out, int* kmax, int64_t* bmax) {
    out->resize((size_t)nq);
    *kmax = 1;
    *bmax = 1;
    for (int64_t i = 0; i < nq; ++i) {
        const pmlsh_query_args& q = args[i];
        try {
            validate_ann(x, nullptr, 0, q.k, nullptr, nullptr, q.r_min);
            pmlsh_plan plan;
            plan_params(x->n, x->m, q.k, q.c, q.confidence, q.beta, &plan);
            double r_min = q.r_min;
            if (!(r_min > 0.0)) r_min = index_default_r_min(x, plan.budget);
            if (!std::isfinite(r_min)) fail(PMLSH_EINVAL, "r_min must be finite");
            AnnQueryParams& p = (*out)[(size_t)i];
            p.c = q.c;
            p.t = plan.t;
            p.r_min = r_min;
            p.k = q.k;
            p.budget = (int32_t)plan.budget;
            *kmax = std::max(*kmax, q.k);
            *bmax = std::max<int64_t>(*bmax, plan.budget);
        } catch (const Error& e) {
            fail(e.code, "query " + std::to_string(i) + ": " + e.msg);
        }
    }
}

void run_ann_planned(const pmlsh_index* x, const float* queries, int64_t nq,
                     const AnnQueryParams& p, int64_t* out_ids, float* out_dist, hipStream_t st,
                     void* region, int64_t region_bytes) {
    if (nq == 0) return;
    const AnnWorkspace w = ann_workspace_in(x, nq, p.k, p.budget, region_bytes);
    if (w.batch < 1) fail(PMLSH_ENOMEM, "the workspace region holds no query");
    const AnnCall call{p.k, p.budget, p.c, p.t, p.r_min, nullptr, p.k, 0};
    run_ann_region(x, queries, nq, call, out_ids, out_dist, nullptr, st, w, region);
}

int64_t ann_workspace_bytes_mixed(const pmlsh_index* x, int64_t nq, int kmax, int64_t bmax) {
    return nq > 0 ? ann_workspace(x, nq, kmax, bmax).bytes : 0;
}

void run_ann_mixed(const pmlsh_index* x, const float* queries, int64_t nq,
                   const AnnQueryParams* qpar, int kmax, int64_t bmax, int out_stride,
                   int64_t* out_ids, float* out_dist, int32_t* out_stats, hipStream_t st,
                   void* region, int64_t region_bytes) {
    if (nq == 0) return;
    const AnnCall call{kmax, bmax, 0.0, 0.0, 0.0, qpar, out_stride, 0};
    if (region) {
        const AnnWorkspace w = ann_workspace_in(x, nq, kmax, bmax, region_bytes);
        if (w.batch < 1) fail(PMLSH_ENOMEM, "the workspace region holds no query");
        run_ann_region(x, queries, nq, call, out_ids, out_dist, out_stats, st, w, region);
        return;
    }
    const AnnWorkspace w = ann_workspace(x, nq, kmax, bmax);
    void* ws = ws_alloc((size_t)w.bytes, st);
    try {
        run_ann_region(x, queries, nq, call, out_ids, out_dist, out_stats, st, w, ws);
    } catch (...) {
        ws_free(ws, st);
        throw;
    }
    ws_free(ws, st);
}

}  // namespace pmlsh

using namespace pmlsh;

extern "C" {

int pmlsh_build(const pmlsh_build_args* args, pmlsh_index** out) {
    return guarded([&] {
        if (!out) fail(PMLSH_EINVAL, "out is NULL");
        *out = index_build(args);
    });
}

void pmlsh_free(pmlsh_index* index) { index_release(index); }

int pmlsh_plan_params(int64_t n, int32_t m, int32_t k, double c, double confidence,
                      double beta, pmlsh_plan* out) {
    return guarded([&] {
        if (!out) fail(PMLSH_EINVAL, "out is NULL");
        pmlsh_plan p;
        plan_params(n, m, k, c, confidence, beta, &p);
        *out = p;
    });
}

int pmlsh_default_r_min(const pmlsh_index* index, int64_t budget, double* r_min) {
    return guarded([&] {
        if (!index || !r_min) fail(PMLSH_EINVAL, "NULL argument");
        if (budget < 1) fail(PMLSH_EINVAL, "budget must be >= 1");
        *r_min = index_default_r_min(index, budget);
    });
}

int pmlsh_ann(const pmlsh_index* index, const float* queries, int64_t nq, int32_t k,
              double c, double confidence, double beta, double r_min, int64_t* out_ids,
              float* out_dist, int32_t* out_stats, void* stream) {
    return guarded([&] {
        validate_ann(index, queries, nq, k, out_ids, out_dist, r_min);
        run_ann(index, queries, nq, k, c, confidence, beta, r_min, out_ids, out_dist,
                out_stats, static_cast<hipStream_t>(stream));
    });
}

int pmlsh_ann_mixed(const pmlsh_index* index, const float* queries, int64_t nq,
                    const pmlsh_query_args* args, int32_t out_stride, int64_t* out_ids,
                    float* out_dist, int32_t* out_stats, void* stream) {
    return guarded([&] {
        if (!index) fail(PMLSH_EINVAL, "index is NULL");
        if (nq < 0) fail(PMLSH_EINVAL, "nq must be >= 0");
        if (nq == 0) return;
        if (!queries || !args || !out_ids || !out_dist)
            fail(PMLSH_EINVAL, "queries, args and outputs must not be NULL");
        std::vector<AnnQueryParams> params;
        int kmax = 1;
        int64_t bmax = 1;
        plan_queries(index, args, nq, &params, &kmax, &bmax);
        if (out_stride < kmax) fail(PMLSH_EINVAL, "out_stride must be >= every k");
        hipStream_t st = static_cast<hipStream_t>(stream);
        void* dp = ws_alloc(params.size() * sizeof(AnnQueryParams), st);
        try {
            PMLSH_HIP(hipMemcpyAsync(dp, params.data(), params.size() * sizeof(AnnQueryParams),
                                     hipMemcpyHostToDevice, st));
            // the host copy of the parameters lives until this call returns
            PMLSH_HIP(hipStreamSynchronize(st));
            run_ann_mixed(index, queries, nq, static_cast<const AnnQueryParams*>(dp), kmax, bmax,
                          out_stride, out_ids, out_dist, out_stats, st, nullptr, 0);
        } catch (...) {
            ws_free(dp, st);
            throw;
        }
        ws_free(dp, st);
    });
}

int pmlsh_bc(const pmlsh_index* index, const float* queries, int64_t nq, double r, double c,
             double confidence, double beta, int64_t* out_ids, float* out_dist,
             int32_t* out_stats, void* stream) {
    return guarded([&] {
        validate_ann(index, queries, nq, 1, out_ids, out_dist, r);
        if (!(r > 0.0) || !std::isfinite(r)) fail(PMLSH_EINVAL, "r must be positive and finite");
        pmlsh_plan plan;
        plan_params(index->n, index->m, 1, c, confidence, beta, &plan);
        if (nq == 0) return;
        hipStream_t st = static_cast<hipStream_t>(stream);
        int32_t* stats = out_stats;
        void* tmp = nullptr;
        if (!stats) {
            tmp = ws_alloc((size_t)nq * 4 * sizeof(int32_t), st);
            stats = static_cast<int32_t*>(tmp);
        }
        try {
            run_ann(index, queries, nq, 1, c, confidence, beta, r, out_ids, out_dist, stats, st, 1);
            launch_bc_finalize(out_ids, out_dist, stats, nq, (float)(c * r), st);
        } catch (...) {
            ws_free(tmp, st);
            throw;
        }
        ws_free(tmp, st);
    });
}

int pmlsh_acp(const pmlsh_index* index, int32_t k, double c, double confidence,
              double beta, int64_t* out_pairs, float* out_dist, pmlsh_acp_stats* stats,
              void* stream) {
    return guarded([&] {
        if (!index) fail(PMLSH_EINVAL, "index is NULL");
        if (!out_pairs || !out_dist) fail(PMLSH_EINVAL, "outputs must not be NULL");
        if (index->n < 2) fail(PMLSH_EINVAL, "ACP needs n >= 2");
        if (k < 1) fail(PMLSH_EINVAL, "k must be >= 1");
        const double pairs = (double)index->n * (double)(index->n - 1) / 2.0;
        if ((double)k > pairs) fail(PMLSH_EINVAL, "k must be <= n(n-1)/2");
        if (k > PMLSH_MAX_K) fail(PMLSH_EUNSUPPORTED, "k above PMLSH_MAX_K");
        run_acp(index, k, c, confidence, beta, out_pairs, out_dist, stats,
                static_cast<hipStream_t>(stream));
    });
}

int pmlsh_acp_bb(const pmlsh_index* index, int32_t k, double c, double confidence,
                 double beta, int64_t* out_pairs, float* out_dist, pmlsh_acp_stats* stats,
                 void* stream) {
    return guarded([&] {
        if (!index) fail(PMLSH_EINVAL, "index is NULL");
        if (!out_pairs || !out_dist) fail(PMLSH_EINVAL, "outputs must not be NULL");
        if (index->n < 2) fail(PMLSH_EINVAL, "ACP needs n >= 2");
        if (k < 1) fail(PMLSH_EINVAL, "k must be >= 1");
        const double pairs = (double)index->n * (double)(index->n - 1) / 2.0;
        if ((double)k > pairs) fail(PMLSH_EINVAL, "k must be <= n(n-1)/2");
        if (k > PMLSH_MAX_K) fail(PMLSH_EUNSUPPORTED, "k above PMLSH_MAX_K");
        run_acp_bb(index, k, c, confidence, beta, out_pairs, out_dist, stats,
                   static_cast<hipStream_t>(stream));
    });
}

int pmlsh_acp_lca(const pmlsh_index* index, int32_t k, double c, double confidence,
                  double beta, double gamma, int64_t* out_pairs, float* out_dist,
                  pmlsh_acp_stats* stats, double* gamma_used, void* stream) {
    return guarded([&] {
        if (!index) fail(PMLSH_EINVAL, "index is NULL");
        if (!out_pairs || !out_dist) fail(PMLSH_EINVAL, "outputs must not be NULL");
        if (index->n < 2) fail(PMLSH_EINVAL, "ACP needs n >= 2");
        if (k < 1) fail(PMLSH_EINVAL, "k must be >= 1");
        const double pairs = (double)index->n * (double)(index->n - 1) / 2.0;
        if ((double)k > pairs) fail(PMLSH_EINVAL, "k must be <= n(n-1)/2");
        if (k > PMLSH_MAX_K) fail(PMLSH_EUNSUPPORTED, "k above PMLSH_MAX_K");
        if (std::isnan(gamma) || std::isinf(gamma)) fail(PMLSH_EINVAL, "gamma must be finite");
        run_acp_lca(index, k, c, confidence, beta, gamma, out_pairs, out_dist, stats, gamma_used,
                    static_cast<hipStream_t>(stream));
    });
}

int pmlsh_index_export_nodes(const pmlsh_index* index, int32_t* level, int32_t* first_leaf,
                             int32_t* end_leaf, float* radius) {
    return guarded([&] {
        if (!index || !level || !first_leaf || !end_leaf || !radius)
            fail(PMLSH_EINVAL, "NULL argument");
        export_nodes(index, level, first_leaf, end_leaf, radius);
    });
}

int pmlsh_get_index_info(const pmlsh_index* index, pmlsh_index_info* out) {
    return guarded([&] {
        if (!index || !out) fail(PMLSH_EINVAL, "NULL argument");
        pmlsh_index_info i{};
        i.n = index->n;
        i.d = index->d;
        i.m = index->m;
        i.leaf_size = index->leaf_size;
        i.fanout = index->fanout;
        i.num_pivots = index->num_pivots;
        i.levels = index->levels;
        i.n_leaves = index->n_leaves;
        i.n_nodes = index->n_nodes;
        i.sample_size = (int64_t)index->sample_sorted.size();
        i.device_bytes = index->device_bytes;
        i.filter_gemm = index->filter_gemm;
        i.eps_max = index->eps_max;
        *out = i;
    });
}

int pmlsh_index_filter_projection(const pmlsh_index* index, float* proj, float* eps) {
    return guarded([&] {
        if (!index || !proj || !eps) fail(PMLSH_EINVAL, "NULL argument");
        if (!index->filter_gemm) fail(PMLSH_EINVAL, "the index was built with filter_gemm = 0");
        const int64_t n = index->n;
        PMLSH_HIP(hipSetDevice(index->device));
        struct Buf {
            float* p = nullptr;
            ~Buf() { if (p) (void)hipFree(p); }
        } dp, de;
        PMLSH_HIP(hipMalloc(&dp.p, (size_t)n * MP * sizeof(float)));
        PMLSH_HIP(hipMalloc(&de.p, (size_t)n * sizeof(float)));
        launch_project_lp(index->data, n, index->d, index->d_pad, index->hash,
                          index->filter_gemm, dp.p, de.p, nullptr);
        std::vector<float> hp((size_t)n * MP), he((size_t)n);
        PMLSH_HIP(hipMemcpy(hp.data(), dp.p, hp.size() * sizeof(float), hipMemcpyDeviceToHost));
        PMLSH_HIP(hipMemcpy(he.data(), de.p, he.size() * sizeof(float), hipMemcpyDeviceToHost));
        // leaf order -> id order
        const int m = index->m;
        for (int64_t j = 0; j < n; ++j) {
            const int64_t id = index->perm_host[(size_t)j];
            for (int i = 0; i < m; ++i) proj[id * m + i] = hp[(size_t)j * MP + i];
            eps[id] = he[(size_t)j];
        }
    });
}

int pmlsh_index_export_leaves(const pmlsh_index* index, int32_t* perm, int64_t* offsets) {
    return guarded([&] {
        if (!index || !perm || !offsets) fail(PMLSH_EINVAL, "NULL argument");
        std::memcpy(perm, index->perm_host.data(), index->perm_host.size() * sizeof(int32_t));
        const int64_t L = index->leaf_size;
        for (int64_t b = 0; b <= index->n_leaves; ++b) offsets[b] = std::min(index->n, b * L);
    });
}

int pmlsh_ann_timing_enable(int stage_mask) {
    return guarded([&] {
        if (stage_mask < 0 || stage_mask >= (1 << PMLSH_N_STAGES))
            fail(PMLSH_EINVAL, "stage_mask must be a mask of the PMLSH_N_STAGES stages");
        timing_set((unsigned)stage_mask);
    });
}

int pmlsh_ann_timing_read(pmlsh_ann_timing* out, int reset) {
    return guarded([&] {
        if (!out) fail(PMLSH_EINVAL, "out is NULL");
        timing_read(out, reset != 0);
    });
}

int pmlsh_tune(int key, int64_t value) {
    return guarded([&] {
        if (key < 0 || key >= PMLSH_N_TUNE) fail(PMLSH_EINVAL, "unknown tuning key");
        if (value == -1) value = tune_default(key);
        const int64_t hi = key == PMLSH_TUNE_GROUP_LIST      ? 2048
                           : key == PMLSH_TUNE_ACP_FIRST_CAP ? (int64_t(1) << 20)
                           : key == PMLSH_TUNE_SCAN_SHAPE    ? 2
                                                             : 1;
        if (value < 0 || value > hi) fail(PMLSH_EINVAL, "tuning value out of range");
        tune_set(key, value);
    });
}

const char* pmlsh_last_error(void) { return error_cstr(); }

}  // extern "C"
