/*
 * pmlsh.h - C ABI of the PM-LSH query path on AMD Instinct MI355X (gfx950).
 *
 * PM-LSH (Zheng et al., "PM-LSH: a fast and accurate in-memory framework for
 * high-dimensional approximate NN and closest pair search") answers
 *   (c,k)-ANN  (Definition 2, Section 2.1) with Algorithm 2 (Section 5.2), and
 *   (c,k)-ACP  (Definition 4, Section 2.1) with radius filtering (Section 6.3)
 * over points projected by m Gaussian hash functions h*(o) = a . o (Eq. 3,
 * Section 3.2) and indexed by a PM-tree in the projected space (Section 4.1).
 *
 * Conventions shared by every entry point
 *   - Return value: PMLSH_OK (0) on success, a negative PMLSH_E* code on error.
 *     On error no output buffer has been written and a message is available
 *     from pmlsh_last_error() on the calling thread. No C++ exception crosses
 *     this interface.
 *   - Argument validation happens before any HIP call: invalid arguments are
 *     reported without touching the GPU.
 *   - Matrices are row-major FP32. Ids are 0-based row numbers of the data
 *     matrix passed to pmlsh_build, int64 at this interface.
 *   - Distances returned are Euclidean (not squared), FP32. Results are
 *     sorted ascending by (distance, id) for ANN and by (distance, i, j) with
 *     i < j for ACP.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Work is
 *     enqueued on it; pmlsh_ann returns before the results are ready (read
 *     them after synchronising the stream), pmlsh_build and pmlsh_acp return
 *     after their work on the stream has completed.
 *   - An index may be used by several threads for concurrent queries on
 *     different streams; calls on the same index and the same stream are
 *     serialised by the stream.
 */
#ifndef PMLSH_H
#define PMLSH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PMLSH_OK 0
#define PMLSH_EINVAL (-1)       /* invalid argument                          */
#define PMLSH_ENOMEM (-2)       /* device or host memory exhausted           */
#define PMLSH_EDEVICE (-3)      /* a HIP call failed                         */
#define PMLSH_EUNSUPPORTED (-4) /* valid but outside this build's limits     */

#define PMLSH_MAX_M 16          /* hash functions per index                  */
#define PMLSH_MAX_PIVOTS 8      /* global pivots of the PM-tree              */
#define PMLSH_MAX_K 1024        /* results per ANN query / ACP call          */

/* exit kinds reported per ANN query (Algorithm 2)                          */
#define PMLSH_EXIT_NEAR 1      /* k verified points within c*r              */
#define PMLSH_EXIT_BUDGET 2     /* the range query reached beta*n + k points */

typedef struct pmlsh_index pmlsh_index; /* opaque, owned by the caller once built */

/*
 * Index construction (Sections 3.2 and 4.1).
 *   data   n x d FP32, row-major. Device pointer if data_on_device != 0, else
 *          host pointer. Read only; the index keeps its own copy (rows
 *          permuted to leaf order), so the caller may free `data` on return.
 *   hash   m x d FP32, row-major: the m projection vectors a_1..a_m, whose
 *          entries the caller draws i.i.d. from N(0,1) (2-stable, Section 2.2).
 *          Same residency as `data`. Copied.
 *   n >= 1, 1 <= d <= 65536, 1 <= m <= PMLSH_MAX_M. Every value must be finite.
 *   num_pivots   s, 0..PMLSH_MAX_PIVOTS (the paper uses 5, Section 7.1).
 *   leaf_size    points per leaf, 8..256 (0 = 64).
 *   fanout       children per inner node, a power of two in 2..64 (0 = 16).
 *   sample_seed  seed of the pair sample that estimates the distance
 *                distribution F used for r_min (Section 5.2).
 *   r_min_kappa  r_min = kappa * F^-1(B/n); in (0, 1]; 0 selects 0.9.
 *   filter_gemm  projection behind the FP16 rows of the batched range
 *                filter: 0 rounds the FP64 projection (Eq. 3, Section 3.2);
 *                PMLSH_FILTER_GEMM_FP16 / _BF16 compute it on the matrix cores
 *                from FP16 / BF16 inputs with FP32 accumulation (points at
 *                build, queries per batch), each row with a bound eps on its
 *                distance to the exact projection; the filter then widens
 *                its radius by eps(query) + max eps(point), so it still passes
 *                every point the exact projection would. Every later decision
 *                (pool distances, budget cut, rounds, verification) uses the
 *                FP64-accurate projection, so answers do not depend on this
 *                choice; the pool, and with it the time, grows with the
 *                widening. EUNSUPPORTED if a value exceeds the input format.
 * Errors: EINVAL (arguments, non-finite values), ENOMEM, EDEVICE,
 * EUNSUPPORTED. On success *out receives the index; free it with pmlsh_free.
 */
#define PMLSH_FILTER_GEMM_FP16 1
#define PMLSH_FILTER_GEMM_BF16 2

typedef struct {
    const float* data;
    int64_t n;
    int32_t d;
    const float* hash;
    int32_t m;
    int32_t data_on_device;
    int32_t num_pivots;
    int32_t leaf_size;
    int32_t fanout;
    int32_t filter_gemm;
    uint64_t sample_seed;
    double r_min_kappa;
    void* stream;
} pmlsh_build_args;

int pmlsh_build(const pmlsh_build_args* args, pmlsh_index** out);

/* Releases every host and device resource of the index. NULL is a no-op.
 * The caller must make sure no work using the index is still in flight. */
void pmlsh_free(pmlsh_index* index);

/*
 * Query parameters of Algorithm 2 (Lemma 3, Section 4.3; Eq. 10 and Lemma 5,
 * Section 5.3; the budget of Section 5.2).
 * Host-only computation: never touches the GPU.
 *   confidence  Pr[E1] = 1 - alpha1 in (0,1): t = sqrt(chi^2_{alpha1}(m)),
 *               the upper alpha1 quantile (Lemma 3, first line of Eq. 10).
 *   c > 1       approximation ratio; alpha2 solves t^2 = c^2 chi^2_{1-alpha2}(m).
 *   beta        fraction of false positives budgeted; beta < 0 selects
 *               2 * alpha2 (Lemma 5); beta must be <= 1.
 *   budget      B = ceil(beta * n) + k, capped at n (candidates of Algorithm 2).
 *   acp_budget  T = ceil(beta * n (n-1) / 2) + k (pairs of Section 6.3).
 * Errors: EINVAL for n < 1, m outside 1..16, k < 1, c <= 1 or not finite,
 * confidence outside (0,1), beta > 1 or NaN.
 */
typedef struct {
    double t;          /* radius factor                                  */
    double alpha1;
    double alpha2;
    double beta;       /* the beta actually used                         */
    int64_t budget;    /* B                                              */
    int64_t acp_budget;/* T                                              */
} pmlsh_plan;

int pmlsh_plan_params(int64_t n, int32_t m, int32_t k, double c,
                      double confidence, double beta, pmlsh_plan* out);

/* r_min of Section 5.2 for a candidate budget B on this index:
 * kappa * (sample distance at index ceil(min(1, B/n) * S) - 1), S the sample
 * size. Host-only. Errors: EINVAL for a NULL argument or budget < 1. */
int pmlsh_default_r_min(const pmlsh_index* index, int64_t budget, double* r_min);

/*
 * (c,k)-ANN, Algorithm 2 (Section 5.2), for a batch of queries.
 *   queries   nq x d FP32 device pointer (row-major).
 *   nq >= 0 (0 is a no-op), 1 <= k <= min(n, PMLSH_MAX_K), c, confidence,
 *   beta as in pmlsh_plan_params; r_min > 0 is the first radius, r_min <= 0
 *   selects pmlsh_default_r_min for the budget B.
 *   out_ids   nq x k int64 device pointer; out_dist nq x k FP32 device pointer.
 *   out_stats optional (NULL allowed) nq x 4 int32 device pointer; per query:
 *             range queries issued, final |C|, exit kind (PMLSH_EXIT_*),
 *             points scanned in leaves over all rounds (saturating at 2^31-1).
 * Each query: project q with the index's hash matrix; starting at r = r_min,
 * (a) from the second round on, stop if k candidates lie within c*r of q;
 * (b) collect the points whose projected distance to q' is <= t*r, using
 *     the PM-tree's node test (Eq. 5) to skip subtrees;
 * (c) if they number >= B, the candidate set C is the B of them nearest to q'
 *     in the projected space (ties by id) and the loop stops; otherwise
 *     C is all of them and r <- c*r.
 * The answer is the k members of C nearest to q by exact distance, in
 * (distance, id) order; out_dist holds Euclidean distances (not squared).
 * Precision: projected and exact distances are computed in FP32; where the
 * FP32 values leave the order open within their rounding error, the budget
 * cut in (c) and the order of the answer are decided on FP64 values (the
 * FP64 projection and FP64 distances from the FP32 rows), and out_dist is
 * the FP32 rounding of the FP64 distance (more than 512 members within FP32
 * rounding of the k-th keep the FP32 order and distances).
 * Asynchronous on `stream`. Errors: EINVAL, ENOMEM (workspace), EDEVICE,
 * EUNSUPPORTED (k > PMLSH_MAX_K).
 */
int pmlsh_ann(const pmlsh_index* index, const float* queries, int64_t nq,
              int32_t k, double c, double confidence, double beta, double r_min,
              int64_t* out_ids, float* out_dist, int32_t* out_stats,
              void* stream);

/*
 * (c,k)-ANN, Algorithm 2 (Section 5.2), for a batch whose queries carry
 * their own parameters: query i is answered exactly as pmlsh_ann would
 * answer it alone with k = args[i].k, c = args[i].c, confidence =
 * args[i].confidence, beta = args[i].beta and r_min = args[i].r_min (each
 * as in pmlsh_ann). Algorithm 2 is run per query, so one launch serves all
 * of them and no answer depends on the others.
 *   args        host array of nq entries.
 *   out_stride  row stride of out_ids / out_dist, >= the largest k; query
 *               i's answer is written to row i, the first args[i].k entries.
 *   out_ids     nq x out_stride int64 device pointer; out_dist the same FP32.
 *   out_stats   optional nq x 4 int32 device pointer, as for pmlsh_ann.
 * The per-query parameters are copied to the device on `stream`; the call
 * returns after that copy (it waits for the work queued on the stream before
 * it) and leaves the search itself asynchronous. Errors: EINVAL (an entry or
 * out_stride invalid, naming the entry), EUNSUPPORTED (a k above
 * PMLSH_MAX_K), ENOMEM, EDEVICE.
 */
typedef struct {
    int32_t k;
    int32_t reserved;
    double c;
    double confidence;
    double beta;
    double r_min;
} pmlsh_query_args;

int pmlsh_ann_mixed(const pmlsh_index* index, const float* queries, int64_t nq,
                    const pmlsh_query_args* args, int32_t out_stride, int64_t* out_ids,
                    float* out_dist, int32_t* out_stats, void* stream);

/*
 * pmlsh_ann for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Arguments, results and errors are those of pmlsh_ann; the same kernels
 * run. The workspace is a fixed array of PMLSH_NOALLOC_SCRATCH_BYTES in the
 * library's code object, one copy per device (held until the process ends),
 * instead of the caching allocator: no hipMalloc, hipFree or other
 * allocating routine is called, and per-stage timing is skipped. The
 * queries run in batches that fit the array; EUNSUPPORTED when not even one
 * query of this index fits (its message gives the bytes one query needs).
 * Every call on a device shares that device's array and leaves its contents
 * behind (the kernels initialise all they read): calls that overlap on one
 * device, on any streams, race and must be serialised by the caller.
 */
#define PMLSH_NOALLOC_SCRATCH_BYTES (64LL * 1024 * 1024)

int pmlsh_ann_noalloc(const pmlsh_index* index, const float* queries, int64_t nq,
                      int32_t k, double c, double confidence, double beta, double r_min,
                      int64_t* out_ids, float* out_dist, int32_t* out_stats,
                      void* stream);

/*
 * (r,c)-BC (ball cover) query, Algorithm 1 (Section 5.1), for a batch of
 * queries: one range query of radius t*r around q' with the budget
 * B = beta*n + 1 (the same reading of the budget as pmlsh_ann: when the ball
 * holds at least B points, C is the B of them nearest to q' in the projected
 * space, ties by id; otherwise C is the ball). The answer is the point of C
 * nearest to q (ties by id) when the ball reached B points, or when that
 * point lies within c*r of q; otherwise nothing.
 *   queries   nq x d FP32 device pointer; r > 0 finite; c, confidence,
 *             beta as in pmlsh_plan_params (k = 1).
 *   out_ids   nq int64 device pointer: the point's id, or -1 for nothing.
 *   out_dist  nq FP32 device pointer: its Euclidean distance, or +inf.
 *   out_stats optional nq x 4 int32 device pointer, as for pmlsh_ann (1
 *             range query; exit kind PMLSH_EXIT_BUDGET or 0).
 * Asynchronous on `stream`. Errors: EINVAL, ENOMEM, EDEVICE.
 */
int pmlsh_bc(const pmlsh_index* index, const float* queries, int64_t nq, double r,
             double c, double confidence, double beta, int64_t* out_ids,
             float* out_dist, int32_t* out_stats, void* stream);

/*
 * (c,k)-ACP by radius filtering (Section 6.3, Algorithm 4), canonical form.
 *   1. every pair inside one leaf is verified; ub = the k-th smallest such
 *      distance (+inf if fewer than k pairs). With leaves of at most 64
 *      points every such pair first gets rigorous bounds from the Gram
 *      matrix of its leaf (FP16 matrix cores), and only the pairs whose
 *      bounds reach the k-th smallest upper bound get exact distances: ub
 *      and the answer are those of verifying them all;
 *   2. every pair (i<j) in different leaves with projected distance < t*ub is
 *      a candidate; pairs of leaves whose Mindist (Eq. 11) is at least t*ub
 *      are skipped whole;
 *   3. at most T pairs are verified in total; above that the candidates with
 *      the smallest projected distance (ties by (i,j)) are kept;
 *   4. the k verified pairs with the smallest exact distance are returned.
 *   n >= 2, 1 <= k <= min(n(n-1)/2, PMLSH_MAX_K); c, confidence, beta as in
 *   pmlsh_plan_params.
 *   out_pairs k x 2 int64 device pointer (i < j); out_dist k FP32 device.
 *   stats     optional host pointer, filled on success.
 * Precision: distances are computed in FP32; the order of the answer (step 4,
 * ties by (i, j)) is decided on FP64 distances from the FP32 rows for every
 * pair within FP32 rounding of the k-th one, and out_dist is the FP32
 * rounding of the FP64 distance (more than 1,024 such pairs keep the FP32
 * order and distances). The same holds for pmlsh_acp_bb and pmlsh_acp_lca.
 * Synchronous: returns after the work on `stream` has completed.
 * Errors: EINVAL, ENOMEM (candidate buffers), EDEVICE, EUNSUPPORTED.
 */
typedef struct {
    double t;
    double ub;            /* k-th smallest self-join distance                 */
    int64_t budget;       /* T                                                */
    int64_t n_seed;       /* pairs inside one leaf (the self-join's seeds)    */
    int64_t n_cand_raw;   /* cross-leaf pairs with projected distance < t*ub  */
    int64_t n_cand;       /* candidates verified after the T cut              */
    int64_t tiles_total;  /* leaf pairs (e1 < e2)                             */
    int64_t tiles_scanned;/* leaf pairs that survived the Mindist test        */
} pmlsh_acp_stats;

int pmlsh_acp(const pmlsh_index* index, int32_t k, double c, double confidence,
              double beta, int64_t* out_pairs, float* out_dist,
              pmlsh_acp_stats* stats, void* stream);

/*
 * Serving loop: continuous batching of (c,k)-ANN requests on a resident
 * index. Each request is Algorithm 2 (Section 5.2) for its own queries with
 * its own k, c, confidence and beta, exactly as pmlsh_ann would answer it
 * alone (results are identical bit for bit).
 *
 * A server owns one host worker thread and one HIP stream of the index's
 * device (default priority). Requests wait in arrival order; the worker
 * forms each launch from the oldest waiting request and the requests after
 * it with the same (k, c, confidence, beta, r_min), up to max_batch queries
 * (a larger request is split over several launches), gathers their queries
 * into a staging buffer, runs the batched ANN path on it and scatters the
 * answers to each request's outputs. Up to max_inflight launches are queued
 * on the stream at once, so requests that arrive while others run on the GPU
 * are admitted as soon as a launch slot and the HBM budget allow: a launch
 * is admitted while the staging and workspace bytes of the launches in
 * flight, its own included, stay within hbm_budget (one launch is always
 * admitted when none is in flight).
 *
 *   max_batch     queries per launch, 1..65535 (0 selects 1024)
 *   max_inflight  launches queued at once, 1..64 (0 selects 2)
 *   hbm_budget    bytes, 0 selects 8 GiB
 * pmlsh_server_create errors: EINVAL, EDEVICE (stream or thread creation).
 */
typedef struct pmlsh_server pmlsh_server;

typedef struct {
    int64_t max_batch;
    int32_t max_inflight;
    int64_t hbm_budget;
} pmlsh_server_args;

int pmlsh_server_create(const pmlsh_index* index, const pmlsh_server_args* args,
                        pmlsh_server** out);

/* Submits one request: queries nq x d FP32 device pointer, outputs nq x k
 * int64 ids and FP32 distances (device), arguments as in pmlsh_ann. The
 * caller keeps the buffers alive and untouched until the request completes.
 * When `stream` is not NULL, the server waits for the work queued on it so
 * far before reading the queries; otherwise the queries must already be
 * complete. Validation happens here (EINVAL / EUNSUPPORTED as pmlsh_ann);
 * on success *ticket identifies the request (nq = 0 completes at once). */
int pmlsh_server_submit(pmlsh_server* server, const float* queries, int64_t nq,
                        int32_t k, double c, double confidence, double beta,
                        double r_min, int64_t* out_ids, float* out_dist,
                        void* stream, uint64_t* ticket);

/* *done = 1 when the request has completed (its outputs are written), else
 * 0. EINVAL for an unknown ticket. */
int pmlsh_server_test(pmlsh_server* server, uint64_t ticket, int* done);

/* Blocks until the request has completed and releases the ticket. Returns
 * the request's result: PMLSH_OK, or the error its launch hit. */
int pmlsh_server_wait(pmlsh_server* server, uint64_t ticket);

/* Counters since creation: requests and queries completed, launches, and
 * request latency (submission to completion seen by the worker) in ms. */
typedef struct {
    int64_t requests;
    int64_t queries;
    int64_t launches;
    double latency_p50_ms;
    double latency_p99_ms;
    double latency_max_ms;
} pmlsh_server_stats;

int pmlsh_server_get_stats(pmlsh_server* server, pmlsh_server_stats* out);

/* Completes every submitted request, stops the worker and frees the server
 * (its tickets become invalid). */
void pmlsh_server_destroy(pmlsh_server* server);

/*
 * (c,k)-ACP by the branch-and-bound algorithm (Algorithm 3, Section 6.1):
 * the T = beta*n(n-1)/2 + k pairs (capped at n(n-1)/2) with the smallest
 * projected distances over all pairs, ties by (i, j), are verified and the k
 * with the smallest exact distance (ties by (i, j)) are returned. Arguments,
 * outputs and errors as pmlsh_acp; EUNSUPPORTED when T exceeds 2^28 (known
 * before any GPU work) or more than 2^28 pairs lie within the T-th smallest
 * projected distance. In stats, ub is that
 * distance's bound d_T used by the scan, n_seed is 0, n_cand_raw the pairs
 * within d_T, n_cand = T. Synchronous.
 */
int pmlsh_acp_bb(const pmlsh_index* index, int32_t k, double c, double confidence,
                 double beta, int64_t* out_pairs, float* out_dist,
                 pmlsh_acp_stats* stats, void* stream);

/*
 * (c,k)-ACP by radius filtering with FindLCA (Algorithm 4 with Algorithm 5,
 * Section 6.3):
 *   1. every pair inside one leaf is verified; ub = the k-th smallest exact
 *      distance; count = the number of verified pairs;
 *   2. FindLCA: walking down from the root, the inner nodes whose radius is
 *      below gamma * t * ub (a found node's subtree is not searched further);
 *   3. the found nodes in ascending order of radius (ties by node index);
 *      in each, every pair of points in different leaves of its subtree
 *      with projected distance below t * ub is verified; then ub becomes the
 *      k-th smallest verified distance and count grows by those pairs; the
 *      scan stops after the first node that leaves count > T;
 *   4. the k verified pairs with the smallest (distance, i, j).
 * ub and count are updated after each node (the paper updates them after
 * each verified pair). gamma > 0 is used as given; gamma <= 0 estimates it
 * so that Pr(gamma) = 0.85 over 100,000 random pairs (the ratio of the
 * radius of their lowest common ancestor to their projected distance).
 * gamma_used (optional host pointer) receives the gamma applied. Other
 * arguments, outputs and errors as pmlsh_acp; stats: ub is the final ub,
 * n_cand_raw = n_cand = the candidates verified, tiles_total the leaf pairs
 * under the found nodes, tiles_scanned those scanned. Synchronous.
 */
int pmlsh_acp_lca(const pmlsh_index* index, int32_t k, double c, double confidence,
                  double beta, double gamma, int64_t* out_pairs, float* out_dist,
                  pmlsh_acp_stats* stats, double* gamma_used, void* stream);

/* Node structure of the index, for checking pmlsh_acp_lca against an
 * independent implementation: for each of the n_nodes nodes (levels top
 * down, the leaves last), its level (0 = root level), the range
 * [first_leaf, end_leaf) of leaves under it (leaf b holds the ids listed by
 * pmlsh_index_export_leaves for b) and its covering radius in the projected
 * space. Host buffers of n_nodes entries each. */
int pmlsh_index_export_nodes(const pmlsh_index* index, int32_t* level, int32_t* first_leaf,
                             int32_t* end_leaf, float* radius);

/* Shape and size of a built index. Host-only. */
typedef struct {
    int64_t n;
    int32_t d;
    int32_t m;
    int32_t leaf_size;
    int32_t fanout;
    int32_t num_pivots;
    int32_t levels;       /* tree levels including the leaf level           */
    int64_t n_leaves;
    int64_t n_nodes;      /* all levels                                       */
    int64_t sample_size;  /* pairs in the r_min sample                        */
    int64_t device_bytes; /* HBM held by the index                            */
    int32_t filter_gemm;  /* as built (0, PMLSH_FILTER_GEMM_FP16 or _BF16)     */
    float eps_max;        /* largest point bound eps of that projection (0 for 0) */
} pmlsh_index_info;

int pmlsh_get_index_info(const pmlsh_index* index, pmlsh_index_info* out);

/* The low-precision projection of an index built with filter_gemm != 0, for
 * checking its bound: recomputes, for every point in id order, the m
 * coordinates the filter's rows come from (host buffer of n x m floats) and
 * the bound eps on their Euclidean distance to the exact projection (host
 * buffer of n floats). EINVAL if the index was built with filter_gemm = 0. */
int pmlsh_index_filter_projection(const pmlsh_index* index, float* proj, float* eps);

/* Leaf partition of the index, for checking ACP against an independent
 * implementation: leaf b holds the ids perm[offsets[b] .. offsets[b+1]).
 * perm: n int32 host buffer; offsets: n_leaves + 1 int64 host buffer.
 * Host-only (copied at build). */
int pmlsh_index_export_leaves(const pmlsh_index* index, int32_t* perm,
                              int64_t* offsets);

/*
 * Tracing aid: per-stage GPU time of pmlsh_ann and pmlsh_acp.
 * pmlsh_ann_timing_enable takes
 * a process-wide mask of stages (bit s = stage s; 0 turns timing off,
 * (1 << PMLSH_N_STAGES) - 1 times every stage; other values: PMLSH_EINVAL).
 * Each launch of a timed stage is bracketed by two HIP events on the caller's
 * stream; pmlsh_ann_timing_read() waits for the recorded events and returns
 * the summed milliseconds and launch counts per stage since the last reset
 * (reset != 0 clears the totals after reading). Stages:
 *   PMLSH_STAGE_PROJECT   query projection (FP64 matrix cores)
 *   PMLSH_STAGE_TAU       per-query bound on the B-th projected distance and the
 *                         chunk-ball test of Eq. 5
 *   PMLSH_STAGE_FILTER    range filter on the FP16 matrix cores, candidate pools
 *   PMLSH_STAGE_FINISH    budget cut, rounds of Algorithm 2, verification, top-k
 *   PMLSH_STAGE_PERQUERY  per-query kernel (queries outside the batched path)
 *   PMLSH_STAGE_DIST      squared distances from every query to every 64-point
 *                         chunk centre (input of the bound and of Eq. 5)
 * and of pmlsh_acp (Section 6.3), one launch each per call:
 *   PMLSH_STAGE_ACP_SELFJOIN  exact distances of every within-leaf pair
 *   PMLSH_STAGE_ACP_SELECT    ub = the k-th smallest of them (on the device)
 *   PMLSH_STAGE_ACP_TILES     parent distances and the Mindist (Eq. 11) leaf-pair test
 *   PMLSH_STAGE_ACP_SCAN      projected pair scan of the surviving leaf pairs
 *   PMLSH_STAGE_ACP_VERIFY    seeds of the top-k band and exact distances of the candidates
 *   PMLSH_STAGE_ACP_TOPK      top-k of the verified pairs (FP64 order in the band)
 * Host-side bookkeeping only; enabling it does not change any result.
 */
#define PMLSH_STAGE_PROJECT 0
#define PMLSH_STAGE_TAU 1
#define PMLSH_STAGE_FILTER 2
#define PMLSH_STAGE_FINISH 3
#define PMLSH_STAGE_PERQUERY 4
#define PMLSH_STAGE_DIST 5
#define PMLSH_STAGE_ACP_SELFJOIN 6
#define PMLSH_STAGE_ACP_SELECT 7
#define PMLSH_STAGE_ACP_TILES 8
#define PMLSH_STAGE_ACP_SCAN 9
#define PMLSH_STAGE_ACP_VERIFY 10
#define PMLSH_STAGE_ACP_TOPK 11
#define PMLSH_N_STAGES 12

typedef struct {
    double ms[PMLSH_N_STAGES];
    int64_t launches[PMLSH_N_STAGES];
} pmlsh_ann_timing;

int pmlsh_ann_timing_enable(int stage_mask);
int pmlsh_ann_timing_read(pmlsh_ann_timing* out, int reset);

/*
 * Test aid: process-wide switches of the ANN path: the group filter of the
 * bound kernel (the minima of 64-chunk groups that rule out the groups unable
 * to hold a chunk chosen for tau or a chunk passing Eq. 5), and the choice of
 * the plain FP32 per-query path for whole launches, the block shape of the
 * range filter; and the first buffer capacities of pmlsh_acp. Results are the same under every setting; only
 * the work differs.
 *   PMLSH_TUNE_GROUP_LIST         most groups (and 256-chunk blocks of the
 *                                 Eq. 5 test) one query lists, 0..2048
 *                                 (default 2048); when more qualify, or at 0,
 *                                 the passes read the query's whole row
 *   PMLSH_TUNE_GROUP_MINIMA_LDS   1 (default): the group minima are copied to
 *                                 LDS when they fit (about 28,000 groups);
 *                                 0: read from HBM in every pass
 *   PMLSH_TUNE_FP32_PATH          0 (default): the batched path (FP16 matrix-core
 *                                 filter, FP16 verification rows with bounds);
 *                                 1: every query of a launch takes the per-query
 *                                 kernel (PM-tree walk with Eq. 5, FP32 projected
 *                                 and exact distances), the plain FP32 path
 *   PMLSH_TUNE_ACP_FIRST_CAP      0 (default): pmlsh_acp's first capacities
 *                                 for the candidate pairs (2^20, or 4 k) and
 *                                 the band of seeds verified exactly (2^16, or
 *                                 4 k); 1..2^20: both start at this value, so
 *                                 that the passes that redo a stage at the
 *                                 full count run on small inputs
 *   PMLSH_TUNE_SCAN_SHAPE         0 (default): the range filter's query block
 *                                 follows the index's size (512 queries per
 *                                 workgroup below 32,768 chunks of 64 points,
 *                                 1,024 from there on); 1: always 512; 2:
 *                                 always 1,024
 * value -1 restores the default; a key or value out of range: PMLSH_EINVAL.
 * A call running while a switch changes may see either setting.
 */
#define PMLSH_TUNE_GROUP_LIST 0
#define PMLSH_TUNE_GROUP_MINIMA_LDS 1
#define PMLSH_TUNE_FP32_PATH 2
#define PMLSH_TUNE_ACP_FIRST_CAP 3
#define PMLSH_TUNE_SCAN_SHAPE 4
#define PMLSH_N_TUNE 5

int pmlsh_tune(int key, int64_t value);

/* Message of the last failed call on this thread ("" if none). The pointer
 * stays valid until the next failing call on the same thread. */
const char* pmlsh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMLSH_H */
