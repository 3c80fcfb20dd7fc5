// Internal declarations shared by the host-side translation units of the
// PM-LSH library: error reporting, the index object and the device layout.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <functional>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "pmlsh.h"

namespace pmlsh {

// Projected coordinates are padded from m to MP floats (zero pad lanes).
constexpr int MP = 16;
// Weight cm of the per-pair rounding margin cm * ||q'|| * ||o'|| of the FP16
// scan: 2^-9 bounds the FP16 rounding of the projected dot product, the extra
// 2^-14 absorbs the rounding of the margin term itself.
constexpr float kScanMarginWeight = 0.001953125f + 0.00006103515625f;
// halves per FP16 row of the matrix-core scan: 21 terms (16 coordinates,
// the hi and lo halves of the norm, two ones and the margin term) padded to
// a multiple of eight; the eight halves the 32-deep MFMA reads beyond them
// are zero and are not stored
constexpr int kScanRow = 24;
// Chunks the ANN bound may choose per query (64 points each; at least twice
// the largest budget of the batched path).
constexpr int kSelCap = 1024;

// The batch's chunk-distance matrix (bf16 values) is stored in blocks of 64
// queries x 64 chunks (8 KB, a query's 64 chunks contiguous inside), the
// blocks of one band of 64 queries in chunk order, so that a workgroup tile
// of the kernels that write and read it is one contiguous run; then the
// minimum of every group of 64 chunks, a row of cdist_gmin_len entries per
// query.
inline int64_t cdist_groups(int64_t n_chunk) { return (n_chunk + 63) / 64; }
inline int64_t cdist_gmin_len(int64_t n_chunk) { return (cdist_groups(n_chunk) + 15) / 16 * 16; }
inline int64_t cdist_block_elems(int64_t batch, int64_t n_chunk) {
    return (batch + 63) / 64 * 4096 * cdist_groups(n_chunk);
}
inline int64_t cdist_elems(int64_t batch, int64_t n_chunk) {
    return cdist_block_elems(batch, n_chunk) + batch * cdist_gmin_len(n_chunk);
}

// Thread-local error message returned by pmlsh_last_error().
void set_error(const std::string& msg);
void clear_error();
const char* error_cstr();

struct Error {
    int code;
    std::string msg;
};

// Throws pmlsh::Error; caught at the C boundary.
[[noreturn]] void fail(int code, const std::string& msg);

// Runs fn and turns any exception into an error code and message.
template <class F>
int guarded(F&& fn) {
    try {
        fn();
        return PMLSH_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host memory exhausted");
        return PMLSH_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return PMLSH_EDEVICE;
    } catch (...) {
        set_error("unknown error");
        return PMLSH_EDEVICE;
    }
}

#define PMLSH_HIP(call)                                                          \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess)                                                    \
            ::pmlsh::fail(e_ == hipErrorOutOfMemory ? PMLSH_ENOMEM : PMLSH_EDEVICE, \
                          std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

// ---------------------------------------------------------------- workspace
// Device memory from the library's per-device caching allocator: a released
// block is reused at once on the stream it was released on, and on other
// streams once the work queued before its release has completed. ws_free
// never throws.
void* ws_alloc(size_t bytes, hipStream_t st);
void ws_free(void* p, hipStream_t st);

// Parameters of one query of a launch whose queries differ in k, c,
// confidence, beta or r_min (device array, one entry per query).
struct AnnQueryParams {
    double c, t, r_min;
    int32_t k, budget;
};

// ---------------------------------------------------------------- ANN host path
// Argument checks of pmlsh_ann (throw EINVAL / EUNSUPPORTED).
void validate_ann(const pmlsh_index* index, const float* queries, int64_t nq, int k,
                  const int64_t* out_ids, const float* out_dist, double r_min);
// Bytes of the device workspace one pmlsh_ann call on nq queries allocates.
int64_t ann_workspace_bytes(const pmlsh_index* x, int64_t nq, int k, double c,
                            double confidence, double beta);
// pmlsh_ann after validation: asynchronous on st. max_rounds > 0 stops
// Algorithm 2 after that many range queries.
void run_ann(const pmlsh_index* x, const float* queries, int64_t nq, int k, double c,
             double confidence, double beta, double r_min, int64_t* out_ids,
             float* out_dist, int32_t* out_stats, hipStream_t st, int max_rounds = 0);
// A batch of queries with per-query parameters: the device array qpar (nq
// entries, from plan_queries), the largest k and budget among them, and the
// row stride of the outputs (>= kmax). region / region_bytes: a fixed
// device region for the workspace (null: the caching allocator).
void run_ann_mixed(const pmlsh_index* x, const float* queries, int64_t nq,
                   const AnnQueryParams* qpar, int kmax, int64_t bmax, int out_stride,
                   int64_t* out_ids, float* out_dist, int32_t* out_stats, hipStream_t st,
                   void* region, int64_t region_bytes);
// A batch of queries sharing one plan (from plan_queries), its answers
// written with row stride k, the workspace in the given device region.
void run_ann_planned(const pmlsh_index* x, const float* queries, int64_t nq,
                     const AnnQueryParams& p, int64_t* out_ids, float* out_dist, hipStream_t st,
                     void* region, int64_t region_bytes);
// Host plan of per-query parameters (t, B and the default r_min resolved);
// throws EINVAL / EUNSUPPORTED like pmlsh_ann for an invalid entry.
void plan_queries(const pmlsh_index* x, const pmlsh_query_args* args, int64_t nq,
                  std::vector<AnnQueryParams>* out, int* kmax, int64_t* bmax);
// Workspace bytes of run_ann_mixed on nq queries with these largest k, B.
int64_t ann_workspace_bytes_mixed(const pmlsh_index* x, int64_t nq, int kmax, int64_t bmax);
// pmlsh_ann over a fixed device region of region_bytes instead of the
// caching allocator: the queries go through in batches that fit it;
// EUNSUPPORTED (before any HIP call) when not even one query fits. The
// region's address is asked of region_of_device only after that check.
// Allocates no device memory.
void run_ann_in(const pmlsh_index* x, const float* queries, int64_t nq, int k, double c,
                double confidence, double beta, double r_min, int64_t* out_ids,
                float* out_dist, int32_t* out_stats, hipStream_t st,
                const std::function<void*()>& region_of_device, int64_t region_bytes);
// (r,c)-BC answers from the per-query stats of one round with k = 1.
void launch_bc_finalize(int64_t* ids, float* dist, const int32_t* stats, int64_t nq, float cr,
                        hipStream_t stream);

// ---------------------------------------------------------------- planner
double chi2_cdf(double x, int m);
double chi2_upper_quantile(double alpha, int m);
uint64_t splitmix64(uint64_t x);
void plan_params(int64_t n, int m, int k, double c, double confidence,
                 double beta, pmlsh_plan* out);  // throws on invalid input

// ---------------------------------------------------------------- tree
// Flattened PM-tree, structure-of-arrays over all nodes; levels are stored
// top-down and contiguously, level l holding nodes
// [level_begin[l], level_begin[l+1]). Leaves form the last level and hold
// the contiguous point range [child_begin, child_end) of the leaf order.
struct HostTree {
    int levels = 0;
    int64_t n_nodes = 0;
    std::vector<int64_t> level_begin;     // levels + 1
    std::vector<float> centre;            // MP x n_nodes (dimension-major)
    std::vector<float> radius;            // n_nodes
    std::vector<float> hr_min, hr_max;    // s x n_nodes
    std::vector<int32_t> child_begin, child_end;
    std::vector<int32_t> npts;            // points in the subtree of each node
    std::vector<float> pivots;            // s x MP
    std::vector<int32_t> perm;            // leaf position -> original id
    float coord_scale = 0.f;              // max ||o'|| + max ||p_i||
};

// Binary split tree of the leaf order: node 0 is the root; a node covers the
// leaves [leaf_begin, leaf_end); left and right are -1 for a leaf.
struct SplitNode {
    int64_t leaf_begin, leaf_end;
    int32_t left, right;
};

// Recursive gap-aware splits of the leaf order on the device, level by level
// (bulkload.hip): proj is the device projection (n x MP, original order);
// returns the leaf order (leaf position -> id) and the split tree.
void device_split(const float* proj, int64_t n, int leaf, hipStream_t st,
                  std::vector<int32_t>* perm, std::vector<SplitNode>* nodes);

// Device reductions of the bulk-load (bulkload.hip). device_all_finite:
// whether count floats are all finite. device_pivots: s pivots by
// farthest-point selection over the ids (started from the point farthest
// from the centroid, smallest id on ties) and the largest FP64 norm of a
// point. device_ball_summaries: for every range [p0, p1) of the leaf order
// (perm on the device), the FP64 mean rounded to FP32 (m x MP), the largest
// FP64 distance of its points to that centre, and per pivot the smallest and
// largest FP64 distance (m x 2 s, min then max).
bool device_all_finite(const float* x, int64_t count, hipStream_t st);
void device_pivots(const float* proj, int64_t n, int s, hipStream_t st, std::vector<float>* pivots,
                   double* max_norm);
void device_ball_summaries(const float* proj, const int32_t* perm, const std::vector<int64_t>& p0,
                           const std::vector<int64_t>& p1, const float* pivots, int s,
                           hipStream_t st, std::vector<float>* centre, std::vector<double>* radius,
                           std::vector<double>* ring);

// Bulk-loads the tree over the device projection proj (n x MP, original
// order) from the leaf order (host perm, and its device copy perm_dev) and
// the split tree of device_split.
void build_tree(const float* proj, int64_t n, int leaf_size, int fanout, int num_pivots,
                std::vector<int32_t> perm, const int32_t* perm_dev,
                const std::vector<SplitNode>& split, hipStream_t st, HostTree* out);

// ---------------------------------------------------------------- index
struct DeviceTree {
    float* centre = nullptr;
    float* radius = nullptr;
    float* hr_min = nullptr;
    float* hr_max = nullptr;
    int32_t* child_begin = nullptr;
    int32_t* child_end = nullptr;
    int32_t* npts = nullptr;
    float* pivots = nullptr;
};

}  // namespace pmlsh

struct pmlsh_index {
    int64_t n = 0;
    int d = 0, d_pad = 0, m = 0;
    int leaf_size = 0, fanout = 0, num_pivots = 0, levels = 0;
    int64_t n_leaves = 0, n_nodes = 0;
    int device = 0;
    // device buffers, all in leaf order
    float* data = nullptr;       // n x d_pad, zero padded
    float* proj_hi = nullptr;    // n x MP: FP32 rounding of the FP64 projection
    float* proj_lo = nullptr;    // n x MP: FP32 rounding of (projection - hi)
    uint16_t* proj16 = nullptr;  // n_pad16 x kScanRow FP16 rows of the matrix-core scan
    int64_t n_pad16 = 0;         // n rounded up to 64
    float scale16 = 1.f;         // power-of-two scale s of those rows
    float* chunk_cen = nullptr;  // n_pad16 / 64 x MP: centre of each 64-point chunk
    float* chunk_rad = nullptr;  // n_pad16 / 64: radius covering the chunk's points
    uint16_t* data16 = nullptr;  // n x d16 FP16 copy of D_leaf, rows scaled by a power of two
    float* data16_scale = nullptr;  // n: that power of two
    float* data16_eps = nullptr;    // n: bound on |row - scale * FP16 row|
    int d16 = 0;                    // d rounded up to a multiple of 8
    int32_t* perm = nullptr;     // leaf position -> id
    int32_t* inv_perm = nullptr; // id -> leaf position
    float* hash = nullptr;       // MP x d, zero rows beyond m
    pmlsh::DeviceTree tree;
    int64_t device_bytes = 0;
    // host copies
    std::vector<int64_t> level_begin;
    std::vector<int32_t> perm_host;
    std::vector<double> sample_sorted;   // ascending pair distances (r_min rule)
    double kappa = 0.9;
    float coord_scale = 0.f;
    // projection behind the scan rows (0: the FP64 one; else the FP16/BF16
    // matrix-core one), the largest bound of its points and the bound on the
    // norm of every scan-row projection (coord_scale + eps_max)
    int filter_gemm = 0;
    float eps_max = 0.f;
    float scan_scale = 0.f;      // bound on |o' - scan_centre| over the scan rows
    float scan_centre[pmlsh::MP] = {};  // centre of the scan rows (mean projected point)
    // (c,k)-ACP workspace kept between calls: one device buffer per role,
    // grown on demand, freed with the index; calls on one index serialise on
    // the mutex
    mutable std::mutex acp_mu;
    mutable std::vector<std::pair<void*, size_t>> acp_bufs;
    // pinned host staging of the ACP calls' small device-to-host reads
    mutable void* acp_host = nullptr;
    // FindLCA's gamma at Pr(gamma) = 0.85 (a fixed sample of the index, so
    // computed once), 0 until the first call that estimates it
    mutable double acp_gamma085 = 0.0;
};

namespace pmlsh {

// ---------------------------------------------------------------- timing
bool timing_enabled(int stage);
// process-wide switches of pmlsh_tune
int64_t tune_default(int key);
int64_t tune_get(int key);
void tune_set(int key, int64_t value);
void timing_set(unsigned stage_mask);
void timing_read(pmlsh_ann_timing* out, bool reset);

// While an object of this class lives, StageTimer on the same thread times
// nothing (no events are created or recorded).
class TimingOff {
public:
    TimingOff();
    ~TimingOff();
    TimingOff(const TimingOff&) = delete;
    TimingOff& operator=(const TimingOff&) = delete;

private:
    bool prev_;
};

// Brackets the launches issued during its lifetime with HIP events when
// per-stage timing is enabled.
class StageTimer {
public:
    StageTimer(int stage, hipStream_t st);
    ~StageTimer();
    StageTimer(const StageTimer&) = delete;
    StageTimer& operator=(const StageTimer&) = delete;

private:
    int stage_;
    hipStream_t st_;
    bool on_ = false;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// ---------------------------------------------------------------- kernels
// Launch wrappers (defined in the .hip translation units). All take the
// stream the work is enqueued on and throw on launch failure.
void launch_project(const float* x, int64_t rows, int d, int64_t ld,
                    const float* hash, float* out_hi, float* out_lo,
                    hipStream_t stream);
void launch_gather_rows(const float* src, int d, int64_t ld_src, const int32_t* perm,
                        int64_t rows, float* dst, int d_pad, hipStream_t stream);
void launch_gather_proj(const float* src, const int32_t* perm, int64_t rows,
                        float* dst, hipStream_t stream);
// Low-precision projection (FP16 or BF16 inputs, FP32 accumulation) of rows
// x (stride ld) with its per-row bound eps (mode: PMLSH_FILTER_GEMM_*).
void launch_project_lp(const float* x, int64_t rows, int d, int64_t ld, const float* hash,
                       int mode, float* out, float* eps, hipStream_t stream);
void launch_augment16(const float* proj, int64_t n, int64_t n_pad, float s, float cm, const float* centre,
                      uint16_t* out, hipStream_t stream);
void launch_half_rows(const float* data, int64_t n, int d_pad, int d16, uint16_t* out,
                      float* scale, float* eps, hipStream_t stream);
void launch_pair_dist_f64(const float* x, int d, int64_t ld, const int64_t* pairs,
                          int64_t count, double* out, hipStream_t stream);

struct AnnLaunch {
    const pmlsh_index* idx;
    const float* queries;   // nq x d (caller layout)
    const float* qproj;     // nq x MP
    const float* qproj_lo;  // nq x MP: FP32 rounding of (projection - qproj)
    int64_t nq;
    int k;
    double c, t, r_min;
    int max_rounds;         // range queries per query at most (0: no limit)
    int64_t budget;
    int32_t* ws_front;      // front_slots x 2 x n_leaves: frontier lists of the tree walk
    int64_t front_slots;    // workgroups of the per-query kernel (one frontier pair each)
    int32_t* ws_cpos;       // nq x budget
    float* ws_cdist;        // nq x budget
    float* ws_clo;          // nq x budget: lower bounds of the verified distances
    int32_t* ws_topk;       // nq x 3 x k
    // leaf-major fast path, per query
    int32_t* q_flag;
    uint32_t* l_count;
    uint32_t* q_scanned;
    uint32_t* pq_list;      // count, then the queries flagged for the per-query kernel
    uint32_t* l_list;       // nq x pool_cap leaf positions (candidate pool)
    uint16_t* ws_qaug;      // nq x 32 FP16 query rows of the matrix-core scan
    float* ws_qlp;          // nq x MP low-precision query projections (filter_gemm), or null
    float* ws_qeps;         // nq: their bounds
    float2* ws_qtest;       // nq: radius and margin of each query's chunk-ball test
    uint64_t* ws_cmask;     // the same, chunk-major in blocks of 256 chunks x ceil(nq / 64) words
    uint16_t* ws_cdist2;    // squared distances to the chunk centres (bf16, rounded down), in
                            // blocks of 64 queries x 64 chunks
    uint16_t* ws_cgmin;     // nq x cdist_gmin_len: their minimum per group of 64 chunks
    int64_t pool_cap;       // candidate region per query
    int64_t* out_ids;
    float* out_dist;
    int32_t* out_stats;
    const AnnQueryParams* qpar = nullptr;   // per-query parameters (then k, budget: the largest)
    int out_stride = 0;                     // output row stride (0: k)
    bool fast = false;                      // the batched path (its workspace fields are set)
};
void launch_ann(const AnnLaunch& a, hipStream_t stream);
int ann_lds_bytes(int d_pad);
int64_t ann_pool_per_query(int64_t n);
bool ann_fast_path(int64_t budget);

}  // namespace pmlsh
