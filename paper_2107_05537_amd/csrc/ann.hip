// (c,k)-ANN query kernel (gfx950): Algorithm 2 of PM-LSH, one workgroup per
// query, all rounds on the device.
//
// Per round i (radius r_i = r_min * c^i):
//   1. from the second round on, count the verified candidates within c*r_i
//      of q and stop when there are at least k (the stopping test of Algorithm 2);
//   2. walk the flattened PM-tree level by level, keeping the nodes that pass
//      the PM-tree access test of Eq. 5 for the range query (q', t*r_i); the
//      surviving leaves go to a per-query list in global memory;
//   3. scan those leaves: every point of the new shell t*r_{i-1} < pd <= t*r_i
//      is counted and histogrammed on its 64-bit key (pd^2 bits, id);
//   4. if the ball holds at least B points, the B - |C| smallest keys of the
//      shell are added to C (exact radix select, see block_select); otherwise
//      the whole shell is added and r grows by c;
//   5. the new members of C are verified: exact FP32 squared distance to q,
//      by direct differences (never by the |q|^2 + |o|^2 - 2 q.o expansion).
// The answer is the k members of C with the smallest (distance, id).
//
// Candidate membership and ordering are decided on bit patterns of FP32 values
// computed by one inlined routine with explicit fused multiply-adds, so every
// scan pass recomputes bit-identical projected distances and the counts of
// different passes agree exactly.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstddef>
#include <cstdint>

#include "internal.hpp"

namespace pmlsh {
namespace {

constexpr int WG = 256;
constexpr int NWAVE = WG / 64;
constexpr int NB = 2048;    // histogram bins of one radix-select step
constexpr int CAP = 2048;   // keys sorted in LDS at once (power of two)
static_assert(kSelCap * 64 >= 2 * CAP + 64, "the chosen-chunk list must hold 2 * budget points");
constexpr int MAX_LEVELS = 16;
constexpr int MAX_ROUNDS = 1000;
constexpr int64_t kScanBlocks = 1024;   // scan workgroups if the occupancy query fails

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

struct AnnArgs {
    const float* data;
    const float* proj;
    const int32_t* perm;
    const float* ncen;
    const float* nrad;
    const float* hrmin;
    const float* hrmax;
    const int32_t* cb;
    const int32_t* ce;
    const int32_t* npts;
    const float* piv;
    int64_t n_nodes;
    int64_t n_leaves;
    int levels;
    int s;
    int d, d_pad;
    int32_t level_begin[MAX_LEVELS + 1];
    float coord_scale;
    float scan_scale;           // bound on |o' - scen| over the scan rows
    float scen[MP];             // centre of the scan rows
    const float* qlp;           // low-precision query projections of the filter, or null
    const float* qeps;          // their bounds
    float eps_max;              // largest bound of the points' scan-row projections
    const float* q;
    const float* qp;
    const float* qp_lo;         // FP32 rounding of (projection - qp)
    const float* proj_lo;       // the same for the data, leaf order
    // Algorithm 2's parameters, the same for every query of the launch, or
    // per query from qpar (then k and budget here are the largest of the
    // launch and serve as strides of the per-query workspace)
    int k;
    int32_t budget;
    double c, t, r_min;
    const AnnQueryParams* qpar;
    int out_stride;             // row stride of out_ids / out_dist (>= every k)
    int max_rounds;             // range queries per query at most ((r,c)-BC: 1)
    int32_t* ws_front;
    int32_t* ws_cpos;
    float* ws_cdist;
    int32_t* ws_topk;
    int64_t* out_ids;
    float* out_dist;
    int32_t* out_stats;
    // leaf-major fast path (per query): radius bound, its square and test
    // slack, fallback flag, candidate count, scanned points, candidate list
    int32_t* q_flag;
    uint32_t* pq_list;          // count, then the queries flagged for the per-query kernel
    uint32_t* l_count;          // candidates per query
    uint32_t* q_scanned;
    uint32_t* l_list;           // nq x q_cap leaf positions (candidate pool)
    int q_cap;
    int nq;
    int64_t n;
    // matrix-core scan: FP16 point rows, their count (padded to 64), scale,
    // and the per-query FP16 rows
    const uint16_t* proj16;
    int64_t n_pad16;
    float scale16;
    uint16_t* qaug;
    // chunk balls, and per query the radius tq of their test (Eq. 5) and
    // the margin of the stored squared distances, from the bound kernel
    const float* chunk_cen;
    const float* chunk_rad;
    float2* qtest;
    // the same mask chunk-major, in blocks of 256 chunks: word (chunk c, query
    // band qb) at cmask_at(c, qb), cwords = ceil(nq / 64) bands
    uint64_t* cmask;
    int cwords;
    // squared distances from every query to every chunk centre, as bf16 bit
    // patterns rounded toward zero (lower bounds), in blocks of 64 queries x
    // 64 chunks (cdist_at); the minimum of each group of 64 chunks (row
    // stride gld)
    uint16_t* cdist;
    uint16_t* cgmin;
    int64_t cgroups, gld;
    int glds;                   // bound kernel: group minima copied to LDS
    int grp_cap;                // bound kernel: most groups or blocks listed (<= kGrpCap)
    // bounded verification: FP16 rows (stride d16), their scales and error
    // bounds, and per C member a lower bound of its squared distance (the
    // upper bound goes to ws_cdist; equal bounds mean the exact value)
    const uint16_t* data16;
    const float* d16_scale;
    const float* d16_eps;
    int d16;
    float* ws_clo;
};

// Element (query q, chunk c) of the blocked chunk-distance matrix.
__device__ __forceinline__ int64_t cdist_at(const AnnArgs& a, int64_t q, int64_t c) {
    return (((q >> 6) * a.cgroups + (c >> 6)) << 12) + ((q & 63) << 6) + (c & 63);
}

// Mask word of chunk c and query band qb (queries 64 qb .. 64 qb + 63): the
// 256 words of one band and one block of 256 chunks are contiguous.
__device__ __forceinline__ int64_t cmask_at(const AnnArgs& a, int64_t c, int64_t qb) {
    return (((c >> 8) * a.cwords + qb) << 8) + (c & 255);
}

// skey and spos come last: the bound kernel uses only the fields before
// them and keeps its row of centre distances in their place.
struct Smem {
    uint32_t hist[NB];
    int32_t red[NWAVE * 2];
    int32_t cnt0, cnt1, cnt2;
    int32_t thr_bin, thr_below, thr_in;
    int32_t pad_[2];
    uint64_t skey[CAP];
    int32_t spos[CAP];
};
static_assert(offsetof(Smem, skey) % 16 == 0, "row area must be 16-byte aligned");

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// The parameters of query qi of the launch.
__device__ __forceinline__ AnnQueryParams query_params(const AnnArgs& a, int64_t qi) {
    if (a.qpar) return a.qpar[qi];
    AnnQueryParams p;
    p.c = a.c;
    p.t = a.t;
    p.r_min = a.r_min;
    p.k = a.k;
    p.budget = a.budget;
    return p;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

// Slot for each lane with take == true, one LDS atomic per wave.
__device__ __forceinline__ int wave_append(bool take, int32_t* counter) {
    const uint64_t m = __ballot(take);
    if (m == 0) return -1;
    const int leader = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    return base + __popcll(m & lanemask_lt());
}

__device__ __forceinline__ int block_sum(int v, Smem& sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane_id() == 0) sh.red[threadIdx.x >> 6] = v;
    __syncthreads();
    int s = 0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) s += sh.red[w];
    __syncthreads();
    return s;
}

// Exclusive prefix sum over the workgroup.
__device__ __forceinline__ int block_exclusive_scan(int v, Smem& sh) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh.red[NWAVE + wave] = x;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += sh.red[NWAVE + w];
    __syncthreads();
    return before + x - v;
}

// Squared projected distance, always the same operation sequence.
__device__ __forceinline__ float proj_dist2(const float* __restrict__ o, const float* qp) {
    const float4* o4 = reinterpret_cast<const float4*>(o);
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < MP / 4; ++j) {
        const float4 v = o4[j];
        float t;
        t = __fsub_rn(qp[4 * j + 0], v.x); acc = __fmaf_rn(t, t, acc);
        t = __fsub_rn(qp[4 * j + 1], v.y); acc = __fmaf_rn(t, t, acc);
        t = __fsub_rn(qp[4 * j + 2], v.z); acc = __fmaf_rn(t, t, acc);
        t = __fsub_rn(qp[4 * j + 3], v.w); acc = __fmaf_rn(t, t, acc);
    }
    return acc;
}

__device__ __forceinline__ float node_dist(const AnnArgs& a, int node, const float* qp) {
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
        const float t = qp[j] - a.ncen[(int64_t)j * a.n_nodes + node];
        acc = fmaf(t, t, acc);
    }
    return sqrtf(acc);
}

// Eq. 5: the node is accessed iff its covering ball and every pivot ring can
// hold a point within R of q'. `slack` absorbs FP32 rounding (conservative).
// All of the node's data is loaded before any test, so the loads overlap.
__device__ __forceinline__ bool node_pass(const AnnArgs& a, int node, const float* qp,
                                          const float* qpiv, float R, float slack) {
    float hmn[PMLSH_MAX_PIVOTS], hmx[PMLSH_MAX_PIVOTS];
#pragma unroll
    for (int i = 0; i < PMLSH_MAX_PIVOTS; ++i) {
        hmn[i] = hmx[i] = 0.f;
        if (i < a.s) {
            hmn[i] = a.hrmin[(int64_t)i * a.n_nodes + node];
            hmx[i] = a.hrmax[(int64_t)i * a.n_nodes + node];
        }
    }
    const float rad = a.nrad[node];
    bool pass = node_dist(a, node, qp) <= rad + R + slack;
#pragma unroll
    for (int i = 0; i < PMLSH_MAX_PIVOTS; ++i)
        if (i < a.s)
            pass = pass & (qpiv[i] - R <= hmx[i] + slack) & (qpiv[i] + R >= hmn[i] - slack);
    return pass;
}

__device__ __forceinline__ int shift_for(uint64_t lo, uint64_t hi) {
    const uint64_t span = hi - lo;
    if (span < (uint64_t)NB) return 0;
    const int bits = 64 - __clzll((long long)span);
    return bits - 11;
}

__device__ __forceinline__ void clear_hist(Smem& sh) {
    for (int i = threadIdx.x; i < NB; i += WG) sh.hist[i] = 0;
    __syncthreads();
}

// Finds the bin where the running count of the histogram reaches `need`.
__device__ void find_threshold(int need, Smem& sh) {
    constexpr int PER = NB / WG;
    const int base = threadIdx.x * PER;
    int local[PER];
    int s = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) { local[j] = (int)sh.hist[base + j]; s += local[j]; }
    const int excl = block_exclusive_scan(s, sh);
    if (excl < need && excl + s >= need) {
        int acc = excl;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (acc + local[j] >= need) {
                sh.thr_bin = base + j;
                sh.thr_below = acc;
                sh.thr_in = local[j];
                break;
            }
            acc += local[j];
        }
    }
    __syncthreads();
}

// Histogram bin of a non-negative radius below R: 256 bins per octave over
// [R / 2^8, R], everything smaller in bin 0.
__device__ __forceinline__ int radius_bin(float v, uint32_t base) {
    const uint32_t b = __float_as_uint(v) >> 15;
    return b <= base ? 0 : (int)(b - base);
}

// Level-by-level traversal with Eq. 5; returns the number of leaves that pass
// and leaves their ids in fa (the first of the two per-query buffers).
//
// With `shrink`, the radius R (in/out) is lowered level by level to an upper
// bound tau on the budget-th smallest projected distance: the passing nodes
// whose every point lies within dist(q', centre) + radius <= tau hold at least
// `budget` points. Then every point of the final ball of radius tau lies in a
// kept leaf, the ball holds at least `budget` points, and its `budget`
// nearest points are those of the ball of the original radius.
__device__ int traverse(const AnnArgs& a, const float* qp, const float* qpiv, float& R,
                        float slack, bool shrink, int budget, int32_t* fa, int32_t* fb,
                        Smem& sh) {
    int ncur = a.level_begin[1] - a.level_begin[0];
    for (int l = 0; l < a.levels; ++l) {
        const bool leaf_level = (l == a.levels - 1);
        // A: test the candidates of this level at R; the passing ones go to fb
        if (threadIdx.x == 0) sh.cnt0 = 0;
        __syncthreads();
        for (int base = 0; base < ncur; base += WG) {
            const int i = base + threadIdx.x;
            bool pass = false;
            int node = 0;
            if (i < ncur) {
                node = (l == 0) ? a.level_begin[0] + i : fa[i];
                // entries always lie in this level; the check only keeps a
                // corrupted list from reading outside the node arrays
                if (node >= a.level_begin[l] && node < a.level_begin[l + 1])
                    pass = node_pass(a, node, qp, qpiv, R, slack);
            }
            const int slot = wave_append(pass, &sh.cnt0);
            if (pass && slot < a.n_leaves) fb[slot] = node;
        }
        __syncthreads();
        const int np = sh.cnt0 < a.n_leaves ? sh.cnt0 : (int)a.n_leaves;
        __syncthreads();
        // B: weighted histogram of the nodes' distance upper bounds -> tau
        float Rn = R;
        if (shrink) {
            const uint32_t hb = __float_as_uint(R) >> 15;
            const uint32_t base = hb > (uint32_t)(NB - 1) ? hb - (uint32_t)(NB - 1) : 0u;
            clear_hist(sh);
            int loc = 0;
            for (int i = threadIdx.x; i < np; i += WG) {
                const int node = fb[i];
                const float ub = node_dist(a, node, qp) + a.nrad[node] + slack;
                if (ub <= R) {
                    atomicAdd(&sh.hist[radius_bin(ub, base)], (uint32_t)a.npts[node]);
                    loc += a.npts[node];
                }
            }
            __syncthreads();
            if (block_sum(loc, sh) >= budget) {
                if (threadIdx.x == 0) sh.thr_bin = NB - 1;
                __syncthreads();
                find_threshold(budget, sh);
                // upper edge of the threshold bin: every counted ub is below it
                const float tau = __uint_as_float((base + (uint32_t)sh.thr_bin + 1u) << 15);
                Rn = tau < R ? tau : R;
            }
            __syncthreads();
        }
        // C: keep what passes at the lowered radius; expand inner nodes into fa
        if (threadIdx.x == 0) sh.cnt1 = 0;
        __syncthreads();
        for (int base = 0; base < np; base += WG) {
            const int i = base + threadIdx.x;
            bool keep = false;
            int node = 0;
            if (i < np) {
                node = fb[i];
                keep = Rn == R || node_pass(a, node, qp, qpiv, Rn, slack);
            }
            if (leaf_level) {
                const int slot = wave_append(keep, &sh.cnt1);
                if (keep && slot < a.n_leaves) fa[slot] = node;
            } else if (keep) {
                const int b = a.cb[node], e = a.ce[node];
                const int slot = atomicAdd(&sh.cnt1, e - b);
                if (slot + (e - b) <= a.n_leaves)
                    for (int j = b; j < e; ++j) fa[slot + (j - b)] = j;
            }
        }
        __syncthreads();
        ncur = sh.cnt1 < a.n_leaves ? sh.cnt1 : (int)a.n_leaves;
        R = Rn;
        __syncthreads();
    }
    return ncur;
}

// Calls f(valid, pos, pd2) for every point of the listed leaves; wave-uniform.
template <class F>
__device__ __forceinline__ void scan_leaves(const AnnArgs& a, const int32_t* leaves, int nl,
                                            const float* qp, F&& f) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    for (int li = wave; li < nl; li += NWAVE) {
        const int leaf = leaves[li];
        const int p0 = a.cb[leaf], p1 = a.ce[leaf];
        for (int base = p0; base < p1; base += 64) {
            const int pos = base + lane;
            const bool valid = pos < p1;
            const float pd2 = valid ? proj_dist2(a.proj + (int64_t)pos * MP, qp) : FLT_MAX;
            f(valid, pos, pd2);
        }
    }
}

__device__ void bitonic_sort(int count, Smem& sh) {
    int P = 1;
    while (P < count) P <<= 1;
    for (int i = count + threadIdx.x; i < P; i += WG) { sh.skey[i] = ~0ull; sh.spos[i] = -1; }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += WG) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t x = sh.skey[i], y = sh.skey[ixj];
                    if ((x > y) == up) {
                        sh.skey[i] = y; sh.skey[ixj] = x;
                        const int32_t t = sh.spos[i]; sh.spos[i] = sh.spos[ixj]; sh.spos[ixj] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// The need-th smallest (need in [1, n]) of the n <= CAP distinct 64-bit keys
// in sh.skey: NB-bin histogram passes over LDS, each narrowing the key range
// to the bin that holds it.
__device__ uint64_t lds_select(int n, int need, Smem& sh) {
    uint64_t lo = ~0ull, hi = 0ull;
    for (int i = threadIdx.x; i < n; i += WG) {
        const uint64_t k = sh.skey[i];
        lo = k < lo ? k : lo;
        hi = k > hi ? k : hi;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t l2 = __shfl_xor(lo, off), h2 = __shfl_xor(hi, off);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
    }
    uint64_t* red = reinterpret_cast<uint64_t*>(sh.hist);
    if (lane_id() == 0) {
        red[threadIdx.x >> 6] = lo;
        red[NWAVE + (threadIdx.x >> 6)] = hi;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) {
        lo = red[w] < lo ? red[w] : lo;
        hi = red[NWAVE + w] > hi ? red[NWAVE + w] : hi;
    }
    __syncthreads();
    for (;;) {
        const int sft = shift_for(lo, hi);
        clear_hist(sh);
        for (int i = threadIdx.x; i < n; i += WG) {
            const uint64_t k = sh.skey[i];
            if (k >= lo && k <= hi) atomicAdd(&sh.hist[(int)((k - lo) >> sft)], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) sh.thr_bin = NB - 1;
        __syncthreads();
        find_threshold(need, sh);
        const int T = sh.thr_bin, below = sh.thr_below, inT = sh.thr_in;
        const uint64_t nlo = lo + ((uint64_t)T << sft);
        const uint64_t span = (1ull << sft) - 1ull;
        const uint64_t nhi = hi - nlo > span ? nlo + span : hi;
        __syncthreads();
        if (sft == 0) return nlo;
        if (inT == 1) {
            // the bin holds one key: that key
            for (int i = threadIdx.x; i < n; i += WG) {
                const uint64_t k = sh.skey[i];
                if (k >= nlo && k <= nhi) red[0] = k;
            }
            __syncthreads();
            const uint64_t key = red[0];
            __syncthreads();
            return key;
        }
        need -= below;
        lo = nlo;
        hi = nhi;
    }
}

// Exact selection of the `need` smallest 64-bit keys among the members of a
// source with key in [lo, hi] (radix select with NB-bin steps). src(v) calls
// v(valid, key, payload) wave-uniformly over all members; emit(payload, slot)
// receives every selected payload exactly once, slot in [0, need).
// If hist_ready, sh.hist already holds the histogram of [lo, hi] at
// shift_for(lo, hi) and `total` is the member count in [lo, hi].
template <class Src, class Emit>
__device__ void block_select(Src&& src, Emit&& emit, uint64_t lo, uint64_t hi, int need,
                             bool hist_ready, int total, Smem& sh) {
    int emitted = 0;
    for (;;) {
        const int shift = shift_for(lo, hi);
        if (!hist_ready) {
            clear_hist(sh);
            src([&](bool valid, uint64_t key, int32_t) {
                if (valid && key >= lo && key <= hi) atomicAdd(&sh.hist[(key - lo) >> shift], 1u);
            });
            __syncthreads();
            int loc = 0;
            for (int i = threadIdx.x; i < NB; i += WG) loc += (int)sh.hist[i];
            total = block_sum(loc, sh);
        }
        hist_ready = false;
        if (total <= CAP) {
            if (threadIdx.x == 0) sh.cnt1 = 0;
            __syncthreads();
            src([&](bool valid, uint64_t key, int32_t payload) {
                const bool take = valid && key >= lo && key <= hi;
                const int slot = wave_append(take, &sh.cnt1);
                if (take && slot < CAP) { sh.skey[slot] = key; sh.spos[slot] = payload; }
            });
            __syncthreads();
            bitonic_sort(total, sh);
            for (int i = threadIdx.x; i < need; i += WG) emit(sh.spos[i], emitted + i);
            __syncthreads();
            return;
        }
        if (threadIdx.x == 0) { sh.thr_bin = NB - 1; sh.thr_below = 0; sh.thr_in = 0; }
        __syncthreads();
        find_threshold(need, sh);
        const int T = sh.thr_bin, below = sh.thr_below, inT = sh.thr_in;
        if (threadIdx.x == 0) { sh.cnt1 = 0; sh.cnt2 = 0; }
        __syncthreads();
        const bool gather_T = inT <= CAP;
        src([&](bool valid, uint64_t key, int32_t payload) {
            const bool in = valid && key >= lo && key <= hi;
            const int bin = in ? (int)((key - lo) >> shift) : NB;
            const bool lower = in && bin < T;
            const int s1 = wave_append(lower, &sh.cnt1);
            if (lower && s1 < below) emit(payload, emitted + s1);
            const bool at = gather_T && in && bin == T;
            const int s2 = wave_append(at, &sh.cnt2);
            if (at && s2 < CAP) { sh.skey[s2] = key; sh.spos[s2] = payload; }
        });
        __syncthreads();
        emitted += below;
        need -= below;
        if (gather_T) {
            bitonic_sort(inT, sh);
            for (int i = threadIdx.x; i < need; i += WG) emit(sh.spos[i], emitted + i);
            __syncthreads();
            return;
        }
        const uint64_t nlo = lo + ((uint64_t)T << shift);
        const uint64_t nhi = nlo + ((1ull << shift) - 1ull);
        lo = nlo;
        hi = nhi < hi ? nhi : hi;
    }
}

// Exact squared distances of C entries [v0, v1): 16 lanes per row, each
// 16-lane group keeping VR rows in flight (VR independent loads per column
// step) so the gather of 1 KB rows runs at HBM rate rather than at latency.
constexpr int VR = 4;

__device__ void verify(const AnnArgs& a, const float* qs, const int32_t* cpos, float* cdist,
                       int v0, int v1) {
    const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int d4 = a.d_pad >> 2;
    const float4* q4 = reinterpret_cast<const float4*>(qs);
    constexpr int GROUPS = WG / 16;
    for (int base = v0; base < v1; base += GROUPS * VR) {
        const float4* row[VR];
        bool ok[VR];
        float acc[VR];
#pragma unroll
        for (int r = 0; r < VR; ++r) {
            const int i = base + g + GROUPS * r;
            ok[r] = i < v1;
            row[r] = reinterpret_cast<const float4*>(a.data + (int64_t)cpos[ok[r] ? i : v0] * a.d_pad);
            acc[r] = 0.f;
        }
#pragma unroll 2
        for (int c = l16; c < d4; c += 16) {
            float4 x[VR];
#pragma unroll
            for (int r = 0; r < VR; ++r) x[r] = row[r][c];
            const float4 y = q4[c];
#pragma unroll
            for (int r = 0; r < VR; ++r) {
                float t;
                t = y.x - x[r].x; acc[r] = __fmaf_rn(t, t, acc[r]);
                t = y.y - x[r].y; acc[r] = __fmaf_rn(t, t, acc[r]);
                t = y.z - x[r].z; acc[r] = __fmaf_rn(t, t, acc[r]);
                t = y.w - x[r].w; acc[r] = __fmaf_rn(t, t, acc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < VR; ++r) {
            float v = acc[r];
            v += __shfl_xor(v, 8, 16);
            v += __shfl_xor(v, 4, 16);
            v += __shfl_xor(v, 2, 16);
            v += __shfl_xor(v, 1, 16);
            if (ok[r] && l16 == 0) cdist[base + g + GROUPS * r] = v;
        }
    }
}

// Exact squared distances (same operation sequence as verify) of the C
// members listed in idx[0, cnt); both bounds of each become the exact value.
__device__ void verify_list(const AnnArgs& a, const float* qs, const int32_t* cpos,
                            const int32_t* idx, int cnt, float* lo2, float* hi2) {
    const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int d4 = a.d_pad >> 2;
    const float4* q4 = reinterpret_cast<const float4*>(qs);
    constexpr int GROUPS = WG / 16;
    for (int base = 0; base < cnt; base += GROUPS * VR) {
        const float4* row[VR];
        bool ok[VR];
        float acc[VR];
        int mi[VR];
#pragma unroll
        for (int r = 0; r < VR; ++r) {
            const int j = base + g + GROUPS * r;
            ok[r] = j < cnt;
            mi[r] = idx[ok[r] ? j : 0];
            row[r] = reinterpret_cast<const float4*>(a.data + (int64_t)cpos[mi[r]] * a.d_pad);
            acc[r] = 0.f;
        }
        // two words of every row per lane and step, all loads issued before
        // the first use; the operations and their order are those of verify
        for (int c0 = l16; c0 < d4; c0 += 32) {
            float4 x[VR][2];
#pragma unroll
            for (int r = 0; r < VR; ++r) {
                x[r][0] = row[r][c0];
                x[r][1] = c0 + 16 < d4 ? row[r][c0 + 16] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int c = c0 + 16 * u;
                if (u == 1 && c >= d4) break;
                const float4 y = q4[c];
#pragma unroll
                for (int r = 0; r < VR; ++r) {
                    float t;
                    t = y.x - x[r][u].x; acc[r] = __fmaf_rn(t, t, acc[r]);
                    t = y.y - x[r][u].y; acc[r] = __fmaf_rn(t, t, acc[r]);
                    t = y.z - x[r][u].z; acc[r] = __fmaf_rn(t, t, acc[r]);
                    t = y.w - x[r][u].w; acc[r] = __fmaf_rn(t, t, acc[r]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < VR; ++r) {
            float v = acc[r];
            v += __shfl_xor(v, 8, 16);
            v += __shfl_xor(v, 4, 16);
            v += __shfl_xor(v, 2, 16);
            v += __shfl_xor(v, 1, 16);
            if (ok[r] && l16 == 0) {
                lo2[mi[r]] = v;
                hi2[mi[r]] = v;
            }
        }
    }
}

// Bounds on the exact FP32 squared distance (the value verify would compute)
// of C members [v0, v1), from the FP16 rows: with D16 the distance to the
// FP16 row (accumulated in FP32 like verify, relative error <= gamma) and eps
// the row's bound |x - s x16|, the true distance lies in [D16 - eps, D16 +
// eps] and the FP32 value within a further factor (1 +- gamma); every
// rounding of the bound arithmetic is covered by extra factors of a few u.
__device__ void verify16(const AnnArgs& a, const float* qs, const int32_t* cpos,
                         float* lo2, float* hi2, int v0, int v1) {
    const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int d8 = a.d16 >> 3;
    constexpr int GROUPS = WG / 16;
    const float u = 5.9604645e-08f;
    const float gam = 2.f * u * (float)(a.d16 / 16 + 8);
    for (int base = v0; base < v1; base += GROUPS * VR) {
        const uint4* row[VR];
        bool ok[VR];
        float acc[VR], sc[VR];
        int pr[VR];
#pragma unroll
        for (int r = 0; r < VR; ++r) {
            const int i = base + g + GROUPS * r;
            ok[r] = i < v1;
            pr[r] = cpos[ok[r] ? i : v0];
            row[r] = reinterpret_cast<const uint4*>(a.data16 + (int64_t)pr[r] * a.d16);
            sc[r] = a.d16_scale[pr[r]];
            acc[r] = 0.f;
        }
        // two 16-byte words of every row per lane and step, all loads issued
        // before the first use (words past the row read as zero halves, and
        // the query's zero padding makes their terms zero)
        for (int c0 = l16; c0 < d8; c0 += 32) {
            uint4 h[VR][2];
#pragma unroll
            for (int r = 0; r < VR; ++r) {
                h[r][0] = row[r][c0];
                h[r][1] = c0 + 16 < d8 ? row[r][c0 + 16] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int c = c0 + 16 * u;
                if (u == 1 && c >= d8) break;
                float y[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) y[e] = qs[8 * c + e];
#pragma unroll
                for (int r = 0; r < VR; ++r) {
                    const uint32_t w[4] = {h[r][u].x, h[r][u].y, h[r][u].z, h[r][u].w};
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const uint16_t bits = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
                        const float xv = (float)__builtin_bit_cast(_Float16, bits);
                        const float t = __fmaf_rn(-sc[r], xv, y[e]);
                        acc[r] = __fmaf_rn(t, t, acc[r]);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < VR; ++r) {
            float v = acc[r];
            v += __shfl_xor(v, 8, 16);
            v += __shfl_xor(v, 4, 16);
            v += __shfl_xor(v, 2, 16);
            v += __shfl_xor(v, 1, 16);
            if (ok[r] && l16 == 0) {
                const float eps = a.d16_eps[pr[r]];
                const float dlo = sqrtf(v * (1.f - gam)) * (1.f - 4.f * u);
                const float dhi = sqrtf(v * (1.f + 2.f * gam)) * (1.f + 4.f * u);
                const float tlo = fmaxf((dlo - eps) * (1.f - 2.f * u), 0.f);
                const float thi = (dhi + eps) * (1.f + 2.f * u);
                lo2[base + g + GROUPS * r] = tlo * tlo * (1.f - gam) * (1.f - 4.f * u);
                hi2[base + g + GROUPS * r] = thi * thi * (1.f + gam) * (1.f + 4.f * u);
            }
        }
    }
}

// Loads the query into LDS (zero padded), its projection and pivot
// distances into registers.
struct QueryCtx {
    float qp[MP];
    float qpiv[PMLSH_MAX_PIVOTS];
    float qn2;
};

__device__ __forceinline__ void load_query(const AnnArgs& a, int64_t qi, float* qs, QueryCtx& c) {
    const float* qrow = a.q + qi * a.d;
    if (qs)
        for (int j = threadIdx.x; j < a.d16; j += WG) qs[j] = j < a.d ? qrow[j] : 0.f;
#pragma unroll
    for (int j = 0; j < MP; ++j) c.qp[j] = a.qp[qi * MP + j];
    c.qn2 = 0.f;
#pragma unroll
    for (int j = 0; j < MP; ++j) c.qn2 = fmaf(c.qp[j], c.qp[j], c.qn2);
#pragma unroll
    for (int i = 0; i < PMLSH_MAX_PIVOTS; ++i) {
        float acc = 0.f;
        if (i < a.s) {
#pragma unroll
            for (int j = 0; j < MP; ++j) {
                const float t = c.qp[j] - a.piv[i * MP + j];
                acc = fmaf(t, t, acc);
            }
        }
        c.qpiv[i] = sqrtf(acc);
    }
}

// Writes the k members of C (the first n_ver entries, n_ver >= k) with the
// smallest (distance^2 bits, id), in that order, and the per-query statistics.
// Relative error bound of the FP32 squared distance that verify computes
// (16 lanes, d_pad / 16 terms each, four shuffle additions).
__device__ __forceinline__ float verify_gamma(const AnnArgs& a) {
    return 2.f * 5.9604645e-08f * (float)(a.d_pad / 16 + 8);
}

constexpr int kRerankCap = 512;   // members the FP64 re-rank takes at most

// FP64 re-rank of the top-k, for near ties of the FP32 distances: every
// member whose exact FP32 squared distance v32 is at most kth32 (1 + 4 gamma),
// kth32 the k-th smallest v32 (+inf with at most k members), gets its squared
// distance in FP64 from its FP32 row; since v32 is within a factor 1 +- gamma
// of that value, no member outside can be among the k nearest in FP64. The k
// smallest (FP64 value, id) are written, each distance as the FP32 rounding
// of the FP64 root. src(j, v32, member) gives the cnt candidates. Returns
// false, writing nothing, when more than kRerankCap members qualify.
template <class Src>
__device__ bool rerank_topk64(const AnnArgs& a, int64_t qi, const float* qs, const int32_t* cpos,
                              int cnt, float kth32, Src&& src, Smem& sh) {
    const int k = query_params(a, qi).k;
    double* d64 = reinterpret_cast<double*>(sh.hist);
    int32_t* mem = reinterpret_cast<int32_t*>(d64 + kRerankCap);
    int32_t* pid = mem + kRerankCap;
    static_assert(NB * sizeof(uint32_t) >= kRerankCap * 16, "re-rank lists must fit the histogram");
    const double lim = (double)kth32 * (1.0 + 4.0 * (double)verify_gamma(a));
    __syncthreads();
    if (threadIdx.x == 0) sh.cnt2 = 0;
    __syncthreads();
    for (int b0 = 0; b0 < cnt; b0 += WG) {
        const int j = b0 + threadIdx.x;
        float v = 0.f;
        int mi = 0;
        if (j < cnt) src(j, v, mi);
        const bool take = j < cnt && (double)v <= lim;
        const int slot = wave_append(take, &sh.cnt2);
        if (take && slot < kRerankCap) {
            mem[slot] = mi;
            pid[slot] = a.perm[cpos[mi]];
        }
    }
    __syncthreads();
    const int np = sh.cnt2;
    if (np > kRerankCap) return false;
    // FP64 squared distances, 16 lanes per member (differences of FP32
    // values are exact in FP64)
    {
        const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
        const int d4 = a.d_pad >> 2;
        const float4* q4 = reinterpret_cast<const float4*>(qs);
        for (int base = 0; base < np; base += WG / 16) {
            const int j = base + g;
            double acc = 0.0;
            if (j < np) {
                const float4* row = reinterpret_cast<const float4*>(a.data + (int64_t)cpos[mem[j]] * a.d_pad);
                // four words per lane and step, loaded before their first use
                for (int c0 = l16; c0 < d4; c0 += 64) {
                    float4 x[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        x[u] = c0 + 16 * u < d4 ? row[c0 + 16 * u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (c0 + 16 * u >= d4) break;
                        const float4 y = q4[c0 + 16 * u];
                        double t;
                        t = (double)y.x - (double)x[u].x; acc = fma(t, t, acc);
                        t = (double)y.y - (double)x[u].y; acc = fma(t, t, acc);
                        t = (double)y.z - (double)x[u].z; acc = fma(t, t, acc);
                        t = (double)y.w - (double)x[u].w; acc = fma(t, t, acc);
                    }
                }
            }
            acc += __shfl_xor(acc, 8, 16);
            acc += __shfl_xor(acc, 4, 16);
            acc += __shfl_xor(acc, 2, 16);
            acc += __shfl_xor(acc, 1, 16);
            if (j < np && l16 == 0) d64[j] = acc;
        }
    }
    __syncthreads();
    // rank by (FP64 value, id); ids are distinct
    for (int j = threadIdx.x; j < np; j += WG) {
        const double v = d64[j];
        const int32_t id = pid[j];
        int rank = 0;
        for (int y = 0; y < np; ++y) rank += d64[y] < v || (d64[y] == v && pid[y] < id);
        if (rank < k) {
            a.out_ids[qi * a.out_stride + rank] = (int64_t)id;
            a.out_dist[qi * a.out_stride + rank] = (float)sqrt(v);
        }
    }
    __syncthreads();
    return true;
}

__device__ void write_topk(const AnnArgs& a, int64_t qi, const float* qs, const int32_t* cpos,
                           const float* cdist, int n_ver, int rounds, int exit_kind,
                           int64_t scanned, Smem& sh) {
    const int32_t* perm = a.perm;
    const int k = query_params(a, qi).k;
    bool done = false;
    if (n_ver <= CAP) {
        // the k-th smallest FP32 value, then the FP64 re-rank
        float kth32 = __int_as_float(0x7f800000);
        if (n_ver > k) {
            for (int i = threadIdx.x; i < n_ver; i += WG)
                sh.skey[i] = ((uint64_t)__float_as_uint(cdist[i]) << 32) | (uint32_t)perm[cpos[i]];
            __syncthreads();
            kth32 = __uint_as_float((uint32_t)(lds_select(n_ver, k, sh) >> 32));
        }
        done = rerank_topk64(a, qi, qs, cpos, n_ver, kth32,
                             [&](int j, float& v, int& mi) { v = cdist[j]; mi = j; }, sh);
    }
    if (done) {
    } else if (n_ver <= CAP) {
        for (int i = threadIdx.x; i < n_ver; i += WG)
            sh.skey[i] = ((uint64_t)__float_as_uint(cdist[i]) << 32) | (uint32_t)perm[cpos[i]];
        __syncthreads();
        int m = n_ver;
        if (n_ver > k) {
            const uint64_t kth = lds_select(n_ver, k, sh);
            // the k smallest keys, gathered through the histogram space
            uint64_t* tmp = reinterpret_cast<uint64_t*>(sh.hist);
            static_assert(NB * sizeof(uint32_t) >= PMLSH_MAX_K * sizeof(uint64_t),
                          "top-k staging must fit the histogram");
            if (threadIdx.x == 0) sh.cnt1 = 0;
            __syncthreads();
            for (int b0 = 0; b0 < n_ver; b0 += WG) {
                const int i = b0 + threadIdx.x;
                const bool take = i < n_ver && sh.skey[i] <= kth;
                const int slot = wave_append(take, &sh.cnt1);
                if (take) tmp[slot] = sh.skey[i];
            }
            __syncthreads();
            for (int j = threadIdx.x; j < k; j += WG) sh.skey[j] = tmp[j];
            __syncthreads();
            m = k;
        }
        bitonic_sort(m, sh);
        for (int j = threadIdx.x; j < k; j += WG) {
            const uint64_t key = sh.skey[j];
            a.out_ids[qi * a.out_stride + j] = (int64_t)(uint32_t)key;
            a.out_dist[qi * a.out_stride + j] = sqrtf(__uint_as_float((uint32_t)(key >> 32)));
        }
    } else {
        auto c_src = [&](auto&& v) {
            for (int base = 0; base < n_ver; base += WG) {
                const int i = base + threadIdx.x;
                const bool valid = i < n_ver;
                uint64_t key = 0;
                if (valid) key = ((uint64_t)__float_as_uint(cdist[i]) << 32) | (uint32_t)perm[cpos[i]];
                v(valid, key, i);
            }
        };
        int32_t* topk = a.ws_topk + qi * 3 * (int64_t)a.k;
        block_select(c_src, [&](int32_t i, int slot) { if (slot < k) topk[slot] = i; }, 0ull,
                     ~0ull, k, false, 0, sh);
        __syncthreads();
        // the k-th smallest FP32 value (the largest of the k selected), then
        // the FP64 re-rank
        float kmax = 0.f;
        for (int j = threadIdx.x; j < k; j += WG) kmax = fmaxf(kmax, cdist[topk[j]]);
        for (int off = 32; off > 0; off >>= 1) kmax = fmaxf(kmax, __shfl_xor(kmax, off));
        if (lane_id() == 0) sh.red[threadIdx.x >> 6] = __float_as_int(kmax);
        __syncthreads();
#pragma unroll
        for (int w = 0; w < NWAVE; ++w) kmax = fmaxf(kmax, __int_as_float(sh.red[w]));
        __syncthreads();
        if (rerank_topk64(a, qi, qs, cpos, n_ver, kmax,
                          [&](int j, float& v, int& mi) { v = cdist[j]; mi = j; }, sh))
            done = true;
    }
    if (!done && n_ver > CAP) {
        const int32_t* topk = a.ws_topk + qi * 3 * (int64_t)a.k;
        for (int j = threadIdx.x; j < k; j += WG) {
            const int i = topk[j];
            sh.skey[j] = ((uint64_t)__float_as_uint(cdist[i]) << 32) | (uint32_t)perm[cpos[i]];
        }
        __syncthreads();
        bitonic_sort(k, sh);
        for (int j = threadIdx.x; j < k; j += WG) {
            const uint64_t key = sh.skey[j];
            a.out_ids[qi * a.out_stride + j] = (int64_t)(uint32_t)key;
            a.out_dist[qi * a.out_stride + j] = sqrtf(__uint_as_float((uint32_t)(key >> 32)));
        }
    }
    if (a.out_stats && threadIdx.x == 0) {
        int32_t* st = a.out_stats + qi * 4;
        st[0] = rounds;
        st[1] = n_ver;
        st[2] = exit_kind;
        st[3] = scanned > 0x7fffffffll ? 0x7fffffff : (int32_t)scanned;
    }
}

__device__ void ann_one(const AnnArgs& a, int64_t qi, int32_t* fa, int32_t* fb, float* qs,
                        Smem& sh);

__global__ __launch_bounds__(WG) void ann_kernel(AnnArgs args) {
    // the argument block read in place (constant memory): naming the
    // parameter itself lets the compiler copy all of it into scratch memory
    (void)args;
    const AnnArgs& a = *(const AnnArgs*)__builtin_amdgcn_kernarg_segment_ptr();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem& sh = *reinterpret_cast<Smem*>(smem_raw);
    float* qs = reinterpret_cast<float*>(smem_raw + ((sizeof(Smem) + 15) & ~size_t(15)));

    // workgroup b answers queries b, b + G, b + 2G, ... with the frontier
    // lists of slot b (G = gridDim.x slots)
    int32_t* fa = a.ws_front + (int64_t)blockIdx.x * 2 * a.n_leaves;
    int32_t* fb = fa + a.n_leaves;
    // every query, or only those the batched path flagged (a.pq_list)
    const int64_t total = a.pq_list ? (int64_t)a.pq_list[0] : a.nq;
    for (int64_t j = blockIdx.x; j < total; j += gridDim.x) {
        __syncthreads();
        ann_one(a, a.pq_list ? (int64_t)a.pq_list[1 + j] : j, fa, fb, qs, sh);
    }
}

// The budget cut of the per-query path in the FP64 order, as cut_fp64 does
// for the batched path: the need members chosen from the shell (FP32 keys,
// in cpos[n_ver, n_ver + need)) are replaced by the shell's entries below a
// band of 2E around the largest chosen FP32 pd^2 and the first band entries
// by (FP64 pd^2, id). The band stays inside the shell (entries of earlier
// rounds are in C by ball membership). Nothing changes when the band holds
// more than 512 entries.
template <class BallSrc>
__device__ void shell_cut_fp64(const AnnArgs& a, int64_t qi, const QueryCtx& qc, BallSrc& ball_src,
                               uint32_t lo_hi, int n_ver, int need, int32_t* cpos, Smem& sh) {
    constexpr int kBandCap = 512;
    int32_t* bpos = reinterpret_cast<int32_t*>(sh.hist);
    uint32_t* bid = reinterpret_cast<uint32_t*>(sh.hist + kBandCap);
    double* b64 = reinterpret_cast<double*>(sh.hist + 2 * kBandCap);
    static_assert(NB >= 4 * kBandCap, "the band must fit the histogram");
    // the largest FP32 pd^2 among the chosen
    float kmax = 0.f;
    for (int j = threadIdx.x; j < need; j += WG)
        kmax = fmaxf(kmax, proj_dist2(a.proj + (int64_t)cpos[n_ver + j] * MP, qc.qp));
    for (int off = 32; off > 0; off >>= 1) kmax = fmaxf(kmax, __shfl_xor(kmax, off));
    if (lane_id() == 0) sh.red[threadIdx.x >> 6] = __float_as_int(kmax);
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) kmax = fmaxf(kmax, __int_as_float(sh.red[w]));
    __syncthreads();
    const float big = sqrtf(qc.qn2) + a.coord_scale;
    const float e = 2.f * (2.384185791015625e-07f * sqrtf(kmax) * big + 1.9073486328125e-06f * kmax);
    const float blo = fmaxf(kmax - 2.f * e, __uint_as_float(lo_hi)), bhi = kmax + 2.f * e;
    if (threadIdx.x == 0) sh.cnt2 = 0;
    __syncthreads();
    int below = 0;
    ball_src([&](bool mem, uint64_t key, int32_t pos) {
        const float v = __uint_as_float((uint32_t)(key >> 32));
        below += mem && v < blo;
        const bool inb = mem && v >= blo && v <= bhi;
        const int slot = wave_append(inb, &sh.cnt2);
        if (inb && slot < kBandCap) {
            bpos[slot] = pos;
            bid[slot] = (uint32_t)key;
        }
    });
    below = block_sum(below, sh);
    const int nb = sh.cnt2;
    // a band that is taken whole leaves the FP32 choice as it is
    if (nb > kBandCap || below > need || below + nb <= need) return;
    for (int j = threadIdx.x; j < nb; j += WG) {
        const int64_t pos = bpos[j];
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < MP; ++t) {
            const double o = (double)a.proj[pos * MP + t] + (double)a.proj_lo[pos * MP + t];
            const double q = (double)a.qp[qi * MP + t] + (double)a.qp_lo[qi * MP + t];
            const double dd = q - o;
            acc = fma(dd, dd, acc);
        }
        b64[j] = acc;
    }
    __syncthreads();
    // C's shell part again: the entries below the band, then the band's
    // first need - below
    if (threadIdx.x == 0) sh.cnt2 = 0;
    __syncthreads();
    ball_src([&](bool mem, uint64_t key, int32_t pos) {
        const bool take = mem && __uint_as_float((uint32_t)(key >> 32)) < blo;
        const int slot = wave_append(take, &sh.cnt2);
        if (take) cpos[n_ver + slot] = pos;
    });
    __syncthreads();
    const int keep = need - below;
    for (int j = threadIdx.x; j < nb; j += WG) {
        const double v = b64[j];
        const uint32_t id = bid[j];
        int rank = 0;
        for (int y = 0; y < nb; ++y) rank += b64[y] < v || (b64[y] == v && bid[y] < id);
        if (rank < keep) cpos[n_ver + below + rank] = bpos[j];
    }
    __syncthreads();
}

// Algorithm 2 for query qi, round by round with PM-tree walks.
__device__ void ann_one(const AnnArgs& a, int64_t qi, int32_t* fa, int32_t* fb, float* qs,
                        Smem& sh) {
    QueryCtx qc;
    load_query(a, qi, qs, qc);
    const float* qp = qc.qp;
    const float* qpiv = qc.qpiv;
    const float qn2 = qc.qn2;
    __syncthreads();

    const AnnQueryParams qpar = query_params(a, qi);
    int32_t* cpos = a.ws_cpos + qi * (int64_t)a.budget;
    float* cdist = a.ws_cdist + qi * (int64_t)a.budget;
    const int32_t* perm = a.perm;
    const int B = qpar.budget;

    double r = qpar.r_min;
    int n_ver = 0;
    int rounds = 0;
    int exit_kind = 0;
    int64_t scanned = 0;
    uint32_t prev_hi = 0;     // bits of the previous squared radius
    bool first = true;

    for (;;) {
        if (rounds > 0) {
            const double cr = qpar.c * r;
            const float thr2 = (float)(cr * cr);
            int loc = 0;
            for (int i = threadIdx.x; i < n_ver; i += WG) loc += cdist[i] <= thr2;
            if (block_sum(loc, sh) >= qpar.k) { exit_kind = PMLSH_EXIT_NEAR; break; }
        }
        if (rounds >= MAX_ROUNDS) r = __longlong_as_double(0x7ff0000000000000ll);
        const double Rd = qpar.t * r;
        const float R = (float)Rd;
        const float R2 = (float)(Rd * Rd);
        ++rounds;
        const float slack = 1e-5f * (sqrtf(qn2) + a.coord_scale + R);

        // range query (q', R), shrunk to the budget when the ball is large
        float Rq = R;
        int nl = traverse(a, qp, qpiv, Rq, slack, true, B, fa, fb, sh);
        const int32_t* leaves = fa;
        const float R2q = Rq < R ? (float)((double)Rq * (double)Rq) : R2;

        // shell (prev, R2q] on the 64-bit keys (pd^2 bits << 32 | id)
        const uint32_t lo_hi = first ? 0u : prev_hi + 1u;
        uint32_t hi_hi = __float_as_uint(R2q);
        const uint64_t klo = (uint64_t)lo_hi << 32;
        uint64_t khi = ((uint64_t)hi_hi << 32) | 0xffffffffull;
        int sh0 = shift_for(klo, khi);
        auto ball_src = [&](auto&& v) {
            scan_leaves(a, leaves, nl, qp, [&](bool valid, int pos, float pd2) {
                const uint32_t b = __float_as_uint(pd2);
                const bool mem = valid && b >= lo_hi && b <= hi_hi;
                const uint64_t key = mem ? (((uint64_t)b << 32) | (uint32_t)perm[pos]) : 0ull;
                v(mem, key, pos);
            });
        };
        auto count_pass = [&]() {
            clear_hist(sh);
            int loc = 0, sc = 0;
            ball_src([&](bool mem, uint64_t key, int32_t) {
                if (mem) { ++loc; atomicAdd(&sh.hist[(key - klo) >> sh0], 1u); }
            });
            for (int li = threadIdx.x; li < nl; li += WG) sc += a.ce[leaves[li]] - a.cb[leaves[li]];
            scanned += block_sum(sc, sh);
            return block_sum(loc, sh);
        };
        int shell = count_pass();
        if (Rq < R && n_ver + shell < B) {
            // the lowered radius fell short (rounding at the bound): redo the
            // range query at the full radius
            Rq = R;
            nl = traverse(a, qp, qpiv, Rq, slack, false, B, fa, fb, sh);
            hi_hi = __float_as_uint(R2);
            khi = ((uint64_t)hi_hi << 32) | 0xffffffffull;
            sh0 = shift_for(klo, khi);
            shell = count_pass();
        }

        if (n_ver + shell >= B) {
            const int need = B - n_ver;
            block_select(ball_src,
                         [&](int32_t pos, int slot) {
                             if (slot < need) cpos[n_ver + slot] = pos;
                         },
                         klo, khi, need, true, shell, sh);
            __syncthreads();
            shell_cut_fp64(a, qi, qc, ball_src, lo_hi, n_ver, need, cpos, sh);
            verify(a, qs, cpos, cdist, n_ver, B);
            n_ver = B;
            exit_kind = PMLSH_EXIT_BUDGET;
            __syncthreads();
            break;
        }
        if (threadIdx.x == 0) sh.cnt1 = 0;
        __syncthreads();
        ball_src([&](bool mem, uint64_t, int32_t pos) {
            const int slot = wave_append(mem, &sh.cnt1);
            if (mem && n_ver + slot < B) cpos[n_ver + slot] = pos;
        });
        __syncthreads();
        verify(a, qs, cpos, cdist, n_ver, n_ver + shell);
        n_ver += shell;
        __syncthreads();
        prev_hi = hi_hi;
        first = false;
        if (rounds >= a.max_rounds) break;
        r = qpar.c * r;
    }

    write_topk(a, qi, qs, cpos, cdist, n_ver, rounds, exit_kind, scanned, sh);
}

// ------------------------------------------------------------------------
// Leaf-major fast path for B <= CAP.
//
// Every candidate set of Algorithm 2 is a prefix of the order of the data by
// (projected distance, id) (the ball of a round holds the points up to t*r;
// a budget exit keeps the B first), and "the ball holds at least B points"
// is "the B-th projected distance is <= t*r". So the list L of the B
// projected-nearest points, verified as far as the rounds need, decides
// every round. The path finds L in three kernels:
//   tau     per query: an upper bound tau on the B-th projected distance
//           from the tree alone (the traversal's budget shrink);
//   filter  per leaf block x query block: each leaf's points are loaded once
//           into registers and tested against every query of the block whose
//           range query (q', tau) reaches the leaf (Eq. 5); points with
//           pd^2 <= tau^2 are appended to the query's candidate list;
//   finish  per query: exact radix select of L from the list, the rounds of
//           Algorithm 2 on L with incremental verification, the top-k.
// Queries whose list overflows (or that fall outside the path) are flagged
// and answered by the per-query kernel above.

// Squared FP32 distances from every query of the batch to every chunk centre,
// as |q'|^2 + |c|^2 - 2 q'.c (clamped at 0), on the FP32 matrix cores: a
// workgroup takes 64 queries x 256 chunks in four sub-tiles of 64 chunks,
// each wave a strip of 16 queries x 64 chunks per sub-tile (four 16 x 16
// tiles of v_mfma_f32_16x16x4_f32, K = 16 in four steps; the next
// sub-tile's centres are loaded meanwhile); each sub-tile goes through LDS
// and leaves as one block of the matrix (64 queries x 64 chunks, 8 KB
// contiguous). The values are bf16 bit patterns, rounded toward zero (the
// FP32 value's upper half), so each stored value is at most the FP32 value
// and above it by less than a factor 1 + 2^-7. The expansion's rounding error, in any
// summation order of the 16 products, stays below 64 u (|q'| + S)^2 (S
// bounds every centre norm); the chunk-ball test adds that much to its
// threshold and tests the rounded-down value, and the choice of chunks for
// the bound needs no exactness.
constexpr int DQB = 64;    // queries per workgroup
constexpr int DCS = 64;    // chunks per sub-tile
constexpr int DCB = 256;   // chunks per workgroup (four sub-tiles)

__global__ __launch_bounds__(WG) void dist_kernel(AnnArgs a) {
    __shared__ float sq[DQB][MP + 1];
    __shared__ float sc[DCS][MP + 1];
    __shared__ float sqn[DQB], scn[DCS];
    __shared__ __align__(16) uint16_t tile[DQB][DCS];
    const int q0 = blockIdx.y * DQB;
    const int nch = (int)(a.n_pad16 >> 6);
    const int nqb = min(DQB, a.nq - q0);
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // one centre coordinate quadruple per thread: centre e / 4, columns 4 (e % 4)
    const int ce = threadIdx.x >> 2, cq = (threadIdx.x & 3) * 4;
    auto load_cen = [&](int c0) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (c0 + ce < nch) v = *reinterpret_cast<const float4*>(a.chunk_cen + (int64_t)(c0 + ce) * MP + cq);
        return v;
    };
    float4 cnext = load_cen(blockIdx.x * DCB);
    {
        // every load of the staging goes out before the LDS stores
        constexpr int PER = DQB * MP / WG;
        float v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * WG, r = e / MP;
            v[u] = r < nqb ? a.qp[(int64_t)(q0 + r) * MP + e % MP] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * WG;
            sq[e / MP][e % MP] = v[u];
        }
    }
    __syncthreads();
    if (threadIdx.x < DQB) {
        float n2 = 0.f;
#pragma unroll
        for (int t = 0; t < MP; ++t) n2 = fmaf(sq[threadIdx.x][t], sq[threadIdx.x][t], n2);
        sqn[threadIdx.x] = n2;
    }
    // A operand (16 queries x 16): lane holds row li, columns lk, 4 + lk, ...
    float av[MP / 4];
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < MP / 4; ++kk) av[kk] = sq[16 * wave + li][4 * kk + lk];
    for (int sub = 0; sub < DCB / DCS; ++sub) {
        const int c0 = blockIdx.x * DCB + sub * DCS;
        if (c0 >= nch) break;
        sc[ce][cq] = cnext.x;
        sc[ce][cq + 1] = cnext.y;
        sc[ce][cq + 2] = cnext.z;
        sc[ce][cq + 3] = cnext.w;
        if (sub + 1 < DCB / DCS) cnext = load_cen(c0 + DCS);
        __syncthreads();
        if (threadIdx.x < DCS) {
            float n2 = 0.f;
#pragma unroll
            for (int t = 0; t < MP; ++t) n2 = fmaf(sc[threadIdx.x][t], sc[threadIdx.x][t], n2);
            scn[threadIdx.x] = n2;
        }
        // B (16 x 16 chunks): lane holds row lk, column li; result register v
        // of lane l is query 4 (l / 16) + v and chunk l % 16 of the tile
        float4_t acc[4] = {};
#pragma unroll
        for (int kk = 0; kk < MP / 4; ++kk)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], sc[16 * t + li][4 * kk + lk],
                                                              acc[t], 0, 0, 0);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int cl = 16 * t + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ql = 16 * wave + 4 * lk + v;
                const float d2 = fmaxf(fmaf(-2.f, acc[t][v], sqn[ql] + scn[cl]), 0.f);
                tile[ql][cl] = (uint16_t)(__float_as_uint(d2) >> 16);
            }
        }
        __syncthreads();
        // four threads per query row, 16 chunks (32 bytes) each: the sub-tile
        // (64 queries x 64 chunks) is one block of the matrix, written as
        // one contiguous 8 KB run
        const int ql = threadIdx.x >> 2, seg = (threadIdx.x & 3) * 16;
        uint32_t gm = 0xffffu;
        {
            const uint4* src = reinterpret_cast<const uint4*>(&tile[ql][seg]);
            const uint4 x0 = src[0], x1 = src[1];
            if (ql < nqb) {
                uint4* dst = reinterpret_cast<uint4*>(a.cdist + cdist_at(a, q0 + ql, c0 + seg));
                dst[0] = x0;
                dst[1] = x1;
            }
            const uint32_t w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const uint32_t h = (e & 1) ? (w[e >> 1] >> 16) : (w[e >> 1] & 0xffffu);
                if (c0 + seg + e < nch) gm = min(gm, h);
            }
        }
        // the group minimum over the four threads of the row
        gm = min(gm, (uint32_t)__shfl_xor((int)gm, 1));
        gm = min(gm, (uint32_t)__shfl_xor((int)gm, 2));
        if ((threadIdx.x & 3) == 0 && ql < nqb)
            a.cgmin[(int64_t)(q0 + ql) * a.gld + (c0 >> 6)] = (uint16_t)gm;
    }
}

// float bits >> 19 of 2^-64: the first of the fixed centre-distance bins
constexpr uint32_t kCenBinBase = 63u << 4;
// Groups (and 256-chunk blocks) the bound kernel lists per query at most, and
// the largest LDS footprint of its group minima and group list (beyond it the
// minima are read from HBM in every pass).
constexpr int kGrpCap = 2048;
constexpr size_t kTauGroupLds = 64 * 1024;

// Upper bound tau on the budget-th smallest projected distance of one query,
// and the query's row of the chunk mask:
//   1. the squared distances from q' to every 64-point chunk centre (computed
//      by dist_kernel, bf16 lower bounds), read four chunks per thread, and
//      the minimum of every group of 64 chunks, which rules out the groups
//      that cannot hold a chosen chunk or a passing one;
//   2. the chunks nearest to q' that hold at least min(n, 2 * budget) points,
//      chosen with a histogram of those distances weighted by chunk sizes;
//   3. over the points of the chosen chunks, the budget-th smallest pd^2
//      (upper edge of its histogram bin) is tau^2;
//   4. the radius of the chunk-ball test of Eq. 5 (a chunk can hold a point
//      within tau of q' only if |q' - centre| <= radius + tau), applied to
//      every chunk by mask_kernel.
// The chosen points are data points, so the ball of radius tau holds at least
// `budget` points and therefore the budget nearest points by projected
// distance. The choice of chunks only affects how tight tau is, never its
// validity.
__global__ __launch_bounds__(WG) void tau_kernel(AnnArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem& sh = *reinterpret_cast<Smem*>(smem_raw);
    const int64_t qi = blockIdx.x;
    QueryCtx qc;
    load_query(a, qi, nullptr, qc);
    const int nch = (int)(a.n_pad16 >> 6);
    const int ng4 = (nch + 3) >> 2;
    const int ngr = (nch + 63) >> 6;
    // four bf16 distances per 8-byte element (element g: chunks 4 g .. 4 g + 3;
    // the 16 elements of a group of 64 chunks are contiguous)
    const uint2* cd4 = reinterpret_cast<const uint2*>(a.cdist + cdist_at(a, qi, 0));
    const int64_t band_stride4 = 1024;   // uint2 elements per block
    auto row4 = [&](int g) { return cd4[(int64_t)(g >> 4) * band_stride4 + (g & 15)]; };
    const uint16_t* grow16 = a.cgmin + qi * a.gld;
    // the group minima (copied to LDS when a.glds is set, else read in the
    // row), then the list of candidate groups and the list of chosen chunks
    unsigned char* lds_free = smem_raw + offsetof(Smem, skey);
    const uint16_t* gmin = grow16;
    if (a.glds) {
        uint16_t* g = reinterpret_cast<uint16_t*>(lds_free);
        // eight loads per thread go out before their LDS stores
        for (int j0 = threadIdx.x; j0 < ngr; j0 += 8 * WG) {
            uint16_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = j0 + u * WG;
                v[u] = j < ngr ? grow16[j] : (uint16_t)0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = j0 + u * WG;
                if (j < ngr) g[j] = v[u];
            }
        }
        gmin = g;
        lds_free += 2 * (size_t)((ngr + 7) & ~7);
    }
    int32_t* glist = reinterpret_cast<int32_t*>(lds_free);
    // the chunks chosen for the bound (step 2)
    int32_t* sel = glist + kGrpCap;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    // bf16 bit pattern k of an element (non-negative values: ordered as
    // unsigned integers)
    auto half_k = [](const uint2& v, int k) {
        const uint32_t w = k < 2 ? v.x : v.y;
        return (k & 1) ? (w >> 16) : (w & 0xffffu);
    };
    const uint32_t hbase = kCenBinBase;
    auto cbin = [&](uint32_t h) { return min(max(h >> 3, hbase) - hbase, (uint32_t)(NB - 1)); };
    const int32_t budget = query_params(a, qi).budget;
    const int64_t want = a.n < 2 * (int64_t)budget ? a.n : 2 * (int64_t)budget;
    const int wc = (int)min<int64_t>(nch, (want + 63) / 64 + 1);

    // b0 bounds the bin sought in step 1 from above: every group holds a
    // chunk at its minimum, so with wc groups whose minima lie in bins <= b0
    // at least wc chunks lie there, and only chunks in those bins need to be
    // counted. A group whose minimum lies above b0 holds none of them: the
    // passes visit only the ngl groups listed (the whole row when more than
    // a.grp_cap groups qualify).
    clear_hist(sh);
    for (int j = threadIdx.x; j < ngr; j += WG) atomicAdd(&sh.hist[cbin(gmin[j])], 1u);
    if (threadIdx.x == 0) {
        sh.thr_bin = NB - 1;
        sh.cnt0 = 0;
    }
    __syncthreads();
    uint32_t b0 = NB - 1;
    if (ngr >= wc) {
        find_threshold(wc, sh);
        b0 = (uint32_t)sh.thr_bin;
    }
    for (int j0 = 0; j0 < ngr; j0 += WG) {
        const int j = j0 + threadIdx.x;
        const bool take = j < ngr && cbin(gmin[j]) <= b0;
        const int slot = wave_append(take, &sh.cnt0);
        if (take && slot < a.grp_cap) glist[slot] = j;
    }
    __syncthreads();
    const int ngl = sh.cnt0;
    const bool grp = ngl <= a.grp_cap;
    __syncthreads();
    // f(g, element g of the row) for every element of the listed groups, or
    // of the whole row (16 consecutive threads read a group's 128 bytes)
    auto for_elems = [&](auto&& f) {
        if (grp) {
            for (int e = threadIdx.x; e < 16 * ngl; e += WG) {
                const int g = 16 * glist[e >> 4] + (e & 15);
                if (g < ng4) f(g, row4(g));
            }
        } else {
            for (int g = threadIdx.x; g < ng4; g += WG) f(g, row4(g));
        }
    };

    // 1: histogram of the centre distances (chunk counts) on fixed bins: 16
    // per octave of the squared distance over [2^-64, 2^64), clamped at both
    // ends, so no range pass is needed. The chosen chunks are those of the
    // bins up to the one where the running count reaches wc = min(n_chunks,
    // ceil(want / 64) + 1) chunks, want = min(n, 2 * budget) points (the
    // extra chunk covers the one chunk with fewer than 64 points).
    clear_hist(sh);
    for_elems([&](int g, const uint2& v) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t b = cbin(half_k(v, k));
            if (4 * g + k < nch && b <= b0) atomicAdd(&sh.hist[b], 1u);
        }
    });
    __syncthreads();
    if (threadIdx.x == 0) sh.thr_bin = NB - 1;
    __syncthreads();
    find_threshold(wc, sh);
    const uint32_t tbin = (uint32_t)sh.thr_bin;
    const int nlow = sh.thr_below;         // chunks of the bins below tbin (< wc)
    const int need = wc - nlow;           // chunks still wanted from bin tbin
    const int in_bin = sh.thr_in;
    // every chunk with a stored value <= tlim is chosen: all of bin tbin, or,
    // when that bin holds more than eight chunks beyond those wanted, only
    // its sub-bins (the three low bits of the bf16 pattern) up to the one
    // where the count reaches `need` (the clamped end bins stay whole)
    uint32_t tlim = tbin == (uint32_t)(NB - 1) ? 0xffffu : ((tbin + hbase) << 3) | 7u;
    if (in_bin - need > 8 && tbin != 0u && tbin != (uint32_t)(NB - 1)) {
        __syncthreads();
        clear_hist(sh);
        for_elems([&](int g, const uint2& v) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t h = half_k(v, k);
                if (4 * g + k < nch && (h >> 3) == tbin + hbase) atomicAdd(&sh.hist[h & 7u], 1u);
            }
        });
        __syncthreads();
        if (threadIdx.x == 0) sh.thr_bin = NB - 1;
        __syncthreads();
        find_threshold(need, sh);
        tlim = ((tbin + hbase) << 3) | (uint32_t)sh.thr_bin;
    }
    if (threadIdx.x == 0) sh.cnt1 = 0;
    __syncthreads();

    // 2: the chosen chunks, and the largest distance bound over their points.
    // The list holds kSelCap chunks: those of the bins below tbin (fewer than
    // wc) come first, then as many of bin tbin's as fit; any kSelCap chunks
    // hold at least 64 kSelCap >= 2 * budget points, so the bound stays valid
    if (threadIdx.x == 0) sh.cnt2 = 0;
    __syncthreads();
    float rmax = 0.f;
    for_elems([&](int g, const uint2& v) {
        bool tk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) tk[k] = 4 * g + k < nch && half_k(v, k) <= tlim;
        if (tk[0] | tk[1] | tk[2] | tk[3]) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (tk[k]) {
                    const int i = 4 * g + k;
                    const uint32_t h = half_k(v, k);
                    const int slot = cbin(h) < tbin ? atomicAdd(&sh.cnt1, 1)
                                                    : nlow + atomicAdd(&sh.cnt2, 1);
                    if (slot < kSelCap) {
                        // the stored distance is low by less than a factor 1 + 2^-7
                        const float d = sqrtf(__uint_as_float(h << 16)) * 1.0079f;
                        rmax = fmaxf(rmax, d + a.chunk_rad[i]);
                        sel[slot] = i;
                    }
                }
            }
        }
    });
    for (int off = 32; off > 0; off >>= 1) rmax = fmaxf(rmax, __shfl_xor(rmax, off));
    if (lane == 0) sh.red[wave] = __float_as_int(rmax);
    __syncthreads();
    const int nsel = min(nlow + sh.cnt2, kSelCap);
    float R = 0.f;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) R = fmaxf(R, __int_as_float(sh.red[w]));
    __syncthreads();
    // every chosen point lies within R up to rounding; the margin keeps the
    // histogram range above all of them
    R = R * 1.0001f + 1e-5f * (sqrtf(qc.qn2) + a.coord_scale);
    float R2 = (float)((double)R * (double)R);

    // 3: histogram of pd^2 over the chosen points -> budget-th smallest
    const uint32_t hb2 = __float_as_uint(R2) >> 15;
    const uint32_t base2 = hb2 > (uint32_t)(NB - 1) ? hb2 - (uint32_t)(NB - 1) : 0u;
    clear_hist(sh);
    int cnt = 0;
    {
        // four points per thread in flight: their row loads go out together
        constexpr int PU = 4;
        for (int e0 = threadIdx.x; e0 < nsel * 64; e0 += PU * WG) {
            float pd2[PU];
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const int e = e0 + u * WG;
                const int64_t pos = e < nsel * 64 ? ((int64_t)sel[e >> 6] << 6) + (e & 63) : a.n;
                pd2[u] = pos < a.n ? proj_dist2(a.proj + pos * MP, qc.qp)
                                   : __int_as_float(0x7f800000);
            }
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                if (pd2[u] <= R2) {
                    atomicAdd(&sh.hist[radius_bin(pd2[u], base2)], 1u);
                    ++cnt;
                }
            }
        }
    }
    __syncthreads();
    if (block_sum(cnt, sh) >= budget) {
        if (threadIdx.x == 0) sh.thr_bin = NB - 1;
        __syncthreads();
        find_threshold(budget, sh);
        const float e2 = __uint_as_float((base2 + (uint32_t)sh.thr_bin + 1u) << 15);
        if (e2 < R2) R2 = e2;
    } else {
        // rounding left fewer than `budget` chosen points inside R: no bound
        R2 = __int_as_float(0x7f800000);
    }

    // 4: the radius of the chunk-ball test, which mask_kernel applies: it
    // covers the FP32 errors of pd^2 and of the test's own distance
    // (relative 2^-16 and 1e-5 (tau + S)); the margin covers the rounding
    // of the expanded squared distance (64 u (|q'| + S)^2)
    if (threadIdx.x == 0) {
        const float tq0 = sqrtf(R2);
        const float tq = tq0 * (1.f + 1.52587890625e-05f) + 1e-5f * (tq0 + a.coord_scale);
        const float big = sqrtf(qc.qn2) + a.coord_scale;
        a.qtest[qi] = make_float2(tq, 64.f * 5.9604645e-08f * big * big);
    }

    if (threadIdx.x == 0) {
        a.l_count[qi] = 0u;
        a.q_scanned[qi] = 0u;   // mask_kernel adds 64 per passing chunk
        a.q_flag[qi] = 0;
        if (qi == 0) a.pq_list[0] = 0u;   // the flagged list of the batch starts empty
        // The query's FP16 row of the matrix-core scan, q' taken relative to
        // the centre of the rows. thr = tau^2 - |q'|^2 plus 96 u (|q'| + S)^2
        // (S bounds every |o'| of a scan row) covers the FP32 errors of the
        // exact pd^2, of the centring and of |q'|^2; the further
        // 2^-15 (|q'| + S)^2 covers the FP32 accumulation of the scan and its
        // hi/lo splits. When the rows come from the low-precision projection,
        // q' is the query's own low-precision projection and tau grows by
        // eps(query) + eps_max, which bounds how far a point's low-precision
        // projected distance lies from its exact one.
        const float u = 5.9604645e-08f;   // 2^-24
        const float* qsrc = a.qlp ? a.qlp + qi * MP : qc.qp;
        float qv[MP];
        float qv2 = 0.f, R2s = R2;
#pragma unroll
        for (int t = 0; t < MP; ++t) {
            qv[t] = qsrc[t] - a.scen[t];
            qv2 = fmaf(qv[t], qv[t], qv2);
        }
        if (a.qlp) {
            const float tw = (sqrtf(R2) + (a.qeps[qi] + a.eps_max)) * (1.f + 2.384185791015625e-07f);
            R2s = tw * tw * (1.f + 2.384185791015625e-07f);
        }
        const float qn = sqrtf(qv2);
        const float big = qn + a.scan_scale;
        const float thr = (R2s + 96.f * u * big * big) - qv2 + 3.0517578e-05f * big * big;
        const float s = a.scale16;
        const float v = -(s * s) * thr;
        float qmax = 0.f;
#pragma unroll
        for (int t = 0; t < MP; ++t) qmax = fmaxf(qmax, fabsf(qv[t]));
        const bool ok = fabsf(v) < 30000.f && 2.f * s * qmax < 30000.f && s * qn < 30000.f;
        _Float16 w[32];
#pragma unroll
        for (int i = 0; i < 32; ++i) w[i] = (_Float16)0.f;
        if (ok) {
#pragma unroll
            for (int t = 0; t < MP; ++t) w[t] = (_Float16)(-2.f * s * qv[t]);
            w[16] = (_Float16)1.f;
            w[17] = (_Float16)1.f;
            const _Float16 hi = (_Float16)v;
            w[18] = hi;
            w[19] = (_Float16)(v - (float)hi);
            w[20] = (_Float16)(-s * qn);
        } else {
            // outside the FP16 range (or no finite bound): every product is
            // +1, no candidate, and the per-query path answers the query
            w[18] = (_Float16)1.f;
        }
        uint4* dst = reinterpret_cast<uint4*>(a.qaug + qi * 32);
        const uint4* src = reinterpret_cast<const uint4*>(w);
#pragma unroll
        for (int i = 0; i < 4; ++i) dst[i] = src[i];
    }
}

// The chunk-ball test of Eq. 5 for every (query, chunk) pair of the batch,
// written as the chunk-major mask the scan reads: bit l of word qb of chunk
// c is query 64 qb + l. A workgroup takes 64 queries x 256 chunks: thread t
// holds the eight chunks 8 (t % 32) .. + 7 of its block and the eight
// queries 8 (t / 32) .. + 7, reads the eight stored squared centre distances
// of each of its query rows in one 16-byte load (eight threads cover a
// query's 128-byte row of a 64-chunk block) and tests d^2 <= (radius +
// tq)^2 + margin with the query's (tq, margin) from the bound kernel. The
// eight query bits of every chunk are one byte of its word, stored in LDS as
// one 8-byte run per thread and assembled per chunk; each query's passing
// chunks, 64 points each, are added to its scan count.
constexpr int MQB = 64;    // queries per workgroup (one mask word)
constexpr int MCH = 256;   // chunks per workgroup: eight per thread of a query octet
static_assert(MCH == 8 * 32 && MQB == 8 * (WG / 32), "thread t: chunk octet t % 32, query octet t / 32");

__global__ __launch_bounds__(WG) void mask_kernel(AnnArgs a) {
    __shared__ float2 qt[MQB];
    __shared__ __align__(16) uint8_t lb[MQB / 8][MCH];   // row qo: byte qo of every chunk's word
    __shared__ uint32_t cnt[MQB];
    const int nch = (int)(a.n_pad16 >> 6);
    const int q0 = blockIdx.y * MQB;
    const int nqb = min(MQB, a.nq - q0);
    const int co = threadIdx.x & 31, qo = threadIdx.x >> 5;
    const int c0 = blockIdx.x * MCH + 8 * co;   // the thread's first chunk
    if (threadIdx.x < MQB) {
        qt[threadIdx.x] = (int)threadIdx.x < nqb ? a.qtest[q0 + threadIdx.x] : make_float2(0.f, 0.f);
        cnt[threadIdx.x] = 0u;
    }
    // the eight rows' loads go out before any test
    uint4 w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int q = 8 * qo + u;
        w[u] = q < nqb && c0 < nch
                   ? *reinterpret_cast<const uint4*>(a.cdist + cdist_at(a, q0 + q, c0))
                   : make_uint4(0u, 0u, 0u, 0u);
    }
    float rad[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) rad[e] = c0 + e < nch ? a.chunk_rad[c0 + e] : 0.f;
    __syncthreads();
    uint32_t bits[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};   // chunk e: the eight query bits
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int q = 8 * qo + u;
        const float2 t = qt[q];
        const uint32_t h[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
        uint32_t np = 0u;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t hb = (e & 1) ? (h[e >> 1] & 0xffff0000u) : (h[e >> 1] << 16);
            const float ra = rad[e] + t.x;
            const bool p = q < nqb && c0 + e < nch && __uint_as_float(hb) <= fmaf(ra, ra, t.y);
            bits[e] |= (uint32_t)p << u;
            np += p;
        }
        // the query's passing chunks over the 32 chunk octets (half a wave)
        np += (uint32_t)__shfl_xor((int)np, 1);
        np += (uint32_t)__shfl_xor((int)np, 2);
        np += (uint32_t)__shfl_xor((int)np, 4);
        np += (uint32_t)__shfl_xor((int)np, 8);
        np += (uint32_t)__shfl_xor((int)np, 16);
        if (co == 0 && np) cnt[q] = np;
    }
    // the eight chunks' bytes of this query octet in one 8-byte store
    *reinterpret_cast<uint2*>(&lb[qo][8 * co]) =
        make_uint2(bits[0] | (bits[1] << 8) | (bits[2] << 16) | (bits[3] << 24),
                   bits[4] | (bits[5] << 8) | (bits[6] << 16) | (bits[7] << 24));
    __syncthreads();
    for (int i = threadIdx.x; i < MCH; i += WG) {
        const int c = blockIdx.x * MCH + i;
        uint64_t wd = 0ull;
#pragma unroll
        for (int o = 0; o < MQB / 8; ++o) wd |= (uint64_t)lb[o][i] << (8 * o);
        if (c < nch) a.cmask[cmask_at(a, c, blockIdx.y)] = wd;
    }
    if ((int)threadIdx.x < nqb && cnt[threadIdx.x])
        atomicAdd(&a.q_scanned[q0 + threadIdx.x], 64u * cnt[threadIdx.x]);
}

// ---- Matrix-core scan (the range filter of the batched path) ----
//
// For every (point, query) pair of the batch one FP16 MFMA dot product of
// 32-half rows decides whether the point can lie within tau of the query:
//   point row P: s*o'_0..s*o'_15, hi(s^2|o'|^2), lo(s^2|o'|^2), 1, 1,
//                cm*s*|o'|, zeros
//   query row Q: -2s*q'_0..-2s*q'_15, 1, 1, hi(-s^2 thr), lo(-s^2 thr),
//                -s*|q'|, zeros
// so P.Q = s^2 (|o'|^2 - 2 q'.o' - thr - cm |q'||o'|), accumulated in FP32.
// thr is tau^2 - |q'|^2 plus margins for the FP32 errors of the exact pd^2 and
// of the split terms; the FP16 rounding of the dot product is bounded by
// 2^-9 |q'||o'|, which the cm term covers pair by pair. Hence every point
// whose FP32 direct-difference pd^2 is within tau^2 gives P.Q < 0, and the
// pool also receives a few points just outside, which the finishing kernel
// removes with the exact pd^2. This is the PM-tree range query of the
// paper computed without the tree: the node tests of Eq. 5 only save work on
// a processor that compares one pair at a time, while the matrix cores
// compare all pairs of a batch at 16 x 16 x 32 per instruction.
//
// Grid: x strides over 64-point chunks, y over blocks of 1,024 queries; wave
// w of a workgroup owns a quarter of the block's mask words (256 queries).
// For each chunk a wave packs the queries whose chunk-ball test passed (the
// set bits of its mask words) into a list and runs the MFMA on groups of 16
// listed queries, so a group's 16 columns are all queries that may hold
// candidates in the chunk (the last group is padded with a row whose product
// with every point is positive). The FP16 rows of the block's queries sit in
// LDS as B operands (lane l: listed query 16 g + l % 16, halves
// 8 (l / 16) .. + 7); the chunk's four 16-point tiles are the A operands
// (lane l: point 16 t + l % 16, same halves). Halves 24..31 are zero in every
// point and query row: neither is stored, and lanes 48..63 hold zeros. A
// result register r of lane l holds point 4 (l / 16) + r of the tile and
// listed query l % 16.

// Two block shapes of the scan: 512 queries per workgroup (128 per wave,
// three workgroups per compute unit) for indexes of fewer than
// kScanLargeChunks chunks, 1,024 (256 per wave, two per compute unit) above:
// staging a block's query rows is a fixed cost per workgroup, paid back only
// when a workgroup has many chunks to scan, and a wave's list of passing
// queries then fills more of each 16-query group.
#ifndef PMLSH_SCAN_QB
#define PMLSH_SCAN_QB 512
#endif
#ifndef PMLSH_SCAN_QB_LARGE
#define PMLSH_SCAN_QB_LARGE 1024
#endif
#ifndef PMLSH_SCAN_STAGE
#define PMLSH_SCAN_STAGE 1024
#endif
#ifndef PMLSH_SCAN_WAVES_PER_EU
#define PMLSH_SCAN_WAVES_PER_EU 3
#endif
#ifndef PMLSH_SCAN_WAVES_PER_EU_LARGE
#define PMLSH_SCAN_WAVES_PER_EU_LARGE 2
#endif
constexpr int64_t kScanLargeChunks = 32768;   // 2,097,152 points
constexpr int SSTG = PMLSH_SCAN_STAGE;        // candidates staged per wave

// Query rows, then per-wave candidate stages: every wave packs, stages,
// counts and flushes its own candidates, so after the rows are loaded the
// scan needs no workgroup barrier. QB queries per block.
template <int QB>
struct __align__(16) ScanShared {
    uint16_t qrow[QB + 1][kScanRow];    // FP16 query rows of the block, padding row last
    uint32_t pos[NWAVE][SSTG];          // staged candidates: leaf position
    uint8_t qid[NWAVE][SSTG];           // and query within the wave's range
    uint32_t hits[NWAVE][QB / NWAVE], base[NWAVE][QB / NWAVE];
    // queries of the wave passing the chunk, by column: slot 16 g + j of the
    // list is lcol[j][g]
    uint8_t lcol[NWAVE][16][QB / NWAVE / 16];
};
template <int QB, int WPE>
constexpr bool scan_shape_ok() {
    return (QB / NWAVE) % 64 == 0 && QB / NWAVE / 64 <= 4 && QB / NWAVE <= 256 &&
           sizeof(ScanShared<QB>) * WPE <= 160 * 1024;
}
static_assert(scan_shape_ok<PMLSH_SCAN_QB, PMLSH_SCAN_WAVES_PER_EU>() &&
                  scan_shape_ok<PMLSH_SCAN_QB_LARGE, PMLSH_SCAN_WAVES_PER_EU_LARGE>(),
              "a wave's queries are whole mask words (ids below 256), and the scan "
              "workgroups of a compute unit fit its LDS");

__device__ __forceinline__ half8_t load_half8(const uint16_t* p) {
    return __builtin_bit_cast(half8_t, *reinterpret_cast<const uint4*>(p));
}

__device__ __forceinline__ void scan_mfma(const half8_t (&av)[4], half8_t b, float4_t (&cc)[4]) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
        cc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[mt], b, float4_t{}, 0, 0, 0);
}

// Writes the wave's staged candidates to the pool with one reservation per
// query (queries qw0 .. qw0 + nqw - 1 of the batch) and empties the stage.
// Only this wave touches its part of the shared memory.
template <int QB>
__device__ __forceinline__ void scan_flush(const AnnArgs& a, ScanShared<QB>& ss, int wave, int lane,
                                           uint32_t& wn, int64_t qw0, int nqw) {
    uint32_t* hits = ss.hits[wave];
    uint32_t* base = ss.base[wave];
    for (uint32_t e = lane; e < wn; e += 64) atomicAdd(&hits[ss.qid[wave][e]], 1u);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int e = lane; e < nqw; e += 64) {
        const uint32_t h = hits[e];
        if (h) base[e] = atomicAdd(&a.l_count[qw0 + e], h);
        hits[e] = 0u;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (uint32_t e = lane; e < wn; e += 64) {
        const int q = ss.qid[wave][e];
        const uint32_t slot = base[q] + atomicAdd(&hits[q], 1u);
        if (slot < (uint32_t)a.q_cap) a.l_list[(qw0 + q) * a.q_cap + slot] = ss.pos[wave][e];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int e = lane; e < nqw; e += 64) hits[e] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    wn = 0;
}

// Stages the negative results of one 64-point x 16-query group (q: the
// lane's query within the wave's range), flushing the stage first whenever
// a ballot's candidates would not fit, so no candidate is lost. The group is
// skipped when no result is negative; otherwise register r of the four tiles
// is tested together first, since most register positions hold no candidate.
template <int QB>
__device__ __forceinline__ void scan_emit(const AnnArgs& a, ScanShared<QB>& ss, int wave, int lane,
                                          uint32_t& wn, const float4_t (&cc)[4], int64_t p0, int q,
                                          int64_t qw0, int nqw) {
    // a result is a candidate when its sign bit is set
    uint32_t z[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        z[r] = __float_as_uint(cc[0][r]) | __float_as_uint(cc[1][r]) | __float_as_uint(cc[2][r]) |
               __float_as_uint(cc[3][r]);
    if (!__builtin_amdgcn_ballot_w64((int32_t)(z[0] | z[1] | z[2] | z[3]) < 0)) return;
    const uint32_t prow = (uint32_t)p0 + 4u * (uint32_t)(lane >> 4);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (!__builtin_amdgcn_ballot_w64((int32_t)z[r] < 0)) continue;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bool c = __float_as_int(cc[mt][r]) < 0;
            const uint64_t m = __builtin_amdgcn_ballot_w64(c);
            if (!m) continue;
            const uint32_t nh = (uint32_t)__popcll(m);
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (wn + nh > (uint32_t)SSTG) scan_flush(a, ss, wave, lane, wn, qw0, nqw);
            if (c) {
                ss.pos[wave][wn + rank] = prow + (uint32_t)(mt * 16 + r);
                ss.qid[wave][wn + rank] = (uint8_t)q;
            }
            wn += nh;
        }
    }
}

template <int QB, int WPE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WPE))) void scan_kernel(AnnArgs a) {
    constexpr int SQB = QB;           // queries per scan block
    constexpr int SQW = SQB / NWAVE;  // queries per wave
    constexpr int QPL = SQW / 64;     // queries per lane in the list building
    constexpr int SPAD = SQB;         // index of the padding row
    __shared__ ScanShared<QB> ss;
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lq = lane >> 4;
    const int q0 = blockIdx.y * SQB;
    const int nqb = min(SQB, a.nq - q0);
    const int nwq = (nqb + 63) >> 6;            // mask words of this query block
    // mask words per wave: the block's words split evenly, whole words each
    const int wpw = (nwq + NWAVE - 1) / NWAVE;
    const int w0 = wave * wpw;                  // first word of this wave
    const int nw = max(0, min(nwq - w0, wpw));
    const int64_t qw0 = (int64_t)q0 + w0 * 64;  // first query of this wave
    const int nqw = max(0, min(nqb - w0 * 64, nw * 64));   // its queries

    // the block's query rows (halves 0..23; 16 bytes per thread and step)
    for (int e = threadIdx.x; e < (SQB + 1) * 3; e += WG) {
        const int r = e / 3, part = e - 3 * r;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (r < nqb) {
            v = *reinterpret_cast<const uint4*>(a.qaug + (int64_t)(q0 + r) * 32 + part * 8);
        } else if (r == SPAD && part == 2) {
            v.y = 0x3c00u;   // half 18 = 1: the product with any point is >= 0
        }
        *reinterpret_cast<uint4*>(&ss.qrow[r][part * 8]) = v;
    }
    for (int e = lane; e < SQW; e += 64) ss.hits[wave][e] = 0u;
    __syncthreads();

    uint32_t wn = 0;
    // Point chunks, strided over the workgroups. Four slots of FP16 rows and
    // mask words are in flight per wave (12 KB of rows); the loop is unrolled
    // over the slots so that each is refilled in place after its chunk.
    const int64_t nchunk = a.n_pad16 >> 6;
    const int64_t G = gridDim.x;
    const int l16 = lane & 15;
    // lane i packs the QPL queries QPL i .. QPL i + QPL - 1 of the wave's
    // range, held in mask word i / (64 / QPL) (those lanes load it together)
    const int pk_word = lane / (64 / QPL), pk_shift = QPL * (lane % (64 / QPL));
    const bool mword = pk_word < nw;
    // Every slot load is unconditional, so that the compiler waits for the
    // slot in use only (a load under a branch makes it wait for every slot in
    // flight): a chunk past the end reads the last chunk (such a slot is never
    // used), a lane without a mask word reads the block's first word, and
    // lanes 48..63, whose halves 24..31 of the A operand are zero, read halves
    // 16..23. What is not the chunk's is cleared where the slot is used.
    const int64_t mband = (q0 >> 6) + (mword ? w0 + pk_word : 0);
    const uint16_t* rbase = a.proj16 + (l16 * kScanRow + (lq < 3 ? lq : 2) * 8);
    const uint32_t rkeep = lq < 3 ? 0xffffffffu : 0u;

    struct Slot {
        half8_t r[4];
        uint64_t m;
    };
    auto load = [&](int64_t cc, Slot& dst) {
        const int64_t ccl = cc < nchunk ? cc : nchunk - 1;
        dst.m = a.cmask[cmask_at(a, ccl, mband)];
        const uint16_t* rp = rbase + ccl * (64 * kScanRow);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) dst.r[mt] = load_half8(rp + mt * 16 * kScanRow);
    };
    uint8_t (*lcol)[SQW / 16] = ss.lcol[wave];
    auto chunk = [&](const Slot& cur, int64_t cc) {
        // the list of passing queries: each lane's set bits at the count of
        // set bits in the lanes below it
        const uint64_t cm = mword ? cur.m : 0ull;
        const uint32_t pk = (uint32_t)(cm >> pk_shift) & ((1u << QPL) - 1u);
        int total = 0;
        uint32_t at = 0;
#pragma unroll
        for (int b = 0; b < QPL; ++b) {
            const uint64_t bb = __builtin_amdgcn_ballot_w64((pk >> b) & 1u);
            total += __popcll(bb);
            at += __builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0u));
        }
        if (total == 0) return;
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        half8_t av[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            av[mt] = __builtin_bit_cast(half8_t, __builtin_bit_cast(u32x4, cur.r[mt]) & rkeep);
#pragma unroll
        for (int b = 0; b < QPL; ++b)
            if ((pk >> b) & 1u) {
                lcol[at & 15][at >> 4] = (uint8_t)(QPL * lane + b);
                ++at;
            }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // room for a chunk's typical candidates (a fuller chunk flushes
        // inside the emit)
        if (wn > (uint32_t)(SSTG - 256)) scan_flush(a, ss, wave, lane, wn, qw0, nqw);
        const uint8_t* mycol = lcol[l16];
        // two groups per step: their row reads and matrix products go out
        // before either result is examined
        for (int g = 0; g < total; g += 32) {
            const bool two = g + 16 < total;
            const int qa = g + l16 < total ? (int)mycol[g >> 4] : -1;
            const int qb = two && g + 16 + l16 < total ? (int)mycol[(g >> 4) + 1] : -1;
            half8_t ba = half8_t{}, bb = half8_t{};
            if (lq < 3) {
                ba = load_half8(&ss.qrow[qa >= 0 ? w0 * 64 + qa : SPAD][lq * 8]);
                if (two) bb = load_half8(&ss.qrow[qb >= 0 ? w0 * 64 + qb : SPAD][lq * 8]);
            }
            float4_t ca[4], cb[4];
            scan_mfma(av, ba, ca);
            if (two) scan_mfma(av, bb, cb);
            scan_emit(a, ss, wave, lane, wn, ca, cc << 6, qa, qw0, nqw);
            if (two) scan_emit(a, ss, wave, lane, wn, cb, cc << 6, qb, qw0, nqw);
        }
    };
    int64_t c = blockIdx.x;
    Slot s0, s1, s2, s3;
    load(c, s0);
    load(c + G, s1);
    load(c + 2 * G, s2);
    load(c + 3 * G, s3);
    for (; c < nchunk; c += 4 * G) {
        chunk(s0, c);
        load(c + 4 * G, s0);
        if (c + G >= nchunk) break;
        chunk(s1, c + G);
        load(c + 5 * G, s1);
        if (c + 2 * G >= nchunk) break;
        chunk(s2, c + 2 * G);
        load(c + 6 * G, s2);
        if (c + 3 * G >= nchunk) break;
        chunk(s3, c + 3 * G);
        load(c + 7 * G, s3);
    }
    scan_flush(a, ss, wave, lane, wn, qw0, nqw);
}

// The budget cut of L in the FP64 order. The FP32 pd^2 of a pool entry
// (direct differences of the FP32 projections) is within
// E = 2^-22 pd (|q'| + S) + 2^-19 pd^2 of its value from the FP64 projections
// (the FP32 roundings of both projections and of the differences, and the
// FP32 sum of 16 squares), so only entries whose FP32 value lies within a
// band of 2E around the B-th value (kth) can be ordered differently in FP64.
// Their pd^2 is recomputed in FP64 from the hi and lo halves of both
// projections: the entries below the band are in L, the first B - below of
// the band by (FP64 pd^2, id) join them, everything else leaves (key ~0).
// Returns false, marking nothing, when the band holds more than 512 entries.
__device__ bool cut_fp64(const AnnArgs& a, int64_t qi, const QueryCtx& qc, int n, int B,
                         uint64_t kth, Smem& sh) {
    constexpr int kBandCap = 512;
    int32_t* band = reinterpret_cast<int32_t*>(sh.hist);            // entry, ~entry if out
    uint32_t* bid = reinterpret_cast<uint32_t*>(sh.hist + kBandCap); // its id
    double* b64 = reinterpret_cast<double*>(sh.hist + 2 * kBandCap); // its FP64 pd^2
    static_assert(NB >= 4 * kBandCap, "the band must fit the histogram");
    const float k2 = __uint_as_float((uint32_t)(kth >> 32));
    const float big = sqrtf(qc.qn2) + a.coord_scale;
    const float e = 2.f * (2.384185791015625e-07f * sqrtf(k2) * big + 1.9073486328125e-06f * k2);
    const float blo = k2 - 2.f * e, bhi = k2 + 2.f * e;
    __syncthreads();
    if (threadIdx.x == 0) sh.cnt2 = 0;
    __syncthreads();
    int below = 0;
    for (int b0 = 0; b0 < n; b0 += WG) {
        const int i = b0 + threadIdx.x;
        const float v = i < n ? __uint_as_float((uint32_t)(sh.skey[i] >> 32)) : __int_as_float(0x7f800000);
        below += i < n && v < blo;
        const bool inb = i < n && v >= blo && v <= bhi;
        const int slot = wave_append(inb, &sh.cnt2);
        if (inb && slot < kBandCap) {
            band[slot] = i;
            bid[slot] = (uint32_t)sh.skey[i];
        }
    }
    below = block_sum(below, sh);
    const int nb = sh.cnt2;
    if (nb > kBandCap || below >= B || below + nb < B) return false;
    if (below + nb == B) {
        // the whole band is in L whatever its FP64 order
        for (int i = threadIdx.x; i < n; i += WG)
            if (__uint_as_float((uint32_t)(sh.skey[i] >> 32)) > bhi) sh.skey[i] = ~0ull;
        __syncthreads();
        return true;
    }
    for (int j = threadIdx.x; j < nb; j += WG) {
        const int64_t pos = sh.spos[band[j]];
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < MP; ++t) {
            const double o = (double)a.proj[pos * MP + t] + (double)a.proj_lo[pos * MP + t];
            const double q = (double)a.qp[qi * MP + t] + (double)a.qp_lo[qi * MP + t];
            const double dd = q - o;
            acc = fma(dd, dd, acc);
        }
        b64[j] = acc;
    }
    __syncthreads();
    const int need = B - below;
    for (int j = threadIdx.x; j < nb; j += WG) {
        const double v = b64[j];
        const uint32_t id = bid[j];
        int rank = 0;
        for (int y = 0; y < nb; ++y) rank += b64[y] < v || (b64[y] == v && bid[y] < id);
        if (rank >= need) band[j] = ~band[j];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nb; j += WG)
        if (band[j] < 0) sh.skey[~band[j]] = ~0ull;
    for (int i = threadIdx.x; i < n; i += WG)
        if (__uint_as_float((uint32_t)(sh.skey[i] >> 32)) > bhi) sh.skey[i] = ~0ull;
    __syncthreads();
    return true;
}

__global__ __launch_bounds__(WG) void finish_kernel(AnnArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem& sh = *reinterpret_cast<Smem*>(smem_raw);
    float* qs = reinterpret_cast<float*>(smem_raw + ((sizeof(Smem) + 15) & ~size_t(15)));
    const int64_t qi = blockIdx.x;
    const AnnQueryParams qpar = query_params(a, qi);
    const int B = qpar.budget;
    const int k = qpar.k;
    const uint32_t cnt = a.l_count[qi];
    if (cnt > (uint32_t)a.q_cap || cnt < (uint32_t)B) {
        // list overflow, or the bound fell short: the per-query kernel answers
        if (threadIdx.x == 0) {
            a.q_flag[qi] = 1;
            a.pq_list[1 + atomicAdd(&a.pq_list[0], 1u)] = (uint32_t)qi;
        }
        return;
    }
    QueryCtx qc;
    load_query(a, qi, qs, qc);
    int32_t* cpos = a.ws_cpos + qi * (int64_t)a.budget;
    float* cdist = a.ws_cdist + qi * (int64_t)a.budget;
    const uint32_t* list = a.l_list + qi * a.q_cap;
    const int32_t* perm = a.perm;
    const int n = (int)cnt;

    // L: the B smallest (pd^2 bits, id) of the list, kept in LDS as keys and
    // leaf positions (entries outside L get the key ~0). Every ball of the
    // rounds below holds the members of L with pd^2 bits <= its radius bits,
    // which is the prefix of L in (pd^2, id) order, so L needs no sorting.
    int nl;
    __syncthreads();
    if (n <= CAP) {
        // four entries per thread in flight: their list, projection and id
        // loads are issued together
        constexpr int PU = 4;
        for (int i0 = threadIdx.x; i0 < n; i0 += PU * WG) {
            int32_t pos[PU];
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const int i = i0 + u * WG;
                pos[u] = (int32_t)list[i < n ? i : i0];
            }
            float pd2[PU];
            int32_t id[PU];
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                pd2[u] = proj_dist2(a.proj + (int64_t)pos[u] * MP, qc.qp);
                id[u] = perm[pos[u]];
            }
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const int i = i0 + u * WG;
                if (i < n) {
                    sh.skey[i] = ((uint64_t)__float_as_uint(pd2[u]) << 32) | (uint32_t)id[u];
                    sh.spos[i] = pos[u];
                }
            }
        }
        __syncthreads();
        if (n > B) {
            const uint64_t kth = lds_select(n, B, sh);
            if (!cut_fp64(a, qi, qc, n, B, kth, sh)) {
                for (int i = threadIdx.x; i < n; i += WG)
                    if (sh.skey[i] > kth) sh.skey[i] = ~0ull;
                __syncthreads();
            }
        }
        nl = n;
    } else {
        auto list_src = [&](auto&& v) {
            for (int base = 0; base < n; base += WG) {
                const int i = base + threadIdx.x;
                const bool valid = i < n;
                uint64_t key = 0;
                int32_t pos = 0;
                if (valid) {
                    pos = (int32_t)list[i];
                    const float pd2 = proj_dist2(a.proj + (int64_t)pos * MP, qc.qp);
                    key = ((uint64_t)__float_as_uint(pd2) << 32) | (uint32_t)perm[pos];
                }
                v(valid, key, pos);
            }
        };
        block_select(list_src, [&](int32_t pos, int slot) { if (slot < B) cpos[slot] = pos; },
                     0ull, ~0ull, B, false, 0, sh);
        __syncthreads();
        for (int j = threadIdx.x; j < B; j += WG) {
            const int32_t pos = cpos[j];
            sh.skey[j] = ((uint64_t)__float_as_uint(proj_dist2(a.proj + (int64_t)pos * MP, qc.qp)) << 32) |
                         (uint32_t)perm[pos];
            sh.spos[j] = pos;
        }
        __syncthreads();
        nl = B;
    }

    // Verification keeps, per member of C, bounds lo2 <= exact <= hi2 on the
    // FP32 squared distance that verify would compute (FP16 rows, verify16);
    // a decision that the bounds cannot settle reads the FP32 rows of the
    // members concerned (verify_list), so every decision equals the one
    // taken on exact values. The index lists live in the histogram space.
    float* lo2 = a.ws_clo + qi * (int64_t)a.budget;
    float* hi2 = cdist;
    int32_t* ilist = reinterpret_cast<int32_t*>(sh.hist);
    double r = qpar.r_min;
    int n_ver = 0, rounds = 0, exit_kind = 0;
    uint32_t prev_bits = 0;
    for (;;) {
        if (rounds > 0) {
            // the c r stop: at least k verified members within c r
            const double cr = qpar.c * r;
            const float thr2 = (float)(cr * cr);
            int sure = 0, maybe = 0;
            for (int i = threadIdx.x; i < n_ver; i += WG) {
                sure += hi2[i] <= thr2;
                maybe += lo2[i] <= thr2 && hi2[i] > thr2;
            }
            sure = block_sum(sure, sh);
            maybe = block_sum(maybe, sh);
            if (sure < k && sure + maybe >= k) {
                if (threadIdx.x == 0) sh.cnt1 = 0;
                __syncthreads();
                for (int b0 = 0; b0 < n_ver; b0 += WG) {
                    const int i = b0 + threadIdx.x;
                    const bool take = i < n_ver && lo2[i] <= thr2 && hi2[i] > thr2;
                    const int slot = wave_append(take, &sh.cnt1);
                    if (take) ilist[slot] = i;
                }
                __syncthreads();
                verify_list(a, qs, cpos, ilist, sh.cnt1, lo2, hi2);
                __syncthreads();
                int loc = 0;
                for (int i = threadIdx.x; i < n_ver; i += WG) loc += hi2[i] <= thr2;
                sure = block_sum(loc, sh);
            }
            if (sure >= k) { exit_kind = PMLSH_EXIT_NEAR; break; }
        }
        if (rounds >= MAX_ROUNDS) r = __longlong_as_double(0x7ff0000000000000ll);
        const double Rd = qpar.t * r;
        const uint32_t r2bits = __float_as_uint((float)(Rd * Rd));
        // members of L that the ball gains this round go to C after the
        // n_ver verified ones
        if (threadIdx.x == 0) sh.cnt1 = n_ver;
        __syncthreads();
        for (int b0 = 0; b0 < nl; b0 += WG) {
            const int i = b0 + threadIdx.x;
            bool take = false;
            if (i < nl) {
                const uint64_t key = sh.skey[i];
                const uint32_t kb = (uint32_t)(key >> 32);
                take = key != ~0ull && kb <= r2bits && (rounds == 0 || kb > prev_bits);
            }
            const int slot = wave_append(take, &sh.cnt1);
            if (take && slot < B) cpos[slot] = sh.spos[i];
        }
        __syncthreads();
        const int nb = sh.cnt1 < B ? sh.cnt1 : B;
        ++rounds;
        verify16(a, qs, cpos, lo2, hi2, n_ver, nb);
        n_ver = nb;
        prev_bits = r2bits;
        __syncthreads();
        if (nb == B) { exit_kind = PMLSH_EXIT_BUDGET; break; }
        if (rounds >= a.max_rounds) break;
        r = qpar.c * r;
    }

    // Top-k: the k smallest upper bounds give hk; only members with lo2 <= hk
    // can be among the k nearest, and those are verified exactly.
    __syncthreads();
    for (int i = threadIdx.x; i < n_ver; i += WG)
        sh.skey[i] = ((uint64_t)__float_as_uint(hi2[i]) << 32) | (uint32_t)i;
    __syncthreads();
    const float hk = n_ver > k ? __uint_as_float((uint32_t)(lds_select(n_ver, k, sh) >> 32))
                                 : __int_as_float(0x7f800000);
    // members that the FP64 order of the re-rank could still place among the
    // k nearest: lower bound within a factor 1 + 4 gamma of hk
    const float hkw = (float)((double)hk * (1.0 + 4.0 * (double)verify_gamma(a)) * (1.0 + 1e-7));
    if (threadIdx.x == 0) sh.cnt1 = 0;
    __syncthreads();
    for (int b0 = 0; b0 < n_ver; b0 += WG) {
        const int i = b0 + threadIdx.x;
        const bool take = i < n_ver && lo2[i] <= hkw;
        const int slot = wave_append(take, &sh.cnt1);
        if (take) sh.spos[slot] = i;
    }
    __syncthreads();
    const int m = sh.cnt1;
    // all of them go to the FP64 re-rank, which decides their order from
    // their rows (no FP32 value is needed; the set holds every member the
    // FP64 order can place among the k nearest)
    bool done = false;
    if (m <= kRerankCap)
        done = rerank_topk64(
            a, qi, qs, cpos, m, __int_as_float(0x7f800000),
            [&](int j, float& v, int& mi) {
                v = 0.f;
                mi = sh.spos[j];
            },
            sh);
    if (!done) {
        // the FP32 order: exact values for the members still bounded, then
        // keys (distance^2 bits, id)
        if (threadIdx.x == 0) sh.cnt2 = 0;
        __syncthreads();
        for (int b0 = 0; b0 < m; b0 += WG) {
            const int j = b0 + threadIdx.x;
            const int i = j < m ? sh.spos[j] : 0;
            const bool take = j < m && lo2[i] != hi2[i];
            const int slot = wave_append(take, &sh.cnt2);
            if (take) ilist[slot] = i;
        }
        __syncthreads();
        verify_list(a, qs, cpos, ilist, sh.cnt2, lo2, hi2);
        __syncthreads();
        for (int j = threadIdx.x; j < m; j += WG) {
            const int i = sh.spos[j];
            sh.skey[j] = ((uint64_t)__float_as_uint(hi2[i]) << 32) | (uint32_t)perm[cpos[i]];
        }
        __syncthreads();
    }
    if (done) {
    } else if (m <= WG) {
        // keys are distinct (ids): the rank of each among the m is its slot
        if (threadIdx.x < m) {
            const uint64_t key = sh.skey[threadIdx.x];
            int rank = 0;
            for (int y = 0; y < m; ++y) rank += sh.skey[y] < key;
            if (rank < k) {
                a.out_ids[qi * a.out_stride + rank] = (int64_t)(uint32_t)key;
                a.out_dist[qi * a.out_stride + rank] = sqrtf(__uint_as_float((uint32_t)(key >> 32)));
            }
        }
    } else {
        const uint64_t kth = lds_select(m, k, sh);
        uint64_t* tmp = reinterpret_cast<uint64_t*>(sh.hist);
        if (threadIdx.x == 0) sh.cnt1 = 0;
        __syncthreads();
        for (int b0 = 0; b0 < m; b0 += WG) {
            const int i = b0 + threadIdx.x;
            const bool take = i < m && sh.skey[i] <= kth;
            const int slot = wave_append(take, &sh.cnt1);
            if (take) tmp[slot] = sh.skey[i];
        }
        __syncthreads();
        for (int j2 = threadIdx.x; j2 < k; j2 += WG) sh.skey[j2] = tmp[j2];
        __syncthreads();
        bitonic_sort(k, sh);
        for (int j2 = threadIdx.x; j2 < k; j2 += WG) {
            const uint64_t key = sh.skey[j2];
            a.out_ids[qi * a.out_stride + j2] = (int64_t)(uint32_t)key;
            a.out_dist[qi * a.out_stride + j2] = sqrtf(__uint_as_float((uint32_t)(key >> 32)));
        }
    }
    if (a.out_stats && threadIdx.x == 0) {
        int32_t* st = a.out_stats + qi * 4;
        st[0] = rounds;
        st[1] = n_ver;
        st[2] = exit_kind;
        st[3] = (int32_t)a.q_scanned[qi];
    }
}

}  // namespace

int64_t ann_pool_per_query(int64_t n) { return n < 16384 ? n : 16384; }

namespace {

// (r,c)-BC answer from one round of Algorithm 2 with k = 1 (Algorithm 1):
// when the ball fell short of the budget, the nearest candidate is the
// answer only if it lies within c r; otherwise (and for an empty ball) the
// answer is "nothing", id -1 and distance +inf.
__global__ __launch_bounds__(WG) void bc_finalize_kernel(int64_t* ids, float* dist,
                                                         const int32_t* stats, int64_t nq,
                                                         float cr) {
    const int64_t q = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (q >= nq) return;
    const int32_t n_cand = stats[q * 4 + 1], exit_kind = stats[q * 4 + 2];
    if (exit_kind == PMLSH_EXIT_BUDGET) return;
    if (n_cand == 0 || !(dist[q] <= cr)) {
        ids[q] = -1;
        dist[q] = __int_as_float(0x7f800000);
    }
}

}  // namespace

void launch_bc_finalize(int64_t* ids, float* dist, const int32_t* stats, int64_t nq, float cr,
                        hipStream_t stream) {
    if (nq <= 0) return;
    hipLaunchKernelGGL(bc_finalize_kernel, dim3((unsigned)((nq + WG - 1) / WG)), dim3(WG), 0,
                       stream, ids, dist, stats, nq, cr);
    PMLSH_HIP(hipGetLastError());
}

bool ann_fast_path(int64_t budget) { return budget <= CAP; }

int ann_lds_bytes(int d_pad) {
    return (int)(((sizeof(Smem) + 15) & ~size_t(15)) + (size_t)d_pad * sizeof(float));
}

void launch_ann(const AnnLaunch& L, hipStream_t stream) {
    const pmlsh_index& x = *L.idx;
    if (L.nq <= 0) return;
    if (x.levels > MAX_LEVELS) fail(PMLSH_EUNSUPPORTED, "tree deeper than 16 levels");
    AnnArgs a{};
    a.data = x.data;
    a.proj = x.proj_hi;
    a.perm = x.perm;
    a.ncen = x.tree.centre;
    a.nrad = x.tree.radius;
    a.hrmin = x.tree.hr_min;
    a.hrmax = x.tree.hr_max;
    a.cb = x.tree.child_begin;
    a.ce = x.tree.child_end;
    a.npts = x.tree.npts;
    a.piv = x.tree.pivots;
    a.n_nodes = x.n_nodes;
    a.n_leaves = x.n_leaves;
    a.levels = x.levels;
    a.s = x.num_pivots;
    a.d = x.d;
    a.d_pad = x.d_pad;
    for (int l = 0; l <= x.levels; ++l) a.level_begin[l] = (int32_t)x.level_begin[l];
    a.coord_scale = x.coord_scale;
    a.scan_scale = x.scan_scale;
    for (int t = 0; t < MP; ++t) a.scen[t] = x.scan_centre[t];
    a.eps_max = x.eps_max;
    a.qlp = nullptr;
    a.qeps = nullptr;
    a.q = L.queries;
    a.qp = L.qproj;
    a.qp_lo = L.qproj_lo;
    a.proj_lo = x.proj_lo;
    a.qpar = L.qpar;
    a.out_stride = L.out_stride > 0 ? L.out_stride : L.k;
    a.k = L.k;
    a.budget = (int32_t)L.budget;
    a.c = L.c;
    a.t = L.t;
    a.r_min = L.r_min;
    a.max_rounds = L.max_rounds > 0 ? L.max_rounds : 0x7fffffff;
    a.ws_front = L.ws_front;
    a.ws_cpos = L.ws_cpos;
    a.ws_cdist = L.ws_cdist;
    a.ws_topk = L.ws_topk;
    a.out_ids = L.out_ids;
    a.out_dist = L.out_dist;
    a.out_stats = L.out_stats;
    a.nq = (int)L.nq;
    a.n = x.n;
    a.proj16 = x.proj16;
    a.n_pad16 = x.n_pad16;
    a.scale16 = x.scale16;
    a.chunk_cen = x.chunk_cen;
    a.chunk_rad = x.chunk_rad;
    a.data16 = x.data16;
    a.d16_scale = x.data16_scale;
    a.d16_eps = x.data16_eps;
    a.d16 = x.d16;
    const int lds = ann_lds_bytes(x.d16);
    PMLSH_HIP(hipFuncSetAttribute((const void*)ann_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    if (L.fast) {
        a.qaug = L.ws_qaug;
        a.qlp = L.ws_qlp;
        a.qeps = L.ws_qeps;
        a.qtest = L.ws_qtest;
        a.cmask = L.ws_cmask;
        a.cwords = (int)((L.nq + 63) / 64);
        a.cdist = L.ws_cdist2;
        a.cgmin = L.ws_cgmin;
        a.cgroups = cdist_groups(x.n_pad16 / 64);
        a.gld = cdist_gmin_len(x.n_pad16 / 64);
        a.ws_clo = L.ws_clo;
        a.q_flag = L.q_flag;
        a.pq_list = L.pq_list;
        a.l_count = L.l_count;
        a.q_scanned = L.q_scanned;
        a.l_list = L.l_list;
        a.q_cap = (int)L.pool_cap;
        const int lds0 = ann_lds_bytes(0);
        const int64_t nchunk = x.n_pad16 / 64;
        {
            StageTimer tm(PMLSH_STAGE_DIST, stream);
            dim3 dgrid((unsigned)((nchunk + DCB - 1) / DCB), (unsigned)((L.nq + DQB - 1) / DQB));
            hipLaunchKernelGGL(dist_kernel, dgrid, dim3(WG), 0, stream, a);
            PMLSH_HIP(hipGetLastError());
        }
        {
            StageTimer tm(PMLSH_STAGE_TAU, stream);
            const int64_t ngr = (nchunk + 63) / 64;
            a.grp_cap = (int)std::min<int64_t>(kGrpCap, std::max<int64_t>(0, tune_get(PMLSH_TUNE_GROUP_LIST)));
            const size_t min_bytes = 2 * (size_t)((ngr + 7) & ~7);
            a.glds = tune_get(PMLSH_TUNE_GROUP_MINIMA_LDS) != 0 &&
                     min_bytes + 4 * (size_t)kGrpCap <= kTauGroupLds;
            const size_t lds_t = std::max((size_t)lds0, offsetof(Smem, skey) +
                                          (a.glds ? min_bytes : 0) +
                                          4 * (size_t)(kGrpCap + kSelCap));
            PMLSH_HIP(hipFuncSetAttribute((const void*)tau_kernel,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_t));
            hipLaunchKernelGGL(tau_kernel, dim3((unsigned)L.nq), dim3(WG), (unsigned)lds_t, stream, a);
            PMLSH_HIP(hipGetLastError());
            dim3 mgrid((unsigned)((nchunk + MCH - 1) / MCH), (unsigned)((L.nq + MQB - 1) / MQB));
            hipLaunchKernelGGL(mask_kernel, mgrid, dim3(WG), 0, stream, a);
            PMLSH_HIP(hipGetLastError());
        }
        // one resident wave of workgroups striding over the chunks, in the
        // block shape that suits the index's size
        const int64_t shape = tune_get(PMLSH_TUNE_SCAN_SHAPE);
        const bool large = shape == 0 ? nchunk >= kScanLargeChunks : shape == 2;
        const void* scan_fn =
            large ? (const void*)scan_kernel<PMLSH_SCAN_QB_LARGE, PMLSH_SCAN_WAVES_PER_EU_LARGE>
                  : (const void*)scan_kernel<PMLSH_SCAN_QB, PMLSH_SCAN_WAVES_PER_EU>;
        const int sqb = large ? PMLSH_SCAN_QB_LARGE : PMLSH_SCAN_QB;
        static thread_local int scan_slots[64][2] = {};
        int& slots = scan_slots[x.device & 63][large ? 1 : 0];
        if (slots == 0) {
            int per_cu = 0, cus = 0;
            PMLSH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, scan_fn, WG, 0));
            PMLSH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, x.device));
            slots = per_cu > 0 && cus > 0 ? per_cu * cus : (int)kScanBlocks;
        }
        const int64_t ny = (L.nq + sqb - 1) / sqb;
        int64_t gx = std::max<int64_t>(1, slots / ny);
        gx = std::min(gx, nchunk);   // at least one chunk per workgroup on average
        dim3 sgrid((unsigned)gx, (unsigned)ny);
        {
            StageTimer tm(PMLSH_STAGE_FILTER, stream);
            if (large)
                hipLaunchKernelGGL((scan_kernel<PMLSH_SCAN_QB_LARGE, PMLSH_SCAN_WAVES_PER_EU_LARGE>),
                                   sgrid, dim3(WG), 0, stream, a);
            else
                hipLaunchKernelGGL((scan_kernel<PMLSH_SCAN_QB, PMLSH_SCAN_WAVES_PER_EU>), sgrid,
                                   dim3(WG), 0, stream, a);
            PMLSH_HIP(hipGetLastError());
        }
        PMLSH_HIP(hipFuncSetAttribute((const void*)finish_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds));
        {
            StageTimer tm(PMLSH_STAGE_FINISH, stream);
            hipLaunchKernelGGL(finish_kernel, dim3((unsigned)L.nq), dim3(WG), lds, stream, a);
            PMLSH_HIP(hipGetLastError());
        }
    }
    // per-query path: every query when the fast path does not apply, else only
    // the queries the fast path flagged
    StageTimer tm(PMLSH_STAGE_PERQUERY, stream);
    const int64_t slots = std::max<int64_t>(1, std::min<int64_t>(L.front_slots, L.nq));
    hipLaunchKernelGGL(ann_kernel, dim3((unsigned)slots), dim3(WG), lds, stream, a);
    PMLSH_HIP(hipGetLastError());
}

}  // namespace pmlsh
