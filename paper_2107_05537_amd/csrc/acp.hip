// (c,k)-ACP by radius filtering (Section 6.3) on gfx950.
//
//   seeds    every pair inside one leaf: lower and upper bounds of its squared
//            distance from an FP16 matrix-core Gram kernel, and the exact FP32
//            distance of the seeds that can reach the top-k (leaves of at most
//            64 points; acp_seed_gram_kernel), else exact FP32 squared
//            distances by direct differences for all (acp_seed_join_kernel,
//            acp_self_join_kernel);
//   ub       the k-th smallest seed distance (device-wide radix select);
//   tiles    leaf pairs (e1 < e2) whose Mindist of Eq. 11 can fall below
//            t*ub (acp_tile_filter_kernel), a lossless skip of whole leaf pairs;
//   scan     all point pairs of the surviving tiles: pairs whose parent-
//            distance bound (PD, Sec. 4.1) already reaches t*ub are dropped,
//            the others get the projected distance from the hi/lo coordinate
//            pairs and are kept when strictly below t*ub (acp_pd_kernel,
//            acp_tile_scan_kernel);
//   budget   at most T verified pairs: the projected-nearest candidates are
//            kept (device-wide radix select on (pd^2, i, j));
//   verify   exact FP32 squared distance of the kept candidates;
//   top-k    the k smallest (dist^2, i, j) over seeds and candidates.
//
// Pairs are carried as three uint32 arrays: the FP32 bit pattern of a squared
// distance (monotone for non-negative floats), then the ids i < j. Ordering by
// the 96-bit concatenation is ordering by (distance, i, j).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace pmlsh {
namespace {

constexpr int WG = 256;
constexpr int NB = 2048;
constexpr int SJ_KC = 16;          // columns staged per self-join step
constexpr int SJ_PER = 8;          // pairs owned by a thread per batch

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Slot for lanes with take == true, one global atomic per wave; returns -1
// for lanes that do not take.
__device__ __forceinline__ int64_t wave_append_global(bool take, unsigned long long* counter) {
    const uint64_t m = __ballot(take);
    if (m == 0) return -1;
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    return (int64_t)base + __popcll(m & ((1ull << lane_id()) - 1ull));
}

// ---------------------------------------------------------------- seeds
__global__ __launch_bounds__(WG) void acp_self_join_kernel(
    const float* __restrict__ data, int d_pad, const int32_t* __restrict__ perm, int64_t n,
    int L, const int64_t* __restrict__ seed_off, uint32_t* __restrict__ k0,
    uint32_t* __restrict__ ii, uint32_t* __restrict__ jj) {
    __shared__ float xs[256][SJ_KC + 1];
    const int64_t leaf = blockIdx.x;
    const int64_t p0 = leaf * L;
    const int cnt = (int)(n - p0 < L ? n - p0 : L);
    const int P = cnt * (cnt - 1) / 2;
    const int64_t out0 = seed_off[leaf];
    for (int base = 0; base < P; base += WG * SJ_PER) {
        int ra[SJ_PER], rb[SJ_PER];
        float acc[SJ_PER];
#pragma unroll
        for (int u = 0; u < SJ_PER; ++u) {
            const int p = base + threadIdx.x + u * WG;
            ra[u] = -1; rb[u] = -1; acc[u] = 0.f;
            if (p < P) {
                int a = 0, rem = p;
                while (rem >= cnt - 1 - a) { rem -= cnt - 1 - a; ++a; }
                ra[u] = a;
                rb[u] = a + 1 + rem;
            }
        }
        for (int c0 = 0; c0 < d_pad; c0 += SJ_KC) {
            for (int e = threadIdx.x; e < cnt * SJ_KC; e += WG) {
                const int r = e / SJ_KC, c = e % SJ_KC;
                xs[r][c] = (c0 + c < d_pad) ? data[(p0 + r) * d_pad + c0 + c] : 0.f;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < SJ_PER; ++u) {
                if (ra[u] >= 0) {
#pragma unroll
                    for (int c = 0; c < SJ_KC; ++c) {
                        const float t = xs[ra[u]][c] - xs[rb[u]][c];
                        acc[u] = __fmaf_rn(t, t, acc[u]);
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < SJ_PER; ++u) {
            if (ra[u] >= 0) {
                const int p = base + threadIdx.x + u * WG;
                const uint32_t ia = (uint32_t)perm[p0 + ra[u]], ib = (uint32_t)perm[p0 + rb[u]];
                k0[out0 + p] = __float_as_uint(acc[u]);
                ii[out0 + p] = ia < ib ? ia : ib;
                jj[out0 + p] = ia < ib ? ib : ia;
            }
        }
    }
}

// ---------------------------------------------------------------- tiles
struct NodeView {
    const float* cen;
    const float* rad;
    const float* hrmin;
    const float* hrmax;
    int64_t n_nodes;
    int s;
};

// Mindist of Eq. 11: the larger of the pivot-ring gap and the centre gap.
// Once the centre gap exceeds `limit` the rings cannot change whether the
// result exceeds it, and they are not read.
__device__ __forceinline__ float mindist(const NodeView& v, int64_t a, int64_t b,
                                         float limit = INFINITY) {
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
        const float t = v.cen[(int64_t)j * v.n_nodes + a] - v.cen[(int64_t)j * v.n_nodes + b];
        acc = fmaf(t, t, acc);
    }
    float m = sqrtf(acc) - v.rad[a] - v.rad[b];
    if (m > limit) return m;
    for (int i = 0; i < v.s; ++i) {
        const int64_t oa = (int64_t)i * v.n_nodes + a, ob = (int64_t)i * v.n_nodes + b;
        m = fmaxf(m, v.hrmin[ob] - v.hrmax[oa]);
        m = fmaxf(m, v.hrmin[oa] - v.hrmax[ob]);
    }
    return m;
}

// The radii of one canonical call, computed on the device from the selected
// seed distance so that no host round trip separates the seeds from the
// tile filter and the pair scan (the same arithmetic as the host's).
struct AcpRadius {
    float R2;          // (t ub)^2, the pair filter's squared radius
    float limit;       // t ub plus the rounding slack of the node tests
    uint32_t seed_lim; // bits of ub^2 (1 + 4 gamma) rounded up: seeds the pool takes
    uint32_t pad;
};

// Leaf pairs (e1 < e2; with diag also e1 = e2) whose Mindist can fall below
// `limit`. One workgroup per first leaf e1: its kept tiles are compacted in
// LDS and appended with one global atomic per flush, so a row's tiles lie
// together in the list (the tile scan keeps e1's rows across them) and the
// single counter sees a few thousand atomics instead of one per wave.
constexpr int kRowBuf = 2048;
__global__ __launch_bounds__(WG) void acp_tile_filter_kernel(
    NodeView v, int64_t leaf_base, int64_t n_leaves, float limit, int diag,
    int2* __restrict__ tiles, int64_t cap, unsigned long long* __restrict__ counter,
    const AcpRadius* __restrict__ rad) {
    if (rad) limit = rad->limit;
    __shared__ int rowbuf[kRowBuf];
    __shared__ int wcount[WG / 64];
    __shared__ int nrow;
    __shared__ unsigned long long gbase;
    const int64_t e1 = blockIdx.x;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) nrow = 0;
    __syncthreads();
    for (int64_t s0 = diag ? e1 : e1 + 1; s0 < n_leaves; s0 += WG) {
        const int64_t e2 = s0 + threadIdx.x;
        bool keep = false;
        if (e2 < n_leaves)
            keep = e2 == e1 || mindist(v, leaf_base + e1, leaf_base + e2, limit) <= limit;
        const uint64_t m = __ballot(keep);
        if (lane == 0) wcount[wave] = __popcll(m);
        __syncthreads();
        int off = nrow, tot = 0;
        for (int w = 0; w < WG / 64; ++w) {
            if (w < wave) off += wcount[w];
            tot += wcount[w];
        }
        if (keep) rowbuf[off + __popcll(m & ((1ull << lane) - 1ull))] = (int)e2;
        __syncthreads();
        if (threadIdx.x == 0) nrow += tot;
        __syncthreads();
        const int cnt = nrow;
        if (cnt > 0 && (cnt > kRowBuf - WG || s0 + WG >= n_leaves)) {
            if (threadIdx.x == 0) gbase = atomicAdd(counter, (unsigned long long)cnt);
            __syncthreads();
            for (int q = threadIdx.x; q < cnt; q += WG) {
                const int64_t slot = (int64_t)gbase + q;
                if (slot < cap) tiles[slot] = make_int2((int)e1, rowbuf[q]);
            }
            __syncthreads();
            if (threadIdx.x == 0) nrow = 0;
            __syncthreads();
        }
    }
}

// Distance from every point (hi + lo) to the centre of its own leaf, FP32:
// the parent distance PD that the PM-tree keeps for leaf entries.
__global__ __launch_bounds__(WG) void acp_pd_kernel(
    const float* __restrict__ phi, const float* __restrict__ plo, NodeView v, int64_t leaf_base,
    int64_t n, int L, float* __restrict__ pd) {
    const int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (j >= n) return;
    const int64_t node = leaf_base + j / L;
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < MP; ++t) {
        const float dt = __fadd_rn(__fsub_rn(phi[j * MP + t], v.cen[(int64_t)t * v.n_nodes + node]),
                                   plo[j * MP + t]);
        acc = __fmaf_rn(dt, dt, acc);
    }
    pd[j] = sqrtf(acc);
}

// All point pairs (a in leaf e1, b in leaf e2; a < b when e1 = e2) of the
// surviving tiles.
//   1. PD filter: |dist(a, centre of e2) - PD(b)| is a lower bound of the
//      projected distance (triangle inequality); pairs whose bound (less its
//      FP32 error) reaches R cannot pass and are dropped. One wave takes one a
//      at a time, lanes take b; the passing pairs are compacted in LDS.
//   2. the remaining pairs get the projected distance from the hi/lo
//      coordinate pairs and are kept when pd^2 < R2.
// The kept set is exactly the set a scan of every pair would keep.
__global__ __launch_bounds__(WG) void acp_tile_scan_kernel(
    const float* __restrict__ phi, const float* __restrict__ plo, const float* __restrict__ ppd,
    NodeView v, int64_t leaf_base, const int32_t* __restrict__ perm, int64_t n, int L,
    const int2* __restrict__ tiles, int64_t n_tiles, float R2, float Rlim,
    uint32_t* __restrict__ ck0, uint32_t* __restrict__ cii, uint32_t* __restrict__ cjj,
    int64_t cap, unsigned long long* __restrict__ counter) {
    extern __shared__ __align__(16) float lds[];
    float* h1 = lds;
    float* l1 = h1 + L * MP;
    float* h2 = l1 + L * MP;
    float* l2 = h2 + L * MP;
    float* da = l2 + L * MP;              // dist(a, centre of e2)
    float* pb = da + L;                   // PD(b)
    int32_t* id1 = reinterpret_cast<int32_t*>(pb + L);
    int32_t* id2 = id1 + L;
    uint32_t* plist = reinterpret_cast<uint32_t*>(id2 + L);   // 64 x 64 pairs (a << 16 | b)
    __shared__ float cen[MP];
    __shared__ int npl;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const float u = 5.9604645e-08f;
    // a contiguous run of the tile list per workgroup: the filter appends the
    // tiles of one first leaf in runs, so the first leaf's rows stay in LDS
    // from one tile to the next
    const int64_t per = (n_tiles + gridDim.x - 1) / gridDim.x;
    const int64_t t_end = min(n_tiles, ((int64_t)blockIdx.x + 1) * per);
    int held = -1;
    for (int64_t t = (int64_t)blockIdx.x * per; t < t_end; ++t) {
        const int2 tl = tiles[t];
        const int64_t a0 = (int64_t)tl.x * L, b0 = (int64_t)tl.y * L;
        const int ca = (int)(n - a0 < L ? n - a0 : L);
        const int cb = (int)(n - b0 < L ? n - b0 : L);
        if (tl.x != held) {
            for (int e = threadIdx.x; e < ca * MP; e += WG) {
                h1[e] = phi[a0 * MP + e];
                l1[e] = plo[a0 * MP + e];
            }
            for (int e = threadIdx.x; e < ca; e += WG) id1[e] = perm[a0 + e];
            held = tl.x;
        }
        for (int e = threadIdx.x; e < cb * MP; e += WG) {
            h2[e] = phi[b0 * MP + e];
            l2[e] = plo[b0 * MP + e];
        }
        for (int e = threadIdx.x; e < cb; e += WG) {
            id2[e] = perm[b0 + e];
            pb[e] = ppd[b0 + e];
        }
        if (threadIdx.x < MP) cen[threadIdx.x] = v.cen[(int64_t)threadIdx.x * v.n_nodes + leaf_base + tl.y];
        if (threadIdx.x == 0) npl = 0;
        __syncthreads();
        for (int a = threadIdx.x; a < ca; a += WG) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < MP; ++j) {
                const float dt = __fadd_rn(__fsub_rn(h1[a * MP + j], cen[j]), l1[a * MP + j]);
                acc = __fmaf_rn(dt, dt, acc);
            }
            da[a] = sqrtf(acc);
        }
        __syncthreads();
        // pairs in blocks of 64 x 64, so the compacted list holds at most 4,096
        for (int ab = 0; ab < ca; ab += 64) {
            for (int bb = 0; bb < cb; bb += 64) {
                // 1: PD filter and compaction
                const int ae = min(ca, ab + 64);
                for (int a = ab + wave; a < ae; a += WG / 64) {
                    const float x = da[a];
                    const int b = bb + lane;
                    bool pass = false;
                    if (b < cb && (tl.x != tl.y || b > a)) {
                        const float y = pb[b];
                        // each distance carries at most ~12 u of relative error
                        pass = fabsf(x - y) - 32.f * u * (x + y) < Rlim;
                    }
                    const uint64_t m = __ballot(pass);
                    if (m) {
                        const int leader = __ffsll((unsigned long long)m) - 1;
                        int base = 0;
                        if (lane == leader) base = atomicAdd(&npl, __popcll(m));
                        base = __shfl(base, leader);
                        if (pass) plist[base + __popcll(m & ((1ull << lane) - 1ull))] =
                            ((uint32_t)a << 16) | (uint32_t)b;
                    }
                }
                __syncthreads();
                // 2: projected distance of the remaining pairs
                const int np = npl;
                for (int base = 0; base < np; base += WG) {
                    const int q = base + threadIdx.x;
                    bool hit = false;
                    float pd2 = 0.f;
                    int a = 0, b = 0;
                    if (q < np) {
                        a = (int)(plist[q] >> 16);
                        b = (int)(plist[q] & 0xffffu);
                        const float* x1 = h1 + a * MP;
                        const float* y1 = l1 + a * MP;
                        const float* x2 = h2 + b * MP;
                        const float* y2 = l2 + b * MP;
#pragma unroll
                        for (int j = 0; j < MP; ++j) {
                            // (hi1 - hi2) is exact for nearby points (Sterbenz);
                            // the lo parts restore what rounding to FP32 lost
                            const float dt = __fadd_rn(__fsub_rn(x1[j], x2[j]), __fsub_rn(y1[j], y2[j]));
                            pd2 = __fmaf_rn(dt, dt, pd2);
                        }
                        hit = pd2 < R2;
                    }
                    const int64_t slot = wave_append_global(hit, counter);
                    if (hit && slot < cap) {
                        const uint32_t ia = (uint32_t)id1[a], ib = (uint32_t)id2[b];
                        ck0[slot] = __float_as_uint(pd2);
                        cii[slot] = ia < ib ? ia : ib;
                        cjj[slot] = ia < ib ? ib : ia;
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) npl = 0;
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- wave scan
// Leaves of at most 64 points: one wave per leaf computes the parent
// distances PD of its points (as acp_pd_kernel) and sorts them ascending
// (ties by position) across its lanes: spd holds the sorted values (+inf
// past the leaf's count), sidx the position of each in the leaf.
__global__ __launch_bounds__(WG) void acp_pd_sorted_kernel(
    const float* __restrict__ phi, const float* __restrict__ plo, NodeView v, int64_t leaf_base,
    int64_t n, int L, int64_t n_leaves, float* __restrict__ ppd, float* __restrict__ spd,
    uint8_t* __restrict__ sidx) {
    const int64_t leaf = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    if (leaf >= n_leaves) return;          // the whole wave leaves together
    const int lane = lane_id();
    const int64_t p0 = leaf * L;
    const int cnt = (int)(n - p0 < L ? n - p0 : L);
    float val = INFINITY;
    if (lane < cnt) {
        const int64_t node = leaf_base + leaf;
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < MP; ++t) {
            const float dt = __fadd_rn(
                __fsub_rn(phi[(p0 + lane) * MP + t], v.cen[(int64_t)t * v.n_nodes + node]),
                plo[(p0 + lane) * MP + t]);
            acc = __fmaf_rn(dt, dt, acc);
        }
        val = sqrtf(acc);
        ppd[p0 + lane] = val;
    }
    int idx = lane;
    // bitonic network over the 64 lanes on (value, position)
    for (int s = 2; s <= 64; s <<= 1) {
        for (int j = s >> 1; j > 0; j >>= 1) {
            const float ov = __shfl_xor(val, j);
            const int oi = __shfl_xor(idx, j);
            const bool keep_min = ((lane & j) == 0) == ((lane & s) == 0);
            const bool other_less = ov < val || (ov == val && oi < idx);
            if (keep_min == other_less) {
                val = ov;
                idx = oi;
            }
        }
    }
    spd[leaf * 64 + lane] = val;
    sidx[leaf * 64 + lane] = (uint8_t)idx;
}

// Number of the 64 ascending values y (one per lane) below v (strict) or at
// most v; every lane of the wave must call it.
__device__ __forceinline__ int count_sorted(float y, float v, bool strict) {
    int pos = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const float yy = __shfl(y, pos + step - 1);
        if (strict ? yy < v : yy <= v) pos += step;
    }
    const float yy = __shfl(y, pos);
    if (strict ? yy < v : yy <= v) ++pos;
    return pos;
}

__device__ __forceinline__ float readlane_f(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}

// Lanes with a PD candidate range of at most this many pairs each take them
// one by one; a wider tile is scanned whole.
constexpr int kSparseMax = 40;

// The pairs of the surviving tiles (leaves of at most 64 points), one wave
// per contiguous run of the tile list; lane a holds point a of the first
// leaf (its hi/lo projection in registers, kept while the first leaf stays
// the same).
//   1. lane a computes x = dist(a, centre of e2); the pairs (a, b) whose PD
//      bound |x - PD(b)| (less its FP32 error, as in acp_tile_scan_kernel)
//      stays below Rlim have PD(b) inside an interval around x, found by
//      binary search in e2's sorted PDs (the interval is widened so that it
//      holds every such b);
//   2. each b of the interval gets the same per-pair PD test and, when it
//      passes, the projected distance from the hi/lo coordinates; pairs
//      with pd^2 < R2 are emitted. When some lane's interval is wide, the
//      whole tile is scanned instead: lanes take b, the loop takes a.
// The emitted set is the set acp_tile_scan_kernel emits for the same tiles.
__global__ __launch_bounds__(WG) void acp_tile_scan_wave_kernel(
    const float* __restrict__ phi, const float* __restrict__ plo, const float* __restrict__ ppd,
    const float* __restrict__ spd, const uint8_t* __restrict__ sidx, NodeView v,
    int64_t leaf_base, const int32_t* __restrict__ perm, int64_t n, int L,
    const int2* __restrict__ tiles, int64_t n_tiles, float R2, float Rlim,
    uint32_t* __restrict__ ck0, uint32_t* __restrict__ cii, uint32_t* __restrict__ cjj,
    int64_t cap, unsigned long long* __restrict__ counter,
    const unsigned long long* __restrict__ dn_tiles, const AcpRadius* __restrict__ rad) {
    if (dn_tiles) n_tiles = (int64_t)*dn_tiles;
    if (rad) {
        R2 = rad->R2;
        Rlim = rad->limit;
    }
    const int lane = lane_id();
    const int64_t gw = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (WG / 64);
    const int64_t per = (n_tiles + nw - 1) / nw;
    const int64_t t_beg = gw * per;
    const int64_t t_end = t_beg + per < n_tiles ? t_beg + per : n_tiles;
    const float u = 5.9604645e-08f;
    float h1[MP], l1[MP];
    int held = -1, ca = 0;
    uint32_t id1 = 0;
    // Two tiles ahead the tile's index is loaded, one tile ahead its second
    // leaf's centre and sorted PDs (which need that index): a tile then waits
    // for one memory round trip begun a whole tile earlier instead of two in
    // a row. These loads are unconditional (past the wave's last tile they
    // read it again), so the compiler waits for the oldest ones only.
    const int64_t t_last = t_end - 1;
    int2 nt = t_beg < t_end ? tiles[t_beg] : make_int2(0, 0);
    float ncen[MP], ny = 0.f;
    int nsb = 0;
    auto fetch = [&](int e) {
        const int64_t node = leaf_base + e;
#pragma unroll
        for (int j = 0; j < MP; ++j) ncen[j] = v.cen[(int64_t)j * v.n_nodes + node];
        ny = spd[(int64_t)e * 64 + lane];
        nsb = sidx[(int64_t)e * 64 + lane];
    };
    int2 nt2 = nt;
    if (t_beg < t_end) {
        fetch(__builtin_amdgcn_readfirstlane(nt.y));
        nt2 = tiles[t_beg + 1 <= t_last ? t_beg + 1 : t_last];
    }
    for (int64_t t = t_beg; t < t_end; ++t) {
        const int e1 = __builtin_amdgcn_readfirstlane(nt.x);
        const int e2 = __builtin_amdgcn_readfirstlane(nt.y);
        float cen[MP];
#pragma unroll
        for (int j = 0; j < MP; ++j) cen[j] = ncen[j];
        const float y = ny;
        const int sb = nsb;
        nt = nt2;                                          // tile t + 1 (or t_last)
        fetch(__builtin_amdgcn_readfirstlane(nt.y));
        nt2 = tiles[t + 2 <= t_last ? t + 2 : t_last];     // tile t + 2 (or t_last)
        const int64_t a0 = (int64_t)e1 * L, b0 = (int64_t)e2 * L;
        if (e1 != held) {
            ca = (int)(n - a0 < L ? n - a0 : L);
            const int a = lane < ca ? lane : 0;
            const float4* hp = reinterpret_cast<const float4*>(phi + (a0 + a) * MP);
            const float4* lp = reinterpret_cast<const float4*>(plo + (a0 + a) * MP);
#pragma unroll
            for (int q = 0; q < MP / 4; ++q) {
                const float4 hv = hp[q], lv = lp[q];
                h1[4 * q] = hv.x; h1[4 * q + 1] = hv.y; h1[4 * q + 2] = hv.z; h1[4 * q + 3] = hv.w;
                l1[4 * q] = lv.x; l1[4 * q + 1] = lv.y; l1[4 * q + 2] = lv.z; l1[4 * q + 3] = lv.w;
            }
            id1 = (uint32_t)perm[a0 + a];
            held = e1;
        }
        const int cb = (int)(n - b0 < L ? n - b0 : L);
        const bool diag = e1 == e2;
        // 1. distance to the centre of e2, interval of PD(b)
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < MP; ++j) {
            const float dt = __fadd_rn(__fsub_rn(h1[j], cen[j]), l1[j]);
            acc = __fmaf_rn(dt, dt, acc);
        }
        const float x = sqrtf(acc);
        // |x - y| - 32u (x + y) < Rlim implies y in (lov, hiv) in exact
        // arithmetic; the bounds are widened by 1e-6 (x + Rlim), far more than
        // the FP32 rounding of that test and of the bounds themselves
        float lov = (x * (1.f - 32.f * u) - Rlim) / (1.f + 32.f * u);
        float hiv = (x * (1.f + 32.f * u) + Rlim) / (1.f - 32.f * u);
        const float wid = (x + (Rlim < INFINITY ? Rlim : 0.f)) * 1e-6f + 1e-30f;
        lov -= wid;
        hiv += wid;
        if (lane >= ca) {
            lov = INFINITY;
            hiv = -INFINITY;
        }
        const int lo = count_sorted(y, lov, true);
        int hi = count_sorted(y, hiv, false);
        hi = hi < cb ? hi : cb;
        const int mine = hi > lo ? hi - lo : 0;
        const int widest = wave_max(mine);
        if (widest == 0) continue;
        if (widest <= kSparseMax) {
            // 2a. lane by lane
            for (int it = 0; it < widest; ++it) {
                const int pos = lo + (it < mine ? it : 0);
                const float yb = __shfl(y, pos);
                const int b = __shfl(sb, pos);
                bool hit = false;
                float pd2 = 0.f;
                uint32_t id2 = 0;
                if (it < mine && (!diag || b > lane) &&
                    fabsf(x - yb) - 32.f * u * (x + yb) < Rlim) {
                    const float4* hp = reinterpret_cast<const float4*>(phi + (b0 + b) * MP);
                    const float4* lp = reinterpret_cast<const float4*>(plo + (b0 + b) * MP);
#pragma unroll
                    for (int q = 0; q < MP / 4; ++q) {
                        const float4 hv = hp[q], lv = lp[q];
                        float dt;
                        dt = __fadd_rn(__fsub_rn(h1[4 * q], hv.x), __fsub_rn(l1[4 * q], lv.x));
                        pd2 = __fmaf_rn(dt, dt, pd2);
                        dt = __fadd_rn(__fsub_rn(h1[4 * q + 1], hv.y), __fsub_rn(l1[4 * q + 1], lv.y));
                        pd2 = __fmaf_rn(dt, dt, pd2);
                        dt = __fadd_rn(__fsub_rn(h1[4 * q + 2], hv.z), __fsub_rn(l1[4 * q + 2], lv.z));
                        pd2 = __fmaf_rn(dt, dt, pd2);
                        dt = __fadd_rn(__fsub_rn(h1[4 * q + 3], hv.w), __fsub_rn(l1[4 * q + 3], lv.w));
                        pd2 = __fmaf_rn(dt, dt, pd2);
                    }
                    hit = pd2 < R2;
                    id2 = (uint32_t)perm[b0 + b];
                }
                const int64_t slot = wave_append_global(hit, counter);
                if (hit && slot < cap) {
                    ck0[slot] = __float_as_uint(pd2);
                    cii[slot] = id1 < id2 ? id1 : id2;
                    cjj[slot] = id1 < id2 ? id2 : id1;
                }
            }
        } else {
            // 2b. the whole tile: lane b holds point b of e2, the loop takes a
            const int b = lane < cb ? lane : 0;
            float h2[MP], l2[MP];
            const float4* hp = reinterpret_cast<const float4*>(phi + (b0 + b) * MP);
            const float4* lp = reinterpret_cast<const float4*>(plo + (b0 + b) * MP);
#pragma unroll
            for (int q = 0; q < MP / 4; ++q) {
                const float4 hv = hp[q], lv = lp[q];
                h2[4 * q] = hv.x; h2[4 * q + 1] = hv.y; h2[4 * q + 2] = hv.z; h2[4 * q + 3] = hv.w;
                l2[4 * q] = lv.x; l2[4 * q + 1] = lv.y; l2[4 * q + 2] = lv.z; l2[4 * q + 3] = lv.w;
            }
            const float yb = ppd[b0 + b];
            const uint32_t id2 = (uint32_t)perm[b0 + b];
            for (int a = 0; a < ca; ++a) {
                const float xa = readlane_f(x, a);
                bool hit = false;
                float pd2 = 0.f;
                if (lane < cb && (!diag || lane > a) &&
                    fabsf(xa - yb) - 32.f * u * (xa + yb) < Rlim) {
#pragma unroll
                    for (int j = 0; j < MP; ++j) {
                        const float dt = __fadd_rn(__fsub_rn(readlane_f(h1[j], a), h2[j]),
                                                   __fsub_rn(readlane_f(l1[j], a), l2[j]));
                        pd2 = __fmaf_rn(dt, dt, pd2);
                    }
                    hit = pd2 < R2;
                }
                const uint32_t ia = (uint32_t)__builtin_amdgcn_readlane((int)id1, a);
                const int64_t slot = wave_append_global(hit, counter);
                if (hit && slot < cap) {
                    ck0[slot] = __float_as_uint(pd2);
                    cii[slot] = ia < id2 ? ia : id2;
                    cjj[slot] = ia < id2 ? id2 : ia;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- seeds
// Device-side radix select of the need-th smallest of `count` 32-bit keys:
// the state holds the bits resolved so far (prefix, pbits) and the rank
// still to find among the keys with that prefix. A histogram pass counts the
// next `width` bits of the keys that carry the prefix; the pick kernel finds
// the bin holding the rank, extends the prefix, and clears the histogram.
struct SelState {
    uint32_t prefix;
    int32_t pbits;
    int64_t need;
};

// Rank selection in a histogram of NB bins by a workgroup of WG threads:
// the bin b with cum(b) < need <= cum(b) + h[b] (cum(b) = the count of the
// bins below b) and cum(b). Thread t sums bins [8t, 8t + 8), a block-wide
// inclusive scan of those sums finds the one thread whose range holds the
// rank, which walks its eight bins.
__device__ void pick_bin(const uint32_t* h, int64_t need, int* out_bin, int64_t* out_cum) {
    __shared__ int64_t wtot[WG / 64];
    const int per = NB / WG, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t v = 0;
    for (int i = 0; i < per; ++i) v += h[threadIdx.x * per + i];
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    for (int w = 0; w < wave; ++w) incl += wtot[w];
    const int64_t excl = incl - v;
    if (excl < need && incl >= need) {
        int64_t cum = excl;
        int bin = threadIdx.x * per + per - 1;
        for (int i = 0; i < per; ++i) {
            const int64_t c = h[threadIdx.x * per + i];
            if (cum + c >= need) { bin = threadIdx.x * per + i; break; }
            cum += c;
        }
        *out_bin = bin;
        *out_cum = cum;
    }
    __syncthreads();
}

// The pick step (one workgroup of WG threads): the bin of the device-wide
// histogram holding rank `need`, the prefix extended by it, the rank within
// it; the histogram is cleared for the next pass.
__global__ __launch_bounds__(WG) void acp_sel_pick_kernel(uint32_t* __restrict__ ghist,
                                                          SelState* __restrict__ state,
                                                          int width, int64_t need0) {
    __shared__ uint32_t h[NB];
    __shared__ int s_bin;
    __shared__ int64_t s_cum;
    for (int i = threadIdx.x; i < NB; i += WG) h[i] = ghist[i];
    if (threadIdx.x == 0) {
        s_bin = (1 << width) - 1;       // unreachable while need <= count
        s_cum = 0;
    }
    __syncthreads();
    // need0 >= 0: the first pass (the state is not read, it starts empty)
    const bool first = need0 >= 0;
    const int64_t need = first ? need0 : state->need;
    pick_bin(h, need, &s_bin, &s_cum);
    if (threadIdx.x == 0) {
        state->prefix = ((first ? 0u : state->prefix) << width) | (uint32_t)s_bin;
        state->pbits = (first ? 0 : state->pbits) + width;
        state->need = need - s_cum;
    }
    for (int i = threadIdx.x; i < NB; i += WG) ghist[i] = 0;
}

// ub^2 = the key left in state->prefix (has_ub), else ub = +inf. When the
// band it was selected from outgrew its capacity (*band_count > band_cap) the
// key means nothing and the call redoes these stages: the radii are then
// empty, so that the tile filter and the pair scan in between do no work.
__global__ void acp_radius_kernel(const SelState* __restrict__ state, int has_ub, double t,
                                  double gamma, float coord_scale,
                                  const unsigned long long* __restrict__ band_count,
                                  int64_t band_cap, AcpRadius* __restrict__ out) {
    if ((int64_t)*band_count > band_cap) {
        AcpRadius r;
        r.R2 = -1.f;
        r.limit = -INFINITY;
        r.seed_lim = 0u;
        r.pad = 0u;
        *out = r;
        return;
    }
    const float ub2 = has_ub ? __uint_as_float(state->prefix) : INFINITY;
    const double ub = has_ub ? sqrt((double)ub2) : HUGE_VAL;
    const double R = t * ub;
    const bool inf = isinf(R);
    const float slack = (float)(1e-5 * (2.0 * (double)coord_scale + (inf ? 0.0 : R)));
    AcpRadius r;
    r.R2 = inf ? INFINITY : (float)(R * R);
    r.limit = inf ? INFINITY : (float)R + slack;
    r.seed_lim = has_ub ? __float_as_uint(nextafterf((float)((double)ub2 * (1.0 + 4.0 * gamma)), INFINITY))
                        : 0xffffffffu;
    r.pad = 0u;
    *out = r;
}

// The need-th smallest of the first min(*dev_count, cap) keys, by one
// workgroup (three radix passes of 11, 11 and 10 bits over keys that stay in
// L2); the key is left in state->prefix (all 32 bits).
__global__ __launch_bounds__(WG) void acp_kth_small_kernel(const uint32_t* __restrict__ keys,
                                                           int64_t cap,
                                                           const unsigned long long* __restrict__ dev_count,
                                                           int64_t need, SelState* __restrict__ state) {
    __shared__ uint32_t h[NB];
    __shared__ int s_bin;
    __shared__ int64_t s_cum;
    const int64_t real = (int64_t)*dev_count;
    const int64_t cnt = real < cap ? real : cap;
    uint32_t prefix = 0;
    int pbits = 0;
    for (int pass = 0; pass < 3; ++pass) {
        const int width = pass < 2 ? 11 : 10;
        const int shift = 32 - pbits - width;
        const uint32_t mask = (1u << width) - 1u;
        for (int i = threadIdx.x; i < NB; i += WG) h[i] = 0;
        if (threadIdx.x == 0) {
            s_bin = (1 << width) - 1;
            s_cum = 0;
        }
        __syncthreads();
        for (int64_t e = threadIdx.x; e < cnt; e += WG) {
            const uint32_t x = keys[e];
            if (pbits == 0 || (x >> (32 - pbits)) == prefix) atomicAdd(&h[(x >> shift) & mask], 1u);
        }
        __syncthreads();
        pick_bin(h, need, &s_bin, &s_cum);
        prefix = (prefix << width) | (uint32_t)s_bin;
        pbits += width;
        need -= s_cum;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        state->prefix = prefix;
        state->pbits = 32;
        state->need = need;
    }
}

// Self-join of leaves of at most 64 points, one workgroup per leaf: the
// squared distance of every pair a < b, FP32 direct differences. The
// triangle of 4 x 4 point blocks (136 blocks) is split over two halves of
// every 64-dimension chunk (272 tasks); a task keeps its block's 16 pairs in
// two interleaved accumulators each, so every FP32 sum is a chain of
// d_pad / 4 terms and the squared distance carries a relative error of at
// most (d_pad / 4 + 4) u (two chains per half, two halves). Writes the
// distance bits of pair (a, b) at seed_off[leaf] + a (2 cnt - a - 1) / 2 +
// b - a - 1 (and, with ii/jj, the ids i < j), and adds the top 11 bits of
// every distance to the device-wide histogram ghist (first radix pass of the
// k-th smallest seed).
constexpr int SJ_THREADS = 320;
constexpr int SJ_TASKS = 272;
constexpr int SJ_CK = 64;
__global__ __launch_bounds__(SJ_THREADS) void acp_seed_join_kernel(
    const float* __restrict__ data, int d_pad, const int32_t* __restrict__ perm, int64_t n,
    int L, const int64_t* __restrict__ seed_off, uint32_t* __restrict__ k0,
    uint32_t* __restrict__ ii, uint32_t* __restrict__ jj, uint32_t* __restrict__ ghist) {
    __shared__ float xs[64][SJ_CK + 1];
    __shared__ float part[SJ_TASKS / 2][16];
    __shared__ uint32_t hist[NB];
    const int64_t leaf = blockIdx.x;
    const int64_t p0 = leaf * L;
    const int cnt = (int)(n - p0 < L ? n - p0 : L);
    const int t = threadIdx.x;
    for (int i = t; i < NB; i += SJ_THREADS) hist[i] = 0;
    const bool task = t < SJ_TASKS;
    const int bl = t >> 1, half = t & 1;
    int bi = 0, rem = task ? bl : 0;
    while (rem >= 16 - bi) {
        rem -= 16 - bi;
        ++bi;
    }
    const int bj = bi + rem;
    float acc0[16], acc1[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) { acc0[q] = 0.f; acc1[q] = 0.f; }
    for (int c0 = 0; c0 < d_pad; c0 += SJ_CK) {
        const int w = d_pad - c0 < SJ_CK ? d_pad - c0 : SJ_CK;
        __syncthreads();
        for (int e = t; e < 64 * (SJ_CK / 4); e += SJ_THREADS) {
            const int r = e / (SJ_CK / 4), q = e % (SJ_CK / 4);
            float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < cnt && 4 * q < w)
                val = *reinterpret_cast<const float4*>(data + (p0 + r) * d_pad + c0 + 4 * q);
            xs[r][4 * q] = val.x;
            xs[r][4 * q + 1] = val.y;
            xs[r][4 * q + 2] = val.z;
            xs[r][4 * q + 3] = val.w;
        }
        __syncthreads();
        if (task) {
            for (int i = 0; i < SJ_CK / 2; i += 2) {
                const int dd = half * (SJ_CK / 2) + i;
                float xa[4], xb[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) { xa[r] = xs[4 * bi + r][dd]; xb[r] = xs[4 * bj + r][dd]; }
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float df = __fsub_rn(xa[r], xb[s]);
                        acc0[4 * r + s] = __fmaf_rn(df, df, acc0[4 * r + s]);
                    }
#pragma unroll
                for (int r = 0; r < 4; ++r) { xa[r] = xs[4 * bi + r][dd + 1]; xb[r] = xs[4 * bj + r][dd + 1]; }
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float df = __fsub_rn(xa[r], xb[s]);
                        acc1[4 * r + s] = __fmaf_rn(df, df, acc1[4 * r + s]);
                    }
            }
        }
    }
    // combine: the two chains of each half, then the two halves
    if (task && half == 1) {
#pragma unroll
        for (int q = 0; q < 16; ++q) part[bl][q] = __fadd_rn(acc0[q], acc1[q]);
    }
    __syncthreads();
    if (task && half == 0) {
        const int64_t out0 = seed_off[leaf];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int a = 4 * bi + r, b = 4 * bj + s;
                if (a < b && b < cnt) {
                    const float d2 = __fadd_rn(__fadd_rn(acc0[4 * r + s], acc1[4 * r + s]),
                                               part[bl][4 * r + s]);
                    const uint32_t bits = __float_as_uint(d2);
                    const int64_t p = out0 + (int64_t)a * (2 * cnt - a - 1) / 2 + (b - a - 1);
                    k0[p] = bits;
                    if (ii) {
                        const uint32_t ia = (uint32_t)perm[p0 + a], ib = (uint32_t)perm[p0 + b];
                        ii[p] = ia < ib ? ia : ib;
                        jj[p] = ia < ib ? ib : ia;
                    }
                    atomicAdd(&hist[bits >> 21], 1u);
                }
            }
    }
    __syncthreads();
    for (int i = t; i < NB; i += SJ_THREADS)
        if (hist[i]) atomicAdd(&ghist[i], hist[i]);
}

// Seed bounds of leaves of at most 64 points on the FP16 matrix cores: the
// squared distances by the Gram identity |a - b|^2 = |a|^2 + |b|^2 - 2 a.b,
// over the leaf's rows taken relative to its first point x0, scaled by the
// power of two sc = 1 / (2 S) (S the largest FP16-row scale of the leaf, so
// every |a_i - x0_i| sc < 2^15) and rounded to FP16: a~ = fp16(sc fl(a - x0)).
// One workgroup per leaf. The 64 x 64 Gram matrix is the ten 16 x 16 tiles on
// or above the diagonal (v_mfma_f32_16x16x32_f16, FP32 sums), three, three,
// two and two per wave; the rows pass through LDS SG_W coordinates at a
// time, their loads issued SG_DEPTH steps ahead. With X0L the first point's
// row is read into LDS once (d_pad <= SG_X0), so a step loads only the
// leaf's own rows; otherwise its coordinates are loaded beside them at every
// step.
//
// Bounds (rigorous, in scaled units, K the coordinates summed):
//   rounding to FP16 and the FP32 centring: |a~ - sc (a - x0)| <= rho_a =
//     4.9e-4 |a~| + 1.02 2^-14 sqrt(K) (the last term covers inputs below the
//     FP16 normal range, flushed or not);
//   FP32 sums of K exact FP16 products in any order (a truncating adder
//     included): |G_ab - a~.b~| <= g_K |a~| |b~|, g_K = K 2^-23 / (1 - K 2^-23),
//     so |a~| <= A_a = sqrt(G_aa / (1 - g_K));
//   d2 = (G_aa + G_bb) - 2 G_ab lies within E = (g_K + 2^-22) (A_a + A_b)^2 of
//     |a~ - b~|^2.
// So sc |a - b| lies in [sqrt(d2 - E) - rho_a - rho_b, sqrt(d2 + E) + rho_a +
// rho_b]. Both ends, squared and divided by sc^2 (widened by 2^-18 for their
// own FP32 evaluation), are written as the pair's bounds (FP32 bit patterns)
// in the triangular layout of the seeds (leaf b's pairs from b L (L - 1) / 2
// on); the top 11 bits of every upper bound go to ghist (first radix pass of
// the k-th smallest upper bound).
// Two steps of row loads in flight, one 32-coordinate slice per step: wider
// steps (up to 128 coordinates, 512 contiguous bytes per row) and deeper
// rings are no faster, the kernel moving its bytes at about nine tenths of
// a plain device copy's rate.
constexpr int SG_DEPTH = 2;                  // steps of row loads in flight
constexpr int SG_KS = 1;                     // 32-coordinate slices per step
constexpr int SG_W = 32 * SG_KS;             // coordinates per step
constexpr int SG_LD = SG_W + 8;              // LDS row stride of the staged FP16 rows, in halves
constexpr int SG_X0 = 2048;                  // LDS floats for the first point's row
static_assert(SG_DEPTH >= 2 && SG_X0 % 32 == 0, "at least two steps in flight; whole steps");

template <bool X0L>
__global__ __launch_bounds__(WG) void acp_seed_gram_kernel(
    const float* __restrict__ data, int d_pad, const float* __restrict__ row_scale, int64_t n,
    int L, float gk, uint32_t* __restrict__ hi_out,
    uint32_t* __restrict__ lo_out, uint32_t* __restrict__ ghist) {
    typedef _Float16 h8 __attribute__((ext_vector_type(8)));
    typedef float f4v __attribute__((ext_vector_type(4)));
    __shared__ __align__(16) _Float16 xs[2][64][SG_LD];
    __shared__ __align__(16) float x0s[X0L ? SG_X0 : 4];
    __shared__ float gnorm[64], anorm[64], rho[64];
    const int64_t leaf = blockIdx.x;
    const int64_t p0 = leaf * L;
    const int cnt = (int)(n - p0 < L ? n - p0 : L);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    // staging: thread t converts coordinates 8 (t % 4) .. + 7 of row t / 4
    const int r = t >> 2, q = (t & 3) * 8;
    const bool rv = r < cnt;
    const float* rowp = data + (p0 + (rv ? r : 0)) * d_pad;
    const float* x0p = data + p0 * d_pad;
    // Every global load of the steady state is unconditional (columns past
    // d_pad read the row's last four and are zeroed when staged), so the
    // compiler waits for the oldest step's loads only: a load under a branch
    // would make it wait for all of them at every step.
    struct Stage { float4 a[2 * SG_KS], z[2 * SG_KS]; };
    auto ld4 = [&](const float* p, int c) {
        return *reinterpret_cast<const float4*>(p + (c < d_pad ? c : d_pad - 4));
    };
    auto load = [&](Stage& s, int k0) {
#pragma unroll
        for (int i = 0; i < SG_KS; ++i) {
            s.a[2 * i] = ld4(rowp, k0 + 32 * i + q);
            s.a[2 * i + 1] = ld4(rowp, k0 + 32 * i + q + 4);
            if (!X0L) {
                s.z[2 * i] = ld4(x0p, k0 + 32 * i + q);
                s.z[2 * i + 1] = ld4(x0p, k0 + 32 * i + q + 4);
            }
        }
    };
    const int nst = (d_pad + SG_W - 1) / SG_W;
    // steps padded to whole rounds of the ring: the extra steps stage zeros
    const int nsp = (nst + SG_DEPTH - 1) / SG_DEPTH * SG_DEPTH;
    // the power-of-two scale, in every wave: sc = 1 / (2 S)
    float smax = row_scale[p0 + (lane < cnt ? lane : 0)];
    // the first row into LDS (its loads before the ring's, 2 * 4 WG = 2,048
    // floats at most, zero past d_pad)
    float4 xa = make_float4(0.f, 0.f, 0.f, 0.f), xb = xa;
    if (X0L) {
        static_assert(!X0L || SG_X0 == 8 * WG, "two float4 loads per thread fill the first row's array");
        xa = ld4(x0p, 4 * t);
        xb = ld4(x0p, 4 * t + 4 * WG);
    }
    // set j of the ring holds the steps j, j + SG_DEPTH, ...
    Stage sr[SG_DEPTH];
#pragma unroll
    for (int j = 0; j < SG_DEPTH; ++j) load(sr[j], SG_W * j);
    for (int off = 32; off > 0; off >>= 1) smax = fmaxf(smax, __shfl_xor(smax, off));
    const float sc = 0.5f / smax;
    if (X0L) {
        // the whole array, unconditionally (SG_X0 = 8 WG floats)
        const bool oa = 4 * t < d_pad, ob = 4 * t + 4 * WG < d_pad;
        *reinterpret_cast<float4*>(&x0s[4 * t]) =
            make_float4(oa ? xa.x : 0.f, oa ? xa.y : 0.f, oa ? xa.z : 0.f, oa ? xa.w : 0.f);
        *reinterpret_cast<float4*>(&x0s[4 * t + 4 * WG]) =
            make_float4(ob ? xb.x : 0.f, ob ? xb.y : 0.f, ob ? xb.z : 0.f, ob ? xb.w : 0.f);
    }
    __syncthreads();
    auto store = [&](Stage s, int buf, int k0) {
#pragma unroll
        for (int i = 0; i < SG_KS; ++i) {
            const int kc = k0 + 32 * i + q;
            const bool lo_ok = rv && kc < d_pad, hi_ok = rv && kc + 4 < d_pad;
            float4 z0, z1;
            if (X0L) {
                // columns past d_pad read column 0 (and are zeroed below)
                z0 = *reinterpret_cast<const float4*>(&x0s[lo_ok ? kc : 0]);
                z1 = *reinterpret_cast<const float4*>(&x0s[hi_ok ? kc + 4 : 0]);
            } else {
                z0 = s.z[2 * i];
                z1 = s.z[2 * i + 1];
            }
            const float4 a0 = s.a[2 * i], a1 = s.a[2 * i + 1];
            h8 v;
            v[0] = (_Float16)(__fsub_rn(a0.x, z0.x) * sc);
            v[1] = (_Float16)(__fsub_rn(a0.y, z0.y) * sc);
            v[2] = (_Float16)(__fsub_rn(a0.z, z0.z) * sc);
            v[3] = (_Float16)(__fsub_rn(a0.w, z0.w) * sc);
            v[4] = (_Float16)(__fsub_rn(a1.x, z1.x) * sc);
            v[5] = (_Float16)(__fsub_rn(a1.y, z1.y) * sc);
            v[6] = (_Float16)(__fsub_rn(a1.z, z1.z) * sc);
            v[7] = (_Float16)(__fsub_rn(a1.w, z1.w) * sc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (!lo_ok) v[e] = (_Float16)0.f;
                if (!hi_ok) v[4 + e] = (_Float16)0.f;
            }
            *reinterpret_cast<h8*>(&xs[buf][r][32 * i + q]) = v;
        }
    };
    // the wave's tiles (bi, bj): w0 (0,0) (1,1) (0,1), w1 (2,2) (3,3) (2,3),
    // w2 (0,2) (0,3), w3 (1,2) (1,3)
    const int nt = wave < 2 ? 3 : 2;
    int bi[3], bj[3];
    if (wave < 2) {
        bi[0] = 2 * wave; bj[0] = 2 * wave;
        bi[1] = 2 * wave + 1; bj[1] = 2 * wave + 1;
        bi[2] = 2 * wave; bj[2] = 2 * wave + 1;
    } else {
        bi[0] = wave - 2; bj[0] = 2;
        bi[1] = wave - 2; bj[1] = 3;
        bi[2] = 0; bj[2] = 0;
    }
    f4v acc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[j] = f4v{0.f, 0.f, 0.f, 0.f};
    auto mma = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < SG_KS; ++kk)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (j < nt) {
                    const h8 fa = *reinterpret_cast<const h8*>(&xs[buf][16 * bi[j] + l16][32 * kk + 8 * lq]);
                    const h8 fb = *reinterpret_cast<const h8*>(&xs[buf][16 * bj[j] + l16][32 * kk + 8 * lq]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(fa, fb, acc[j], 0, 0, 0);
                }
            }
    };
    // step st is staged in LDS buffer st % 2 from ring set st % SG_DEPTH,
    // which then loads step st + SG_DEPTH (the last step stages into a buffer
    // nobody reads and its loads are never used)
    auto step = [&](int st, Stage& nxt) {
        mma(st & 1);
        store(nxt, (st + 1) & 1, SG_W * (st + 1));
        load(nxt, SG_W * (st + 1 + SG_DEPTH));
        __syncthreads();
    };
    store(sr[0], 0, 0);
    load(sr[0], SG_W * SG_DEPTH);
    __syncthreads();
    for (int st = 0; st < nsp; st += SG_DEPTH) {
#pragma unroll
        for (int j = 0; j < SG_DEPTH; ++j) step(st + j, sr[(j + 1) % SG_DEPTH]);
    }

    // the squared norms from the diagonal tiles; the staging area becomes the
    // histogram
    uint32_t* hist = reinterpret_cast<uint32_t*>(&xs[0][0][0]);
    static_assert(sizeof(xs) >= NB * sizeof(uint32_t), "the histogram reuses the staging area");
    for (int i = t; i < NB; i += WG) hist[i] = 0;
    if (wave < 2) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (l16 == 4 * lq + v) gnorm[16 * bi[j] + l16] = acc[j][v];
    }
    __syncthreads();
    const float Kf = (float)(32 * ((d_pad + 31) / 32));
    if (t < 64) {
        const float A = sqrtf(fmaxf(gnorm[t], 0.f) / (1.f - gk)) * (1.f + 9.5367431640625e-07f);
        anorm[t] = A;
        rho[t] = 4.9e-4f * A + 1.02f * 6.103515625e-05f * sqrtf(Kf) * (1.f + 9.5367431640625e-07f);
    }
    __syncthreads();
    const float ek = (gk + 2.384185791015625e-07f) * (1.f + 3.814697265625e-06f);
    const float inv = 1.f / sc;            // a power of two: exact
    const float up = 1.f + 3.814697265625e-06f, dn = 1.f - 3.814697265625e-06f;
    // every leaf before the last holds L points
    const int64_t out0 = leaf * (int64_t)(L * (L - 1) / 2);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (j < nt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = 16 * bi[j] + 4 * lq + v, b = 16 * bj[j] + l16;
                if (a < b && b < cnt) {
                    const float d2 = (gnorm[a] + gnorm[b]) - 2.f * acc[j][v];
                    const float sA = anorm[a] + anorm[b];
                    const float E = ek * sA * sA;
                    const float rr = rho[a] + rho[b];
                    const float sh = sqrtf(fmaxf(d2 + E, 0.f)) * up + rr;
                    const float sl = sqrtf(fmaxf(d2 - E, 0.f)) * dn - rr * up;
                    const float hi = (sh * inv) * (sh * inv) * up;
                    const float lo = sl > 0.f ? (sl * inv) * (sl * inv) * dn : 0.f;
                    const uint32_t hb = __float_as_uint(hi);
                    const int64_t p = out0 + (int64_t)a * (2 * cnt - a - 1) / 2 + (b - a - 1);
                    hi_out[p] = hb;
                    lo_out[p] = __float_as_uint(lo);
                    atomicAdd(&hist[hb >> 21], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int i = t; i < NB; i += WG)
        if (hist[i]) atomicAdd(&ghist[i], hist[i]);
}

// Seeds whose lower bound is at most U (1 + widen), U the upper edge of the
// radix bin that holds the k-th smallest upper bound (the selection's prefix
// of state->pbits bits), or every seed when all is set: their ids (i < j)
// are appended. One wave per leaf (leaves of at most 64 points, at most
// 2,016 pairs, all loaded before any test), sixteen leaves per workgroup:
// the workgroup's pairs are gathered in LDS and appended with one global
// atomic (a few thousand pairs spread over as many leaves would otherwise
// queue that many atomics on one counter); pairs beyond the LDS buffer (mass
// ties) are appended one wave at a time.
constexpr int kBandWaves = 16;
constexpr int kBandLds = 2048;

__global__ __launch_bounds__(64 * kBandWaves) void acp_seed_gram_band_kernel(
    const uint32_t* __restrict__ lo, const int32_t* __restrict__ perm, int64_t n, int L,
    int64_t n_leaves, const SelState* __restrict__ state, float widen, int all,
    uint32_t* __restrict__ oii, uint32_t* __restrict__ ojj, int64_t cap,
    unsigned long long* __restrict__ counter) {
    __shared__ uint32_t bi[kBandLds], bj[kBandLds];
    __shared__ unsigned int nl;
    __shared__ unsigned long long gbase;
    const int lane = threadIdx.x & 63;
    const int64_t leaf = (int64_t)blockIdx.x * kBandWaves + (threadIdx.x >> 6);
    if (threadIdx.x == 0) nl = 0u;
    __syncthreads();
    if (leaf < n_leaves) {
        const int64_t p0 = leaf * L;
        const int cnt = (int)(n - p0 < L ? n - p0 : L);
        const int P = cnt * (cnt - 1) / 2;
        const int64_t off = leaf * (int64_t)(L * (L - 1) / 2);
        constexpr int PER = (64 * 63 / 2 + 63) / 64;
        float v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int p = u * 64 + lane;
            v[u] = p < P ? __uint_as_float(lo[off + p]) : INFINITY;
        }
        float lim = INFINITY;
        if (!all) {
            const int pb = state->pbits;
            const uint32_t low = pb >= 32 ? 0u : (1u << (32 - pb)) - 1u;
            const uint32_t top = pb >= 32 ? state->prefix : state->prefix << (32 - pb);
            lim = __uint_as_float(top | low) * (1.f + widen) * (1.f + 3.814697265625e-06f);
        }
        uint64_t any = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) any |= __ballot(v[u] <= lim);
        if (any) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int p = u * 64 + lane;
                const bool take = p < P && v[u] <= lim;
                const uint64_t m = __ballot(take);
                if (m == 0) continue;
                uint32_t i = 0, j = 0;
                if (take) {
                    int a = 0, rem = p;
                    while (rem >= cnt - 1 - a) { rem -= cnt - 1 - a; ++a; }
                    const uint32_t ia = (uint32_t)perm[p0 + a], ib = (uint32_t)perm[p0 + a + 1 + rem];
                    i = ia < ib ? ia : ib;
                    j = ia < ib ? ib : ia;
                }
                const int leader = __ffsll((unsigned long long)m) - 1;
                unsigned int base = 0u;
                if (lane == leader) base = atomicAdd(&nl, (unsigned int)__popcll(m));
                base = (unsigned int)__shfl((int)base, leader);
                const unsigned int slot = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
                const bool spill = take && slot >= (unsigned int)kBandLds;
                if (take && !spill) {
                    bi[slot] = i;
                    bj[slot] = j;
                }
                const int64_t g = wave_append_global(spill, counter);
                if (spill && g < cap) {
                    oii[g] = i;
                    ojj[g] = j;
                }
            }
        }
    }
    __syncthreads();
    const unsigned int tot = nl < (unsigned int)kBandLds ? nl : (unsigned int)kBandLds;
    if (tot == 0u) return;
    if (threadIdx.x == 0) gbase = atomicAdd(counter, (unsigned long long)tot);
    __syncthreads();
    for (unsigned int t = threadIdx.x; t < tot; t += 64 * kBandWaves) {
        const unsigned long long g = gbase + t;
        if ((int64_t)g < cap) {
            oii[g] = bi[t];
            ojj[g] = bj[t];
        }
    }
}

__global__ __launch_bounds__(WG) void acp_sel_hist_kernel(
    const uint32_t* __restrict__ keys, int64_t count, const SelState* __restrict__ state,
    int shift, int width, uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[NB];
    for (int i = threadIdx.x; i < NB; i += WG) h[i] = 0;
    __syncthreads();
    // shift 21: the first pass (the state is not read)
    const uint32_t prefix = shift == 21 ? 0u : state->prefix;
    const int pbits = shift == 21 ? 0 : state->pbits;
    const uint32_t mask = (1u << width) - 1u;
    for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * WG) {
        const uint32_t x = keys[e];
        if (pbits == 0 || (x >> (32 - pbits)) == prefix) atomicAdd(&h[(x >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NB; i += WG)
        if (h[i]) atomicAdd(&ghist[i], h[i]);
}

// Within-leaf pairs whose distance bits are at most lim (the band of the
// top-k, or every seed when lim is +inf): (bits, i, j) appended to the pool.
__global__ __launch_bounds__(WG) void acp_seed_band_kernel(
    const uint32_t* __restrict__ k0, const int64_t* __restrict__ seed_off,
    const int32_t* __restrict__ perm, int64_t n, int L, uint32_t lim,
    uint32_t* __restrict__ ok0, uint32_t* __restrict__ oii, uint32_t* __restrict__ ojj,
    int64_t cap, unsigned long long* __restrict__ counter) {
    const int64_t leaf = blockIdx.x;
    const int64_t p0 = leaf * L;
    const int cnt = (int)(n - p0 < L ? n - p0 : L);
    const int P = cnt * (cnt - 1) / 2;
    const int64_t off = seed_off[leaf];
    for (int base = 0; base < P; base += WG) {
        const int p = base + threadIdx.x;
        uint32_t key = 0;
        bool take = false;
        if (p < P) {
            key = k0[off + p];
            take = key <= lim;
        }
        uint32_t i = 0, j = 0;
        if (take) {
            int a = 0, rem = p;
            while (rem >= cnt - 1 - a) { rem -= cnt - 1 - a; ++a; }
            const uint32_t ia = (uint32_t)perm[p0 + a], ib = (uint32_t)perm[p0 + a + 1 + rem];
            i = ia < ib ? ia : ib;
            j = ia < ib ? ib : ia;
        }
        const int64_t slot = wave_append_global(take, counter);
        if (take && slot < cap) { ok0[slot] = key; oii[slot] = i; ojj[slot] = j; }
    }
}

// ---------------------------------------------------------------- verify
// FP32 squared distance of two rows over one lane's float4 columns l16,
// l16 + 16, ... (d4 columns in all), summed in that ascending order with the
// eight columns' loads issued together (clamped into the row, the extra ones
// unused): one memory round trip per 128 columns.
__device__ __forceinline__ float row_dist2_f32(const float4* __restrict__ r1,
                                               const float4* __restrict__ r2, int l16, int d4) {
    float acc = 0.f;
    for (int c0 = l16; c0 < d4; c0 += 128) {
        float4 x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int c = c0 + 16 * u < d4 ? c0 + 16 * u : c0;
            x[u] = r1[c];
            y[u] = r2[c];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (c0 + 16 * u < d4) {
                float t;
                t = x[u].x - y[u].x; acc = __fmaf_rn(t, t, acc);
                t = x[u].y - y[u].y; acc = __fmaf_rn(t, t, acc);
                t = x[u].z - y[u].z; acc = __fmaf_rn(t, t, acc);
                t = x[u].w - y[u].w; acc = __fmaf_rn(t, t, acc);
            }
        }
    }
    return acc;
}

// Exact FP32 squared distance of `count` pairs (16 lanes per pair). With
// dev_count the pairs are the first min(*dev_count, count) and the keys of the
// rest of the `count` slots are set to +inf bits (ignored by a selection of
// a rank within the real pairs).
__global__ __launch_bounds__(WG) void acp_verify_kernel(
    const float* __restrict__ data, int d_pad, const int32_t* __restrict__ inv_perm,
    const uint32_t* __restrict__ cii, const uint32_t* __restrict__ cjj, int64_t count,
    uint32_t* __restrict__ k0, uint32_t* __restrict__ ii, uint32_t* __restrict__ jj,
    const unsigned long long* __restrict__ dev_count) {
    const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int d4 = d_pad >> 2;
    if (dev_count) {
        const int64_t real = (int64_t)*dev_count;
        const int64_t lim = real < count ? real : count;
        for (int64_t e = lim + (int64_t)blockIdx.x * WG + threadIdx.x; e < count;
             e += (int64_t)gridDim.x * WG)
            k0[e] = 0xffffffffu;
        count = lim;
    }
    for (int64_t base = (int64_t)blockIdx.x * (WG / 16); base < count;
         base += (int64_t)gridDim.x * (WG / 16)) {
        const int64_t e = base + g;
        float acc = 0.f;
        if (e < count) {
            const float4* r1 = reinterpret_cast<const float4*>(data + (int64_t)inv_perm[cii[e]] * d_pad);
            const float4* r2 = reinterpret_cast<const float4*>(data + (int64_t)inv_perm[cjj[e]] * d_pad);
            acc = row_dist2_f32(r1, r2, l16, d4);
        }
        acc += __shfl_xor(acc, 8, 16);
        acc += __shfl_xor(acc, 4, 16);
        acc += __shfl_xor(acc, 2, 16);
        acc += __shfl_xor(acc, 1, 16);
        if (e < count && l16 == 0) {
            k0[e] = __float_as_uint(acc);
            ii[e] = cii[e];
            jj[e] = cjj[e];
        }
    }
}

// ---------------------------------------------------------------- select
// Radix-select step over the 96-bit keys (k0, ii, jj): elements whose leading
// sub-keys equal v0 (depth >= 1) and v1 (depth 2) take part; their sub-key at
// `depth` contributes its bits [shift, shift + 11) to the histogram when its
// higher bits equal `prefix` (prefix_bits of them).
struct SelStep {
    int depth;
    uint32_t v0, v1;
    int shift;
    uint32_t mask;
    int prefix_bits;
    uint32_t prefix;
};

__device__ __forceinline__ bool sel_member(const SelStep& s, uint32_t a, uint32_t b, uint32_t c,
                                           uint32_t* sub) {
    if (s.depth >= 1 && a != s.v0) return false;
    if (s.depth >= 2 && b != s.v1) return false;
    const uint32_t x = s.depth == 0 ? a : (s.depth == 1 ? b : c);
    if (s.prefix_bits > 0 && (x >> (32 - s.prefix_bits)) != s.prefix) return false;
    *sub = x;
    return true;
}

__global__ __launch_bounds__(WG) void acp_hist_kernel(
    const uint32_t* __restrict__ k0, const uint32_t* __restrict__ ii,
    const uint32_t* __restrict__ jj, int64_t count, SelStep s, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[NB];
    for (int i = threadIdx.x; i < NB; i += WG) h[i] = 0;
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * WG) {
        uint32_t x;
        if (sel_member(s, k0[e], ii[e], jj[e], &x)) atomicAdd(&h[(x >> s.shift) & s.mask], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NB; i += WG)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

struct SelKey {
    int depth;
    uint32_t v0, v1, v2;
};

// (a, b, c) <= the selected key, comparing the first depth+1 sub-keys
__device__ __forceinline__ bool key_le(const SelKey& K, uint32_t a, uint32_t b, uint32_t c) {
    if (a != K.v0) return a < K.v0;
    if (K.depth == 0) return true;
    if (b != K.v1) return b < K.v1;
    if (K.depth == 1) return true;
    return c <= K.v2;
}

__global__ __launch_bounds__(WG) void acp_gather_kernel(
    const uint32_t* __restrict__ k0, const uint32_t* __restrict__ ii,
    const uint32_t* __restrict__ jj, int64_t count, SelKey K, uint32_t* __restrict__ ok0,
    uint32_t* __restrict__ oii, uint32_t* __restrict__ ojj, int64_t cap,
    unsigned long long* __restrict__ counter) {
    for (int64_t base = (int64_t)blockIdx.x * WG; base < count; base += (int64_t)gridDim.x * WG) {
        const int64_t e = base + threadIdx.x;
        bool take = false;
        uint32_t a = 0, b = 0, c = 0;
        if (e < count) {
            a = k0[e]; b = ii[e]; c = jj[e];
            take = key_le(K, a, b, c);
        }
        const int64_t slot = wave_append_global(take, counter);
        if (take && slot < cap) { ok0[slot] = a; oii[slot] = b; ojj[slot] = c; }
    }
}

// Sorts `count` (<= 1024) keys by (k0, ii, jj) and writes the k results.
__global__ __launch_bounds__(WG) void acp_final_kernel(
    const uint32_t* __restrict__ k0, const uint32_t* __restrict__ ii,
    const uint32_t* __restrict__ jj, int count, int64_t* __restrict__ out_pairs,
    float* __restrict__ out_dist) {
    __shared__ uint64_t hk[1024];
    __shared__ uint32_t lk[1024];
    int P = 1;
    while (P < count) P <<= 1;
    for (int i = threadIdx.x; i < P; i += WG) {
        if (i < count) {
            hk[i] = ((uint64_t)k0[i] << 32) | ii[i];
            lk[i] = jj[i];
        } else {
            hk[i] = ~0ull;
            lk[i] = ~0u;
        }
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += WG) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & k) == 0;
                    const bool gt = hk[i] > hk[ixj] || (hk[i] == hk[ixj] && lk[i] > lk[ixj]);
                    if (gt == up) {
                        const uint64_t th = hk[i]; hk[i] = hk[ixj]; hk[ixj] = th;
                        const uint32_t tl = lk[i]; lk[i] = lk[ixj]; lk[ixj] = tl;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < count; i += WG) {
        out_pairs[2 * i] = (int64_t)(uint32_t)(hk[i] & 0xffffffffull);
        out_pairs[2 * i + 1] = (int64_t)lk[i];
        out_dist[i] = sqrtf(__uint_as_float((uint32_t)(hk[i] >> 32)));
    }
}

constexpr int kTopBand = 1024;   // pairs the FP64 top-k takes at most (>= PMLSH_MAX_K)

// FP64 squared distance of two FP32 rows over one lane's float4 columns
// l16, l16 + 16, ... (d4 columns in all), summed in that ascending order; the
// loads of eight columns go out together (clamped into the row, the extra
// ones unused), so a row costs one memory round trip per 128 columns rather
// than one per column.
__device__ __forceinline__ double row_dist2_f64(const float4* __restrict__ r1,
                                                const float4* __restrict__ r2, int l16, int d4) {
    double acc = 0.0;
    for (int c0 = l16; c0 < d4; c0 += 128) {
        float4 x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int c = c0 + 16 * u < d4 ? c0 + 16 * u : c0;
            x[u] = r1[c];
            y[u] = r2[c];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (c0 + 16 * u < d4) {
                double t;
                t = (double)x[u].x - (double)y[u].x; acc = fma(t, t, acc);
                t = (double)x[u].y - (double)y[u].y; acc = fma(t, t, acc);
                t = (double)x[u].z - (double)y[u].z; acc = fma(t, t, acc);
                t = (double)x[u].w - (double)y[u].w; acc = fma(t, t, acc);
            }
        }
    }
    return acc;
}

// Top-k in the FP64 order of Section 6 (distance, then i, then j). The `count`
// pairs are every pair whose FP32 distance lies within the verify error band
// of the FP32 k-th one, so the exact top-k is among them; each gets its squared
// distance in FP64 from the FP32 rows and the k smallest by (d^2, i, j) are
// written (16 lanes per pair, as in the FP32 verify).
__global__ __launch_bounds__(WG) void acp_final64_kernel(
    const float* __restrict__ data, int d_pad, const int32_t* __restrict__ inv_perm,
    const uint32_t* __restrict__ ii, const uint32_t* __restrict__ jj, int count, int k,
    int64_t* __restrict__ out_pairs, float* __restrict__ out_dist) {
    __shared__ double dk[kTopBand];
    __shared__ uint64_t pk[kTopBand];
    const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int d4 = d_pad >> 2;
    int P = 1;
    while (P < count) P <<= 1;
    for (int base = 0; base < P; base += WG / 16) {
        const int e = base + g;
        double acc = 0.0;
        if (e < count) {
            const float4* r1 = reinterpret_cast<const float4*>(data + (int64_t)inv_perm[ii[e]] * d_pad);
            const float4* r2 = reinterpret_cast<const float4*>(data + (int64_t)inv_perm[jj[e]] * d_pad);
            acc = row_dist2_f64(r1, r2, l16, d4);
        }
        acc += __shfl_xor(acc, 8, 16);
        acc += __shfl_xor(acc, 4, 16);
        acc += __shfl_xor(acc, 2, 16);
        acc += __shfl_xor(acc, 1, 16);
        if (l16 == 0 && e < P) {
            dk[e] = e < count ? acc : INFINITY;
            pk[e] = e < count ? (((uint64_t)ii[e] << 32) | jj[e]) : ~0ull;
        }
    }
    __syncthreads();
    for (int s = 2; s <= P; s <<= 1) {
        for (int j = s >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += WG) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & s) == 0;
                    const bool gt = dk[i] > dk[ixj] || (dk[i] == dk[ixj] && pk[i] > pk[ixj]);
                    if (gt == up) {
                        const double td = dk[i]; dk[i] = dk[ixj]; dk[ixj] = td;
                        const uint64_t tp = pk[i]; pk[i] = pk[ixj]; pk[ixj] = tp;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < k; i += WG) {
        out_pairs[2 * i] = (int64_t)(pk[i] >> 32);
        out_pairs[2 * i + 1] = (int64_t)(pk[i] & 0xffffffffull);
        out_dist[i] = (float)sqrt(dk[i]);
    }
}

constexpr int kSmallPool = 16384;   // pools the one-workgroup top-k takes
constexpr size_t kSmallTopkLds =
    (size_t)kSmallPool * 4 + (size_t)NB * 4 + (size_t)kTopBand * 8 + (size_t)kTopBand * 8;

// Top-k of a pool of at most kSmallPool pairs in one workgroup: the k-th
// smallest FP32 key by radix select in LDS (11, 11, 10 bits), the band
// kth (1 + band) rounded up one ulp, and the band's order in FP64 as in
// acp_final64_kernel. status[0] receives the band size m; when m exceeds
// kTopBand nothing is written and the caller falls back to the FP32 order.
__global__ __launch_bounds__(WG) void acp_topk_small_kernel(
    const uint32_t* __restrict__ k0, const uint32_t* __restrict__ ii,
    const uint32_t* __restrict__ jj, int count, int k, double band,
    const float* __restrict__ data, int d_pad, const int32_t* __restrict__ inv_perm,
    int64_t* __restrict__ out_pairs, float* __restrict__ out_dist, int* __restrict__ status,
    const unsigned long long* __restrict__ dn_add) {
    // dn_add: the pool holds a further *dn_add pairs counted on the device
    if (dn_add) count += (int)*dn_add;
    extern __shared__ __align__(16) unsigned char smem[];
    double* dk = reinterpret_cast<double*>(smem);
    uint64_t* pk = reinterpret_cast<uint64_t*>(dk + kTopBand);
    uint32_t* keys = reinterpret_cast<uint32_t*>(pk + kTopBand);
    uint32_t* h = keys + kSmallPool;
    __shared__ uint32_t s_prefix;
    __shared__ int s_pbits, s_need, s_m, s_bin;
    __shared__ int64_t s_cum;
    for (int e = threadIdx.x; e < count; e += WG) keys[e] = k0[e];
    if (threadIdx.x == 0) {
        s_prefix = 0;
        s_pbits = 0;
        s_need = k;
        s_m = 0;
    }
    const int shifts[3] = {21, 10, 0}, widths[3] = {11, 11, 10};
    for (int pass = 0; pass < 3; ++pass) {
        for (int i = threadIdx.x; i < NB; i += WG) h[i] = 0;
        __syncthreads();
        const uint32_t prefix = s_prefix;
        const int pbits = s_pbits;
        const uint32_t mask = (1u << widths[pass]) - 1u;
        for (int e = threadIdx.x; e < count; e += WG) {
            const uint32_t x = keys[e];
            if (pbits == 0 || (x >> (32 - pbits)) == prefix)
                atomicAdd(&h[(x >> shifts[pass]) & mask], 1u);
        }
        __syncthreads();
        const int need = s_need;
        if (threadIdx.x == 0) {
            s_bin = (int)mask;          // unreachable while need <= count
            s_cum = 0;
        }
        __syncthreads();
        pick_bin(h, need, &s_bin, &s_cum);
        if (threadIdx.x == 0) {
            s_prefix = (s_prefix << widths[pass]) | (uint32_t)s_bin;
            s_pbits += widths[pass];
            s_need = need - (int)s_cum;
        }
        __syncthreads();
    }
    const float kth = __uint_as_float(s_prefix);
    const uint32_t lim = __float_as_uint(nextafterf((float)((double)kth * (1.0 + band)), INFINITY));
    for (int e = threadIdx.x; e < count; e += WG) {
        if (keys[e] <= lim) {
            const int slot = atomicAdd(&s_m, 1);
            if (slot < kTopBand) pk[slot] = ((uint64_t)ii[e] << 32) | jj[e];
        }
    }
    __syncthreads();
    const int m = s_m;
    if (threadIdx.x == 0) *status = m;
    if (m > kTopBand) return;
    const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int d4 = d_pad >> 2;
    int P = 1;
    while (P < m) P <<= 1;
    for (int base = 0; base < P; base += WG / 16) {
        const int e = base + g;
        double acc = 0.0;
        if (e < m) {
            const uint64_t key = pk[e];
            const float4* r1 = reinterpret_cast<const float4*>(data + (int64_t)inv_perm[(uint32_t)(key >> 32)] * d_pad);
            const float4* r2 = reinterpret_cast<const float4*>(data + (int64_t)inv_perm[(uint32_t)key] * d_pad);
            acc = row_dist2_f64(r1, r2, l16, d4);
        }
        acc += __shfl_xor(acc, 8, 16);
        acc += __shfl_xor(acc, 4, 16);
        acc += __shfl_xor(acc, 2, 16);
        acc += __shfl_xor(acc, 1, 16);
        if (l16 == 0 && e < P) {
            dk[e] = e < m ? acc : INFINITY;
            if (e >= m) pk[e] = ~0ull;
        }
    }
    __syncthreads();
    for (int sz = 2; sz <= P; sz <<= 1) {
        for (int j = sz >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += WG) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & sz) == 0;
                    const bool gt = dk[i] > dk[ixj] || (dk[i] == dk[ixj] && pk[i] > pk[ixj]);
                    if (gt == up) {
                        const double td = dk[i]; dk[i] = dk[ixj]; dk[ixj] = td;
                        const uint64_t tp = pk[i]; pk[i] = pk[ixj]; pk[ixj] = tp;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < k; i += WG) {
        out_pairs[2 * i] = (int64_t)(pk[i] >> 32);
        out_pairs[2 * i + 1] = (int64_t)(pk[i] & 0xffffffffull);
        out_dist[i] = (float)sqrt(dk[i]);
    }
}

// The pool pairs whose FP32 distance bits are at most the band limit of the
// selected k-th key (state->prefix): kth (1 + band), rounded up one ulp, the
// same limit pool_topk states on the host.
__global__ __launch_bounds__(WG) void acp_band_gather_kernel(
    const uint32_t* __restrict__ k0, const uint32_t* __restrict__ ii,
    const uint32_t* __restrict__ jj, int64_t count, const SelState* __restrict__ state,
    double band, uint32_t* __restrict__ ok0, uint32_t* __restrict__ oii,
    uint32_t* __restrict__ ojj, int64_t cap, unsigned long long* __restrict__ counter) {
    const float kth = __uint_as_float(state->prefix);
    const uint32_t lim = __float_as_uint(nextafterf((float)((double)kth * (1.0 + band)), INFINITY));
    for (int64_t base = (int64_t)blockIdx.x * WG; base < count; base += (int64_t)gridDim.x * WG) {
        const int64_t e = base + threadIdx.x;
        bool take = false;
        uint32_t a = 0;
        if (e < count) {
            a = k0[e];
            take = a <= lim;
        }
        const int64_t slot = wave_append_global(take, counter);
        if (take && slot < cap) { ok0[slot] = a; oii[slot] = ii[e]; ojj[slot] = jj[e]; }
    }
}


// ---------------------------------------------------------------- host side
// Workspace buffer of one role, kept in the index between calls and grown
// (freed and allocated anew) only when a call needs more than it holds.
enum Slot {
    S_HIST, S_COUNT, S_DOFF, S_TILES, S_PPD, S_SEEDS, S_CAND = S_SEEDS + 3, S_KEPT = S_CAND + 3,
    S_POOL = S_KEPT + 3, S_TOP = S_POOL + 3, S_SPD = S_TOP + 3, S_SIDX, S_STATE, S_GHIST,
    S_SLO, S_STATE2, S_COUNTS, S_RADIUS, S_BAND, S_COUNT_ALL = S_BAND + 3
};

struct DevBuf {
    void* p = nullptr;
    const pmlsh_index* x;
    int slot;
    DevBuf(const pmlsh_index* idx, int s) : x(idx), slot(s) {}
    void alloc(size_t bytes) {
        if (bytes == 0) bytes = 1;
        auto& b = x->acp_bufs[slot];
        if (b.second < bytes) {
            if (b.first) {
                (void)hipFree(b.first);
                b = {nullptr, 0};
            }
            PMLSH_HIP(hipMalloc(&b.first, bytes));
            b.second = bytes;
        }
        p = b.first;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Small device-to-host reads of an ACP call (counts, selection states,
// histograms) go through a pinned host buffer of the index, kept with its
// workspace: a copy into pageable host memory is staged by the runtime and
// finishes before the next operation is issued, while copies into pinned
// memory queue like kernels, so the reads of one step cost one
// synchronisation. Calls on one index serialise on its mutex and every
// HostReads waits before the next is made, so one buffer serves them all.
constexpr size_t kHostReadBytes = 16384;
struct HostReads {
    unsigned char* base;
    hipStream_t st;
    size_t used = 0;
    int n = 0;
    struct Item {
        void* dst;
        size_t off, bytes;
    } items[8];
    HostReads(const pmlsh_index* x, hipStream_t s) : st(s) {
        if (!x->acp_host) PMLSH_HIP(hipHostMalloc(&x->acp_host, kHostReadBytes, hipHostMallocDefault));
        base = static_cast<unsigned char*>(x->acp_host);
    }
    void add(void* dst, const void* src, size_t bytes) {
        const size_t off = (used + 15) & ~size_t(15);
        if (n == 8 || off + bytes > kHostReadBytes) fail(PMLSH_EDEVICE, "host read staging overflow");
        PMLSH_HIP(hipMemcpyAsync(base + off, src, bytes, hipMemcpyDeviceToHost, st));
        items[n++] = {dst, off, bytes};
        used = off + bytes;
    }
    void wait() {
        PMLSH_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < n; ++i) std::memcpy(items[i].dst, base + items[i].off, items[i].bytes);
        n = 0;
        used = 0;
    }
};

struct Triplets {
    DevBuf k0, ii, jj;
    int64_t cap = 0;
    Triplets(const pmlsh_index* idx, int s) : k0(idx, s), ii(idx, s + 1), jj(idx, s + 2) {}
    void alloc(int64_t c) {
        cap = c;
        k0.alloc((size_t)c * 4);
        ii.alloc((size_t)c * 4);
        jj.alloc((size_t)c * 4);
    }
};

int grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    g = std::min<int64_t>(std::max<int64_t>(g, 1), 4096);
    return (int)g;
}

// Device-wide selection of the need-th smallest key. With value_only, only the
// first sub-key (the distance bits) is resolved.
SelKey select_kth(const pmlsh_index* x, const uint32_t* k0, const uint32_t* ii, const uint32_t* jj, int64_t count,
                  int64_t need, bool value_only, uint32_t* dhist, hipStream_t st) {
    SelKey K{0, 0, 0, 0};
    uint32_t v[3] = {0, 0, 0};
    std::vector<uint32_t> h(NB);
    for (int depth = 0; depth < 3; ++depth) {
        uint32_t prefix = 0;
        int pbits = 0;
        uint32_t last = 0;
        for (int pass = 0; pass < 3; ++pass) {
            const int width = pass < 2 ? 11 : 10;
            const int shift = 32 - pbits - width;
            SelStep s{depth, v[0], v[1], shift, (1u << width) - 1u, pbits, prefix};
            PMLSH_HIP(hipMemsetAsync(dhist, 0, NB * sizeof(uint32_t), st));
            hipLaunchKernelGGL(acp_hist_kernel, dim3(grid_for(count, WG * 16)), dim3(WG), 0, st,
                               k0, ii, jj, count, s, dhist);
            PMLSH_HIP(hipGetLastError());
            {
                HostReads rd(x, st);
                rd.add(h.data(), dhist, NB * sizeof(uint32_t));
                rd.wait();
            }
            int64_t cum = 0;
            int T = -1;
            for (int b = 0; b < (1 << width); ++b) {
                if (cum + h[b] >= need) { T = b; break; }
                cum += h[b];
            }
            if (T < 0) fail(PMLSH_EDEVICE, "radix select lost elements");
            need -= cum;
            prefix = (prefix << width) | (uint32_t)T;
            pbits += width;
            last = h[T];
        }
        v[depth] = prefix;
        K.depth = depth;
        K.v0 = v[0];
        K.v1 = v[1];
        K.v2 = v[2];
        if (value_only || (int64_t)last == need) return K;
    }
    return K;
}


// Device-side selection of the need-th smallest of `count` 32-bit keys (no
// host round trip): three histogram passes of 11, 11 and 10 bits, each
// followed by the pick kernel; the key is left in state->prefix and ghist is
// left cleared. With first_done the first pass (top 11 bits) is already in
// ghist (the self-join adds it); otherwise ghist must be clear on entry.
// With passes < 3 only the leading 11 or 22 bits of the key are resolved
// (state->pbits of them in state->prefix). The first pass starts from an
// empty state without reading it.
void device_select(const uint32_t* keys, int64_t count, int64_t need, SelState* state,
                   uint32_t* ghist, bool first_done, hipStream_t st, int passes = 3) {
    const int shifts[3] = {21, 10, 0}, widths[3] = {11, 11, 10};
    for (int pass = 0; pass < passes; ++pass) {
        if (pass > 0 || !first_done) {
            hipLaunchKernelGGL(acp_sel_hist_kernel, dim3(grid_for(count, WG * 16)), dim3(WG), 0,
                               st, keys, count, state, shifts[pass], widths[pass], ghist);
            PMLSH_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(acp_sel_pick_kernel, dim3(1), dim3(WG), 0, st, ghist, state,
                           widths[pass], pass == 0 ? need : (int64_t)-1);
        PMLSH_HIP(hipGetLastError());
    }
}

// Relative error bound of the FP32 squared distances in a pool: the verify
// kernel sums d_pad / 16 terms per lane and four shuffle levels, (d_pad / 16
// + 6) u; the self-join of leaves of at most 64 points sums chains of
// d_pad / 4 terms, (d_pad / 4 + 4) u; the self-join of larger leaves one
// chain of d_pad terms, (d_pad + 2) u. The band of the FP64 top-k is sized
// with twice the largest bound of the kernels that filled the pool.
double pool_gamma(const pmlsh_index* x, bool has_seeds) {
    const double u = 5.9604645e-08;
    double g = (double)(x->d_pad / 16 + 8);
    if (has_seeds) g = std::max(g, x->leaf_size <= 64 ? (double)(x->d_pad / 4 + 4)
                                                      : (double)(x->d_pad + 2));
    return 2.0 * u * g;
}

// Self-join of every leaf: distance bits to k0 (and ids to ii/jj when given),
// in the triangular layout of seed_off. For leaves of at most 64 points the
// first radix pass of the k-th seed is added to ghist (returns true).
bool launch_self_join(const pmlsh_index* x, const int64_t* doff, uint32_t* k0, uint32_t* ii,
                      uint32_t* jj, uint32_t* ghist, hipStream_t st) {
    if (x->leaf_size <= 64) {
        hipLaunchKernelGGL(acp_seed_join_kernel, dim3((unsigned)x->n_leaves), dim3(SJ_THREADS), 0,
                           st, x->data, x->d_pad, x->perm, x->n, x->leaf_size, doff, k0, ii, jj,
                           ghist);
        PMLSH_HIP(hipGetLastError());
        return true;
    }
    if (!ii || !jj) fail(PMLSH_EDEVICE, "self-join of large leaves needs id buffers");
    hipLaunchKernelGGL(acp_self_join_kernel, dim3((unsigned)x->n_leaves), dim3(WG), 0, st,
                       x->data, x->d_pad, x->perm, x->n, x->leaf_size, doff, k0, ii, jj);
    PMLSH_HIP(hipGetLastError());
    return false;
}

// Pair scan of a tile list (leaf pairs) against the projected radius: the
// wave-per-tile kernel on the leaves' sorted parent distances when leaves
// hold at most 64 points, the workgroup-per-tile kernel otherwise. Both emit
// exactly the pairs of the tiles with pd^2 < R2 (and a < b on diagonal
// tiles), counted in *counter and written while below cap.
struct TileScan {
    const pmlsh_index* x;
    hipStream_t st;
    NodeView v;
    int64_t leaf_base;
    DevBuf ppd, spd, sidx;
    bool wave = false;
    size_t lds = 0;

    TileScan(const pmlsh_index* idx, hipStream_t s)
        : x(idx), st(s),
          v{idx->tree.centre, idx->tree.radius, idx->tree.hr_min, idx->tree.hr_max, idx->n_nodes,
            idx->num_pivots},
          leaf_base(idx->level_begin[idx->levels - 1]), ppd(idx, S_PPD), spd(idx, S_SPD),
          sidx(idx, S_SIDX) {}

    // parent distances (and their per-leaf sorted copies) of every point
    void prepare() {
        const int64_t n = x->n, NL = x->n_leaves;
        const int L = x->leaf_size;
        ppd.alloc((size_t)n * sizeof(float));
        wave = L <= 64;
        if (wave) {
            spd.alloc((size_t)NL * 64 * sizeof(float));
            sidx.alloc((size_t)NL * 64);
            hipLaunchKernelGGL(acp_pd_sorted_kernel, dim3((unsigned)((NL + 3) / 4)), dim3(WG), 0,
                               st, x->proj_hi, x->proj_lo, v, leaf_base, n, L, NL,
                               ppd.as<float>(), spd.as<float>(), sidx.as<uint8_t>());
            PMLSH_HIP(hipGetLastError());
            return;
        }
        hipLaunchKernelGGL(acp_pd_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, st,
                           x->proj_hi, x->proj_lo, v, leaf_base, n, L, ppd.as<float>());
        PMLSH_HIP(hipGetLastError());
        lds = (size_t)L * MP * 4 * 4 + (size_t)L * 4 * 4 + (size_t)64 * 64 * 4;
        if (lds > 160 * 1024 - 256)
            fail(PMLSH_EUNSUPPORTED, "ACP leaves of this size do not fit the tile scan's LDS");
        PMLSH_HIP(hipFuncSetAttribute((const void*)acp_tile_scan_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }

    // With dn_tiles and rad (leaves of at most 64 points only), the tile count
    // and the radii are read on the device and n_tiles only bounds the count.
    void scan(const int2* tiles, int64_t n_tiles, float R2, float Rlim, uint32_t* k0,
              uint32_t* ii, uint32_t* jj, int64_t cap, unsigned long long* counter,
              const unsigned long long* dn_tiles = nullptr, const AcpRadius* rad = nullptr) {
        if (n_tiles <= 0) return;
        if (wave) {
            const int64_t waves = std::min<int64_t>(n_tiles, 16384);
            hipLaunchKernelGGL(acp_tile_scan_wave_kernel, dim3((unsigned)((waves + 3) / 4)),
                               dim3(WG), 0, st, x->proj_hi, x->proj_lo, ppd.as<float>(),
                               spd.as<float>(), sidx.as<uint8_t>(), v, leaf_base, x->perm, x->n,
                               x->leaf_size, tiles, n_tiles, R2, Rlim, k0, ii, jj, cap, counter,
                               dn_tiles, rad);
        } else {
            if (dn_tiles || rad) fail(PMLSH_EDEVICE, "device radii need leaves of at most 64 points");
            hipLaunchKernelGGL(acp_tile_scan_kernel, dim3(grid_for(n_tiles, 1)), dim3(WG), lds, st,
                               x->proj_hi, x->proj_lo, ppd.as<float>(), v, leaf_base, x->perm,
                               x->n, x->leaf_size, tiles, n_tiles, R2, Rlim, k0, ii, jj, cap,
                               counter);
        }
        PMLSH_HIP(hipGetLastError());
    }
};

}  // namespace

// The k nearest pairs of the verified pool, in (distance, i, j) order. The
// FP32 k-th distance (selected on the device) bounds the band of pairs that
// can belong to the exact top-k: every pool value carries a relative error
// of at most gamma (pool_gamma), so a pair whose exact distance is at most
// the exact k-th one has an FP32 value within kth (1 + 4 gamma); the band's
// order is taken in FP64. A band of more than kTopBand pairs (mass ties)
// keeps the FP32 order.
// With dn_add the pool holds n_pool + *dn_add pairs (counted on the device),
// at most n_max; the count is read back only when the one-workgroup kernel
// cannot finish alone.
void pool_topk(const pmlsh_index* x, Triplets& pool, int64_t n_pool, int k, double gamma,
               Triplets& top, DevBuf& dhist, DevBuf& dcount, int64_t* out_pairs,
               float* out_dist, hipStream_t st, const unsigned long long* dn_add = nullptr,
               int64_t n_max = 0) {
    DevBuf dstate(x, S_STATE), ghist(x, S_GHIST);
    dstate.alloc(sizeof(SelState));
    ghist.alloc(NB * sizeof(uint32_t));
    auto exact_count = [&] {
        unsigned long long extra = 0;
        {
            HostReads rd(x, st);
            rd.add(&extra, dn_add, sizeof(extra));
            rd.wait();
        }
        n_pool += (int64_t)extra;
        dn_add = nullptr;
        if (n_pool < k) fail(PMLSH_EDEVICE, "fewer verified pairs than k");
    };
    if (dn_add && n_max > kSmallPool) exact_count();
    if (n_pool < k && !dn_add) fail(PMLSH_EDEVICE, "fewer verified pairs than k");
    if ((dn_add ? n_max : n_pool) <= kSmallPool) {
        // one workgroup: select, band and FP64 order; falls through on mass ties
        PMLSH_HIP(hipFuncSetAttribute((const void*)acp_topk_small_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)kSmallTopkLds));
        hipLaunchKernelGGL(acp_topk_small_kernel, dim3(1), dim3(WG), kSmallTopkLds, st,
                           pool.k0.as<uint32_t>(), pool.ii.as<uint32_t>(),
                           pool.jj.as<uint32_t>(), (int)n_pool, k, 4.0 * gamma, x->data,
                           x->d_pad, x->inv_perm, out_pairs, out_dist,
                           static_cast<int*>(dcount.p), dn_add);
        PMLSH_HIP(hipGetLastError());
        int m = 0;
        {
            HostReads rd(x, st);
            rd.add(&m, dcount.p, sizeof(m));
            rd.wait();
        }
        if (m < k) fail(PMLSH_EDEVICE, "top-k selection lost pairs");
        if (m <= kTopBand) return;
        if (dn_add) exact_count();
    }
    PMLSH_HIP(hipMemsetAsync(ghist.p, 0, NB * sizeof(uint32_t), st));
    device_select(pool.k0.as<uint32_t>(), n_pool, k, dstate.as<SelState>(),
                  ghist.as<uint32_t>(), false, st);
    top.alloc(kTopBand);
    PMLSH_HIP(hipMemsetAsync(dcount.p, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(acp_band_gather_kernel, dim3(grid_for(n_pool, WG)), dim3(WG), 0, st,
                       pool.k0.as<uint32_t>(), pool.ii.as<uint32_t>(), pool.jj.as<uint32_t>(),
                       n_pool, dstate.as<SelState>(), 4.0 * gamma, top.k0.as<uint32_t>(),
                       top.ii.as<uint32_t>(), top.jj.as<uint32_t>(), (int64_t)kTopBand,
                       static_cast<unsigned long long*>(dcount.p));
    PMLSH_HIP(hipGetLastError());
    unsigned long long m = 0;
    {
        HostReads rd(x, st);
        rd.add(&m, dcount.p, sizeof(m));
        rd.wait();
    }
    if ((int64_t)m < k) fail(PMLSH_EDEVICE, "top-k selection lost pairs");
    if ((int64_t)m <= kTopBand) {
        hipLaunchKernelGGL(acp_final64_kernel, dim3(1), dim3(WG), 0, st, x->data, x->d_pad,
                           x->inv_perm, top.ii.as<uint32_t>(), top.jj.as<uint32_t>(), (int)m,
                           k, out_pairs, out_dist);
    } else {
        // mass ties: the k smallest full keys (distance bits, i, j) in FP32
        const SelKey K = select_kth(x, pool.k0.as<uint32_t>(), pool.ii.as<uint32_t>(),
                                    pool.jj.as<uint32_t>(), n_pool, k, false,
                                    dhist.as<uint32_t>(), st);
        PMLSH_HIP(hipMemsetAsync(dcount.p, 0, sizeof(unsigned long long), st));
        hipLaunchKernelGGL(acp_gather_kernel, dim3(grid_for(n_pool, WG)), dim3(WG), 0, st,
                           pool.k0.as<uint32_t>(), pool.ii.as<uint32_t>(),
                           pool.jj.as<uint32_t>(), n_pool, K, top.k0.as<uint32_t>(),
                           top.ii.as<uint32_t>(), top.jj.as<uint32_t>(), (int64_t)k,
                           static_cast<unsigned long long*>(dcount.p));
        PMLSH_HIP(hipGetLastError());
        unsigned long long g = 0;
        {
            HostReads rd(x, st);
            rd.add(&g, dcount.p, sizeof(g));
            rd.wait();
        }
        if ((int64_t)g != k) fail(PMLSH_EDEVICE, "top-k selection lost pairs");
        hipLaunchKernelGGL(acp_final_kernel, dim3(1), dim3(WG), 0, st, top.k0.as<uint32_t>(),
                           top.ii.as<uint32_t>(), top.jj.as<uint32_t>(), k, out_pairs,
                           out_dist);
    }
    PMLSH_HIP(hipGetLastError());
    PMLSH_HIP(hipStreamSynchronize(st));
}

void run_acp(const pmlsh_index* x, int k, double c, double confidence, double beta,
             int64_t* out_pairs, float* out_dist, pmlsh_acp_stats* stats,
             hipStream_t st) {
    pmlsh_plan plan;
    plan_params(x->n, x->m, k, c, confidence, beta, &plan);
    const int64_t n = x->n;
    const int L = x->leaf_size;
    const int64_t NL = x->n_leaves;

    std::lock_guard<std::mutex> lock(x->acp_mu);
    if ((int)x->acp_bufs.size() < S_COUNT_ALL) x->acp_bufs.resize(S_COUNT_ALL, {nullptr, 0});
    DevBuf dhist(x, S_HIST), dcount(x, S_COUNT), dstate(x, S_STATE), ghist(x, S_GHIST);
    dhist.alloc(NB * sizeof(uint32_t));
    dcount.alloc(sizeof(unsigned long long));
    dstate.alloc(sizeof(SelState));
    ghist.alloc(NB * sizeof(uint32_t));
    auto reset_counter = [&] {
        PMLSH_HIP(hipMemsetAsync(dcount.p, 0, sizeof(unsigned long long), st));
    };
    auto read_counter = [&]() -> int64_t {
        unsigned long long v = 0;
        {
            HostReads rd(x, st);
            rd.add(&v, dcount.p, sizeof(v));
            rd.wait();
        }
        return (int64_t)v;
    };
    // ---- seeds: every within-leaf pair
    std::vector<int64_t> seed_off(NL + 1, 0);
    for (int64_t b = 0; b < NL; ++b) {
        const int64_t cnt = std::min<int64_t>(L, n - b * L);
        seed_off[b + 1] = seed_off[b] + cnt * (cnt - 1) / 2;
    }
    const int64_t n_seed = seed_off[NL];
    Triplets seeds(x, S_SEEDS), band(x, S_BAND);
    DevBuf doff(x, S_DOFF), slo(x, S_SLO);
    double ub = HUGE_VAL;
    uint32_t ub2_bits = 0x7f800000u;
    PMLSH_HIP(hipMemsetAsync(ghist.p, 0, NB * sizeof(uint32_t), st));
    auto read_ub = [&] {
        SelState hs{};
        {
            HostReads rd(x, st);
            rd.add(&hs, dstate.p, sizeof(hs));
            rd.wait();
        }
        ub2_bits = hs.prefix;
        float ub2;
        std::memcpy(&ub2, &ub2_bits, 4);
        ub = std::sqrt((double)ub2);
    };

    // Leaves of at most 64 points: bounds of every seed from the FP16 Gram
    // kernel, U >= the k-th smallest upper bound, and exact FP32 distances
    // (the verify kernel's) for the band of seeds whose lower bound is at most
    // U (1 + 8 gamma) only. The k seeds of smallest exact distance lie in the
    // band (their lower bounds are at most U), so its k-th FP32 distance ub2
    // is at most U (1 + gamma / 2), and any seed outside the band has an FP32
    // distance above U (1 + 8 gamma) (1 - gamma / 2) > ub2 (1 + 4 gamma): ub2
    // is the k-th FP32 seed distance over all seeds, and the band holds every
    // seed the pool takes. A band above band_max (mass ties) falls back to
    // the direct self-join.
    const double gamma_v = pool_gamma(x, false);
    const int gram_k = 32 * ((x->d_pad + 31) / 32);
    const int64_t first_cap = tune_get(PMLSH_TUNE_ACP_FIRST_CAP);   // 0: the defaults
    bool gram = false, deferred = false, all_seeds = n_seed < k;
    int64_t n_band = 0, band_max = 0, bcap = 0;
    DevBuf dstate2(x, S_STATE2), dcnts(x, S_COUNTS), drad(x, S_RADIUS);
    dcnts.alloc(4 * sizeof(unsigned long long));
    drad.alloc(sizeof(AcpRadius));
    auto take_ub = [&](const SelState& hs) {
        ub2_bits = hs.prefix;
        float ub2;
        std::memcpy(&ub2, &ub2_bits, 4);
        ub = std::sqrt((double)ub2);
    };
    // the band at capacity bcap: gathered (its size counted in dcnts[0]),
    // verified, and its k-th selected into dstate2, all on the device
    auto launch_band = [&] {
        unsigned long long* cnt = dcnts.as<unsigned long long>();
        band.alloc(bcap);
        PMLSH_HIP(hipMemsetAsync(dcnts.p, 0, 4 * sizeof(unsigned long long), st));
        hipLaunchKernelGGL(acp_seed_gram_band_kernel, dim3((unsigned)((NL + kBandWaves - 1) / kBandWaves)),
                           dim3(64 * kBandWaves), 0, st, slo.as<uint32_t>(), x->perm, n, L, NL,
                           dstate.as<SelState>(),
                           (float)(8.0 * gamma_v), all_seeds ? 1 : 0, band.ii.as<uint32_t>(),
                           band.jj.as<uint32_t>(), bcap, cnt);
        PMLSH_HIP(hipGetLastError());
        hipLaunchKernelGGL(acp_verify_kernel, dim3(grid_for(bcap, WG / 16)), dim3(WG), 0, st,
                           x->data, x->d_pad, x->inv_perm, band.ii.as<uint32_t>(),
                           band.jj.as<uint32_t>(), bcap, band.k0.as<uint32_t>(),
                           band.ii.as<uint32_t>(), band.jj.as<uint32_t>(),
                           static_cast<const unsigned long long*>(cnt));
        PMLSH_HIP(hipGetLastError());
        if (!all_seeds) {
            hipLaunchKernelGGL(acp_kth_small_kernel, dim3(1), dim3(WG), 0, st,
                               band.k0.as<uint32_t>(), bcap,
                               static_cast<const unsigned long long*>(cnt), (int64_t)k,
                               dstate2.as<SelState>());
            PMLSH_HIP(hipGetLastError());
        }
    };
    // the band's size (and ub) read back: true when the band fit its capacity
    auto read_band = [&]() -> bool {
        unsigned long long nb = 0;
        SelState hs{};
        {
            HostReads rd(x, st);
            rd.add(&nb, dcnts.p, sizeof(nb));
            rd.add(&hs, dstate2.p, sizeof(hs));
            rd.wait();
        }
        n_band = (int64_t)nb;
        if (n_band > bcap) return false;
        if (!all_seeds) take_ub(hs);
        return true;
    };
    // direct self-join: exact distance bits of every seed (the ids of the
    // few seeds the top-k can use are recovered from their position)
    auto direct_seeds = [&] {
        gram = false;
        doff.alloc((NL + 1) * sizeof(int64_t));
        PMLSH_HIP(hipMemcpyAsync(doff.p, seed_off.data(), (NL + 1) * sizeof(int64_t),
                                 hipMemcpyHostToDevice, st));
        seeds.k0.alloc((size_t)n_seed * 4);
        if (L > 64) {
            seeds.ii.alloc((size_t)n_seed * 4);
            seeds.jj.alloc((size_t)n_seed * 4);
        }
        bool first_done;
        {
            StageTimer tm(PMLSH_STAGE_ACP_SELFJOIN, st);
            first_done = launch_self_join(x, doff.as<int64_t>(), seeds.k0.as<uint32_t>(),
                                          L > 64 ? seeds.ii.as<uint32_t>() : nullptr,
                                          L > 64 ? seeds.jj.as<uint32_t>() : nullptr,
                                          ghist.as<uint32_t>(), st);
        }
        // ub: k-th smallest seed distance (selected on the device)
        if (n_seed >= k) {
            StageTimer tm(PMLSH_STAGE_ACP_SELECT, st);
            device_select(seeds.k0.as<uint32_t>(), n_seed, k, dstate.as<SelState>(),
                          ghist.as<uint32_t>(), first_done, st);
            read_ub();
        }
    };
    if (n_seed > 0 && L <= 64 && gram_k <= 65536) {
        seeds.k0.alloc((size_t)n_seed * 4);
        slo.alloc((size_t)n_seed * 4);
        const double ukd = (double)gram_k * std::ldexp(1.0, -23);
        const float gk = (float)(ukd / (1.0 - ukd) * (1.0 + 1e-6));
        {
            StageTimer tm(PMLSH_STAGE_ACP_SELFJOIN, st);
            if (x->d_pad <= SG_X0)
                hipLaunchKernelGGL(acp_seed_gram_kernel<true>, dim3((unsigned)NL), dim3(WG), 0, st,
                                   x->data, x->d_pad, x->data16_scale, n, L, gk,
                                   seeds.k0.as<uint32_t>(), slo.as<uint32_t>(), ghist.as<uint32_t>());
            else
                hipLaunchKernelGGL(acp_seed_gram_kernel<false>, dim3((unsigned)NL), dim3(WG), 0, st,
                                   x->data, x->d_pad, x->data16_scale, n, L, gk,
                                   seeds.k0.as<uint32_t>(), slo.as<uint32_t>(), ghist.as<uint32_t>());
            PMLSH_HIP(hipGetLastError());
        }
        StageTimer tm(PMLSH_STAGE_ACP_SELECT, st);
        all_seeds = n_seed < k;
        // U: the upper edge of the 22-bit radix bin of the k-th smallest upper
        // bound (at least that bound, and at most 2^-19 above it)
        if (!all_seeds)
            device_select(seeds.k0.as<uint32_t>(), n_seed, k, dstate.as<SelState>(),
                          ghist.as<uint32_t>(), true, st, 2);
        // The band is gathered, verified and its k-th selected without a host
        // round trip (the verify and selection kernels read the band's size
        // on the device), and the radii follow on the device: the tile filter
        // and the pair scan run before the host reads anything back. A band
        // beyond its capacity is gathered again at its size, and what
        // followed it is redone.
        dstate2.alloc(sizeof(SelState));
        band_max = std::max<int64_t>(int64_t(1) << 20, n_seed / 8);
        bcap = std::min<int64_t>(n_seed, first_cap > 0 ? first_cap
                                                       : std::max<int64_t>(int64_t(1) << 16, 4 * (int64_t)k));
        launch_band();
        hipLaunchKernelGGL(acp_radius_kernel, dim3(1), dim3(1), 0, st, dstate2.as<SelState>(),
                           all_seeds ? 0 : 1, plan.t, gamma_v, x->coord_scale,
                           static_cast<const unsigned long long*>(dcnts.p), bcap,
                           drad.as<AcpRadius>());
        PMLSH_HIP(hipGetLastError());
        deferred = true;
    }
    if (!deferred && n_seed > 0) direct_seeds();

    // ---- tiles surviving Mindist (Eq. 11), then the pair scan of those tiles
    const int64_t tiles_total = NL * (NL - 1) / 2;
    if (tiles_total > (int64_t(1) << 31) || NL > 65535)
        fail(PMLSH_EUNSUPPORTED, "ACP supports at most 65535 leaves");
    int64_t n_tiles = 0;
    DevBuf tiles(x, S_TILES);
    TileScan scan(x, st);
    constexpr int64_t kMaxCand = int64_t(1) << 28;
    Triplets cand(x, S_CAND);
    int64_t n_raw = 0;
    int64_t cap = first_cap > 0 ? first_cap
                                : std::min<int64_t>(kMaxCand, std::max<int64_t>(int64_t(1) << 20, 4 * (int64_t)k));
    double R = 0.0;
    float R2 = 0.f, limit = 0.f;
    auto set_radii = [&] {
        R = plan.t * ub;
        R2 = std::isinf(R) ? INFINITY : (float)(R * R);
        const float slack = (float)(1e-5 * (2.0 * x->coord_scale + (std::isinf(R) ? 0.0 : R)));
        limit = std::isinf(R) ? INFINITY : (float)R + slack;
    };
    // tile filter and pair scan with host radii and host round trips
    auto tiles_and_scan = [&] {
        n_tiles = 0;
        n_raw = 0;
        if (tiles_total > 0) {
            tiles.alloc((size_t)tiles_total * sizeof(int2));
            reset_counter();
            StageTimer tm(PMLSH_STAGE_ACP_TILES, st);
            scan.prepare();
            hipLaunchKernelGGL(acp_tile_filter_kernel, dim3((unsigned)NL), dim3(WG), 0, st, scan.v,
                               scan.leaf_base, NL, limit, 0, tiles.as<int2>(), tiles_total,
                               static_cast<unsigned long long*>(dcount.p), nullptr);
            PMLSH_HIP(hipGetLastError());
        }
        if (tiles_total > 0) n_tiles = read_counter();
        for (int attempt = 0; n_tiles > 0 && attempt < 2; ++attempt) {
            cand.alloc(cap);
            reset_counter();
            {
                StageTimer tm(PMLSH_STAGE_ACP_SCAN, st);
                scan.scan(tiles.as<int2>(), n_tiles, R2, limit, cand.k0.as<uint32_t>(),
                          cand.ii.as<uint32_t>(), cand.jj.as<uint32_t>(), cap,
                          static_cast<unsigned long long*>(dcount.p));
            }
            n_raw = read_counter();
            if (n_raw <= cap) break;
            if (n_raw > kMaxCand)
                fail(PMLSH_EUNSUPPORTED, "more than 2^28 candidate pairs pass the radius filter");
            cap = n_raw;
        }
    };
    if (deferred) {
        unsigned long long* cnt = dcnts.as<unsigned long long>();
        if (tiles_total > 0) {
            tiles.alloc((size_t)tiles_total * sizeof(int2));
            {
                StageTimer tm(PMLSH_STAGE_ACP_TILES, st);
                scan.prepare();
                hipLaunchKernelGGL(acp_tile_filter_kernel, dim3((unsigned)NL), dim3(WG), 0, st,
                                   scan.v, scan.leaf_base, NL, 0.f, 0, tiles.as<int2>(), tiles_total,
                                   cnt + 1, drad.as<AcpRadius>());
                PMLSH_HIP(hipGetLastError());
            }
            cand.alloc(cap);
            StageTimer tm(PMLSH_STAGE_ACP_SCAN, st);
            scan.scan(tiles.as<int2>(), tiles_total, 0.f, 0.f, cand.k0.as<uint32_t>(),
                      cand.ii.as<uint32_t>(), cand.jj.as<uint32_t>(), cap, cnt + 2, cnt + 1,
                      drad.as<AcpRadius>());
        }
        // the one read of this sequence: band size, ub, tile and candidate counts
        unsigned long long hc[3] = {0, 0, 0};
        SelState hs{};
        {
            HostReads rd(x, st);
            rd.add(hc, dcnts.p, sizeof(hc));
            rd.add(&hs, dstate2.p, sizeof(hs));
            rd.wait();
        }
        n_band = (int64_t)hc[0];
        if (n_band <= bcap) {
            gram = true;
            if (!all_seeds) take_ub(hs);
            set_radii();
            n_tiles = (int64_t)hc[1];
            n_raw = (int64_t)hc[2];
            if (n_raw > cap) {
                // the candidate buffer overflowed: scan again at the full count
                if (n_raw > kMaxCand)
                    fail(PMLSH_EUNSUPPORTED, "more than 2^28 candidate pairs pass the radius filter");
                cap = n_raw;
                cand.alloc(cap);
                reset_counter();
                {
                    StageTimer tm(PMLSH_STAGE_ACP_SCAN, st);
                    scan.scan(tiles.as<int2>(), n_tiles, R2, limit, cand.k0.as<uint32_t>(),
                              cand.ii.as<uint32_t>(), cand.jj.as<uint32_t>(), cap,
                              static_cast<unsigned long long*>(dcount.p));
                }
                if (read_counter() != n_raw) fail(PMLSH_EDEVICE, "pair scan count changed");
            }
        } else {
            // the band outgrew its capacity: gather it again at its size (or
            // take the direct self-join), then the tiles and the scan
            if (n_band <= band_max) {
                bcap = n_band;
                launch_band();
                gram = read_band();
            }
            if (!gram) direct_seeds();
            set_radii();
            tiles_and_scan();
        }
    } else {
        set_radii();
        tiles_and_scan();
    }

    // ---- budget T: keep the projected-nearest candidates
    const int64_t keep = std::max<int64_t>(0, plan.acp_budget - n_seed);
    int64_t n_keep = std::min(n_raw, keep);
    Triplets kept(x, S_KEPT);
    const Triplets* cands = &cand;
    if (n_raw > keep && keep > 0) {
        SelKey K = select_kth(x, cand.k0.as<uint32_t>(), cand.ii.as<uint32_t>(),
                              cand.jj.as<uint32_t>(), n_raw, keep, false, dhist.as<uint32_t>(), st);
        kept.alloc(keep);
        reset_counter();
        hipLaunchKernelGGL(acp_gather_kernel, dim3(grid_for(n_raw, WG)), dim3(WG), 0, st,
                           cand.k0.as<uint32_t>(), cand.ii.as<uint32_t>(), cand.jj.as<uint32_t>(),
                           n_raw, K, kept.k0.as<uint32_t>(), kept.ii.as<uint32_t>(),
                           kept.jj.as<uint32_t>(), keep,
                           static_cast<unsigned long long*>(dcount.p));
        PMLSH_HIP(hipGetLastError());
        if (read_counter() != keep) fail(PMLSH_EDEVICE, "budget cut lost candidates");
        cands = &kept;
    }

    // ---- the pool: the seeds within the band of the top-k (every seed when
    // there are fewer than k), then the verified candidates. The pool's k-th
    // FP32 distance is at most the seeds' k-th (ub^2), so every seed its
    // FP64 band can hold lies within ub^2 (1 + 4 gamma).
    const double gamma = gram ? gamma_v : pool_gamma(x, true);
    uint32_t seed_lim = 0xffffffffu;
    if (n_seed >= k) {
        float ub2;
        std::memcpy(&ub2, &ub2_bits, 4);
        const float lim = std::nextafter((float)((double)ub2 * (1.0 + 4.0 * gamma)), INFINITY);
        std::memcpy(&seed_lim, &lim, 4);
    }
    Triplets pool(x, S_POOL);
    Triplets top(x, S_TOP);
    if (gram) {
        // the verified candidates first (their number is known), then the
        // band's seeds appended on a device counter: the pool's size is read
        // back only if the top-k cannot finish in one workgroup
        pool.alloc(std::max<int64_t>(n_band + n_keep, 1));
        unsigned long long* nseeds = dcnts.as<unsigned long long>() + 3;
        PMLSH_HIP(hipMemsetAsync(nseeds, 0, sizeof(unsigned long long), st));
        {
            StageTimer tm(PMLSH_STAGE_ACP_VERIFY, st);
            if (n_keep > 0) {
                hipLaunchKernelGGL(acp_verify_kernel, dim3(grid_for(n_keep, WG / 16)), dim3(WG), 0, st,
                                   x->data, x->d_pad, x->inv_perm, cands->ii.as<uint32_t>(),
                                   cands->jj.as<uint32_t>(), n_keep, pool.k0.as<uint32_t>(),
                                   pool.ii.as<uint32_t>(), pool.jj.as<uint32_t>(), nullptr);
                PMLSH_HIP(hipGetLastError());
            }
            if (n_band > 0) {
                const SelKey all{0, seed_lim, 0, 0};
                hipLaunchKernelGGL(acp_gather_kernel, dim3(grid_for(n_band, WG)), dim3(WG), 0, st,
                                   band.k0.as<uint32_t>(), band.ii.as<uint32_t>(),
                                   band.jj.as<uint32_t>(), n_band, all,
                                   pool.k0.as<uint32_t>() + n_keep, pool.ii.as<uint32_t>() + n_keep,
                                   pool.jj.as<uint32_t>() + n_keep, n_band, nseeds);
                PMLSH_HIP(hipGetLastError());
            }
        }
        StageTimer tm(PMLSH_STAGE_ACP_TOPK, st);
        pool_topk(x, pool, n_keep, k, gamma, top, dhist, dcount, out_pairs, out_dist, st, nseeds,
                  n_keep + n_band);
    } else {
        int64_t seed_cap = std::min<int64_t>(n_seed, std::max<int64_t>(4096, 4 * (int64_t)k));
        int64_t n_pool_seeds = 0;
        for (int attempt = 0; attempt < 2; ++attempt) {
            pool.alloc(std::max<int64_t>(seed_cap + n_keep, 1));
            if (n_seed == 0) break;
            reset_counter();
            StageTimer tm(PMLSH_STAGE_ACP_VERIFY, st);
            const SelKey all{0, seed_lim, 0, 0};
            if (L > 64) {
                hipLaunchKernelGGL(acp_gather_kernel, dim3(grid_for(n_seed, WG)), dim3(WG), 0, st,
                                   seeds.k0.as<uint32_t>(), seeds.ii.as<uint32_t>(),
                                   seeds.jj.as<uint32_t>(), n_seed, all, pool.k0.as<uint32_t>(),
                                   pool.ii.as<uint32_t>(), pool.jj.as<uint32_t>(), seed_cap,
                                   static_cast<unsigned long long*>(dcount.p));
            } else {
                hipLaunchKernelGGL(acp_seed_band_kernel, dim3((unsigned)NL), dim3(WG), 0, st,
                                   seeds.k0.as<uint32_t>(), doff.as<int64_t>(), x->perm, n, L,
                                   seed_lim, pool.k0.as<uint32_t>(), pool.ii.as<uint32_t>(),
                                   pool.jj.as<uint32_t>(), seed_cap,
                                   static_cast<unsigned long long*>(dcount.p));
            }
            PMLSH_HIP(hipGetLastError());
            n_pool_seeds = read_counter();
            if (n_pool_seeds <= seed_cap) break;
            seed_cap = n_pool_seeds;
        }
        if (n_pool_seeds > seed_cap) fail(PMLSH_EDEVICE, "seed band grew between two passes");
        const int64_t n_pool = n_pool_seeds + n_keep;
        if (n_keep > 0) {
            StageTimer tm(PMLSH_STAGE_ACP_VERIFY, st);
            hipLaunchKernelGGL(acp_verify_kernel, dim3(grid_for(n_keep, WG / 16)), dim3(WG), 0, st,
                               x->data, x->d_pad, x->inv_perm, cands->ii.as<uint32_t>(),
                               cands->jj.as<uint32_t>(), n_keep, pool.k0.as<uint32_t>() + n_pool_seeds,
                               pool.ii.as<uint32_t>() + n_pool_seeds,
                               pool.jj.as<uint32_t>() + n_pool_seeds, nullptr);
            PMLSH_HIP(hipGetLastError());
        }
        if (n_pool < k) fail(PMLSH_EDEVICE, "fewer verified pairs than k");

        // ---- top-k over the pool
        {
            StageTimer tm(PMLSH_STAGE_ACP_TOPK, st);
            pool_topk(x, pool, n_pool, k, gamma, top, dhist, dcount, out_pairs, out_dist, st);
        }
    }

    if (stats) {
        stats->t = plan.t;
        stats->ub = ub;
        stats->budget = plan.acp_budget;
        stats->n_seed = n_seed;
        stats->n_cand_raw = n_raw;
        stats->n_cand = n_keep;
        stats->tiles_total = tiles_total;
        stats->tiles_scanned = n_tiles;
    }
}

// (c,k)-ACP by the branch-and-bound algorithm (Algorithm 3, Section 6.1): the
// T pairs with the smallest projected distances over all pairs (ties by
// (i, j)) are verified and the k nearest returned. Best-first search with
// Mindist pruning finds exactly those T pairs; here a projected distance d_T
// with at least T pairs at or below it is found first (the T-th smallest
// projected distance of the pairs inside leaves, or a radius grown by 4x
// from their largest while fewer than T pairs are found), the pairs at or
// below d_T are collected by the tile scan (leaf pairs whose Mindist
// exceeds d_T skipped whole, as the search would) and the T smallest are
// cut by a radix select on (pd^2, i, j).
void run_acp_bb(const pmlsh_index* x, int k, double c, double confidence, double beta,
                int64_t* out_pairs, float* out_dist, pmlsh_acp_stats* stats, hipStream_t st) {
    pmlsh_plan plan;
    plan_params(x->n, x->m, k, c, confidence, beta, &plan);
    const int64_t n = x->n;
    const int L = x->leaf_size;
    const int64_t NL = x->n_leaves;
    const int64_t n_pairs = n * (n - 1) / 2;
    const int64_t T = std::min<int64_t>(plan.acp_budget, n_pairs);
    constexpr int64_t kMaxCand = int64_t(1) << 28;
    if (NL > 65535) fail(PMLSH_EUNSUPPORTED, "ACP supports at most 65535 leaves");
    // the T projected-closest pairs are collected at once: a larger budget
    // cannot be served, which is known before any scan
    if (T > kMaxCand) fail(PMLSH_EUNSUPPORTED, "the budget T exceeds the 2^28 pairs one call collects");

    std::lock_guard<std::mutex> lock(x->acp_mu);
    if ((int)x->acp_bufs.size() < S_COUNT_ALL) x->acp_bufs.resize(S_COUNT_ALL, {nullptr, 0});
    DevBuf dhist(x, S_HIST), dcount(x, S_COUNT), tiles(x, S_TILES);
    Triplets cand(x, S_CAND), kept(x, S_KEPT), pool(x, S_POOL), top(x, S_TOP);
    dhist.alloc(NB * sizeof(uint32_t));
    dcount.alloc(sizeof(unsigned long long));
    auto read_counter = [&]() -> int64_t {
        unsigned long long v = 0;
        {
            HostReads rd(x, st);
            rd.add(&v, dcount.p, sizeof(v));
            rd.wait();
        }
        return (int64_t)v;
    };
    auto reset_counter = [&] {
        PMLSH_HIP(hipMemsetAsync(dcount.p, 0, sizeof(unsigned long long), st));
    };
    TileScan tscan(x, st);
    tscan.prepare();
    const int64_t leaf_base = tscan.leaf_base;
    const NodeView v = tscan.v;
    const int64_t tiles_all = NL * (NL - 1) / 2 + NL;
    tiles.alloc((size_t)tiles_all * sizeof(int2));

    // tiles: the diagonal ones only (d2 < 0), or every leaf pair whose
    // Mindist can reach the projected distance sqrt(d2)
    auto make_tiles = [&](float d2) -> int64_t {
        if (d2 < 0.f) {
            std::vector<int2> diag((size_t)NL);
            for (int64_t e = 0; e < NL; ++e) diag[(size_t)e] = make_int2((int)e, (int)e);
            PMLSH_HIP(hipMemcpyAsync(tiles.p, diag.data(), diag.size() * sizeof(int2),
                                     hipMemcpyHostToDevice, st));
            PMLSH_HIP(hipStreamSynchronize(st));
            return NL;
        }
        const double R = std::sqrt((double)d2);
        const float limit = std::isinf(R)
                                ? INFINITY
                                : (float)(R + 1e-5 * (2.0 * x->coord_scale + R)) * 1.0001f;
        reset_counter();
        dim3 grid((unsigned)NL);
        hipLaunchKernelGGL(acp_tile_filter_kernel, grid, dim3(WG), 0, st, v, leaf_base, NL,
                           limit, 1, tiles.as<int2>(), tiles_all,
                           static_cast<unsigned long long*>(dcount.p), nullptr);
        PMLSH_HIP(hipGetLastError());
        return read_counter();
    };
    // pairs of the tiles with pd^2 <= d2 (counted; written when cap > 0)
    auto scan = [&](int64_t n_tiles, float d2, float limit, int64_t cap) -> int64_t {
        const float R2 = std::isinf(d2) ? INFINITY : std::nextafter(d2, INFINITY);
        reset_counter();
        tscan.scan(tiles.as<int2>(), n_tiles, R2, limit,
                   cap > 0 ? cand.k0.as<uint32_t>() : nullptr,
                   cap > 0 ? cand.ii.as<uint32_t>() : nullptr,
                   cap > 0 ? cand.jj.as<uint32_t>() : nullptr, cap,
                   static_cast<unsigned long long*>(dcount.p));
        return read_counter();
    };
    auto limit_of = [&](float d2) {
        const double R = std::sqrt((double)d2);
        return std::isinf(R) ? INFINITY
                             : (float)(R + 1e-5 * (2.0 * x->coord_scale + R)) * 1.0001f;
    };

    // d_T: the T-th smallest projected distance inside leaves bounds the
    // global one from above; with fewer such pairs, grow a radius until at
    // least T pairs lie within it
    float d2 = INFINITY;
    if (T < n_pairs) {
        const int64_t nd = make_tiles(-1.f);
        const int64_t n_in = scan(nd, INFINITY, INFINITY, 0);
        if (n_in > kMaxCand) fail(PMLSH_EUNSUPPORTED, "too many pairs inside leaves");
        cand.alloc(std::max<int64_t>(n_in, 1));
        scan(nd, INFINITY, INFINITY, n_in);
        if (n_in >= T && n_in > 0) {
            SelKey K = select_kth(x, cand.k0.as<uint32_t>(), cand.ii.as<uint32_t>(),
                                  cand.jj.as<uint32_t>(), n_in, T, true, dhist.as<uint32_t>(),
                                  st);
            std::memcpy(&d2, &K.v0, 4);
        } else {
            // start from the largest pair distance inside leaves (or, with no
            // such pair, from a millionth of the coordinate range squared)
            float top2 = (float)(4e-6 * (double)x->coord_scale * (double)x->coord_scale);
            if (n_in > 0) {
                SelKey K = select_kth(x, cand.k0.as<uint32_t>(), cand.ii.as<uint32_t>(),
                                      cand.jj.as<uint32_t>(), n_in, n_in, true,
                                      dhist.as<uint32_t>(), st);
                std::memcpy(&top2, &K.v0, 4);
            }
            d2 = std::max(top2, 1e-30f) * 4.f;
            for (;;) {
                const int64_t nt = make_tiles(d2);
                if (scan(nt, d2, limit_of(d2), 0) >= T || std::isinf(d2)) break;
                d2 = d2 * 4.f;
            }
        }
    }
    const int64_t n_tiles = make_tiles(d2);
    const int64_t n_raw = scan(n_tiles, d2, limit_of(d2), 0);
    if (n_raw > kMaxCand)
        fail(PMLSH_EUNSUPPORTED, "more than 2^28 pairs lie within the T-th projected distance");
    if (n_raw < std::min<int64_t>(T, 1)) fail(PMLSH_EDEVICE, "pair scan found no pairs");
    cand.alloc(n_raw);
    if (scan(n_tiles, d2, limit_of(d2), n_raw) != n_raw)
        fail(PMLSH_EDEVICE, "pair scan counts disagree");
    // the T smallest (pd^2, i, j)
    const int64_t keep = std::min(T, n_raw);
    const Triplets* cands = &cand;
    if (n_raw > keep) {
        SelKey K = select_kth(x, cand.k0.as<uint32_t>(), cand.ii.as<uint32_t>(),
                              cand.jj.as<uint32_t>(), n_raw, keep, false, dhist.as<uint32_t>(), st);
        kept.alloc(keep);
        reset_counter();
        hipLaunchKernelGGL(acp_gather_kernel, dim3(grid_for(n_raw, WG)), dim3(WG), 0, st,
                           cand.k0.as<uint32_t>(), cand.ii.as<uint32_t>(), cand.jj.as<uint32_t>(),
                           n_raw, K, kept.k0.as<uint32_t>(), kept.ii.as<uint32_t>(),
                           kept.jj.as<uint32_t>(), keep,
                           static_cast<unsigned long long*>(dcount.p));
        PMLSH_HIP(hipGetLastError());
        if (read_counter() != keep) fail(PMLSH_EDEVICE, "budget cut lost candidates");
        cands = &kept;
    }
    // verify, then the k nearest
    pool.alloc(keep);
    hipLaunchKernelGGL(acp_verify_kernel, dim3(grid_for(keep, WG / 16)), dim3(WG), 0, st, x->data,
                       x->d_pad, x->inv_perm, cands->ii.as<uint32_t>(), cands->jj.as<uint32_t>(),
                       keep, pool.k0.as<uint32_t>(), pool.ii.as<uint32_t>(),
                       pool.jj.as<uint32_t>(), nullptr);
    PMLSH_HIP(hipGetLastError());
    if (keep < k) fail(PMLSH_EDEVICE, "fewer verified pairs than k");
    pool_topk(x, pool, keep, k, pool_gamma(x, false), top, dhist, dcount, out_pairs, out_dist, st);
    if (stats) {
        stats->t = plan.t;
        stats->ub = std::sqrt((double)d2);
        stats->budget = T;
        stats->n_seed = 0;
        stats->n_cand_raw = n_raw;
        stats->n_cand = keep;
        stats->tiles_total = tiles_all;
        stats->tiles_scanned = n_tiles;
    }
}

// Host copy of the node structure of the index: level of every node, the
// range [lf, le) of leaves its subtree covers, its parent and its radius.
struct NodeInfo {
    std::vector<int32_t> level, lf, le, parent;
    std::vector<float> rad;
};

NodeInfo fetch_nodes(const pmlsh_index* x) {
    const int64_t N = x->n_nodes;
    NodeInfo I;
    I.level.assign(N, 0);
    I.lf.assign(N, 0);
    I.le.assign(N, 0);
    I.parent.assign(N, -1);
    I.rad.assign(N, 0.f);
    std::vector<int32_t> cb(N), ce(N);
    PMLSH_HIP(hipMemcpy(cb.data(), x->tree.child_begin, N * 4, hipMemcpyDeviceToHost));
    PMLSH_HIP(hipMemcpy(ce.data(), x->tree.child_end, N * 4, hipMemcpyDeviceToHost));
    PMLSH_HIP(hipMemcpy(I.rad.data(), x->tree.radius, N * 4, hipMemcpyDeviceToHost));
    const int levels = x->levels;
    const int64_t leaf_base = x->level_begin[levels - 1];
    for (int l = levels - 1; l >= 0; --l) {
        for (int64_t i = x->level_begin[l]; i < x->level_begin[l + 1]; ++i) {
            I.level[i] = l;
            if (l == levels - 1) {
                I.lf[i] = (int32_t)(i - leaf_base);
                I.le[i] = I.lf[i] + 1;
            } else {
                I.lf[i] = I.lf[cb[i]];
                I.le[i] = I.le[ce[i] - 1];
                for (int32_t ch = cb[i]; ch < ce[i]; ++ch) I.parent[ch] = (int32_t)i;
            }
        }
    }
    return I;
}

// gamma of Section 6.3 with Pr(gamma) = prob: over pairs of points drawn at
// random (SplitMix64 from a fixed seed), the prob-quantile of the ratio of
// the radius of the pair's lowest common ancestor to its projected distance.
double estimate_gamma(const pmlsh_index* x, const NodeInfo& I, double prob) {
    const int64_t n = x->n;
    const int64_t L = x->leaf_size;
    const int64_t leaf_base = x->level_begin[x->levels - 1];
    std::vector<float> hi((size_t)n * MP), lo((size_t)n * MP);
    PMLSH_HIP(hipMemcpy(hi.data(), x->proj_hi, hi.size() * 4, hipMemcpyDeviceToHost));
    PMLSH_HIP(hipMemcpy(lo.data(), x->proj_lo, lo.size() * 4, hipMemcpyDeviceToHost));
    std::vector<int64_t> pos_of(n);
    for (int64_t p = 0; p < n; ++p) pos_of[x->perm_host[p]] = p;
    // radius of a ball around the top-level nodes' mean centre covering them
    // all (the tree's top level may hold several nodes)
    double r_top = 0;
    {
        const int64_t N = x->n_nodes, t0 = x->level_begin[0], t1 = x->level_begin[1];
        std::vector<float> cen((size_t)MP * N);
        PMLSH_HIP(hipMemcpy(cen.data(), x->tree.centre, cen.size() * 4, hipMemcpyDeviceToHost));
        double mean[MP] = {0};
        for (int64_t i = t0; i < t1; ++i)
            for (int t = 0; t < MP; ++t) mean[t] += cen[(size_t)t * N + i] / (double)(t1 - t0);
        for (int64_t i = t0; i < t1; ++i) {
            double acc = 0;
            for (int t = 0; t < MP; ++t) {
                const double dt = cen[(size_t)t * N + i] - mean[t];
                acc += dt * dt;
            }
            r_top = std::max(r_top, std::sqrt(acc) + (double)I.rad[i]);
        }
    }
    const double pairs = (double)n * (double)(n - 1) / 2.0;
    const int64_t S = (int64_t)std::min(100000.0, pairs);
    const uint64_t seed = 0x6761u;   // fixed: "ga"
    std::vector<double> ratio;
    ratio.reserve(S);
    for (int64_t j = 0; j < S; ++j) {
        const int64_t i = (int64_t)(splitmix64(seed + (uint64_t)j) % (uint64_t)n);
        const int64_t o = 1 + (int64_t)(splitmix64(seed + (uint64_t)S + (uint64_t)j) %
                                         (uint64_t)(n - 1));
        const int64_t pa = pos_of[i], pb = pos_of[(i + o) % n];
        int64_t node = leaf_base + pa / L;
        const int64_t b = pb / L;
        // up to the lowest common ancestor; pairs under different top-level
        // nodes have the covering ball of the whole tree as theirs
        while (node >= 0 && !(I.lf[node] <= b && b < I.le[node])) node = I.parent[node];
        const double r_lca = node >= 0 ? (double)I.rad[node] : r_top;
        double acc = 0;
        for (int t = 0; t < MP; ++t) {
            const double dt = ((double)hi[pa * MP + t] + (double)lo[pa * MP + t]) -
                              ((double)hi[pb * MP + t] + (double)lo[pb * MP + t]);
            acc += dt * dt;
        }
        if (acc > 0) ratio.push_back(r_lca / std::sqrt(acc));
    }
    if (ratio.empty()) return 1.0;
    std::sort(ratio.begin(), ratio.end());
    const size_t at = (size_t)std::max(1.0, std::ceil(prob * (double)ratio.size())) - 1;
    return ratio[std::min(at, ratio.size() - 1)];
}

// (c,k)-ACP by radius filtering with FindLCA (Algorithm 4 with Algorithm 5):
//   1. self-join of every leaf, all seed pairs verified; ub = the k-th
//      smallest exact distance; count = number of verified pairs;
//   2. R = gamma t ub; FindLCA: walking down from the root, the inner nodes
//      with radius below R (a found node's subtree is not searched further);
//   3. the found nodes in ascending order of radius (ties by node); in each,
//      every pair of points in different leaves of the subtree whose
//      projected distance is below t ub is verified, then ub becomes the
//      k-th smallest verified distance and count grows by those pairs;
//      after a node that leaves count > T the scan stops;
//   4. the k verified pairs with the smallest (distance, i, j).
// Reading: ub and count are updated after each node (the paper updates them
// after every verified pair, within the node's own order).
void run_acp_lca(const pmlsh_index* x, int k, double c, double confidence, double beta,
                 double gamma, int64_t* out_pairs, float* out_dist, pmlsh_acp_stats* stats,
                 double* gamma_used, hipStream_t st) {
    pmlsh_plan plan;
    plan_params(x->n, x->m, k, c, confidence, beta, &plan);
    const int64_t n = x->n;
    const int L = x->leaf_size;
    const int64_t NL = x->n_leaves;
    const int64_t T = plan.acp_budget;
    constexpr int64_t kMaxCand = int64_t(1) << 28;

    std::lock_guard<std::mutex> lock(x->acp_mu);
    if ((int)x->acp_bufs.size() < S_COUNT_ALL) x->acp_bufs.resize(S_COUNT_ALL, {nullptr, 0});
    DevBuf dhist(x, S_HIST), dcount(x, S_COUNT), tiles(x, S_TILES), ghist(x, S_GHIST);
    Triplets seeds(x, S_SEEDS), cand(x, S_CAND), pool(x, S_POOL), kept(x, S_KEPT),
        top(x, S_TOP);
    dhist.alloc(NB * sizeof(uint32_t));
    dcount.alloc(sizeof(unsigned long long));
    ghist.alloc(NB * sizeof(uint32_t));
    auto reset_counter = [&] {
        PMLSH_HIP(hipMemsetAsync(dcount.p, 0, sizeof(unsigned long long), st));
    };
    auto read_counter = [&]() -> int64_t {
        unsigned long long v = 0;
        {
            HostReads rd(x, st);
            rd.add(&v, dcount.p, sizeof(v));
            rd.wait();
        }
        return (int64_t)v;
    };

    // 1. seeds
    std::vector<int64_t> seed_off(NL + 1, 0);
    for (int64_t b = 0; b < NL; ++b) {
        const int64_t cnt = std::min<int64_t>(L, n - b * L);
        seed_off[b + 1] = seed_off[b] + cnt * (cnt - 1) / 2;
    }
    const int64_t n_seed = seed_off[NL];
    // the pool of verified pairs: seeds first, candidates appended
    int64_t pool_cap = std::max<int64_t>(n_seed + (int64_t(1) << 20), k);
    pool.alloc(pool_cap);
    if (n_seed > 0) {
        DevBuf doff(x, S_DOFF);
        doff.alloc((NL + 1) * sizeof(int64_t));
        PMLSH_HIP(hipMemcpyAsync(doff.p, seed_off.data(), (NL + 1) * sizeof(int64_t),
                                 hipMemcpyHostToDevice, st));
        PMLSH_HIP(hipMemsetAsync(ghist.p, 0, NB * sizeof(uint32_t), st));
        launch_self_join(x, doff.as<int64_t>(), pool.k0.as<uint32_t>(), pool.ii.as<uint32_t>(),
                         pool.jj.as<uint32_t>(), ghist.as<uint32_t>(), st);
        PMLSH_HIP(hipStreamSynchronize(st));
    }
    int64_t n_pool = n_seed;
    auto kth_dist = [&]() -> double {
        if (n_pool < k) return HUGE_VAL;
        SelKey K = select_kth(x, pool.k0.as<uint32_t>(), pool.ii.as<uint32_t>(),
                              pool.jj.as<uint32_t>(), n_pool, k, true, dhist.as<uint32_t>(), st);
        float v2;
        std::memcpy(&v2, &K.v0, 4);
        return std::sqrt((double)v2);
    };
    double ub = kth_dist();
    int64_t count = n_seed;

    // 2. FindLCA with R = gamma t ub
    NodeInfo I = fetch_nodes(x);
    if (!(gamma > 0.0)) {
        // the estimate depends on the index alone (a fixed sample of pairs)
        if (!(x->acp_gamma085 > 0.0)) x->acp_gamma085 = estimate_gamma(x, I, 0.85);
        gamma = x->acp_gamma085;
    }
    if (gamma_used) *gamma_used = gamma;
    const double Rlca = gamma * plan.t * ub;
    std::vector<int64_t> found;
    {
        std::vector<int64_t> stack;
        for (int64_t i = x->level_begin[0]; i < x->level_begin[1]; ++i) stack.push_back(i);
        while (!stack.empty()) {
            const int64_t e = stack.back();
            stack.pop_back();
            if (I.level[e] == x->levels - 1) continue;            // leaves: self-joined
            if ((double)I.rad[e] < Rlca) {
                found.push_back(e);
            } else {
                for (int64_t ch = x->level_begin[I.level[e] + 1]; ch < x->level_begin[I.level[e] + 2];
                     ++ch)
                    if (I.parent[ch] == e) stack.push_back(ch);
            }
        }
    }
    std::sort(found.begin(), found.end(), [&](int64_t a, int64_t b) {
        return I.rad[a] != I.rad[b] ? I.rad[a] < I.rad[b] : a < b;
    });

    // 3. the found nodes, ascending radius
    TileScan tscan(x, st);
    tscan.prepare();
    int64_t tiles_total = 0, tiles_scanned = 0, n_cand_total = 0;
    for (int64_t e : found) tiles_total += (int64_t)(I.le[e] - I.lf[e]) * (I.le[e] - I.lf[e] - 1) / 2;
    std::vector<int2> tl;
    int64_t cand_cap = 0;
    for (int64_t e : found) {
        if (count > T) break;
        tl.clear();
        for (int32_t a = I.lf[e]; a < I.le[e]; ++a)
            for (int32_t b = a + 1; b < I.le[e]; ++b) tl.push_back(make_int2(a, b));
        if (tl.empty()) continue;
        tiles.alloc(tl.size() * sizeof(int2));
        PMLSH_HIP(hipMemcpyAsync(tiles.p, tl.data(), tl.size() * sizeof(int2),
                                 hipMemcpyHostToDevice, st));
        tiles_scanned += (int64_t)tl.size();
        const double R = plan.t * ub;
        const float R2 = std::isinf(R) ? INFINITY : (float)(R * R);
        const float limit = std::isinf(R)
                                ? INFINITY
                                : (float)R + (float)(1e-5 * (2.0 * x->coord_scale + R));
        int64_t nc = 0;
        for (int attempt = 0; attempt < 2; ++attempt) {
            if (cand_cap < 1) {
                cand_cap = int64_t(1) << 16;
                cand.alloc(cand_cap);
            }
            reset_counter();
            tscan.scan(tiles.as<int2>(), (int64_t)tl.size(), R2, limit, cand.k0.as<uint32_t>(),
                       cand.ii.as<uint32_t>(), cand.jj.as<uint32_t>(), cand_cap,
                       static_cast<unsigned long long*>(dcount.p));
            nc = read_counter();
            if (nc <= cand_cap) break;
            if (nc > kMaxCand)
                fail(PMLSH_EUNSUPPORTED, "more than 2^28 candidate pairs in one node");
            cand_cap = nc;
            cand.alloc(cand_cap);
        }
        if (nc == 0) continue;
        if (n_pool + nc > pool_cap) {
            // grow the pool, keeping what it holds
            const int64_t new_cap = std::max(2 * pool_cap, n_pool + nc);
            kept.alloc(n_pool);
            for (int f = 0; f < 3; ++f) {
                void* src = f == 0 ? pool.k0.p : f == 1 ? pool.ii.p : pool.jj.p;
                void* dst = f == 0 ? kept.k0.p : f == 1 ? kept.ii.p : kept.jj.p;
                PMLSH_HIP(hipMemcpyAsync(dst, src, n_pool * 4, hipMemcpyDeviceToDevice, st));
            }
            PMLSH_HIP(hipStreamSynchronize(st));
            pool.alloc(new_cap);
            for (int f = 0; f < 3; ++f) {
                void* src = f == 0 ? kept.k0.p : f == 1 ? kept.ii.p : kept.jj.p;
                void* dst = f == 0 ? pool.k0.p : f == 1 ? pool.ii.p : pool.jj.p;
                PMLSH_HIP(hipMemcpyAsync(dst, src, n_pool * 4, hipMemcpyDeviceToDevice, st));
            }
            pool_cap = new_cap;
        }
        hipLaunchKernelGGL(acp_verify_kernel, dim3(grid_for(nc, WG / 16)), dim3(WG), 0, st,
                           x->data, x->d_pad, x->inv_perm, cand.ii.as<uint32_t>(),
                           cand.jj.as<uint32_t>(), nc, pool.k0.as<uint32_t>() + n_pool,
                           pool.ii.as<uint32_t>() + n_pool, pool.jj.as<uint32_t>() + n_pool, nullptr);
        PMLSH_HIP(hipGetLastError());
        n_pool += nc;
        count += nc;
        n_cand_total += nc;
        ub = kth_dist();
    }

    // 4. the k nearest verified pairs
    if (n_pool < k) fail(PMLSH_EDEVICE, "fewer verified pairs than k");
    pool_topk(x, pool, n_pool, k, pool_gamma(x, true), top, dhist, dcount, out_pairs, out_dist,
              st);
    if (stats) {
        stats->t = plan.t;
        stats->ub = ub;
        stats->budget = T;
        stats->n_seed = n_seed;
        stats->n_cand_raw = n_cand_total;
        stats->n_cand = n_cand_total;
        stats->tiles_total = tiles_total;
        stats->tiles_scanned = tiles_scanned;
    }
}

void export_nodes(const pmlsh_index* x, int32_t* level, int32_t* first_leaf, int32_t* end_leaf,
                  float* radius) {
    NodeInfo I = fetch_nodes(x);
    std::copy(I.level.begin(), I.level.end(), level);
    std::copy(I.lf.begin(), I.lf.end(), first_leaf);
    std::copy(I.le.begin(), I.le.end(), end_leaf);
    std::copy(I.rad.begin(), I.rad.end(), radius);
}

}  // namespace pmlsh
