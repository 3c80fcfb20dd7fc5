// (c,k)-ANN query kernel (gfx950): Algorithm 2 of PM-LSH, one workgroup per
// query, all rounds on the device.
//
// Per round i (radius r_i = r_min * c^i):
//   1. from the second round on, count the verified candidates within c*r_i
//      of q and stop when there are at least k (Algorithm 2, line 4);
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

#include <cfloat>
#include <cstdint>

#include "internal.hpp"

namespace pmlsh {
namespace {

constexpr int WG = 256;
constexpr int NWAVE = WG / 64;
constexpr int NB = 2048;    // histogram bins of one radix-select step
constexpr int CAP = 2048;   // keys sorted in LDS at once (power of two)
constexpr int MAX_LEVELS = 16;
constexpr int MAX_ROUNDS = 1000;

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
    const float* piv;
    int64_t n_nodes;
    int64_t n_leaves;
    int levels;
    int s;
    int d, d_pad;
    int32_t level_begin[MAX_LEVELS + 1];
    float coord_scale;
    const float* q;
    const float* qp;
    int k;
    int32_t budget;
    double c, t, r_min;
    int32_t* ws_front;
    int32_t* ws_cpos;
    float* ws_cdist;
    int32_t* ws_topk;
    int64_t* out_ids;
    float* out_dist;
    int32_t* out_stats;
};

struct Smem {
    uint32_t hist[NB];
    uint64_t skey[CAP];
    int32_t spos[CAP];
    int32_t red[NWAVE * 2];
    int32_t cnt0, cnt1, cnt2;
    int32_t thr_bin, thr_below, thr_in;
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

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
__device__ __forceinline__ bool node_pass(const AnnArgs& a, int node, const float* qp,
                                          const float* qpiv, float R, float slack) {
    if (node_dist(a, node, qp) > a.nrad[node] + R + slack) return false;
    for (int i = 0; i < a.s; ++i) {
        const int64_t o = (int64_t)i * a.n_nodes + node;
        if (qpiv[i] - R > a.hrmax[o] + slack) return false;
        if (qpiv[i] + R < a.hrmin[o] - slack) return false;
    }
    return true;
}

// Level-by-level traversal; returns the number of leaves passing Eq. 5, whose
// ids are left in *out (one of the two per-query frontier buffers).
__device__ int traverse(const AnnArgs& a, const float* qp, const float* qpiv, float R,
                        float slack, int32_t* fa, int32_t* fb, int32_t** out, Smem& sh) {
    int32_t* cur = fa;
    int32_t* nxt = fb;
    int ncur = a.level_begin[1] - a.level_begin[0];
    for (int l = 0; l < a.levels; ++l) {
        const bool leaf_level = (l == a.levels - 1);
        if (threadIdx.x == 0) sh.cnt0 = 0;
        __syncthreads();
        for (int base = 0; base < ncur; base += WG) {
            const int i = base + threadIdx.x;
            bool pass = false;
            int node = 0;
            if (i < ncur) {
                node = (l == 0) ? a.level_begin[0] + i : cur[i];
                // entries always lie in this level; the check only keeps a
                // corrupted list from reading outside the node arrays
                if (node >= a.level_begin[l] && node < a.level_begin[l + 1])
                    pass = node_pass(a, node, qp, qpiv, R, slack);
            }
            if (leaf_level) {
                const int slot = wave_append(pass, &sh.cnt0);
                if (pass && slot < a.n_leaves) nxt[slot] = node;
            } else if (pass) {
                const int b = a.cb[node], e = a.ce[node];
                const int slot = atomicAdd(&sh.cnt0, e - b);
                if (slot + (e - b) <= a.n_leaves)
                    for (int j = b; j < e; ++j) nxt[slot + (j - b)] = j;
            }
        }
        __syncthreads();
        ncur = sh.cnt0 < a.n_leaves ? sh.cnt0 : (int)a.n_leaves;
        __syncthreads();
        int32_t* t = cur; cur = nxt; nxt = t;
    }
    *out = cur;
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

// Exact squared distances of C entries [v0, v1): 16 lanes per row.
__device__ void verify(const AnnArgs& a, const float* qs, const int32_t* cpos, float* cdist,
                       int v0, int v1) {
    const int g = threadIdx.x >> 4, l16 = threadIdx.x & 15;
    const int d4 = a.d_pad >> 2;
    const float4* q4 = reinterpret_cast<const float4*>(qs);
    for (int base = v0; base < v1; base += WG / 16) {
        const int i = base + g;
        float acc = 0.f;
        if (i < v1) {
            const float4* row = reinterpret_cast<const float4*>(a.data + (int64_t)cpos[i] * a.d_pad);
            for (int c = l16; c < d4; c += 16) {
                const float4 x = row[c], y = q4[c];
                float t;
                t = y.x - x.x; acc = __fmaf_rn(t, t, acc);
                t = y.y - x.y; acc = __fmaf_rn(t, t, acc);
                t = y.z - x.z; acc = __fmaf_rn(t, t, acc);
                t = y.w - x.w; acc = __fmaf_rn(t, t, acc);
            }
        }
        acc += __shfl_xor(acc, 8, 16);
        acc += __shfl_xor(acc, 4, 16);
        acc += __shfl_xor(acc, 2, 16);
        acc += __shfl_xor(acc, 1, 16);
        if (i < v1 && l16 == 0) cdist[i] = acc;
    }
}

__global__ __launch_bounds__(WG) void ann_kernel(AnnArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Smem& sh = *reinterpret_cast<Smem*>(smem_raw);
    float* qs = reinterpret_cast<float*>(smem_raw + ((sizeof(Smem) + 15) & ~size_t(15)));

    const int64_t qi = blockIdx.x;
    const float* qrow = a.q + qi * a.d;
    for (int c = threadIdx.x; c < a.d_pad; c += WG) qs[c] = c < a.d ? qrow[c] : 0.f;

    float qp[MP];
#pragma unroll
    for (int j = 0; j < MP; ++j) qp[j] = a.qp[qi * MP + j];
    float qpiv[PMLSH_MAX_PIVOTS];
    float qn2 = 0.f;
#pragma unroll
    for (int j = 0; j < MP; ++j) qn2 = fmaf(qp[j], qp[j], qn2);
    for (int i = 0; i < a.s; ++i) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < MP; ++j) {
            const float t = qp[j] - a.piv[i * MP + j];
            acc = fmaf(t, t, acc);
        }
        qpiv[i] = sqrtf(acc);
    }
    __syncthreads();

    int32_t* fa = a.ws_front + qi * 2 * a.n_leaves;
    int32_t* fb = fa + a.n_leaves;
    int32_t* cpos = a.ws_cpos + qi * (int64_t)a.budget;
    float* cdist = a.ws_cdist + qi * (int64_t)a.budget;
    const int32_t* perm = a.perm;
    const int B = a.budget;

    double r = a.r_min;
    int n_ver = 0;
    int rounds = 0;
    int exit_kind = 0;
    int64_t scanned = 0;
    uint32_t prev_hi = 0;     // bits of the previous squared radius
    bool first = true;

    for (;;) {
        if (rounds > 0) {
            const double cr = a.c * r;
            const float thr2 = (float)(cr * cr);
            int loc = 0;
            for (int i = threadIdx.x; i < n_ver; i += WG) loc += cdist[i] <= thr2;
            if (block_sum(loc, sh) >= a.k) { exit_kind = PMLSH_EXIT_LINE4; break; }
        }
        if (rounds >= MAX_ROUNDS) r = __longlong_as_double(0x7ff0000000000000ll);
        const double Rd = a.t * r;
        const float R = (float)Rd;
        const float R2 = (float)(Rd * Rd);
        ++rounds;
        const float slack = 1e-5f * (sqrtf(qn2) + a.coord_scale + R);

        int32_t* leaves = nullptr;
        const int nl = traverse(a, qp, qpiv, R, slack, fa, fb, &leaves, sh);

        // shell (prev, R2] on the 64-bit keys (pd^2 bits << 32 | id)
        const uint32_t lo_hi = first ? 0u : prev_hi + 1u;
        const uint32_t hi_hi = __float_as_uint(R2);
        const uint64_t klo = (uint64_t)lo_hi << 32;
        const uint64_t khi = ((uint64_t)hi_hi << 32) | 0xffffffffull;
        const int sh0 = shift_for(klo, khi);
        auto ball_src = [&](auto&& v) {
            scan_leaves(a, leaves, nl, qp, [&](bool valid, int pos, float pd2) {
                const uint32_t b = __float_as_uint(pd2);
                const bool mem = valid && b >= lo_hi && b <= hi_hi;
                const uint64_t key = mem ? (((uint64_t)b << 32) | (uint32_t)perm[pos]) : 0ull;
                v(mem, key, pos);
            });
        };

        clear_hist(sh);
        int loc = 0, sc = 0;
        ball_src([&](bool mem, uint64_t key, int32_t) {
            if (mem) { ++loc; atomicAdd(&sh.hist[(key - klo) >> sh0], 1u); }
        });
        for (int li = threadIdx.x; li < nl; li += WG) sc += a.ce[leaves[li]] - a.cb[leaves[li]];
        scanned += block_sum(sc, sh);
        const int shell = block_sum(loc, sh);

        if (n_ver + shell >= B) {
            const int need = B - n_ver;
            block_select(ball_src,
                         [&](int32_t pos, int slot) {
                             if (slot < need) cpos[n_ver + slot] = pos;
                         },
                         klo, khi, need, true, shell, sh);
            __syncthreads();
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
        r = a.c * r;
    }

    // top-k of C by (distance^2 bits, id)
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
    const int k = a.k;
    if (n_ver <= CAP) {
        if (threadIdx.x == 0) sh.cnt1 = 0;
        __syncthreads();
        c_src([&](bool valid, uint64_t key, int32_t i) {
            const int slot = wave_append(valid, &sh.cnt1);
            if (valid && slot < CAP) { sh.skey[slot] = key; sh.spos[slot] = i; }
        });
        __syncthreads();
        bitonic_sort(n_ver, sh);
    } else {
        block_select(c_src, [&](int32_t i, int slot) { if (slot < k) topk[slot] = i; }, 0ull,
                     ~0ull, k, false, 0, sh);
        __syncthreads();
        for (int j = threadIdx.x; j < k; j += WG) {
            const int i = topk[j];
            sh.skey[j] = ((uint64_t)__float_as_uint(cdist[i]) << 32) | (uint32_t)perm[cpos[i]];
            sh.spos[j] = i;
        }
        __syncthreads();
        bitonic_sort(k, sh);
    }
    for (int j = threadIdx.x; j < k; j += WG) {
        const int i = sh.spos[j];
        a.out_ids[qi * k + j] = (int64_t)perm[cpos[i]];
        a.out_dist[qi * k + j] = sqrtf(cdist[i]);
    }
    if (a.out_stats && threadIdx.x == 0) {
        int32_t* st = a.out_stats + qi * 4;
        st[0] = rounds;
        st[1] = n_ver;
        st[2] = exit_kind;
        st[3] = scanned > 0x7fffffffll ? 0x7fffffff : (int32_t)scanned;
    }
}

}  // namespace

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
    a.piv = x.tree.pivots;
    a.n_nodes = x.n_nodes;
    a.n_leaves = x.n_leaves;
    a.levels = x.levels;
    a.s = x.num_pivots;
    a.d = x.d;
    a.d_pad = x.d_pad;
    for (int l = 0; l <= x.levels; ++l) a.level_begin[l] = (int32_t)x.level_begin[l];
    a.coord_scale = x.coord_scale;
    a.q = L.queries;
    a.qp = L.qproj;
    a.k = L.k;
    a.budget = (int32_t)L.budget;
    a.c = L.c;
    a.t = L.t;
    a.r_min = L.r_min;
    a.ws_front = L.ws_front;
    a.ws_cpos = L.ws_cpos;
    a.ws_cdist = L.ws_cdist;
    a.ws_topk = L.ws_topk;
    a.out_ids = L.out_ids;
    a.out_dist = L.out_dist;
    a.out_stats = L.out_stats;
    const int lds = ann_lds_bytes(x.d_pad);
    PMLSH_HIP(hipFuncSetAttribute((const void*)ann_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    hipLaunchKernelGGL(ann_kernel, dim3((unsigned)L.nq), dim3(WG), lds, stream, a);
    PMLSH_HIP(hipGetLastError());
}

}  // namespace pmlsh
