// Device bulk-load of the leaf order of the PM-tree (Section 4.1): the
// recursive gap-aware splits of the whole point set, computed level by level
// on the GPU. Every node with more than leaf_size points is cut along its
// principal direction (power iteration on the 16 x 16 covariance of its
// projected points, started from the coordinate axis of largest variance)
// at a whole-leaf boundary within the middle 60 % of its leaves, where the
// sorted projections onto that direction show the widest gap, so cuts fall
// between clusters rather than through them.
//
// Per level, for all nodes being cut at once: FP64 coordinate sums and
// centred second moments over pieces of at most kPiece points (one
// workgroup per piece, reduced per node in a fixed order, so a build is
// deterministic), one wave per node for the power iteration, FP64 keys
// (direction . point), a segmented radix sort of the nodes' points by key
// (stable, so equal keys keep their order), and one wave per node for the
// cut. The host only keeps the list of nodes and their children.

#include <hipcub/hipcub.hpp>

#include "internal.hpp"

namespace pmlsh {
namespace {

constexpr int kPiece = 8192;     // points per moment workgroup
constexpr int kCov = MP * (MP + 1) / 2;   // upper triangle of the covariance

struct Piece {
    int32_t seg;                 // node (index into the level's list)
    int32_t b, e;                // positions [b, e) of the leaf order
};

// Coordinate sums of every piece (four waves, shuffle then LDS, fixed order);
// positions are ids when perm is null.
__global__ __launch_bounds__(256) void bl_sum_kernel(const float* __restrict__ proj,
                                                      const int32_t* perm,
                                                      const Piece* __restrict__ pieces,
                                                      double* __restrict__ part) {
    const Piece pc = pieces[blockIdx.x];
    double acc[MP];
#pragma unroll
    for (int j = 0; j < MP; ++j) acc[j] = 0.0;
    for (int i = pc.b + (int)threadIdx.x; i < pc.e; i += 256) {
        const int64_t row = perm ? (int64_t)perm[i] : (int64_t)i;
        const float4* p = reinterpret_cast<const float4*>(proj + row * MP);
#pragma unroll
        for (int q = 0; q < MP / 4; ++q) {
            const float4 v = p[q];
            acc[4 * q] += v.x;
            acc[4 * q + 1] += v.y;
            acc[4 * q + 2] += v.z;
            acc[4 * q + 3] += v.w;
        }
    }
    __shared__ double red[4][MP];
#pragma unroll
    for (int j = 0; j < MP; ++j) {
        double v = acc[j];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        acc[j] = v;
    }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int j = 0; j < MP; ++j) red[threadIdx.x >> 6][j] = acc[j];
    __syncthreads();
    if (threadIdx.x < MP) {
        const int j = threadIdx.x;
        part[(int64_t)blockIdx.x * MP + j] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
    }
}

// Centred second moments (upper triangle) of every piece about its node's
// mean: 64 points at a time through LDS, one thread per matrix entry.
__global__ __launch_bounds__(256) void bl_cov_kernel(const float* __restrict__ proj,
                                                      const int32_t* __restrict__ perm,
                                                      const Piece* __restrict__ pieces,
                                                      const double* __restrict__ mean,
                                                      double* __restrict__ part) {
    const Piece pc = pieces[blockIdx.x];
    __shared__ double tile[64][MP + 1];
    __shared__ double mu[MP];
    if (threadIdx.x < MP) mu[threadIdx.x] = mean[(int64_t)pc.seg * MP + threadIdx.x];
    // entry t of the upper triangle: row j, column k >= j
    int ej = 0, ek = 0;
    if (threadIdx.x < kCov) {
        int t = threadIdx.x, j = 0;
        while (t >= MP - j) { t -= MP - j; ++j; }
        ej = j;
        ek = j + t;
    }
    double acc = 0.0;
    __syncthreads();
    for (int base = pc.b; base < pc.e; base += 64) {
        const int cnt = min(64, pc.e - base);
        {
            const int q = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 4;
            if (q < cnt) {
                const float4 v = *reinterpret_cast<const float4*>(
                    proj + (int64_t)perm[base + q] * MP + c0);
                tile[q][c0] = (double)v.x - mu[c0];
                tile[q][c0 + 1] = (double)v.y - mu[c0 + 1];
                tile[q][c0 + 2] = (double)v.z - mu[c0 + 2];
                tile[q][c0 + 3] = (double)v.w - mu[c0 + 3];
            }
        }
        __syncthreads();
        if (threadIdx.x < kCov)
            for (int q = 0; q < cnt; ++q) acc = fma(tile[q][ej], tile[q][ek], acc);
        __syncthreads();
    }
    if (threadIdx.x < kCov) part[(int64_t)blockIdx.x * kCov + threadIdx.x] = acc;
}

// Per node and entry, the sum of its pieces' partial values in piece order,
// divided by `div[node]` when div is given.
__global__ void bl_reduce_kernel(const double* __restrict__ part, int width,
                                 const int32_t* __restrict__ piece_begin, int m,
                                 const int32_t* __restrict__ div, double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * width) return;
    const int s = (int)(t / width), w = (int)(t % width);
    double v = 0.0;
    for (int p = piece_begin[s]; p < piece_begin[s + 1]; ++p) v += part[(int64_t)p * width + w];
    out[t] = div ? v / (double)div[s] : v;
}

// Principal direction of every node: 30 steps of the power iteration on its
// covariance (lane l < 16 holds row l), started from the axis of largest
// variance (the first one on ties); kept where the product vanishes.
__global__ __launch_bounds__(256) void bl_direction_kernel(const double* __restrict__ cov, int m,
                                                            double* __restrict__ dir_out) {
    const int s = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= m) return;
    const double* c = cov + (int64_t)s * kCov;
    const int l = lane & (MP - 1);
    double row[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) {
        const int a = min(l, k), b = max(l, k);
        // index of (a, b) in the upper triangle
        row[k] = c[a * MP - a * (a - 1) / 2 + (b - a)];
    }
    int ax = 0;
    double best = c[0];
    for (int j = 1; j < MP; ++j) {
        const double v = c[j * MP - j * (j - 1) / 2];
        if (v > best) { best = v; ax = j; }
    }
    double dir[MP];
#pragma unroll
    for (int k = 0; k < MP; ++k) dir[k] = k == ax ? 1.0 : 0.0;
    for (int it = 0; it < 30; ++it) {
        double nd = 0.0;
#pragma unroll
        for (int k = 0; k < MP; ++k) nd += row[k] * dir[k];
        double n2 = nd * nd;
        // sum over the 16 lanes of the row block (each block of 16 lanes
        // holds the same rows), in a fixed order
        for (int off = 8; off > 0; off >>= 1) n2 += __shfl_xor(n2, off, 16);
        const double nrm = sqrt(n2);
        if (!(nrm > 0.0)) break;
        const double v = nd / nrm;
#pragma unroll
        for (int k = 0; k < MP; ++k) dir[k] = __shfl(v, k, 16);
    }
    if (lane < MP) dir_out[(int64_t)s * MP + lane] = dir[lane];
}

// FP64 key direction . point of every position of the pieces, and the
// sort's values (the ids at those positions).
__global__ __launch_bounds__(256) void bl_keys_kernel(const float* __restrict__ proj,
                                                       const int32_t* __restrict__ perm,
                                                       const Piece* __restrict__ pieces,
                                                       const double* __restrict__ dir,
                                                       double* __restrict__ key) {
    const Piece pc = pieces[blockIdx.x];
    __shared__ double dv[MP];
    if (threadIdx.x < MP) dv[threadIdx.x] = dir[(int64_t)pc.seg * MP + threadIdx.x];
    __syncthreads();
    for (int i = pc.b + (int)threadIdx.x; i < pc.e; i += 256) {
        const float* p = proj + (int64_t)perm[i] * MP;
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < MP; ++j) v += dv[j] * (double)p[j];
        key[i] = v;
    }
}

// The sorted ids back into the leaf order, positions of the pieces only.
__global__ __launch_bounds__(256) void bl_copy_kernel(const Piece* __restrict__ pieces,
                                                       const int32_t* __restrict__ src,
                                                       int32_t* __restrict__ perm) {
    const Piece pc = pieces[blockIdx.x];
    for (int i = pc.b + (int)threadIdx.x; i < pc.e; i += 256) perm[i] = src[i];
}

// The cut of every node (one wave each): after j whole leaves, j within the
// middle 60 % of its leaves, at the widest gap of the sorted keys (the
// smallest such j); the middle leaf when no cut position qualifies.
__global__ __launch_bounds__(256) void bl_cut_kernel(const int32_t* __restrict__ seg_b,
                                                      const int32_t* __restrict__ seg_e, int m,
                                                      int leaf, const double* __restrict__ key,
                                                      int32_t* __restrict__ mid) {
    const int s = (int)(((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= m) return;
    const int b = seg_b[s], cnt = seg_e[s] - b;
    const int nleaves = (cnt + leaf - 1) / leaf;
    int jlo = max(1, (nleaves * 2) / 10);
    int jhi = min(nleaves - 1, nleaves - (nleaves * 2) / 10);
    if (jhi < jlo) jlo = jhi = nleaves / 2;
    double gap = -1.0;
    int best = 0x7fffffff;
    for (int j = jlo + lane; j <= jhi; j += 64) {
        const int64_t p = (int64_t)j * leaf;
        if (p <= 0 || p >= cnt) continue;
        const double g = key[b + p] - key[b + p - 1];
        if (g > gap) { gap = g; best = j; }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double og = __shfl_xor(gap, off);
        const int ob = __shfl_xor(best, off);
        if (og > gap || (og == gap && ob < best)) { gap = og; best = ob; }
    }
    if (lane == 0) mid[s] = b + (gap < 0.0 ? nleaves / 2 : best) * leaf;
}

__device__ __forceinline__ double dist64(const float* p, const float* c) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
        const double t = (double)p[j] - (double)c[j];
        acc = fma(t, t, acc);
    }
    return sqrt(acc);
}

// Mean of every node (sums / count, from bl_reduce_kernel) rounded to FP32.
__global__ void bl_centre_kernel(const double* __restrict__ mean, int64_t count,
                                 float* __restrict__ cf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) cf[t] = (float)mean[t];
}

// Per piece: the largest FP64 distance of its points to their node's FP32
// centre, and for every pivot the smallest and largest distance to it
// (width 1 + 2 s per piece; min and max do not depend on the order).
__global__ __launch_bounds__(256) void bl_ring_kernel(const float* __restrict__ proj,
                                                       const int32_t* __restrict__ perm,
                                                       const Piece* __restrict__ pieces,
                                                       const float* __restrict__ cf,
                                                       const float* __restrict__ piv, int s,
                                                       double* __restrict__ part) {
    const Piece pc = pieces[blockIdx.x];
    __shared__ float c[MP];
    __shared__ float pv[PMLSH_MAX_PIVOTS][MP];
    __shared__ double red[4][1 + 2 * PMLSH_MAX_PIVOTS];
    if (threadIdx.x < MP) c[threadIdx.x] = cf[(int64_t)pc.seg * MP + threadIdx.x];
    if (threadIdx.x < s * MP) pv[threadIdx.x / MP][threadIdx.x % MP] = piv[threadIdx.x];
    __syncthreads();
    double rad = 0.0, lo[PMLSH_MAX_PIVOTS], hi[PMLSH_MAX_PIVOTS];
#pragma unroll
    for (int t = 0; t < PMLSH_MAX_PIVOTS; ++t) {
        lo[t] = __longlong_as_double(0x7ff0000000000000ll);
        hi[t] = 0.0;
    }
    for (int i = pc.b + (int)threadIdx.x; i < pc.e; i += 256) {
        float p[MP];
        const float4* src = reinterpret_cast<const float4*>(proj + (int64_t)perm[i] * MP);
#pragma unroll
        for (int q = 0; q < MP / 4; ++q) {
            const float4 v = src[q];
            p[4 * q] = v.x;
            p[4 * q + 1] = v.y;
            p[4 * q + 2] = v.z;
            p[4 * q + 3] = v.w;
        }
        rad = fmax(rad, dist64(p, c));
#pragma unroll
        for (int t = 0; t < PMLSH_MAX_PIVOTS; ++t) {
            if (t < s) {
                const double dd = dist64(p, pv[t]);
                lo[t] = fmin(lo[t], dd);
                hi[t] = fmax(hi[t], dd);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) rad = fmax(rad, __shfl_xor(rad, off));
#pragma unroll
    for (int t = 0; t < PMLSH_MAX_PIVOTS; ++t) {
        for (int off = 32; off > 0; off >>= 1) {
            lo[t] = fmin(lo[t], __shfl_xor(lo[t], off));
            hi[t] = fmax(hi[t], __shfl_xor(hi[t], off));
        }
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = rad;
        for (int t = 0; t < s; ++t) {
            red[w][1 + 2 * t] = lo[t];
            red[w][2 + 2 * t] = hi[t];
        }
    }
    __syncthreads();
    const int width = 1 + 2 * s;
    if (threadIdx.x < width) {
        const int e = threadIdx.x;
        const bool is_min = e >= 1 && (e & 1);
        double v = red[0][e];
        for (int k = 1; k < 4; ++k) v = is_min ? fmin(v, red[k][e]) : fmax(v, red[k][e]);
        part[(int64_t)blockIdx.x * width + e] = v;
    }
}

// Per node and entry, the max (entry 0 and the even ones) or min (odd ones)
// over its pieces.
__global__ void bl_reduce_ring_kernel(const double* __restrict__ part, int width,
                                      const int32_t* __restrict__ piece_begin, int m,
                                      double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * width) return;
    const int sg = (int)(t / width), e = (int)(t % width);
    const bool is_min = e >= 1 && (e & 1);
    double v = part[(int64_t)piece_begin[sg] * width + e];
    for (int p = piece_begin[sg] + 1; p < piece_begin[sg + 1]; ++p) {
        const double x = part[(int64_t)p * width + e];
        v = is_min ? fmin(v, x) : fmax(v, x);
    }
    out[t] = v;
}

// Farthest-point step over the ids [0, n): the distance of every point to
// ref (an FP32 row), folded into mind[i] = min(mind[i], distance) when mind
// is given; per workgroup the largest value and its smallest id.
__global__ __launch_bounds__(256) void bl_far_kernel(const float* __restrict__ proj, int64_t n,
                                                      const float* __restrict__ ref,
                                                      double* mind, double* __restrict__ bval,
                                                      int64_t* __restrict__ bidx) {
    __shared__ float r[MP];
    __shared__ double sv[4];
    __shared__ int64_t si[4];
    if (threadIdx.x < MP) r[threadIdx.x] = ref[threadIdx.x];
    __syncthreads();
    double best = -1.0;
    int64_t bi = 0x7fffffffffffffffll;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double v = dist64(proj + i * MP, r);
        if (mind) {
            v = fmin(mind[i], v);
            mind[i] = v;
        }
        if (v > best) { best = v; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off);
        const int64_t oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = best;
        si[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w)
            if (sv[w] > best || (sv[w] == best && si[w] < bi)) { best = sv[w]; bi = si[w]; }
        bval[blockIdx.x] = best;
        bidx[blockIdx.x] = bi;
    }
}

// The largest value over the workgroups of bl_far_kernel (smallest id on
// ties); its point is copied to dst (an FP32 row) and its value to *val.
__global__ __launch_bounds__(256) void bl_pick_kernel(const float* __restrict__ proj,
                                                       const double* __restrict__ bval,
                                                       const int64_t* __restrict__ bidx, int nb,
                                                       float* __restrict__ dst,
                                                       double* __restrict__ val) {
    __shared__ double sv[4];
    __shared__ int64_t si[4];
    __shared__ int64_t pick;
    double best = -1.0;
    int64_t bi = 0x7fffffffffffffffll;
    for (int b = threadIdx.x; b < nb; b += 256)
        if (bval[b] > best || (bval[b] == best && bidx[b] < bi)) { best = bval[b]; bi = bidx[b]; }
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off);
        const int64_t oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = best;
        si[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w)
            if (sv[w] > best || (sv[w] == best && si[w] < bi)) { best = sv[w]; bi = si[w]; }
        sv[0] = best;
        pick = bi;
    }
    __syncthreads();
    if (threadIdx.x < MP && dst) dst[threadIdx.x] = proj[pick * MP + threadIdx.x];
    if (threadIdx.x == 0 && val) *val = sv[0];
}

// Any non-finite value among count floats sets *flag (a plain store).
__global__ void bl_finite_kernel(const float* __restrict__ x, int64_t count,
                                 int32_t* __restrict__ flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) *flag = 1;
}

__global__ void bl_fill_kernel(double* __restrict__ x, int64_t count, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

template <class T>
struct DevVec {
    T* p = nullptr;
    size_t cap = 0;
    ~DevVec() { if (p) (void)hipFree(p); }
    T* get(size_t count) {
        if (count > cap) {
            if (p) PMLSH_HIP(hipFree(p));
            p = nullptr;
            cap = 0;
            PMLSH_HIP(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)));
            cap = std::max<size_t>(count, 1);
        }
        return p;
    }
};

}  // namespace

void device_split(const float* proj, int64_t n, int leaf, hipStream_t st,
                  std::vector<int32_t>* perm_out, std::vector<SplitNode>* nodes_out) {
    if (n <= 0 || n > 0x7fffffffLL - kPiece) fail(PMLSH_EUNSUPPORTED, "point count out of range");
    std::vector<SplitNode>& nodes = *nodes_out;
    nodes.clear();
    nodes.push_back({0, (n + leaf - 1) / leaf, -1, -1});
    std::vector<int32_t> cur;                          // nodes cut at this level
    std::vector<int32_t> nb{0}, ne{(int32_t)n};        // their point ranges
    if (n > leaf) cur.push_back(0);

    DevVec<int32_t> perm, perm_alt, d_idx;
    DevVec<double> key, key_alt, part, mean, cov, dir;
    DevVec<Piece> d_pieces;
    DevVec<unsigned char> temp;
    {
        std::vector<int32_t> iota((size_t)n);
        for (int64_t i = 0; i < n; ++i) iota[(size_t)i] = (int32_t)i;
        PMLSH_HIP(hipMemcpyAsync(perm.get((size_t)n), iota.data(), (size_t)n * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
        PMLSH_HIP(hipStreamSynchronize(st));
    }
    key.get((size_t)n);
    key_alt.get((size_t)n);
    perm_alt.get((size_t)n);

    std::vector<Piece> pieces;
    std::vector<int32_t> host_idx, mids;
    while (!cur.empty()) {
        const int m = (int)cur.size();
        // per node: begin, end, first piece (m + 1), point count
        pieces.clear();
        host_idx.assign((size_t)4 * m + 1, 0);
        int32_t* sb = host_idx.data();
        int32_t* se = sb + m;
        int32_t* pb = se + m;          // m + 1 entries
        int32_t* cnt = pb + m + 1;
        for (int s = 0; s < m; ++s) {
            const int32_t b = nb[(size_t)cur[(size_t)s]], e = ne[(size_t)cur[(size_t)s]];
            sb[s] = b;
            se[s] = e;
            cnt[s] = e - b;
            pb[s] = (int32_t)pieces.size();
            for (int32_t x = b; x < e; x += kPiece) pieces.push_back({s, x, std::min(e, x + kPiece)});
        }
        pb[m] = (int32_t)pieces.size();
        const int np = (int)pieces.size();
        int32_t* di = d_idx.get(host_idx.size());
        Piece* dp = d_pieces.get(pieces.size());
        PMLSH_HIP(hipMemcpyAsync(di, host_idx.data(), host_idx.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
        PMLSH_HIP(hipMemcpyAsync(dp, pieces.data(), pieces.size() * sizeof(Piece),
                                 hipMemcpyHostToDevice, st));
        const int32_t *dsb = di, *dse = di + m, *dpb = di + 2 * m, *dcnt = di + 3 * m + 1;

        // mean, covariance, direction
        double* dpart = part.get((size_t)np * kCov);
        double* dmean = mean.get((size_t)m * MP);
        double* dcov = cov.get((size_t)m * kCov);
        double* ddir = dir.get((size_t)m * MP);
        hipLaunchKernelGGL(bl_sum_kernel, dim3((unsigned)np), dim3(256), 0, st, proj, perm.p, dp,
                           dpart);
        hipLaunchKernelGGL(bl_reduce_kernel, dim3((unsigned)(((int64_t)m * MP + 255) / 256)),
                           dim3(256), 0, st, dpart, MP, dpb, m, dcnt, dmean);
        hipLaunchKernelGGL(bl_cov_kernel, dim3((unsigned)np), dim3(256), 0, st, proj, perm.p, dp,
                           dmean, dpart);
        hipLaunchKernelGGL(bl_reduce_kernel, dim3((unsigned)(((int64_t)m * kCov + 255) / 256)),
                           dim3(256), 0, st, dpart, kCov, dpb, m, nullptr, dcov);
        hipLaunchKernelGGL(bl_direction_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st,
                           dcov, m, ddir);
        hipLaunchKernelGGL(bl_keys_kernel, dim3((unsigned)np), dim3(256), 0, st, proj, perm.p, dp,
                           ddir, key.p);
        PMLSH_HIP(hipGetLastError());

        // stable sort of every node's points by key
        size_t tbytes = 0;
        PMLSH_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(
            nullptr, tbytes, key.p, key_alt.p, perm.p, perm_alt.p, (int)n, m, dsb, dse, 0,
            (int)(sizeof(double) * 8), st));
        void* tp = temp.get(tbytes);
        PMLSH_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(
            tp, tbytes, key.p, key_alt.p, perm.p, perm_alt.p, (int)n, m, dsb, dse, 0,
            (int)(sizeof(double) * 8), st));
        hipLaunchKernelGGL(bl_copy_kernel, dim3((unsigned)np), dim3(256), 0, st, dp, perm_alt.p,
                           perm.p);
        // the cuts, from the sorted keys
        int32_t* dmid = reinterpret_cast<int32_t*>(dcov);   // free after the directions
        hipLaunchKernelGGL(bl_cut_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, dsb,
                           dse, m, leaf, key_alt.p, dmid);
        PMLSH_HIP(hipGetLastError());
        mids.resize((size_t)m);
        PMLSH_HIP(hipMemcpyAsync(mids.data(), dmid, (size_t)m * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, st));
        PMLSH_HIP(hipStreamSynchronize(st));

        std::vector<int32_t> next;
        for (int s = 0; s < m; ++s) {
            const int32_t id = cur[(size_t)s];
            const int32_t b = sb[s], e = se[s], md = mids[(size_t)s];
            if (md <= b || md >= e || (md - b) % leaf != 0)
                fail(PMLSH_EDEVICE, "device split produced an invalid cut");
            const int32_t l = (int32_t)nodes.size(), r = l + 1;
            nodes.push_back({b / leaf, (md + leaf - 1) / leaf, -1, -1});
            nodes.push_back({md / leaf, (e + leaf - 1) / leaf, -1, -1});
            nb.push_back(b);
            ne.push_back(md);
            nb.push_back(md);
            ne.push_back(e);
            nodes[(size_t)id].left = l;
            nodes[(size_t)id].right = r;
            if (md - b > leaf) next.push_back(l);
            if (e - md > leaf) next.push_back(r);
        }
        cur.swap(next);
    }
    perm_out->resize((size_t)n);
    PMLSH_HIP(hipMemcpyAsync(perm_out->data(), perm.p, (size_t)n * sizeof(int32_t),
                             hipMemcpyDeviceToHost, st));
    PMLSH_HIP(hipStreamSynchronize(st));
}

namespace {

// Pieces of at most kPiece positions for every range [p0[s], p1[s]), and the
// first piece of every range (m + 1 entries).
void make_pieces(const std::vector<int64_t>& p0, const std::vector<int64_t>& p1,
                 std::vector<Piece>* pieces, std::vector<int32_t>* first) {
    pieces->clear();
    first->assign(p0.size() + 1, 0);
    for (size_t sg = 0; sg < p0.size(); ++sg) {
        if (p1[sg] > 0x7fffffffLL - kPiece) fail(PMLSH_EUNSUPPORTED, "point count out of range");
        (*first)[sg] = (int32_t)pieces->size();
        for (int64_t x = p0[sg]; x < p1[sg]; x += kPiece)
            pieces->push_back({(int32_t)sg, (int32_t)x, (int32_t)std::min(p1[sg], x + kPiece)});
    }
    (*first)[p0.size()] = (int32_t)pieces->size();
}

}  // namespace

bool device_all_finite(const float* x, int64_t count, hipStream_t st) {
    DevVec<int32_t> flag;
    int32_t* f = flag.get(1);
    PMLSH_HIP(hipMemsetAsync(f, 0, sizeof(int32_t), st));
    const int64_t blocks = std::min<int64_t>(4096, (count + 255) / 256);
    if (blocks > 0)
        hipLaunchKernelGGL(bl_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, count, f);
    PMLSH_HIP(hipGetLastError());
    int32_t h = 0;
    PMLSH_HIP(hipMemcpyAsync(&h, f, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PMLSH_HIP(hipStreamSynchronize(st));
    return h == 0;
}

void device_pivots(const float* proj, int64_t n, int s, hipStream_t st, std::vector<float>* pivots,
                   double* max_norm) {
    constexpr int kFarBlocks = 1024;
    DevVec<double> bval, mind, part, mean, val;
    DevVec<int64_t> bidx;
    DevVec<float> rows;                 // centroid, zero row, then the s pivots
    DevVec<Piece> d_pieces;
    DevVec<int32_t> d_first;
    const int nb = (int)std::min<int64_t>(kFarBlocks, (n + 255) / 256);
    double* bv = bval.get((size_t)nb);
    int64_t* bi = bidx.get((size_t)nb);
    float* rw = rows.get((size_t)(2 + s) * MP);
    double* dv = val.get(1);
    PMLSH_HIP(hipMemsetAsync(rw, 0, (size_t)(2 + s) * MP * sizeof(float), st));
    // largest norm: the farthest point from the zero row
    hipLaunchKernelGGL(bl_far_kernel, dim3((unsigned)nb), dim3(256), 0, st, proj, n, rw + MP,
                       nullptr, bv, bi);
    hipLaunchKernelGGL(bl_pick_kernel, dim3(1), dim3(256), 0, st, proj, bv, bi, nb, nullptr, dv);
    PMLSH_HIP(hipGetLastError());
    PMLSH_HIP(hipMemcpyAsync(max_norm, dv, sizeof(double), hipMemcpyDeviceToHost, st));
    pivots->assign((size_t)s * MP, 0.f);
    if (s > 0) {
        // centroid: FP64 sums over pieces of the ids, reduced in order
        std::vector<Piece> pieces;
        std::vector<int32_t> first;
        make_pieces({0}, {n}, &pieces, &first);
        Piece* dp = d_pieces.get(pieces.size());
        int32_t* df = d_first.get(first.size());
        PMLSH_HIP(hipMemcpyAsync(dp, pieces.data(), pieces.size() * sizeof(Piece),
                                 hipMemcpyHostToDevice, st));
        PMLSH_HIP(hipMemcpyAsync(df, first.data(), first.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
        double* pt = part.get(pieces.size() * MP);
        double* mn = mean.get(MP);
        hipLaunchKernelGGL(bl_sum_kernel, dim3((unsigned)pieces.size()), dim3(256), 0, st, proj,
                           nullptr, dp, pt);
        hipLaunchKernelGGL(bl_reduce_kernel, dim3(1), dim3(256), 0, st, pt, MP, df, 1, nullptr, mn);
        PMLSH_HIP(hipGetLastError());
        // the reduce kernel sums; the mean divides by n in FP64 on the host
        double sums[MP];
        PMLSH_HIP(hipMemcpyAsync(sums, mn, sizeof(sums), hipMemcpyDeviceToHost, st));
        PMLSH_HIP(hipStreamSynchronize(st));
        float cf[MP];
        for (int j = 0; j < MP; ++j) cf[j] = (float)(sums[j] / (double)n);
        PMLSH_HIP(hipMemcpyAsync(rw, cf, sizeof(cf), hipMemcpyHostToDevice, st));
        // first pivot: the point farthest from the centroid; then each next
        // pivot is the point farthest from the pivots chosen so far
        double* md = mind.get((size_t)n);
        hipLaunchKernelGGL(bl_fill_kernel, dim3(1024), dim3(256), 0, st, md, n,
                           __builtin_huge_val());
        hipLaunchKernelGGL(bl_far_kernel, dim3((unsigned)nb), dim3(256), 0, st, proj, n, rw, nullptr,
                           bv, bi);
        hipLaunchKernelGGL(bl_pick_kernel, dim3(1), dim3(256), 0, st, proj, bv, bi, nb,
                           rw + 2 * MP, nullptr);
        for (int p = 1; p < s; ++p) {
            hipLaunchKernelGGL(bl_far_kernel, dim3((unsigned)nb), dim3(256), 0, st, proj, n,
                               rw + (size_t)(1 + p) * MP, md, bv, bi);
            hipLaunchKernelGGL(bl_pick_kernel, dim3(1), dim3(256), 0, st, proj, bv, bi, nb,
                               rw + (size_t)(2 + p) * MP, nullptr);
        }
        PMLSH_HIP(hipGetLastError());
        PMLSH_HIP(hipMemcpyAsync(pivots->data(), rw + 2 * MP, (size_t)s * MP * sizeof(float),
                                 hipMemcpyDeviceToHost, st));
    }
    PMLSH_HIP(hipStreamSynchronize(st));
}

void device_ball_summaries(const float* proj, const int32_t* perm, const std::vector<int64_t>& p0,
                           const std::vector<int64_t>& p1, const float* pivots, int s,
                           hipStream_t st, std::vector<float>* centre, std::vector<double>* radius,
                           std::vector<double>* ring) {
    const int64_t m = (int64_t)p0.size();
    const int width = 1 + 2 * s;
    centre->assign((size_t)m * MP, 0.f);
    radius->assign((size_t)m, 0.0);
    ring->assign((size_t)m * 2 * s, 0.0);
    if (m == 0) return;
    std::vector<Piece> pieces;
    std::vector<int32_t> first;
    make_pieces(p0, p1, &pieces, &first);
    std::vector<int32_t> cnt((size_t)m);
    for (int64_t i = 0; i < m; ++i) cnt[(size_t)i] = (int32_t)(p1[(size_t)i] - p0[(size_t)i]);
    DevVec<Piece> d_pieces;
    DevVec<int32_t> d_first, d_cnt;
    DevVec<double> part, mean, out;
    DevVec<float> cf, piv;
    Piece* dp = d_pieces.get(pieces.size());
    int32_t* df = d_first.get(first.size());
    int32_t* dc = d_cnt.get((size_t)m);
    PMLSH_HIP(hipMemcpyAsync(dp, pieces.data(), pieces.size() * sizeof(Piece),
                             hipMemcpyHostToDevice, st));
    PMLSH_HIP(hipMemcpyAsync(df, first.data(), first.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, st));
    PMLSH_HIP(hipMemcpyAsync(dc, cnt.data(), cnt.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                             st));
    const int np = (int)pieces.size();
    double* pt = part.get((size_t)np * std::max(MP, width));
    double* mn = mean.get((size_t)m * MP);
    float* c = cf.get((size_t)m * MP);
    double* o = out.get((size_t)m * width);
    float* pv = piv.get((size_t)std::max(1, s) * MP);
    if (s > 0)
        PMLSH_HIP(hipMemcpyAsync(pv, pivots, (size_t)s * MP * sizeof(float), hipMemcpyHostToDevice,
                                 st));
    hipLaunchKernelGGL(bl_sum_kernel, dim3((unsigned)np), dim3(256), 0, st, proj, perm, dp, pt);
    hipLaunchKernelGGL(bl_reduce_kernel, dim3((unsigned)((m * MP + 255) / 256)), dim3(256), 0, st,
                       pt, MP, df, (int)m, dc, mn);
    hipLaunchKernelGGL(bl_centre_kernel, dim3((unsigned)((m * MP + 255) / 256)), dim3(256), 0, st,
                       mn, m * MP, c);
    hipLaunchKernelGGL(bl_ring_kernel, dim3((unsigned)np), dim3(256), 0, st, proj, perm, dp, c, pv,
                       s, pt);
    hipLaunchKernelGGL(bl_reduce_ring_kernel, dim3((unsigned)((m * width + 255) / 256)), dim3(256),
                       0, st, pt, width, df, (int)m, o);
    PMLSH_HIP(hipGetLastError());
    std::vector<double> h((size_t)m * width);
    PMLSH_HIP(hipMemcpyAsync(centre->data(), c, (size_t)m * MP * sizeof(float),
                             hipMemcpyDeviceToHost, st));
    PMLSH_HIP(hipMemcpyAsync(h.data(), o, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    PMLSH_HIP(hipStreamSynchronize(st));
    for (int64_t i = 0; i < m; ++i) {
        (*radius)[(size_t)i] = h[(size_t)(i * width)];
        for (int t = 0; t < 2 * s; ++t) (*ring)[(size_t)(i * 2 * s + t)] = h[(size_t)(i * width + 1 + t)];
    }
}

}  // namespace pmlsh
