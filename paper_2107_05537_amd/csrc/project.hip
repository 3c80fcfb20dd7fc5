// Projection and layout kernels (gfx950).
//
// project_kernel computes o' = (a_1.o, ..., a_m.o) (Eq. 3, Section 3.2) for a
// block of rows with the FP64 matrix cores (v_mfma_f64_16x16x4f64): FP32
// inputs are widened to FP64, accumulated in FP64 and the result is stored as
// the FP32 rounding `hi` plus the FP32 rounding of the remainder `lo`, so
// hi + lo carries the projection to ~2^-48 relative. The hash matrix is padded
// to 16 rows with zeros (m <= 16), which fills the 16-wide MFMA tile.
//
// One workgroup (4 waves) projects 16 rows: the 16 x 16 output tile (16 rows x
// 16 hash functions) is split along the columns, each wave accumulating a
// quarter of every 256-column chunk, and the four partial tiles are summed in
// FP64 at the end. Rows and hash columns are staged through LDS with coalesced
// loads; the row stride of 257 floats keeps the column-wise operand reads free
// of bank conflicts. Small batches (1,024 queries) thus use 64 workgroups.

#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"

namespace pmlsh {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int PJ_ROWS = 16;    // rows per workgroup: one 16 x 16 output tile
constexpr int PJ_KC = 256;     // columns staged per step (64 per wave)

__global__ __launch_bounds__(256) void project_kernel(
    const float* __restrict__ x, int64_t rows, int d, int64_t ld,
    const float* __restrict__ hash, float* __restrict__ out_hi,
    float* __restrict__ out_lo) {
    __shared__ float xs[PJ_ROWS][PJ_KC + 1];
    __shared__ float hs[MP][PJ_KC + 1];
    __shared__ double part[3][64][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * PJ_ROWS;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < d; k0 += PJ_KC) {
        // every load of the step is issued before the LDS stores: thread t
        // reads columns c0 .. c0 + 3 of rows t / 64 + 4 u (u = 0..3), c0 = 4 (t % 64)
        {
            const int c0 = 4 * (tid & 63), r0 = tid >> 6;
            float xv[PJ_ROWS / 4][4], hv[MP / 4][4];
#pragma unroll
            for (int u = 0; u < PJ_ROWS / 4; ++u) {
                const int64_t gr = row0 + r0 + 4 * u;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int gc = k0 + c0 + e;
                    xv[u][e] = (gr < rows && gc < d) ? x[gr * ld + gc] : 0.f;
                }
            }
#pragma unroll
            for (int u = 0; u < MP / 4; ++u) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int gc = k0 + c0 + e;
                    hv[u][e] = gc < d ? hash[(int64_t)(r0 + 4 * u) * d + gc] : 0.f;
                }
            }
#pragma unroll
            for (int u = 0; u < PJ_ROWS / 4; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) xs[r0 + 4 * u][c0 + e] = xv[u][e];
#pragma unroll
            for (int u = 0; u < MP / 4; ++u)
#pragma unroll
                for (int e = 0; e < 4; ++e) hs[r0 + 4 * u][c0 + e] = hv[u][e];
        }
        __syncthreads();
        // each wave takes 64 of the staged columns. A operand: row
        // (lane % 16), k = lane / 16; B operand: hash function (lane % 16).
#pragma unroll 4
        for (int kk = wave * 64; kk < wave * 64 + 64; kk += 4) {
            const double a = (double)xs[lane & 15][kk + (lane >> 4)];
            const double b = (double)hs[lane & 15][kk + (lane >> 4)];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // the four waves' partial tiles are summed by wave 0
    if (wave > 0)
        for (int i = 0; i < 4; ++i) part[wave - 1][lane][i] = acc[i];
    __syncthreads();
    if (wave != 0) return;
    // result element i of a lane: row lane/16 + 4*i, hash function lane % 16
    // (the v_mfma_f64_16x16x4f64 accumulator layout on gfx950)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double v = acc[i] + part[0][lane][i] + part[1][lane][i] + part[2][lane][i];
        const int64_t gr = row0 + (lane >> 4) + 4 * i;
        const int col = lane & 15;
        if (gr < rows) {
            const float hi = (float)v;
            out_hi[gr * MP + col] = hi;
            if (out_lo) out_lo[gr * MP + col] = (float)(v - (double)hi);
        }
    }
}

// Low-precision projection for the matrix-core filter (mixed-precision
// configuration): o' = (a_1.o, ..., a_m.o) with every input rounded to FP16
// or BF16 and the products summed in FP32 on the matrix cores
// (v_mfma_f32_16x16x32_f16 / _bf16), and per row a bound eps on the
// Euclidean norm of (o'_lp - o'), o' being the exact projection of the FP32
// row. With u the unit roundoff of the input format and eta its largest
// absolute error below the normal range (flushed subnormals included), a
// rounded input is a~ = a + da with |da| <= u |a| + eta, so
//   |a~ o~ - a o| <= (2u + u^2) |a o| + (1 + u) eta (|a| + |o|) + eta^2.
// The product of two rounded inputs is exact in FP32, and summing d of them
// in FP32 in any order (a truncating adder included, unit 2^-23) adds at most
// g_d sum |a~ o~|, g_d = d 2^-23 / (1 - d 2^-23). Bounding |a o| through
// |a~| and |o~| and collecting terms (u <= 2^-8), per coordinate
//   e_i <= c1 S_i + eta' (A_i + X) + 2 d eta'^2,
//   c1 = ((2u + u^2) / (1 - u)^2 + g_d) / (1 - g_d),  eta' = 1.02 eta,
// with S_i the FP32 matrix-core sum of |a~_ij| |o~_j| (at least 1 - g_d
// times the exact sum), A_i = sum_j |a_ij| and X = sum_j |o_j| (FP32 sums,
// within the 2% slack of eta'). eps is the FP32 norm of (e_i), enlarged by
// 2^-16 for the rounding of its own evaluation.
//
// A workgroup projects 16 rows; its four waves take the 32-wide input steps
// in turn (wave w: steps w, w + 4, ...) and the partial tiles are summed in
// LDS. Lane l holds row l % 16 and hash function l % 16 for the inputs
// k = 32 s + 8 (l / 16) .. + 7 of a step.
template <bool BF16>
__global__ __launch_bounds__(256) void project_lp_kernel(
    const float* __restrict__ x, int64_t rows, int d, int64_t ld,
    const float* __restrict__ hash, float c1, float eta,
    float* __restrict__ out, float* __restrict__ eps) {
    typedef __attribute__((ext_vector_type(8))) _Float16 h8;
    typedef __attribute__((ext_vector_type(8))) __bf16 b8;
    typedef __attribute__((ext_vector_type(4))) float f4;
    __shared__ float part[3][64][10];   // waves 1..3: acc, accs, xs, as per lane
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * 16;
    const int r = lane & 15, kq = 8 * (lane >> 4);
    const int64_t gr = row0 + r;
    const bool rv = gr < rows;
    f4 acc = {0.f, 0.f, 0.f, 0.f}, accs = {0.f, 0.f, 0.f, 0.f};
    float xs = 0.f, as = 0.f;   // partial sums of |o_j| (row r) and |a_rj| (function r)
    for (int k0 = 32 * wave; k0 < d; k0 += 128) {
        float xv[8], hv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + kq + e;
            xv[e] = rv && k < d ? x[gr * ld + k] : 0.f;
            hv[e] = k < d ? hash[(int64_t)r * d + k] : 0.f;
            xs += fabsf(xv[e]);
            as += fabsf(hv[e]);
        }
        if constexpr (BF16) {
            b8 xa, ha, xb, hb;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                xa[e] = (__bf16)xv[e];
                ha[e] = (__bf16)hv[e];
                xb[e] = (__bf16)fabsf(xv[e]);
                hb[e] = (__bf16)fabsf(hv[e]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, ha, acc, 0, 0, 0);
            accs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xb, hb, accs, 0, 0, 0);
        } else {
            h8 xa, ha, xb, hb;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                xa[e] = (_Float16)xv[e];
                ha[e] = (_Float16)hv[e];
                xb[e] = (_Float16)fabsf(xv[e]);
                hb[e] = (_Float16)fabsf(hv[e]);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(xa, ha, acc, 0, 0, 0);
            accs = __builtin_amdgcn_mfma_f32_16x16x32_f16(xb, hb, accs, 0, 0, 0);
        }
    }
    if (wave > 0) {
        float* p = part[wave - 1][lane];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            p[i] = acc[i];
            p[4 + i] = accs[i];
        }
        p[8] = xs;
        p[9] = as;
    }
    __syncthreads();
    if (wave != 0) return;
    // the sums over the waves, in a fixed order
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        const float* p = part[w][lane];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            acc[i] += p[i];
            accs[i] += p[4 + i];
        }
        xs += p[8];
        as += p[9];
    }
    // the four lanes of a row (function) hold quarters of its sums
    xs += __shfl_xor(xs, 16);
    xs += __shfl_xor(xs, 32);
    as += __shfl_xor(as, 16);
    as += __shfl_xor(as, 32);
    // result register i of lane l: row 4 (l / 16) + i, function l % 16
    const int fn = lane & 15;
    const float a_sum = as;   // lane l holds A for function l % 16
    float e2[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = 4 * (lane >> 4) + i;
        const float x_sum = __shfl(xs, rr);   // lane rr holds X of row rr
        // a zero hash row (m < 16) projects exactly to zero
        const float e = a_sum > 0.f ? c1 * accs[i] + eta * (a_sum + x_sum) + 2.f * (float)d * eta * eta
                                    : 0.f;
        e2[i] = e * e;
        const int64_t g = row0 + rr;
        if (g < rows) out[g * MP + fn] = acc[i];
    }
    // norm over the 16 functions: the 16 lanes of each quarter
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float v = e2[i];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        const int64_t g = row0 + 4 * (lane >> 4) + i;
        if (fn == 0 && g < rows) eps[g] = sqrtf(v) * (1.f + 1.52587890625e-05f);
    }
}

// dst row j = src row perm[j], zero padded from d to d_pad columns.
__global__ __launch_bounds__(256) void gather_rows_kernel(
    const float* __restrict__ src, int d, int64_t ld_src,
    const int32_t* __restrict__ perm, int64_t rows, float* __restrict__ dst,
    int d_pad) {
    const int64_t total = rows * (int64_t)d_pad;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / d_pad;
        const int c = (int)(e - j * d_pad);
        dst[e] = c < d ? src[(int64_t)perm[j] * ld_src + c] : 0.f;
    }
}

__global__ __launch_bounds__(256) void gather_proj_kernel(
    const float* __restrict__ src, const int32_t* __restrict__ perm,
    int64_t rows, float* __restrict__ dst) {
    const int64_t total = rows * MP;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / MP;
        dst[e] = src[(int64_t)perm[j] * MP + (e - j * MP)];
    }
}

// Rows of the FP16 matrix-core scan, kScanRow halves per point (the layout is
// described with scan_kernel), o' taken relative to the centre mu of the
// rows: s * o' (16 dims, pad zero), the hi/lo FP16 pair
// of s^2 ||o'||^2, two ones that carry the query's threshold pair, and
// cm * s * ||o'||, the weight of the rounding margin. Rows from n to n_pad are
// zero, which never produce a candidate.
struct Centre {
    float v[MP];
};

__global__ __launch_bounds__(256) void augment16_kernel(
    const float* __restrict__ proj, int64_t n, int64_t n_pad, float s, float cm, Centre mu,
    uint4* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pad) return;
    _Float16 v[kScanRow];
#pragma unroll
    for (int i = 0; i < kScanRow; ++i) v[i] = (_Float16)0.f;
    if (p < n) {
        float o[MP];
        float on2 = 0.f;
#pragma unroll
        for (int t = 0; t < MP; ++t) {
            o[t] = proj[p * MP + t] - mu.v[t];
            on2 = fmaf(o[t], o[t], on2);
        }
#pragma unroll
        for (int t = 0; t < MP; ++t) v[t] = (_Float16)(s * o[t]);
        const float sn = s * s * on2;
        const _Float16 hi = (_Float16)sn;
        v[16] = hi;
        v[17] = (_Float16)(sn - (float)hi);
        v[18] = (_Float16)1.f;
        v[19] = (_Float16)1.f;
        v[20] = (_Float16)(cm * s * sqrtf(on2));
    }
    const uint4* src = reinterpret_cast<const uint4*>(v);
    constexpr int kParts = kScanRow / 8;
#pragma unroll
    for (int i = 0; i < kParts; ++i) out[p * kParts + i] = src[i];
}

// FP16 copy of the leaf-order data for the bounded verification: one wave
// per row. The row is scaled by a power of two s (its largest magnitude maps
// below 2^15), rounded to FP16, and the exact norm of the rounding error
// |x - s x16| is accumulated in FP64 and rounded up: the distance from any
// query to the FP16 row then lies within eps of the distance to x.
__global__ __launch_bounds__(256) void half_rows_kernel(
    const float* __restrict__ data, int64_t n, int d_pad, int d16,
    uint16_t* __restrict__ out, float* __restrict__ scale, float* __restrict__ eps) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const float* x = data + row * d_pad;
    float mx = 0.f;
    for (int c = lane; c < d_pad; c += 64) mx = fmaxf(mx, fabsf(x[c]));
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    int e = 0;
    if (mx > 0.f) (void)frexpf(mx, &e);
    const float s = ldexpf(1.f, e - 15);          // mx / s < 2^15
    double err = 0.0;
    _Float16* o = reinterpret_cast<_Float16*>(out + row * d16);
    for (int c = lane; c < d16; c += 64) {
        const float v = c < d_pad ? x[c] : 0.f;
        const _Float16 h = (_Float16)(v / s);
        o[c] = h;
        const double dlt = (double)v - (double)s * (double)(float)h;
        err += dlt * dlt;
    }
    for (int off = 32; off > 0; off >>= 1) err += __shfl_xor(err, off);
    if (lane == 0) {
        scale[row] = s;
        const float ef = (float)sqrt(err);
        eps[row] = nextafterf(ef * (1.f + 9.5367431640625e-07f), INFINITY);
    }
}

// FP64 Euclidean distance of row pairs (one wave per pair).
__global__ __launch_bounds__(256) void pair_dist_f64_kernel(
    const float* __restrict__ x, int d, int64_t ld,
    const int64_t* __restrict__ pairs, int64_t count, double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= count) return;
    const float* a = x + pairs[2 * p] * ld;
    const float* b = x + pairs[2 * p + 1] * ld;
    double s = 0.0;
    for (int c = lane; c < d; c += 64) {
        const double t = (double)a[c] - (double)b[c];
        s = fma(t, t, s);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) out[p] = sqrt(s);
}

int grid_for(int64_t work) {
    int64_t g = (work + 255) / 256;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace

void launch_project(const float* x, int64_t rows, int d, int64_t ld,
                    const float* hash, float* out_hi, float* out_lo,
                    hipStream_t stream) {
    if (rows <= 0) return;
    const int64_t blocks = (rows + PJ_ROWS - 1) / PJ_ROWS;
    hipLaunchKernelGGL(project_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                       x, rows, d, ld, hash, out_hi, out_lo);
    PMLSH_HIP(hipGetLastError());
}

void launch_gather_rows(const float* src, int d, int64_t ld_src, const int32_t* perm,
                        int64_t rows, float* dst, int d_pad, hipStream_t stream) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for(rows * d_pad)), dim3(256), 0,
                       stream, src, d, ld_src, perm, rows, dst, d_pad);
    PMLSH_HIP(hipGetLastError());
}

void launch_gather_proj(const float* src, const int32_t* perm, int64_t rows,
                        float* dst, hipStream_t stream) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(gather_proj_kernel, dim3(grid_for(rows * MP)), dim3(256), 0,
                       stream, src, perm, rows, dst);
    PMLSH_HIP(hipGetLastError());
}

void launch_project_lp(const float* x, int64_t rows, int d, int64_t ld, const float* hash,
                       int mode, float* out, float* eps, hipStream_t stream) {
    if (rows <= 0) return;
    // unit roundoff and largest absolute error below the normal range
    const double u = mode == PMLSH_FILTER_GEMM_BF16 ? std::ldexp(1.0, -8) : std::ldexp(1.0, -11);
    const double eta = mode == PMLSH_FILTER_GEMM_BF16 ? std::ldexp(1.0, -126) : std::ldexp(1.0, -14);
    const double ud = (double)d * std::ldexp(1.0, -23);
    const double gd = ud / (1.0 - ud);
    const double c1 = ((2.0 * u + u * u) / ((1.0 - u) * (1.0 - u)) + gd) / (1.0 - gd);
    const float c1f = (float)(c1 * (1.0 + 1e-6));
    const float etaf = (float)(1.02 * eta);
    const unsigned grid = (unsigned)((rows + 15) / 16);
    if (mode == PMLSH_FILTER_GEMM_BF16)
        hipLaunchKernelGGL(project_lp_kernel<true>, dim3(grid), dim3(256), 0, stream, x, rows, d,
                           ld, hash, c1f, etaf, out, eps);
    else
        hipLaunchKernelGGL(project_lp_kernel<false>, dim3(grid), dim3(256), 0, stream, x, rows, d,
                           ld, hash, c1f, etaf, out, eps);
    PMLSH_HIP(hipGetLastError());
}

void launch_augment16(const float* proj, int64_t n, int64_t n_pad, float s, float cm, const float* centre,
                      uint16_t* out, hipStream_t stream) {
    if (n_pad <= 0) return;
    Centre mu{};
    for (int t = 0; t < MP; ++t) mu.v[t] = centre[t];
    hipLaunchKernelGGL(augment16_kernel, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0,
                       stream, proj, n, n_pad, s, cm, mu, reinterpret_cast<uint4*>(out));
    PMLSH_HIP(hipGetLastError());
}

void launch_half_rows(const float* data, int64_t n, int d_pad, int d16, uint16_t* out,
                      float* scale, float* eps, hipStream_t stream) {
    if (n <= 0) return;
    hipLaunchKernelGGL(half_rows_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream,
                       data, n, d_pad, d16, out, scale, eps);
    PMLSH_HIP(hipGetLastError());
}

void launch_pair_dist_f64(const float* x, int d, int64_t ld, const int64_t* pairs,
                          int64_t count, double* out, hipStream_t stream) {
    if (count <= 0) return;
    hipLaunchKernelGGL(pair_dist_f64_kernel, dim3((unsigned)((count + 3) / 4)), dim3(256),
                       0, stream, x, d, ld, pairs, count, out);
    PMLSH_HIP(hipGetLastError());
}

}  // namespace pmlsh
