// Index construction (Sections 3.2, 4.1 and 5.2).
//
//   1. D and A to HBM (if given on the host); A padded to 16 zero-filled rows;
//   2. O' = D A^T on the FP64 matrix cores (hi/lo FP32 pair per coordinate);
//   3. the PM-tree is bulk-loaded on the host over the FP32 `hi` coordinates;
//   4. D, O'_hi and O'_lo are permuted to leaf order on the device, so a leaf
//      is one contiguous run of rows for the scans and the verification;
//   5. the r_min sample: S = min(n(n-1)/2, 100000) SplitMix64-drawn pairs,
//      FP64 distances on the device, sorted on the host.

#include <algorithm>
#include <cmath>
#include <memory>

#include "internal.hpp"

namespace pmlsh {
namespace {

constexpr int64_t kSamplePairs = 100000;

template <class T>
T* dev_alloc(pmlsh_index* idx, int64_t count) {
    if (count <= 0) count = 1;
    void* p = nullptr;
    PMLSH_HIP(hipMalloc(&p, (size_t)count * sizeof(T)));
    idx->device_bytes += count * (int64_t)sizeof(T);
    return static_cast<T*>(p);
}

struct TmpBuf {
    void* p = nullptr;
    ~TmpBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

void index_release(pmlsh_index* x) {
    if (!x) return;
    void* bufs[] = {x->data, x->proj_hi, x->proj_lo, x->proj16, x->chunk_cen, x->chunk_rad,
                    x->data16, x->data16_scale, x->data16_eps, x->perm, x->inv_perm, x->hash,
                    x->tree.centre, x->tree.radius, x->tree.hr_min, x->tree.hr_max,
                    x->tree.child_begin, x->tree.child_end, x->tree.npts,
                    x->tree.pivots};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (auto& b : x->acp_bufs)
        if (b.first) (void)hipFree(b.first);
    if (x->acp_host) (void)hipHostFree(x->acp_host);
    delete x;
}

static void validate_build(const pmlsh_build_args* a) {
    if (!a) fail(PMLSH_EINVAL, "args is NULL");
    if (!a->data || !a->hash) fail(PMLSH_EINVAL, "data and hash must not be NULL");
    if (a->n < 1) fail(PMLSH_EINVAL, "n must be >= 1");
    if (a->n > 0x7fffffffll) fail(PMLSH_EUNSUPPORTED, "n must be < 2^31");
    if (a->d < 1 || a->d > 65536) fail(PMLSH_EINVAL, "d must be in 1..65536");
    if (a->m < 1 || a->m > PMLSH_MAX_M) fail(PMLSH_EINVAL, "m must be in 1..16");
    if (a->num_pivots < 0 || a->num_pivots > PMLSH_MAX_PIVOTS)
        fail(PMLSH_EINVAL, "num_pivots must be in 0..8");
    if (a->leaf_size != 0 && (a->leaf_size < 8 || a->leaf_size > 256))
        fail(PMLSH_EINVAL, "leaf_size must be 0 or in 8..256");
    if (a->fanout != 0 && (a->fanout < 2 || a->fanout > 64 || (a->fanout & (a->fanout - 1))))
        fail(PMLSH_EINVAL, "fanout must be 0 or a power of two in 2..64");
    if (!(a->r_min_kappa >= 0.0 && a->r_min_kappa <= 1.0))
        fail(PMLSH_EINVAL, "r_min_kappa must be in [0, 1]");
    if (a->filter_gemm != 0 && a->filter_gemm != PMLSH_FILTER_GEMM_FP16 &&
        a->filter_gemm != PMLSH_FILTER_GEMM_BF16)
        fail(PMLSH_EINVAL, "filter_gemm must be 0, PMLSH_FILTER_GEMM_FP16 or PMLSH_FILTER_GEMM_BF16");
    if (!a->data_on_device) {
        // host data: finiteness is checked before anything touches the GPU
        const int64_t total = a->n * (int64_t)a->d;
        for (int64_t i = 0; i < total; ++i)
            if (!std::isfinite(a->data[i])) fail(PMLSH_EINVAL, "data holds a non-finite value");
        for (int64_t i = 0; i < (int64_t)a->m * a->d; ++i)
            if (!std::isfinite(a->hash[i])) fail(PMLSH_EINVAL, "hash holds a non-finite value");
    }
}

pmlsh_index* index_build(const pmlsh_build_args* a) {
    validate_build(a);
    hipStream_t st = static_cast<hipStream_t>(a->stream);
    std::unique_ptr<pmlsh_index, void (*)(pmlsh_index*)> idx(new pmlsh_index(), index_release);
    pmlsh_index* x = idx.get();
    x->n = a->n;
    x->d = a->d;
    x->d_pad = (a->d + 3) & ~3;
    x->m = a->m;
    x->num_pivots = a->num_pivots;
    x->leaf_size = a->leaf_size ? a->leaf_size : 64;
    x->fanout = a->fanout ? a->fanout : 16;
    x->kappa = a->r_min_kappa > 0.0 ? a->r_min_kappa : 0.9;
    x->filter_gemm = a->filter_gemm;
    PMLSH_HIP(hipGetDevice(&x->device));
    const int64_t n = a->n;
    const int d = a->d;

    // ---- inputs on the device
    TmpBuf dsrc, hsrc;
    const float* D = a->data;
    const float* H = a->hash;
    if (!a->data_on_device) {
        PMLSH_HIP(hipMalloc(&dsrc.p, (size_t)n * d * sizeof(float)));
        PMLSH_HIP(hipMemcpyAsync(dsrc.p, a->data, (size_t)n * d * sizeof(float),
                                 hipMemcpyHostToDevice, st));
        D = static_cast<const float*>(dsrc.p);
        PMLSH_HIP(hipMalloc(&hsrc.p, (size_t)a->m * d * sizeof(float)));
        PMLSH_HIP(hipMemcpyAsync(hsrc.p, a->hash, (size_t)a->m * d * sizeof(float),
                                 hipMemcpyHostToDevice, st));
        H = static_cast<const float*>(hsrc.p);
    }
    // Device data is not scanned for non-finite values separately: the
    // projection propagates any NaN/inf into O', which is checked below.
    x->hash = dev_alloc<float>(x, (int64_t)MP * d);
    PMLSH_HIP(hipMemsetAsync(x->hash, 0, (size_t)MP * d * sizeof(float), st));
    PMLSH_HIP(hipMemcpyAsync(x->hash, H, (size_t)a->m * d * sizeof(float),
                             hipMemcpyDeviceToDevice, st));

    // ---- projection in original order
    TmpBuf phi, plo;
    PMLSH_HIP(hipMalloc(&phi.p, (size_t)n * MP * sizeof(float)));
    PMLSH_HIP(hipMalloc(&plo.p, (size_t)n * MP * sizeof(float)));
    launch_project(D, n, d, d, x->hash, static_cast<float*>(phi.p), static_cast<float*>(plo.p), st);
    if (!device_all_finite(static_cast<const float*>(phi.p), n * MP, st))
        fail(PMLSH_EINVAL, "data or hash holds a non-finite value");

    // ---- tree
    HostTree T;
    {
        std::vector<int32_t> perm;
        std::vector<SplitNode> split;
        device_split(static_cast<const float*>(phi.p), n, x->leaf_size, st, &perm, &split);
        x->perm = dev_alloc<int32_t>(x, n);
        PMLSH_HIP(hipMemcpyAsync(x->perm, perm.data(), (size_t)n * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
        build_tree(static_cast<const float*>(phi.p), n, x->leaf_size, x->fanout, x->num_pivots,
                   std::move(perm), x->perm, split, st, &T);
    }
    x->levels = T.levels;
    x->n_nodes = T.n_nodes;
    x->level_begin = T.level_begin;
    x->n_leaves = T.level_begin[T.levels] - T.level_begin[T.levels - 1];
    x->coord_scale = T.coord_scale;
    x->perm_host = T.perm;

    auto upload = [&](const auto& vec, auto** dst) {
        using E = typename std::decay<decltype(vec)>::type::value_type;
        *dst = dev_alloc<E>(x, (int64_t)vec.size());
        PMLSH_HIP(hipMemcpyAsync(*dst, vec.data(), vec.size() * sizeof(E),
                                 hipMemcpyHostToDevice, st));
    };
    std::vector<int32_t> inv(n);
    for (int64_t j = 0; j < n; ++j) inv[T.perm[j]] = (int32_t)j;
    upload(inv, &x->inv_perm);
    upload(T.centre, &x->tree.centre);
    upload(T.radius, &x->tree.radius);
    upload(T.hr_min, &x->tree.hr_min);
    upload(T.hr_max, &x->tree.hr_max);
    upload(T.child_begin, &x->tree.child_begin);
    upload(T.child_end, &x->tree.child_end);
    upload(T.npts, &x->tree.npts);
    std::vector<float> piv = T.pivots;
    if (piv.empty()) piv.assign(MP, 0.f);
    upload(piv, &x->tree.pivots);

    // ---- leaf-order copies
    x->data = dev_alloc<float>(x, n * x->d_pad);
    x->proj_hi = dev_alloc<float>(x, n * MP);
    x->proj_lo = dev_alloc<float>(x, n * MP);
    launch_gather_rows(D, d, d, x->perm, n, x->data, x->d_pad, st);
    launch_gather_proj(static_cast<const float*>(phi.p), x->perm, n, x->proj_hi, st);
    launch_gather_proj(static_cast<const float*>(plo.p), x->perm, n, x->proj_lo, st);
    // FP16 copy for the bounded verification
    x->d16 = (x->d + 7) / 8 * 8;
    x->data16 = dev_alloc<uint16_t>(x, n * x->d16);
    x->data16_scale = dev_alloc<float>(x, n);
    x->data16_eps = dev_alloc<float>(x, n);
    launch_half_rows(x->data, n, x->d_pad, x->d16, x->data16, x->data16_scale, x->data16_eps, st);

    // ---- chunk balls, then the FP16 rows of the matrix-core scan
    {
        x->n_pad16 = (n + 63) / 64 * 64;
        // covering ball of every 64-point chunk of the leaf order (the leaves
        // themselves when the leaf size is 64): FP64 mean rounded to FP32,
        // radius measured from that FP32 centre in FP64, widened by 1e-6 and
        // rounded up
        const int64_t nch = x->n_pad16 / 64;
        std::vector<int64_t> c0((size_t)nch), c1((size_t)nch);
        for (int64_t c = 0; c < nch; ++c) {
            c0[(size_t)c] = c * 64;
            c1[(size_t)c] = std::min<int64_t>(n, c * 64 + 64);
        }
        std::vector<float> ccen;
        std::vector<double> r64, unused;
        device_ball_summaries(static_cast<const float*>(phi.p), x->perm, c0, c1, nullptr, 0, st,
                              &ccen, &r64, &unused);
        // radii padded with zeros to a multiple of 16 chunks (vector loads)
        std::vector<float> crad((size_t)((nch + 15) / 16 * 16), 0.f);
        for (int64_t c = 0; c < nch; ++c)
            crad[(size_t)c] = std::nextafter((float)(r64[(size_t)c] * (1.0 + 1e-6)), INFINITY);
        upload(ccen, &x->chunk_cen);
        upload(crad, &x->chunk_rad);

        // The scan rows are centred on mu, the mean of the projected points
        // (from the chunk centres weighted by their counts, FP64, rounded to
        // FP32): distances do not change, and the rounding margin of the
        // FP16 products, which grows with |o' - mu| |q' - mu|, shrinks when
        // the data sits away from the origin. S bounds every |o' - mu|: the
        // largest |centre - mu| + radius over the chunks (FP64, widened by
        // 1e-6, rounded up).
        double mu64[MP] = {};
        for (int64_t c = 0; c < nch; ++c) {
            const double w = (double)(c1[(size_t)c] - c0[(size_t)c]);
            for (int t = 0; t < MP; ++t) mu64[t] += w * (double)ccen[(size_t)(c * MP + t)];
        }
        for (int t = 0; t < MP; ++t) x->scan_centre[t] = (float)(mu64[t] / (double)n);
        double smax = 0.0;
        for (int64_t c = 0; c < nch; ++c) {
            double s2 = 0.0;
            for (int t = 0; t < MP; ++t) {
                const double dd = (double)ccen[(size_t)(c * MP + t)] - (double)x->scan_centre[t];
                s2 += dd * dd;
            }
            smax = std::max(smax, std::sqrt(s2) + (double)crad[(size_t)c]);
        }
        x->scan_scale = std::nextafter((float)(smax * (1.0 + 1e-6)), INFINITY);

        // FP16 rows scaled by a power of two s with s * S < 32, so every
        // entry stays far inside the FP16 range. With filter_gemm the rows
        // come from the low-precision projection of the leaf-order data,
        // whose points are within eps_max of the exact ones.
        const float* proj_scan = x->proj_hi;
        TmpBuf lp, lpe;
        if (x->filter_gemm) {
            PMLSH_HIP(hipMalloc(&lp.p, (size_t)n * MP * sizeof(float)));
            PMLSH_HIP(hipMalloc(&lpe.p, (size_t)n * sizeof(float)));
            float* lpp = static_cast<float*>(lp.p);
            float* lpep = static_cast<float*>(lpe.p);
            launch_project_lp(x->data, n, d, x->d_pad, x->hash, x->filter_gemm, lpp, lpep, st);
            if (!device_all_finite(lpp, n * MP, st) || !device_all_finite(lpep, n, st))
                fail(PMLSH_EUNSUPPORTED, "data exceeds the range of the filter's input format");
            std::vector<float> e(n);
            PMLSH_HIP(hipMemcpyAsync(e.data(), lpep, (size_t)n * sizeof(float),
                                     hipMemcpyDeviceToHost, st));
            PMLSH_HIP(hipStreamSynchronize(st));
            float emax = 0.f;
            for (float v : e) emax = std::max(emax, v);
            x->eps_max = emax;
            // an upper bound of the sum (FP32 addition rounded up twice)
            x->scan_scale = std::nextafter(std::nextafter(x->scan_scale + emax, INFINITY), INFINITY);
            proj_scan = lpp;
        }
        int e = 0;
        const float S = x->scan_scale;
        if (S > 0.f && std::isfinite(S)) (void)std::frexp(S, &e);
        x->scale16 = std::ldexp(1.f, 5 - e);
        x->proj16 = dev_alloc<uint16_t>(x, x->n_pad16 * kScanRow);
        launch_augment16(proj_scan, n, x->n_pad16, x->scale16, kScanMarginWeight, x->scan_centre,
                         x->proj16, st);
        // the temporary projection is released with the scope: the rows are
        // built first
        PMLSH_HIP(hipStreamSynchronize(st));
    }

    // ---- r_min sample (Section 5.2): FP64 distances of sampled pairs
    if (n >= 2) {
        const int64_t S = std::min<int64_t>(n * (n - 1) / 2, kSamplePairs);
        std::vector<int64_t> pairs((size_t)S * 2);
        const uint64_t seed = a->sample_seed;
        for (int64_t j = 0; j < S; ++j) {
            const int64_t i = (int64_t)(splitmix64(seed + (uint64_t)j) % (uint64_t)n);
            const int64_t l =
                (i + 1 + (int64_t)(splitmix64(seed + (uint64_t)S + (uint64_t)j) % (uint64_t)(n - 1))) % n;
            pairs[2 * j] = i;
            pairs[2 * j + 1] = l;
        }
        TmpBuf dp, dd;
        PMLSH_HIP(hipMalloc(&dp.p, pairs.size() * sizeof(int64_t)));
        PMLSH_HIP(hipMalloc(&dd.p, (size_t)S * sizeof(double)));
        PMLSH_HIP(hipMemcpyAsync(dp.p, pairs.data(), pairs.size() * sizeof(int64_t),
                                 hipMemcpyHostToDevice, st));
        launch_pair_dist_f64(D, d, d, static_cast<const int64_t*>(dp.p), S,
                             static_cast<double*>(dd.p), st);
        x->sample_sorted.resize(S);
        PMLSH_HIP(hipMemcpyAsync(x->sample_sorted.data(), dd.p, (size_t)S * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
        PMLSH_HIP(hipStreamSynchronize(st));
        std::sort(x->sample_sorted.begin(), x->sample_sorted.end());
    }
    PMLSH_HIP(hipStreamSynchronize(st));
    return idx.release();
}

// kappa * F^-1(B/n) from the sorted sample. A zero quantile (duplicate
// points) would never grow under r <- c r, so the smallest positive sample
// distance is used instead, and 1 when the sample holds no positive distance.
double index_default_r_min(const pmlsh_index* x, int64_t budget) {
    const std::vector<double>& s = x->sample_sorted;
    if (s.empty()) return 1.0;   // n == 1
    const int64_t S = (int64_t)s.size();
    const double q = std::min(1.0, (double)budget / (double)x->n);
    int64_t i = (int64_t)std::ceil(q * (double)S) - 1;
    if (i < 0) i = 0;
    double v = s[(size_t)i];
    if (!(v > 0.0)) {
        auto it = std::upper_bound(s.begin(), s.end(), 0.0);
        v = it == s.end() ? 1.0 / x->kappa : *it;
    }
    return x->kappa * v;
}

}  // namespace pmlsh
