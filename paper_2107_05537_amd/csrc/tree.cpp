// Host bulk-load of the PM-tree over projected points (Section 4.1).
//
// The paper builds its PM-tree by inserting points one at a time and
// splitting overflowing nodes (Section 6.3, "Promote Methods"). Here the
// whole point set is known up front, so the tree is bulk-loaded:
//   * global pivots p_1..p_s by farthest-point selection (the paper only asks
//     for pivots that keep the node regions small);
//   * leaves by recursive median splits along the coordinate of largest
//     variance, the left part always holding a whole number of leaves, so
//     every leaf has exactly leaf_size points except the last one;
//   * inner levels by grouping `fanout` consecutive nodes of the level below
//     (consecutive leaves of the recursion are spatial neighbours).
// Every node stores what Eq. 5 and Eq. 11 need: a centre e.RO (the mean of
// its points, rounded to FP32), the covering radius e.r about that centre and
// the hyper-ring e.HR[i] = [min, max] distance of its points to pivot i, all
// computed in FP64 from the FP32 coordinates the kernels read and rounded
// outward, so the node tests never reject a node that holds a point the
// kernels would accept.

#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>

#include "internal.hpp"

namespace pmlsh {
namespace {

int hw_threads() {
    unsigned h = std::thread::hardware_concurrency();
    return h == 0 ? 4 : (int)std::min(h, 64u);
}

template <class F>
void parallel_for(int64_t count, F fn) {
    int nt = (int)std::min<int64_t>(hw_threads(), std::max<int64_t>(1, count / 64));
    if (nt <= 1) {
        for (int64_t i = 0; i < count; ++i) fn(i);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int64_t i = t; i < count; i += nt) fn(i);
        });
    for (auto& x : th) x.join();
}

float round_up(double v) {
    float f = (float)v;
    if ((double)f < v) f = std::nextafter(f, std::numeric_limits<float>::infinity());
    return f;
}
float round_down(double v) {
    float f = (float)v;
    if ((double)f > v) f = std::nextafter(f, -std::numeric_limits<float>::infinity());
    return f;
}

double dist64(const float* a, const float* b) {
    double s = 0;
    for (int j = 0; j < MP; ++j) {
        double t = (double)a[j] - (double)b[j];
        s += t * t;
    }
    return std::sqrt(s);
}

// Recursive split of idx[b, e) into whole leaves. A node is cut along its
// principal direction (power iteration on its 16 x 16 covariance) at the
// leaf boundary, within the middle 60 % of its leaves, where the sorted
// projections show the widest gap, so cuts fall between clusters rather
// than through them. Ties in the projection are ordered by id.
struct Splitter {
    const float* proj;
    int64_t leaf;
    std::vector<int32_t>& idx;

    void direction(int64_t b, int64_t e, double* dir) const {
        double mean[MP] = {0};
        for (int64_t i = b; i < e; ++i) {
            const float* p = proj + (int64_t)idx[i] * MP;
            for (int j = 0; j < MP; ++j) mean[j] += p[j];
        }
        const double cnt = (double)(e - b);
        for (int j = 0; j < MP; ++j) mean[j] /= cnt;
        double cov[MP][MP] = {{0}};
        for (int64_t i = b; i < e; ++i) {
            const float* p = proj + (int64_t)idx[i] * MP;
            double c[MP];
            for (int j = 0; j < MP; ++j) c[j] = p[j] - mean[j];
            for (int j = 0; j < MP; ++j)
                for (int k = j; k < MP; ++k) cov[j][k] += c[j] * c[k];
        }
        for (int j = 0; j < MP; ++j)
            for (int k = 0; k < j; ++k) cov[j][k] = cov[k][j];
        // start from the coordinate axis of largest variance
        int ax = 0;
        for (int j = 1; j < MP; ++j)
            if (cov[j][j] > cov[ax][ax]) ax = j;
        for (int j = 0; j < MP; ++j) dir[j] = j == ax ? 1.0 : 0.0;
        for (int it = 0; it < 30; ++it) {
            double nd[MP] = {0}, nrm = 0;
            for (int j = 0; j < MP; ++j) {
                for (int k = 0; k < MP; ++k) nd[j] += cov[j][k] * dir[k];
                nrm += nd[j] * nd[j];
            }
            nrm = std::sqrt(nrm);
            if (!(nrm > 0)) break;
            for (int j = 0; j < MP; ++j) dir[j] = nd[j] / nrm;
        }
    }

    void split(int64_t b, int64_t e, int depth) {
        const int64_t cnt = e - b;
        if (cnt <= leaf) return;
        const int64_t nleaves = (cnt + leaf - 1) / leaf;
        double dir[MP];
        direction(b, e, dir);
        std::vector<std::pair<double, int32_t>> key((size_t)cnt);
        for (int64_t i = 0; i < cnt; ++i) {
            const float* p = proj + (int64_t)idx[b + i] * MP;
            double v = 0;
            for (int j = 0; j < MP; ++j) v += dir[j] * p[j];
            key[(size_t)i] = {v, idx[b + i]};
        }
        std::sort(key.begin(), key.end());
        for (int64_t i = 0; i < cnt; ++i) idx[b + i] = key[(size_t)i].second;
        // candidate cuts after j whole leaves, j in the middle 60 %
        int64_t jlo = std::max<int64_t>(1, (nleaves * 2) / 10);
        int64_t jhi = std::min<int64_t>(nleaves - 1, nleaves - (nleaves * 2) / 10);
        if (jhi < jlo) jlo = jhi = nleaves / 2;
        int64_t best = nleaves / 2;
        double gap = -1;
        for (int64_t j = jlo; j <= jhi; ++j) {
            const int64_t p = j * leaf;
            if (p <= 0 || p >= cnt) continue;
            const double g = key[(size_t)p].first - key[(size_t)p - 1].first;
            if (g > gap) { gap = g; best = j; }
        }
        const int64_t mid = b + best * leaf;
        key.clear();
        key.shrink_to_fit();
        if (depth < 4 && cnt > 200000) {
            std::thread left([&] { split(b, mid, depth + 1); });
            split(mid, e, depth + 1);
            left.join();
        } else {
            split(b, mid, depth + 1);
            split(mid, e, depth + 1);
        }
    }
};

}  // namespace

void build_tree(const float* proj, int64_t n, int leaf_size, int fanout,
                int num_pivots, HostTree* out) {
    HostTree& T = *out;
    const int s = num_pivots;

    // ---- pivots: farthest-point selection, started from the point farthest
    // from the centroid (ties by smallest id)
    T.pivots.assign((size_t)s * MP, 0.f);
    if (s > 0) {
        double cen[MP] = {0};
        for (int64_t i = 0; i < n; ++i)
            for (int j = 0; j < MP; ++j) cen[j] += proj[i * MP + j];
        float cf[MP];
        for (int j = 0; j < MP; ++j) cf[j] = (float)(cen[j] / (double)n);
        std::vector<double> mind(n, std::numeric_limits<double>::infinity());
        int64_t pick = 0;
        double best = -1;
        for (int64_t i = 0; i < n; ++i) {
            double dd = dist64(proj + i * MP, cf);
            if (dd > best) { best = dd; pick = i; }
        }
        for (int p = 0; p < s; ++p) {
            std::copy(proj + pick * MP, proj + pick * MP + MP, T.pivots.begin() + (size_t)p * MP);
            int64_t next = 0;
            double far = -1;
            for (int64_t i = 0; i < n; ++i) {
                double dd = dist64(proj + i * MP, proj + pick * MP);
                if (dd < mind[i]) mind[i] = dd;
                if (mind[i] > far) { far = mind[i]; next = i; }
            }
            pick = next;
        }
    }

    // ---- leaf order by recursive median splits
    T.perm.resize(n);
    std::iota(T.perm.begin(), T.perm.end(), 0);
    Splitter sp{proj, leaf_size, T.perm};
    sp.split(0, n, 0);

    // ---- level sizes, bottom-up; stored top-down
    std::vector<int64_t> sizes;  // bottom-up node counts
    int64_t cnt = (n + leaf_size - 1) / leaf_size;
    sizes.push_back(cnt);
    while (cnt > fanout) {
        cnt = (cnt + fanout - 1) / fanout;
        sizes.push_back(cnt);
    }
    T.levels = (int)sizes.size();
    T.level_begin.assign(T.levels + 1, 0);
    for (int l = 0; l < T.levels; ++l)
        T.level_begin[l + 1] = T.level_begin[l] + sizes[T.levels - 1 - l];
    T.n_nodes = T.level_begin[T.levels];
    const int64_t N = T.n_nodes;
    T.centre.assign((size_t)MP * N, 0.f);
    T.radius.assign(N, 0.f);
    T.hr_min.assign((size_t)std::max(s, 1) * N, 0.f);
    T.hr_max.assign((size_t)std::max(s, 1) * N, 0.f);
    T.child_begin.assign(N, 0);
    T.child_end.assign(N, 0);
    T.npts.assign(N, 0);

    // point range [p0, p1) of every node, in leaf order
    std::vector<int64_t> p0(N), p1(N);
    for (int l = T.levels - 1; l >= 0; --l) {
        const int64_t lb = T.level_begin[l], le = T.level_begin[l + 1];
        const int64_t group = [&] {
            int64_t g = leaf_size;
            for (int u = T.levels - 1; u > l; --u) g *= fanout;
            return g;
        }();
        for (int64_t i = lb; i < le; ++i) {
            const int64_t j = i - lb;
            p0[i] = j * group;
            p1[i] = std::min<int64_t>(n, (j + 1) * group);
            T.npts[i] = (int32_t)(p1[i] - p0[i]);
            if (l == T.levels - 1) {
                T.child_begin[i] = (int32_t)p0[i];
                T.child_end[i] = (int32_t)p1[i];
            } else {
                const int64_t cb = T.level_begin[l + 1] + j * fanout;
                const int64_t ce = std::min<int64_t>(T.level_begin[l + 2], cb + fanout);
                T.child_begin[i] = (int32_t)cb;
                T.child_end[i] = (int32_t)ce;
            }
        }
    }

    // ---- node summaries
    const std::vector<int32_t>& perm = T.perm;
    parallel_for(N, [&](int64_t i) {
        double cen[MP] = {0};
        for (int64_t q = p0[i]; q < p1[i]; ++q) {
            const float* p = proj + (int64_t)perm[q] * MP;
            for (int j = 0; j < MP; ++j) cen[j] += p[j];
        }
        float cf[MP];
        const double c = (double)(p1[i] - p0[i]);
        for (int j = 0; j < MP; ++j) cf[j] = (float)(cen[j] / c);
        double rad = 0, lo[PMLSH_MAX_PIVOTS], hi[PMLSH_MAX_PIVOTS];
        for (int t = 0; t < s; ++t) { lo[t] = std::numeric_limits<double>::infinity(); hi[t] = 0; }
        for (int64_t q = p0[i]; q < p1[i]; ++q) {
            const float* p = proj + (int64_t)perm[q] * MP;
            rad = std::max(rad, dist64(p, cf));
            for (int t = 0; t < s; ++t) {
                double dd = dist64(p, &T.pivots[(size_t)t * MP]);
                lo[t] = std::min(lo[t], dd);
                hi[t] = std::max(hi[t], dd);
            }
        }
        for (int j = 0; j < MP; ++j) T.centre[(size_t)j * N + i] = cf[j];
        T.radius[i] = round_up(rad);
        for (int t = 0; t < s; ++t) {
            T.hr_min[(size_t)t * N + i] = round_down(lo[t]);
            T.hr_max[(size_t)t * N + i] = round_up(hi[t]);
        }
    });

    double maxnorm = 0, pivnorm = 0;
    for (int64_t i = 0; i < n; ++i) {
        double s2 = 0;
        for (int j = 0; j < MP; ++j) s2 += (double)proj[i * MP + j] * proj[i * MP + j];
        maxnorm = std::max(maxnorm, s2);
    }
    for (int t = 0; t < s; ++t) {
        double s2 = 0;
        for (int j = 0; j < MP; ++j) s2 += (double)T.pivots[(size_t)t * MP + j] * T.pivots[(size_t)t * MP + j];
        pivnorm = std::max(pivnorm, s2);
    }
    T.coord_scale = (float)(std::sqrt(maxnorm) + std::sqrt(pivnorm));
}

}  // namespace pmlsh
