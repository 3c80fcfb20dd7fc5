// Host bulk-load of the PM-tree over projected points (Section 4.1).
//
// The paper builds its PM-tree by inserting points one at a time and
// splitting overflowing nodes (Section 6.3, "Promote Methods"). Here the
// whole point set is known up front, so the tree is bulk-loaded:
//   * global pivots p_1..p_s by farthest-point selection (the paper only asks
//     for pivots that keep the node regions small);
//   * leaves by recursive gap-aware splits along each node's principal
//     direction (computed on the device, bulkload.hip), the left part always
//     holding a whole number of leaves, so every leaf has exactly leaf_size
//     points except the last one;
//   * inner levels from the binary split tree: level l holds the maximal
//     subtrees with at most fanout^(H-1-l) leaves, so inner nodes are compact
//     regions and the fanout is about `fanout` (not exactly).
// Every node stores what Eq. 5 and Eq. 11 need: a centre e.RO (the mean of
// its points, rounded to FP32), the covering radius e.r about that centre and
// the hyper-ring e.HR[i] = [min, max] distance of its points to pivot i, all
// computed in FP64 from the FP32 coordinates the kernels read and rounded
// outward, so the node tests never reject a node that holds a point the
// kernels would accept.

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace pmlsh {
namespace {

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

}  // namespace

void build_tree(const float* proj, int64_t n, int leaf_size, int fanout, int num_pivots,
                std::vector<int32_t> perm_in, const int32_t* perm_dev,
                const std::vector<SplitNode>& bt, hipStream_t st, HostTree* out) {
    HostTree& T = *out;
    const int s = num_pivots;

    // ---- pivots: farthest-point selection, started from the point farthest
    // from the centroid (ties by smallest id), on the device
    double maxnorm = 0.0;
    device_pivots(proj, n, s, st, &T.pivots, &maxnorm);

    // ---- leaf order and binary split tree (leaf ranges) of the recursive
    // gap-aware splits; the inner levels are derived from the split tree
    T.perm = std::move(perm_in);
    const int64_t n_leaves = (n + leaf_size - 1) / leaf_size;

    // Level l (of H) holds the maximal binary subtrees with at most
    // fanout^(H-1-l) leaves, left to right: compact regions, nested in the
    // level above, each a contiguous range of leaves. H is the smallest depth
    // whose top level has at most `fanout` nodes.
    auto level_nodes = [&](int64_t cap) {
        std::vector<std::pair<int64_t, int64_t>> out;   // leaf ranges
        std::vector<int32_t> stack{0};
        while (!stack.empty()) {
            const SplitNode& b = bt[stack.back()];
            stack.pop_back();
            if (b.leaf_end - b.leaf_begin <= cap || b.left < 0) {
                out.push_back({b.leaf_begin, b.leaf_end});
            } else {
                stack.push_back(b.right);
                stack.push_back(b.left);
            }
        }
        return out;
    };
    std::vector<int64_t> caps{1};                    // bottom-up
    while (true) {
        const int64_t cap = caps.back();
        if (cap >= n_leaves || (int64_t)level_nodes(cap).size() <= fanout) break;
        caps.push_back(cap * fanout);
    }
    T.levels = (int)caps.size();
    std::vector<std::vector<std::pair<int64_t, int64_t>>> lv(T.levels);
    for (int l = 0; l < T.levels; ++l) lv[l] = level_nodes(caps[T.levels - 1 - l]);
    T.level_begin.assign(T.levels + 1, 0);
    for (int l = 0; l < T.levels; ++l) T.level_begin[l + 1] = T.level_begin[l] + (int64_t)lv[l].size();
    T.n_nodes = T.level_begin[T.levels];
    const int64_t N = T.n_nodes;
    T.centre.assign((size_t)MP * N, 0.f);
    T.radius.assign(N, 0.f);
    T.hr_min.assign((size_t)std::max(s, 1) * N, 0.f);
    T.hr_max.assign((size_t)std::max(s, 1) * N, 0.f);
    T.child_begin.assign(N, 0);
    T.child_end.assign(N, 0);
    T.npts.assign(N, 0);

    // point range [p0, p1) of every node, in leaf order; children are the
    // nodes of the next level inside the node's leaf range
    std::vector<int64_t> p0(N), p1(N);
    for (int l = 0; l < T.levels; ++l) {
        size_t c = 0;   // cursor into the next level
        for (size_t j = 0; j < lv[l].size(); ++j) {
            const int64_t i = T.level_begin[l] + (int64_t)j;
            const int64_t lb = lv[l][j].first, le = lv[l][j].second;
            p0[i] = lb * leaf_size;
            p1[i] = std::min<int64_t>(n, le * leaf_size);
            T.npts[i] = (int32_t)(p1[i] - p0[i]);
            if (l == T.levels - 1) {
                T.child_begin[i] = (int32_t)p0[i];
                T.child_end[i] = (int32_t)p1[i];
            } else {
                const std::vector<std::pair<int64_t, int64_t>>& nx = lv[l + 1];
                const size_t c0 = c;
                while (c < nx.size() && nx[c].second <= le) ++c;
                T.child_begin[i] = (int32_t)(T.level_begin[l + 1] + (int64_t)c0);
                T.child_end[i] = (int32_t)(T.level_begin[l + 1] + (int64_t)c);
            }
        }
    }

    // ---- node summaries (device reductions over each node's points)
    std::vector<float> cen;
    std::vector<double> rad, ring;
    device_ball_summaries(proj, perm_dev, p0, p1, T.pivots.data(), s, st, &cen, &rad, &ring);
    for (int64_t i = 0; i < N; ++i) {
        for (int j = 0; j < MP; ++j) T.centre[(size_t)j * N + i] = cen[(size_t)i * MP + j];
        T.radius[i] = round_up(rad[(size_t)i]);
        for (int t = 0; t < s; ++t) {
            T.hr_min[(size_t)t * N + i] = round_down(ring[(size_t)(i * 2 * s + 2 * t)]);
            T.hr_max[(size_t)t * N + i] = round_up(ring[(size_t)(i * 2 * s + 2 * t + 1)]);
        }
    }

    double pivnorm = 0;
    for (int t = 0; t < s; ++t) {
        double s2 = 0;
        for (int j = 0; j < MP; ++j) s2 += (double)T.pivots[(size_t)t * MP + j] * T.pivots[(size_t)t * MP + j];
        pivnorm = std::max(pivnorm, s2);
    }
    T.coord_scale = (float)(maxnorm + std::sqrt(pivnorm));
}

}  // namespace pmlsh
