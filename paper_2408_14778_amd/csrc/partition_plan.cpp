// Host plan of the subtree-partitioned iteration (no HIP): see partition_plan.hpp.
#include "partition_plan.hpp"

#include <algorithm>

#include "../../include/cfr.h"

namespace cfr {

namespace {

// The canonical layout's children of a consecutive node range are a consecutive range of the next
// level (child_begin is one monotone array over all nodes), so the descendants of the level-cut
// range [x, y) at level l are [down(x, l), down(y, l)).
int64_t down(const Layout& L, int64_t x, int32_t from, int32_t to) {
    for (int32_t l = from; l < to; ++l) x = L.child_begin[x];
    return x;
}

}  // namespace

int plan_partitions(const Layout& L, int32_t cut, int64_t max_window, PartPlan& P, std::string& err) {
    const int32_t D = L.D;
    if (D < 2 || cut < 1 || cut > D - 1) {
        err = "cut level must lie in 1 .. depth - 1 (depth " + std::to_string(D) + ")";
        return CFR_EINVAL;
    }
    if (max_window < 1) {
        err = "max_window_nodes must be positive";
        return CFR_EINVAL;
    }
    P = PartPlan{};
    P.cut = cut;
    P.D = D;
    const int64_t c0 = L.level_offset[cut], c1 = L.level_offset[cut + 1];
    P.base = c1;
    P.total = L.N - c1;
    // window nodes of each level-cut subtree
    std::vector<int64_t> size(c1 - c0, 0);
    for (int64_t v = c0; v < c1; ++v) {
        int64_t x = v, y = v + 1;
        for (int32_t l = cut + 1; l <= D; ++l) {
            x = L.child_begin[x];
            y = L.child_begin[y];
            size[v - c0] += y - x;
        }
    }
    // greedy: consecutive subtrees while the window stays within max_window
    int64_t acc = 0;
    for (int64_t v = c0; v < c1; ++v) {
        const int64_t s = size[v - c0];
        // a subtree with no nodes below the cut (a terminal level-cut node) never opens one
        if (P.a.empty() || (acc > 0 && s > 0 && acc + s > max_window)) {
            if (!P.a.empty()) P.b.push_back(static_cast<int32_t>(v));
            P.a.push_back(static_cast<int32_t>(v));
            acc = 0;
        }
        acc += s;
    }
    P.b.push_back(static_cast<int32_t>(c1));
    P.parts = static_cast<int32_t>(P.a.size());
    const int32_t nl = D - cut;  // window levels cut + 1 .. D
    P.off.assign(P.parts + 1, 0);
    P.lo.assign(static_cast<size_t>(P.parts) * (nl + 1), 0);
    P.patch_off.assign(P.parts + 1, 0);
    P.parent.resize(P.total);
    P.infoset.resize(P.total);
    P.edge.resize(P.total);
    P.player.resize(P.total);
    P.value0.resize(P.total);
    P.child_begin.resize(P.total + P.parts);
    P.patch.resize(static_cast<size_t>(c1 - c0) + P.parts);
    const bool f64 = !L.payoff64.empty();
    std::vector<int64_t> g_lo(D + 2), g_hi(D + 2), off(D + 2);
    for (int32_t p = 0; p < P.parts; ++p) {
        const int64_t a = P.a[p], b = P.b[p];
        int64_t w = 0;
        for (int32_t l = cut + 1; l <= D; ++l) {
            g_lo[l] = down(L, a, cut, l);
            g_hi[l] = down(L, b, cut, l);
            off[l] = w;
            w += g_hi[l] - g_lo[l];
        }
        off[D + 1] = w;
        P.window = std::max(P.window, w);
        P.off[p + 1] = P.off[p] + w;
        for (int32_t l = cut + 1; l <= D + 1; ++l)
            P.lo[static_cast<size_t>(p) * (nl + 1) + (l - cut - 1)] = static_cast<int32_t>(P.base + off[l]);
        const int64_t o = P.off[p];
        int32_t* cb = P.child_begin.data() + o + p;
        for (int32_t l = cut + 1; l <= D; ++l) {
            for (int64_t g = g_lo[l]; g < g_hi[l]; ++g) {
                const int64_t i = off[l] + (g - g_lo[l]);
                const int32_t par = L.parent[g];
                P.parent[o + i] = l == cut + 1
                                      ? par
                                      : static_cast<int32_t>(P.base + off[l - 1] + (par - g_lo[l - 1]));
                cb[i] = l < D ? static_cast<int32_t>(P.base + off[l + 1] +
                                                     (L.child_begin[g] - g_lo[l + 1]))
                              : static_cast<int32_t>(P.base + w);
                P.player[o + i] = L.node_player[g];
                P.infoset[o + i] = L.node_infoset[g];
                P.edge[o + i] = L.node_edge[g];
                P.value0[o + i] = L.node_player[g] < 0 ? (f64 ? L.payoff64[g] : L.payoff[g]) : 0.0;
            }
        }
        cb[w] = static_cast<int32_t>(P.base + w);
        // the level-cut nodes' children in the window, and the end of the last one's
        P.patch_off[p + 1] = P.patch_off[p] + (b - a + 1);
        for (int64_t j = 0; j <= b - a; ++j)
            P.patch[P.patch_off[p] + j] =
                static_cast<int32_t>(P.base + (L.child_begin[a + j] - g_lo[cut + 1]));
    }
    P.patch.resize(P.patch_off[P.parts]);
    return CFR_OK;
}

}  // namespace cfr
