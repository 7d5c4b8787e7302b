// Execution plan builder (see xplan.hpp).
#include "xplan.hpp"

#include <algorithm>
#include <numeric>
#include <tuple>

#include "../../include/cfr.h"

namespace cfr {

namespace {

struct DisjointSets {
    std::vector<int32_t> up;
    explicit DisjointSets(int64_t n) : up(n) { std::iota(up.begin(), up.end(), 0); }
    int32_t find(int32_t x) {
        while (up[x] != x) {
            up[x] = up[up[x]];
            x = up[x];
        }
        return x;
    }
    void unite(int32_t a, int32_t b) {
        a = find(a);
        b = find(b);
        if (a == b) return;
        if (a < b) std::swap(a, b);
        up[a] = b;  // the smaller id represents the set
    }
};

}  // namespace

int build_exec_plan(const Layout& L, ExecPlan& P, std::string& err) {
    if (!L.level_pure) {
        err = "the public-block plan needs level-pure infosets";
        return CFR_ELEVEL;
    }
    const int64_t N = L.N;
    const int32_t D = L.D;
    P = ExecPlan();
    P.N = N; P.D = D; P.Hp = L.Hp; P.Qp = L.Qp; P.Q0 = L.Q0;
    P.level_offset = L.level_offset;
    auto action_of = [&](int64_t c) { return static_cast<int32_t>(c - L.child_begin[L.parent[c]]); };

    DisjointSets ds(N);
    // (a) members of an infoset
    for (int64_t h = 0; h < L.Hp; ++h)
        for (int32_t m = L.member_offset[h] + 1; m < L.member_offset[h + 1]; ++m)
            ds.unite(L.members[L.member_offset[h]], L.members[m]);
    // (b) parents of a block share a block, deepest level first
    {
        std::vector<int32_t> stamp(N, -1), rep(N, -1);
        for (int32_t l = D; l >= 1; --l)
            for (int32_t v = L.level_offset[l]; v < L.level_offset[l + 1]; ++v) {
                const int32_t r = ds.find(v);
                if (stamp[r] != l) {
                    stamp[r] = l;
                    rep[r] = L.parent[v];
                } else {
                    ds.unite(rep[r], L.parent[v]);
                }
            }
    }
    // (c) children by one action of a block of rational-player nodes share a block
    {
        std::vector<std::tuple<int32_t, int32_t, int32_t>> keys;
        for (int32_t l = 1; l <= D; ++l) {
            keys.clear();
            for (int32_t v = L.level_offset[l]; v < L.level_offset[l + 1]; ++v) {
                const int32_t p = L.parent[v];
                if (L.node_player[p] >= 1) keys.emplace_back(ds.find(p), action_of(v), v);
            }
            std::sort(keys.begin(), keys.end());
            for (size_t i = 1; i < keys.size(); ++i)
                if (std::get<0>(keys[i]) == std::get<0>(keys[i - 1]) &&
                    std::get<1>(keys[i]) == std::get<1>(keys[i - 1]))
                    ds.unite(std::get<2>(keys[i - 1]), std::get<2>(keys[i]));
        }
    }

    // blocks per level, ordered by (parent block rank, smallest action, first canonical node)
    P.exec_of.assign(N, -1);
    P.canon_of.assign(N, -1);
    std::vector<int32_t> block_of_root(N, -1), rank_of_node(N, -1);
    struct Block {
        int32_t root, first, min_action, parent_rank, rank;
    };
    std::vector<Block> blocks;
    std::vector<int32_t> order, count;
    for (int32_t l = 0; l <= D; ++l) {
        blocks.clear();
        const int32_t lo = L.level_offset[l], hi = L.level_offset[l + 1];
        for (int32_t v = lo; v < hi; ++v) {
            const int32_t r = ds.find(v);
            int32_t& b = block_of_root[r];
            const int32_t act = l == 0 ? 0 : action_of(v);
            if (b < 0) {
                b = static_cast<int32_t>(blocks.size());
                const int32_t pr = l == 0 ? -1 : rank_of_node[L.parent[v]];
                blocks.push_back({r, v, act, pr, 0});
            } else if (act < blocks[b].min_action) {
                blocks[b].min_action = act;
            }
        }
        order.resize(blocks.size());
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
            const Block& a = blocks[x];
            const Block& b = blocks[y];
            return std::tie(a.parent_rank, a.min_action, a.first) <
                   std::tie(b.parent_rank, b.min_action, b.first);
        });
        for (size_t i = 0; i < order.size(); ++i) blocks[order[i]].rank = static_cast<int32_t>(i);
        P.n_blocks += static_cast<int64_t>(blocks.size());
        // stable counting sort of the level's nodes by block rank
        count.assign(blocks.size() + 1, 0);
        for (int32_t v = lo; v < hi; ++v) ++count[blocks[block_of_root[ds.find(v)]].rank + 1];
        for (size_t i = 1; i < count.size(); ++i) count[i] += count[i - 1];
        for (int32_t v = lo; v < hi; ++v) {
            const int32_t rk = blocks[block_of_root[ds.find(v)]].rank;
            const int32_t x = lo + count[rk]++;
            P.exec_of[v] = x;
            P.canon_of[x] = v;
            rank_of_node[v] = rk;
        }
    }

    // exec infosets: first appearance in exec order (contiguous per level and per block)
    std::vector<int32_t> xh_of_h(L.Hp, -1);
    P.h_level_offset.assign(D + 2, 0);
    P.c_level_offset.assign(D + 2, 0);
    for (int32_t l = 0; l <= D; ++l) {
        P.h_level_offset[l] = static_cast<int32_t>(P.infoset_canon.size());
        P.c_level_offset[l] = static_cast<int32_t>(P.chance_nodes.size());
        for (int32_t x = L.level_offset[l]; x < L.level_offset[l + 1]; ++x) {
            const int32_t c = P.canon_of[x];
            if (L.node_player[c] >= 1) {
                const int32_t h = L.node_infoset[c];
                if (xh_of_h[h] < 0) {
                    xh_of_h[h] = static_cast<int32_t>(P.infoset_canon.size());
                    P.infoset_canon.push_back(h);
                }
            } else if (L.node_player[c] == 0) {
                P.chance_nodes.push_back(x);
            }
        }
    }
    P.h_level_offset[D + 1] = static_cast<int32_t>(P.infoset_canon.size());
    P.c_level_offset[D + 1] = static_cast<int32_t>(P.chance_nodes.size());
    P.C = static_cast<int64_t>(P.chance_nodes.size());
    if (static_cast<int64_t>(P.infoset_canon.size()) != L.Hp) {
        err = "exec plan lost infosets";
        return CFR_EINVAL;
    }
    P.q_offset.assign(L.Hp + 1, 0);
    P.infoset_player.resize(L.Hp);
    for (int64_t hx = 0; hx < L.Hp; ++hx) {
        const int32_t h = P.infoset_canon[hx];
        P.q_offset[hx + 1] = P.q_offset[hx] + (L.q_offset[h + 1] - L.q_offset[h]);
        P.infoset_player[hx] = L.infoset_player[h];
    }
    P.q_input.resize(L.Qp);
    for (int64_t hx = 0; hx < L.Hp; ++hx) {
        const int32_t h = P.infoset_canon[hx];
        for (int32_t a = 0; a < P.q_offset[hx + 1] - P.q_offset[hx]; ++a)
            P.q_input[P.q_offset[hx] + a] = L.q_input[L.q_offset[h] + a];
    }
    // members in exec order
    P.member_offset.assign(L.Hp + 1, 0);
    for (int64_t hx = 0; hx < L.Hp; ++hx) {
        const int32_t h = P.infoset_canon[hx];
        P.member_offset[hx + 1] = P.member_offset[hx] + (L.member_offset[h + 1] - L.member_offset[h]);
    }
    P.members.resize(P.member_offset[L.Hp]);
    P.M = static_cast<int64_t>(P.members.size());
    {
        std::vector<int32_t> fill(P.member_offset.begin(), P.member_offset.end() - 1);
        for (int64_t x = 0; x < N; ++x) {
            const int32_t c = P.canon_of[x];
            if (L.node_player[c] >= 1) P.members[fill[xh_of_h[L.node_infoset[c]]]++] = static_cast<int32_t>(x);
        }
    }

    // per-node arrays
    P.parent.resize(N);
    P.edge.resize(N);
    P.meta.resize(N);
    P.child_begin.assign(N, 0);
    P.child_stride.assign(N, 0);
    P.payoff.resize(N);
    for (int64_t x = 0; x < N; ++x) {
        const int32_t c = P.canon_of[x];
        const int32_t cp = L.parent[c];
        P.parent[x] = cp < 0 ? -1 : P.exec_of[cp];
        P.payoff[x] = L.payoff[c];
        const int kind = L.node_player[c] + 1;
        const int actor = cp < 0 ? 0 : L.node_player[cp] + 1;
        P.meta[x] = static_cast<int8_t>(kind | (actor << 2));
        if (cp < 0) {
            P.edge[x] = -1;
        } else if (L.node_player[cp] >= 1) {
            P.edge[x] = P.q_offset[xh_of_h[L.node_infoset[cp]]] + (c - L.child_begin[cp]);
        } else {
            P.edge[x] = L.node_edge[c];  // chance pairs keep the canonical numbering after Q_+
        }
        const int32_t k = L.child_begin[c + 1] - L.child_begin[c];
        if (k == 0) continue;
        const int32_t e0 = P.exec_of[L.child_begin[c]];
        bool regular = true;
        int32_t d = 1;
        if (k > 1) {
            d = P.exec_of[L.child_begin[c] + 1] - e0;
            regular = d != 0;
            for (int32_t a = 2; a < k && regular; ++a)
                regular = P.exec_of[L.child_begin[c] + a] == e0 + a * d;
        }
        if (regular) {
            P.child_begin[x] = e0;
            P.child_stride[x] = d;
        } else {
            P.child_begin[x] = static_cast<int32_t>(P.child_list.size());
            P.child_stride[x] = 0;
            for (int32_t a = 0; a < k; ++a) P.child_list.push_back(P.exec_of[L.child_begin[c] + a]);
            ++P.n_listed;
        }
    }
    P.L = static_cast<int64_t>(P.child_list.size());
    return CFR_OK;
}

}  // namespace cfr
