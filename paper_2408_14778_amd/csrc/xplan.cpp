// Execution plan builder (see xplan.hpp).
#include "xplan.hpp"

#include <algorithm>
#include <limits>
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
    P.chance_base.resize(P.C);
    P.chance_k.resize(P.C);
    for (int64_t i = 0; i < P.C; ++i) {
        const int32_t hc = L.node_infoset[P.canon_of[P.chance_nodes[i]]];
        P.chance_base[i] = static_cast<int32_t>(L.Qp + L.cq_offset[hc]);
        P.chance_k[i] = L.cq_offset[hc + 1] - L.cq_offset[hc];
    }
    P.chance_prob = L.chance_prob;
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
    build_chunks(P);
    return CFR_OK;
}

void build_chunks(const std::vector<int32_t>& hlo, const std::vector<int32_t>& mo,
                  const int32_t* per_level, std::vector<int32_t>& chunk_first,
                  std::vector<int32_t>& k_level_offset) {
    const int32_t D = static_cast<int32_t>(hlo.size()) - 2;
    chunk_first.clear();
    k_level_offset.assign(D + 2, 0);
    for (int32_t l = 0; l <= D; ++l) {
        const int32_t cap = per_level != nullptr ? per_level[l] : kChunk;
        k_level_offset[l] = static_cast<int32_t>(chunk_first.size());
        int32_t h = hlo[l];
        const int32_t hend = hlo[l + 1];
        while (h < hend) {
            chunk_first.push_back(h);
            int32_t members = mo[h + 1] - mo[h];
            int32_t count = 1;
            ++h;
            if (members > cap) continue;  // a large infoset alone
            while (h < hend && count < cap) {
                const int32_t m = mo[h + 1] - mo[h];
                if (members + m > cap) break;
                members += m;
                ++count;
                ++h;
            }
        }
    }
    k_level_offset[D + 1] = static_cast<int32_t>(chunk_first.size());
    chunk_first.push_back(hlo[D + 1]);
}

void build_chunks(ExecPlan& P, const int32_t* per_level) {
    build_chunks(P.h_level_offset, P.member_offset, per_level, P.chunk_first, P.k_level_offset);
}

int build_forest_plan(const std::vector<ExecPlan>& G, ExecPlan& F, std::string& err) {
    F = ExecPlan();
    const size_t n = G.size();
    if (n == 0) {
        err = "empty batch";
        return CFR_EINVAL;
    }
    int32_t D = 0;
    int64_t N = 0, Hp = 0, Qp = 0, Q0 = 0, M = 0, Lc = 0, C = 0;
    for (const ExecPlan& P : G) {
        D = std::max(D, P.D);
        N += P.N; Hp += P.Hp; Qp += P.Qp; Q0 += P.Q0; M += P.M; Lc += P.L; C += P.C;
    }
    if (N >= std::numeric_limits<int32_t>::max() || Qp + Q0 >= std::numeric_limits<int32_t>::max()) {
        err = "batch exceeds the int32 index range";
        return CFR_EINVAL;
    }
    F.N = N; F.D = D; F.Hp = Hp; F.Qp = Qp; F.Q0 = Q0; F.M = M; F.L = Lc; F.C = C;
    auto lvl = [](const ExecPlan& P, int32_t l, const std::vector<int32_t>& off) {
        return l <= P.D ? off[l + 1] - off[l] : 0;
    };
    // level offsets and per-(game, level) bases for nodes, infosets, chance nodes
    std::vector<std::vector<int64_t>> nb(n, std::vector<int64_t>(D + 1)), hb = nb, cb = nb;
    F.level_offset.assign(D + 2, 0);
    F.h_level_offset.assign(D + 2, 0);
    F.c_level_offset.assign(D + 2, 0);
    int64_t pos = 0, hpos = 0, cpos = 0;
    for (int32_t l = 0; l <= D; ++l) {
        F.level_offset[l] = static_cast<int32_t>(pos);
        F.h_level_offset[l] = static_cast<int32_t>(hpos);
        F.c_level_offset[l] = static_cast<int32_t>(cpos);
        for (size_t g = 0; g < n; ++g) {
            nb[g][l] = pos;
            hb[g][l] = hpos;
            cb[g][l] = cpos;
            pos += lvl(G[g], l, G[g].level_offset);
            hpos += lvl(G[g], l, G[g].h_level_offset);
            cpos += lvl(G[g], l, G[g].c_level_offset);
        }
    }
    F.level_offset[D + 1] = static_cast<int32_t>(pos);
    F.h_level_offset[D + 1] = static_cast<int32_t>(hpos);
    F.c_level_offset[D + 1] = static_cast<int32_t>(cpos);
    // node and infoset maps of every game into the forest
    std::vector<std::vector<int32_t>> node_map(n), h_map(n);
    for (size_t g = 0; g < n; ++g) {
        const ExecPlan& P = G[g];
        node_map[g].resize(P.N);
        h_map[g].resize(P.Hp);
        for (int32_t l = 0; l <= P.D; ++l) {
            for (int32_t x = P.level_offset[l]; x < P.level_offset[l + 1]; ++x)
                node_map[g][x] = static_cast<int32_t>(nb[g][l] + (x - P.level_offset[l]));
            for (int32_t h = P.h_level_offset[l]; h < P.h_level_offset[l + 1]; ++h)
                h_map[g][h] = static_cast<int32_t>(hb[g][l] + (h - P.h_level_offset[l]));
        }
    }
    // forest infosets in forest order: pair offsets, players, members
    std::vector<int32_t> h_game(Hp), h_local(Hp);
    for (size_t g = 0; g < n; ++g)
        for (int64_t h = 0; h < G[g].Hp; ++h) {
            h_game[h_map[g][h]] = static_cast<int32_t>(g);
            h_local[h_map[g][h]] = static_cast<int32_t>(h);
        }
    F.q_offset.assign(Hp + 1, 0);
    F.member_offset.assign(Hp + 1, 0);
    F.infoset_player.resize(Hp);
    F.infoset_canon.resize(Hp);
    for (int64_t h = 0; h < Hp; ++h) {
        const ExecPlan& P = G[h_game[h]];
        const int32_t hl = h_local[h];
        F.q_offset[h + 1] = F.q_offset[h] + (P.q_offset[hl + 1] - P.q_offset[hl]);
        F.member_offset[h + 1] = F.member_offset[h] + (P.member_offset[hl + 1] - P.member_offset[hl]);
        F.infoset_player[h] = P.infoset_player[hl];
        F.infoset_canon[h] = static_cast<int32_t>(h);
    }
    // pair maps: forest pair of (game, local pair); batch input order = concatenated inputs
    std::vector<int64_t> in_base(n + 1, 0), q0_base(n + 1, 0);
    for (size_t g = 0; g < n; ++g) {
        in_base[g + 1] = in_base[g] + G[g].Qp;
        q0_base[g + 1] = q0_base[g] + G[g].Q0;
    }
    std::vector<std::vector<int32_t>> q_map(n);
    for (size_t g = 0; g < n; ++g) q_map[g].resize(G[g].Qp);
    F.q_input.resize(Qp);
    F.members.resize(M);
    for (int64_t h = 0; h < Hp; ++h) {
        const int32_t g = h_game[h];
        const ExecPlan& P = G[g];
        const int32_t hl = h_local[h];
        for (int32_t a = 0; a < P.q_offset[hl + 1] - P.q_offset[hl]; ++a) {
            q_map[g][P.q_offset[hl] + a] = F.q_offset[h] + a;
            F.q_input[F.q_offset[h] + a] = static_cast<int32_t>(in_base[g] + P.q_input[P.q_offset[hl] + a]);
        }
        for (int32_t m = 0; m < P.member_offset[hl + 1] - P.member_offset[hl]; ++m)
            F.members[F.member_offset[h] + m] = node_map[g][P.members[P.member_offset[hl] + m]];
    }
    // per-node arrays
    F.parent.resize(N);
    F.edge.resize(N);
    F.meta.resize(N);
    F.child_begin.assign(N, 0);
    F.child_stride.assign(N, 0);
    F.payoff.resize(N);
    F.canon_of.resize(N);
    F.child_list.reserve(Lc);
    int64_t node_base = 0;
    for (size_t g = 0; g < n; ++g) {
        const ExecPlan& P = G[g];
        const int64_t list_base = static_cast<int64_t>(F.child_list.size());
        for (int64_t x = 0; x < P.N; ++x) {
            const int32_t f = node_map[g][x];
            F.parent[f] = P.parent[x] < 0 ? -1 : node_map[g][P.parent[x]];
            const int32_t e = P.edge[x];
            F.edge[f] = e < 0 ? -1
                        : e < P.Qp ? q_map[g][e]
                                   : static_cast<int32_t>(Qp + q0_base[g] + (e - P.Qp));
            F.meta[f] = P.meta[x];
            F.payoff[f] = P.payoff[x];
            F.canon_of[f] = static_cast<int32_t>(node_base + P.canon_of[x]);
            if ((P.meta[x] & 3) == 0) continue;
            if (P.child_stride[x] != 0) {
                // children at c0 + a * stride in the game map to the same pattern in the forest:
                // a game's level is contiguous in the forest level
                F.child_begin[f] = node_map[g][P.child_begin[x]];
                F.child_stride[f] = P.child_stride[x];
            } else {
                F.child_begin[f] = static_cast<int32_t>(list_base + P.child_begin[x]);
                F.child_stride[f] = 0;
            }
        }
        for (int32_t c : P.child_list) F.child_list.push_back(node_map[g][c]);
        node_base += P.N;
    }
    // chance units, chance probabilities
    F.chance_nodes.resize(C);
    F.chance_base.resize(C);
    F.chance_k.resize(C);
    for (size_t g = 0; g < n; ++g) {
        const ExecPlan& P = G[g];
        for (int32_t l = 0; l <= P.D; ++l)
            for (int32_t i = P.c_level_offset[l]; i < P.c_level_offset[l + 1]; ++i) {
                const int64_t fi = cb[g][l] + (i - P.c_level_offset[l]);
                F.chance_nodes[fi] = node_map[g][P.chance_nodes[i]];
                F.chance_base[fi] = static_cast<int32_t>(Qp + q0_base[g] + (P.chance_base[i] - P.Qp));
                F.chance_k[fi] = P.chance_k[i];
            }
        F.chance_prob.insert(F.chance_prob.end(), P.chance_prob.begin(), P.chance_prob.end());
        F.n_blocks += P.n_blocks;
        F.n_listed += P.n_listed;
    }
    build_chunks(F);
    return CFR_OK;
}

}  // namespace cfr
