// Execution plan builder (see xplan.hpp).
#include "xplan.hpp"

#include <algorithm>
#include <cstring>
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

int build_exec_plan(const Layout& L, ExecPlan& P, std::string& err, bool deep) {
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

    // blocks of every level: first canonical node, smallest action into them, parent block
    struct Block {
        int32_t level, first, min_action, parent, nodes, dec, rank, lo;
        int32_t pairs, members;  // pairs of its infosets, members of its largest infoset
        int32_t ch, kids;        // chance nodes, and their children
        int32_t tier;            // 0: outside every pack
        bool df, root;           // in a pack; the highest block of its pack
    };
    std::vector<Block> blocks;
    std::vector<int32_t> block_of_root(N, -1), block_of(N, -1);
    std::vector<int32_t> level_block(D + 2, 0);
    for (int32_t l = 0; l <= D; ++l) {
        level_block[l] = static_cast<int32_t>(blocks.size());
        for (int32_t v = L.level_offset[l]; v < L.level_offset[l + 1]; ++v) {
            const int32_t r = ds.find(v);
            int32_t& b = block_of_root[r];
            const int32_t act = l == 0 ? 0 : action_of(v);
            if (b < 0) {
                b = static_cast<int32_t>(blocks.size());
                const int32_t pb = l == 0 ? -1 : block_of[L.parent[v]];
                blocks.push_back({l, v, act, pb, 0, 0, 0, 0, 0, 0, 0, 0, 0, false, false});
            } else if (act < blocks[b].min_action) {
                blocks[b].min_action = act;
            }
            block_of[v] = b;
            ++blocks[b].nodes;
            blocks[b].dec += L.node_player[v] >= 0;
            if (L.node_player[v] == 0) {
                ++blocks[b].ch;
                blocks[b].kids += L.child_begin[v + 1] - L.child_begin[v];
            }
        }
    }
    level_block[D + 1] = static_cast<int32_t>(blocks.size());
    for (int64_t h = 0; h < L.Hp; ++h) {
        Block& b = blocks[block_of[L.members[L.member_offset[h]]]];
        b.members = std::max(b.members, L.member_offset[h + 1] - L.member_offset[h]);
        b.pairs += L.q_offset[h + 1] - L.q_offset[h];
    }
    // tiers (children blocks are created after their parents): in pass t, a block's subtree
    // counts its own decision nodes, pairs and levels and those of its children not yet in a
    // pack (blocks already in a pack are leaves of it); the highest unassigned blocks whose
    // subtree fits start packs of tier t, and the unassigned blocks below them join
    if (deep && L.max_actions <= 4) {
        const size_t nb = blocks.size();
        std::vector<int64_t> red_dec(nb), red_pairs(nb), red_ch(nb), red_kids(nb);
        std::vector<int32_t> red_depth(nb), red_members(nb);
        for (int32_t t = 1; t <= kMaxTiers; ++t) {
            for (size_t b = 0; b < nb; ++b) {
                red_dec[b] = blocks[b].dec;
                red_pairs[b] = blocks[b].pairs;
                red_ch[b] = blocks[b].ch;
                red_kids[b] = blocks[b].kids;
                red_depth[b] = 1;
                red_members[b] = blocks[b].members;
            }
            for (int64_t b = static_cast<int64_t>(nb) - 1; b >= 0; --b) {
                const int32_t p = blocks[b].parent;
                if (p < 0 || blocks[b].tier != 0 || blocks[b].dec == 0) continue;
                red_dec[p] += red_dec[b];
                red_pairs[p] += red_pairs[b];
                red_ch[p] += red_ch[b];
                red_kids[p] += red_kids[b];
                red_depth[p] = std::max(red_depth[p], red_depth[b] + 1);
                red_members[p] = std::max(red_members[p], red_members[b]);
            }
            int64_t added = 0, left = 0;
            std::vector<char> in_t(nb, 0);
            for (size_t b = 0; b < nb; ++b) {
                Block& bk = blocks[b];
                if (bk.tier != 0 || bk.dec == 0) continue;
                const bool parent_in = bk.parent >= 0 && in_t[bk.parent];
                const bool fits = red_dec[b] <= kPackDec && red_pairs[b] <= kPackPairs &&
                                  red_ch[b] <= kPackChance && red_kids[b] <= kPackKids &&
                                  red_depth[b] <= kPackLevels && red_members[b] <= kPackSubMembers;
                if (parent_in || fits) {
                    in_t[b] = 1;
                    bk.tier = t;
                    bk.root = !parent_in;
                    ++added;
                }
            }
            for (const Block& bk : blocks) left += bk.tier == 0 && bk.dec > 0;
            P.n_tiers = t;
            if (added == 0) --P.n_tiers;
            if (added == 0 || left == 0) break;
        }
        // blocks of terminals go with their parent block, so that a node's children keep a
        // stride (they are never a pack's work)
        for (Block& bk : blocks)
            if (bk.dec == 0 && bk.parent >= 0) bk.tier = blocks[bk.parent].tier;
        for (Block& bk : blocks) bk.df = bk.tier != 0;
    }
    // order per level: blocks outside the packs first, then (parent block rank, smallest
    // action, first canonical node); the packs' records name their nodes explicitly, so a
    // pack's blocks need not be adjacent, and a block's children stay together
    P.exec_of.assign(N, -1);
    P.canon_of.assign(N, -1);
    P.up_end.assign(D + 1, 0);
    std::vector<int32_t> order;
    for (int32_t l = 0; l <= D; ++l) {
        const int32_t b0 = level_block[l], b1 = level_block[l + 1];
        order.resize(b1 - b0);
        std::iota(order.begin(), order.end(), b0);
        auto key = [&](const Block& b) {
            return std::make_tuple(b.df ? 1 : 0, b.parent < 0 ? -1 : blocks[b.parent].rank,
                                   b.min_action, b.first);
        };
        std::sort(order.begin(), order.end(),
                  [&](int32_t x, int32_t y) { return key(blocks[x]) < key(blocks[y]); });
        int32_t pos = L.level_offset[l];
        P.up_end[l] = pos;
        for (size_t i = 0; i < order.size(); ++i) {
            Block& b = blocks[order[i]];
            b.rank = static_cast<int32_t>(i);
            b.lo = pos;
            pos += b.nodes;
            if (!b.df) P.up_end[l] = pos;
        }
        P.n_blocks += b1 - b0;
        // nodes in block order, canonical order inside a block
        std::vector<int32_t> fill(b1 - b0);
        for (int32_t b = b0; b < b1; ++b) fill[b - b0] = blocks[b].lo;
        for (int32_t v = L.level_offset[l]; v < L.level_offset[l + 1]; ++v) {
            const int32_t x = fill[block_of[v] - b0]++;
            P.exec_of[v] = x;
            P.canon_of[x] = v;
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

    // the prefix of each level outside the packs: its infosets and chance nodes come first too
    P.h_up_end.assign(D + 1, 0);
    P.c_up_end.assign(D + 1, 0);
    for (int32_t l = 0; l <= D; ++l) {
        int32_t h = P.h_level_offset[l];
        while (h < P.h_level_offset[l + 1] && P.members[P.member_offset[h]] < P.up_end[l]) ++h;
        P.h_up_end[l] = h;
        for (int32_t j = h; j < P.h_level_offset[l + 1]; ++j)
            if (P.members[P.member_offset[j]] < P.up_end[l]) {
                err = "exec plan: an infoset outside the packs follows one inside";
                return CFR_EINVAL;
            }
        int32_t c = P.c_level_offset[l];
        while (c < P.c_level_offset[l + 1] && P.chance_nodes[c] < P.up_end[l]) ++c;
        P.c_up_end[l] = c;
    }
    // packs: per tier, runs of consecutive pack-root blocks of one level whose subtrees fit
    // together (in exec order), then each pack's records
    if (P.n_tiers > 0) {
        const size_t nb = blocks.size();
        std::vector<std::vector<int32_t>> kids_of(nb);  // children blocks, in exec order
        for (int32_t l = 1; l <= D; ++l) {
            std::vector<int32_t> lv(level_block[l + 1] - level_block[l]);
            std::iota(lv.begin(), lv.end(), level_block[l]);
            std::sort(lv.begin(), lv.end(),
                      [&](int32_t x, int32_t y) { return blocks[x].rank < blocks[y].rank; });
            for (int32_t b : lv) kids_of[blocks[b].parent].push_back(b);
        }
        // subtree stats of pack blocks within their tier
        std::vector<int64_t> sub_dec(nb, 0), sub_pairs(nb, 0), sub_ch(nb, 0), sub_kids(nb, 0);
        std::vector<int32_t> sub_depth(nb, 0);
        for (int64_t b = static_cast<int64_t>(nb) - 1; b >= 0; --b) {
            if (!blocks[b].df || blocks[b].dec == 0) continue;
            sub_dec[b] += blocks[b].dec;
            sub_pairs[b] += blocks[b].pairs;
            sub_ch[b] += blocks[b].ch;
            sub_kids[b] += blocks[b].kids;
            sub_depth[b] = std::max(sub_depth[b], 1);
            const int32_t p = blocks[b].parent;
            if (p >= 0 && !blocks[b].root) {
                sub_dec[p] += sub_dec[b];
                sub_pairs[p] += sub_pairs[b];
                sub_ch[p] += sub_ch[b];
                sub_kids[p] += sub_kids[b];
                sub_depth[p] = std::max(sub_depth[p], sub_depth[b] + 1);
            }
        }
        std::vector<int32_t> infoset_of_exec(N, -1);
        for (int64_t hx = 0; hx < L.Hp; ++hx)
            for (int32_t m = P.member_offset[hx]; m < P.member_offset[hx + 1]; ++m)
                infoset_of_exec[P.members[m]] = static_cast<int32_t>(hx);
        std::vector<int32_t> chance_index(N, -1);
        for (int64_t i = 0; i < P.C; ++i) chance_index[P.chance_nodes[i]] = static_cast<int32_t>(i);
        std::vector<int32_t> nkids(N, 0);
        for (int64_t v = 0; v < N; ++v)
            if (P.parent[v] >= 0) ++nkids[P.parent[v]];
        auto child = [&](int32_t x, int32_t a) {
            return P.child_stride[x] != 0 ? P.child_begin[x] + a * P.child_stride[x]
                                          : P.child_list[P.child_begin[x] + a];
        };
        std::vector<int32_t> didx_of(N, -1);
        auto word = [](float f) {
            int32_t w;
            std::memcpy(&w, &f, 4);
            return w;
        };
        P.tier_offset.assign(1, 0);
        for (int32_t t = 1; t <= P.n_tiers; ++t) {
            // root blocks of tier t, level by level in exec order
            std::vector<int32_t> roots;
            for (int32_t l = 0; l <= D; ++l) {
                std::vector<int32_t> lv;
                for (int32_t b = level_block[l]; b < level_block[l + 1]; ++b)
                    if (blocks[b].tier == t && blocks[b].root) lv.push_back(b);
                std::sort(lv.begin(), lv.end(),
                          [&](int32_t x, int32_t y) { return blocks[x].rank < blocks[y].rank; });
                roots.insert(roots.end(), lv.begin(), lv.end());
            }
            size_t i = 0;
            while (i < roots.size()) {
                // a run of roots of one level within the caps
                size_t j = i;
                int64_t dec = 0, pairs = 0, chn = 0, kidn = 0;
                int32_t depth = 0;
                while (j < roots.size() && blocks[roots[j]].level == blocks[roots[i]].level &&
                       (j == i || (dec + sub_dec[roots[j]] <= kPackDec &&
                                   pairs + sub_pairs[roots[j]] <= kPackPairs &&
                                   chn + sub_ch[roots[j]] <= kPackChance &&
                                   kidn + sub_kids[roots[j]] <= kPackKids))) {
                    dec += sub_dec[roots[j]];
                    pairs += sub_pairs[roots[j]];
                    chn += sub_ch[roots[j]];
                    kidn += sub_kids[roots[j]];
                    depth = std::max(depth, sub_depth[roots[j]]);
                    ++j;
                }
                PackDesc pk{};
                pk.tier = t;
                pk.level0 = blocks[roots[i]].level;
                pk.nlv = depth;
                // the pack's blocks level by level, in exec order
                std::vector<std::vector<int32_t>> lv_blocks(depth);
                lv_blocks[0].assign(roots.begin() + i, roots.begin() + j);
                for (int32_t d = 0; d + 1 < depth; ++d)
                    for (int32_t b : lv_blocks[d])
                        for (int32_t c : kids_of[b])
                            if (blocks[c].tier == t && !blocks[c].root && blocks[c].dec > 0)
                                lv_blocks[d + 1].push_back(c);
                // decision nodes, members (by infoset), chance nodes and infosets per level
                std::vector<int32_t> dec_nodes, mem_nodes, ch_nodes, infs;
                for (int32_t d = 0; d < depth; ++d) {
                    pk.mlo[d] = static_cast<int32_t>(mem_nodes.size());
                    pk.clo[d] = static_cast<int32_t>(ch_nodes.size());
                    std::vector<int32_t> lv_inf;
                    for (int32_t b : lv_blocks[d])
                        for (int32_t x = blocks[b].lo; x < blocks[b].lo + blocks[b].nodes; ++x) {
                            if ((P.meta[x] & 3) == 0) continue;
                            didx_of[x] = static_cast<int32_t>(dec_nodes.size());
                            dec_nodes.push_back(x);
                            if ((P.meta[x] & 3) == 1) ch_nodes.push_back(x);
                            else if (lv_inf.empty() || lv_inf.back() != infoset_of_exec[x])
                                lv_inf.push_back(infoset_of_exec[x]);
                        }
                    std::sort(lv_inf.begin(), lv_inf.end());
                    lv_inf.erase(std::unique(lv_inf.begin(), lv_inf.end()), lv_inf.end());
                    for (int32_t h : lv_inf) {
                        infs.push_back(h);
                        for (int32_t m = P.member_offset[h]; m < P.member_offset[h + 1]; ++m)
                            mem_nodes.push_back(P.members[m]);
                    }
                }
                for (int32_t d = depth; d <= kPackLevels; ++d) {
                    pk.mlo[d] = static_cast<int32_t>(mem_nodes.size());
                    pk.clo[d] = static_cast<int32_t>(ch_nodes.size());
                }
                pk.n_dec = static_cast<int32_t>(dec_nodes.size());
                pk.n_mem = static_cast<int32_t>(mem_nodes.size());
                pk.n_ch = static_cast<int32_t>(ch_nodes.size());
                pk.n_inf = static_cast<int32_t>(infs.size());
                std::vector<int32_t>& B = P.pack_blob;
                auto align4 = [&]() {  // sections read as 16-byte records start 16-byte aligned
                    while (B.size() % 4 != 0) B.push_back(0);
                };
                auto kid_entry = [&](int32_t c, int32_t& kind) {
                    if (didx_of[c] >= 0) {
                        kind = 0;
                        return didx_of[c];
                    }
                    if ((P.meta[c] & 3) == 0) {
                        kind = 1;
                        return word(P.payoff[c]);
                    }
                    kind = 2;  // the root of a lower tier's pack
                    return c;
                };
                // roots: the decision nodes of the first level
                align4();
                pk.off_root = static_cast<int32_t>(B.size());
                for (int32_t b : lv_blocks[0])
                    for (int32_t x = blocks[b].lo; x < blocks[b].lo + blocks[b].nodes; ++x) {
                        if ((P.meta[x] & 3) == 0) continue;
                        B.push_back(didx_of[x] | ((P.meta[x] >> 2) & 3) << 16);
                        B.push_back(P.parent[x]);
                        B.push_back(P.edge[x]);
                        B.push_back(x);
                        ++pk.n_root;
                    }
                // infosets, with pack-local pair numbering
                pk.off_inf = static_cast<int32_t>(B.size());
                std::vector<int32_t> q_local_of(infs.size());
                int32_t ql = 0, mi = 0;
                for (size_t a = 0; a < infs.size(); ++a) {
                    const int32_t h = infs[a];
                    const int32_t k = P.q_offset[h + 1] - P.q_offset[h];
                    const int32_t nm = P.member_offset[h + 1] - P.member_offset[h];
                    q_local_of[a] = ql;
                    B.push_back(P.q_offset[h]);
                    B.push_back(ql);
                    B.push_back(mi | (mi + nm) << 16);
                    B.push_back(k | P.infoset_player[h] << 8);
                    ql += k;
                    mi += nm;
                }
                pk.n_pairs = ql;
                // members
                pk.off_mem = static_cast<int32_t>(B.size());
                for (size_t a = 0; a < infs.size(); ++a) {
                    const int32_t h = infs[a];
                    const int32_t k = P.q_offset[h + 1] - P.q_offset[h];
                    for (int32_t m = P.member_offset[h]; m < P.member_offset[h + 1]; ++m) {
                        const int32_t x = P.members[m];
                        int32_t w0 = didx_of[x] | k << 16 | (P.infoset_player[h] == 2 ? 1 << 19 : 0);
                        int32_t kidw[4] = {0, 0, 0, 0};
                        for (int32_t c = 0; c < k; ++c) {
                            int32_t kind;
                            kidw[c] = kid_entry(child(x, c), kind);
                            w0 |= kind << (24 + 2 * c);
                            if (kind == 2) w0 |= 1 << 20;
                        }
                        B.push_back(w0);
                        B.push_back(q_local_of[a]);
                        for (int32_t c = 0; c < 4; ++c) B.push_back(kidw[c]);
                    }
                }
                // chance nodes and their children
                align4();
                pk.off_ch = static_cast<int32_t>(B.size());
                int32_t nk = 0;
                for (int32_t x : ch_nodes) {
                    bool bnd = false;
                    for (int32_t c = 0; c < nkids[x]; ++c) bnd |= didx_of[child(x, c)] < 0 &&
                                                                  (P.meta[child(x, c)] & 3) != 0;
                    B.push_back(didx_of[x] | (bnd ? 1 << 20 : 0));
                    B.push_back(nkids[x]);
                    B.push_back(nk);
                    B.push_back(0);
                    nk += nkids[x];
                }
                pk.off_kid = static_cast<int32_t>(B.size());
                pk.n_kid = nk;
                for (int32_t x : ch_nodes) {
                    const int32_t ci = chance_index[x];
                    for (int32_t c = 0; c < nkids[x]; ++c) {
                        int32_t kind;
                        const int32_t e = kid_entry(child(x, c), kind);
                        B.push_back(e);
                        B.push_back(word(P.chance_prob[P.chance_base[ci] - L.Qp + c]));
                        B.push_back(kind);
                    }
                }
                // decision nodes' exec indices
                pk.off_node = static_cast<int32_t>(B.size());
                B.insert(B.end(), dec_nodes.begin(), dec_nodes.end());
                align4();
                for (int32_t x : dec_nodes) didx_of[x] = -1;
                P.packs.push_back(pk);
                i = j;
            }
            P.tier_offset.push_back(static_cast<int32_t>(P.packs.size()));
        }
    }
    build_chunks(P);
    return CFR_OK;
}

void upper_level_stats(const ExecPlan& P, std::vector<int64_t>& decision,
                       std::vector<int8_t>& only_terminal_children) {
    decision.assign(P.D + 1, 0);
    only_terminal_children.assign(P.D + 1, 1);
    std::vector<int32_t> nkids(P.N, 0);
    for (int64_t v = 0; v < P.N; ++v)
        if (P.parent[v] >= 0) ++nkids[P.parent[v]];  // a forest has a root per game
    for (int32_t l = 0; l <= P.D; ++l)
        for (int32_t v = P.level_offset[l]; v < P.up_end[l]; ++v) {
            if ((P.meta[v] & 3) == 0) continue;
            ++decision[l];
            for (int32_t a = 0; a < nkids[v]; ++a) {
                const int32_t ch = P.child_stride[v] != 0 ? P.child_begin[v] + a * P.child_stride[v]
                                                          : P.child_list[P.child_begin[v] + a];
                if ((P.meta[ch] & 3) != 0) only_terminal_children[l] = 0;
            }
        }
}

void build_chunks(const std::vector<int32_t>& hlo, const std::vector<int32_t>& mo,
                  const int32_t* per_level, std::vector<int32_t>& chunk_first,
                  std::vector<int32_t>& k_level_offset, const std::vector<int32_t>* h_split,
                  std::vector<int32_t>* k_split) {
    const int32_t D = static_cast<int32_t>(hlo.size()) - 2;
    chunk_first.clear();
    k_level_offset.assign(D + 2, 0);
    if (k_split != nullptr) k_split->assign(D + 1, 0);
    auto run = [&](int32_t h, int32_t hend, int32_t cap) {
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
    };
    for (int32_t l = 0; l <= D; ++l) {
        const int32_t cap = per_level != nullptr ? per_level[l] : kChunk;
        k_level_offset[l] = static_cast<int32_t>(chunk_first.size());
        const int32_t hs = h_split != nullptr ? (*h_split)[l] : hlo[l + 1];
        run(hlo[l], hs, cap);
        if (k_split != nullptr) (*k_split)[l] = static_cast<int32_t>(chunk_first.size());
        run(hs, hlo[l + 1], cap);
    }
    k_level_offset[D + 1] = static_cast<int32_t>(chunk_first.size());
    chunk_first.push_back(hlo[D + 1]);
}

void build_chunks(ExecPlan& P, const int32_t* per_level) {
    build_chunks(P.h_level_offset, P.member_offset, per_level, P.chunk_first, P.k_level_offset,
                 P.h_up_end.empty() ? nullptr : &P.h_up_end, &P.k_up_end);
}

int build_forest_plan(const std::vector<ExecPlan>& G, ExecPlan& F, std::string& err) {
    F = ExecPlan();
    const size_t n = G.size();
    if (n == 0) {
        err = "empty batch";
        return CFR_EINVAL;
    }
    int32_t D = 0;
    int64_t N = 0, Hp = 0, Qp = 0, Q0 = 0, M = 0, C = 0;
    for (const ExecPlan& P : G) {
        D = std::max(D, P.D);
        N += P.N; Hp += P.Hp; Qp += P.Qp; Q0 += P.Q0; M += P.M; C += P.C;
    }
    if (N >= std::numeric_limits<int32_t>::max() || Qp + Q0 >= std::numeric_limits<int32_t>::max()) {
        err = "batch exceeds the int32 index range";
        return CFR_EINVAL;
    }
    F.N = N; F.D = D; F.Hp = Hp; F.Qp = Qp; F.Q0 = Q0; F.M = M; F.C = C;
    // Forest level l: every game's upper prefix of level l (game order), then every game's
    // pack part of level l. seg(P, l, off, up, s): size of segment s (0 upper, 1 packs).
    auto seg = [](const ExecPlan& P, int32_t l, const std::vector<int32_t>& off,
                  const std::vector<int32_t>& up, int s) -> int64_t {
        if (l > P.D) return 0;
        return s == 0 ? up[l] - off[l] : off[l + 1] - up[l];
    };
    // per (game, level, segment) bases for nodes, infosets, chance nodes
    std::vector<std::vector<int64_t>> nb(n, std::vector<int64_t>(2 * (D + 1))), hb = nb, cb = nb;
    F.level_offset.assign(D + 2, 0);
    F.h_level_offset.assign(D + 2, 0);
    F.c_level_offset.assign(D + 2, 0);
    F.up_end.assign(D + 1, 0);
    F.h_up_end.assign(D + 1, 0);
    F.c_up_end.assign(D + 1, 0);
    int64_t pos = 0, hpos = 0, cpos = 0;
    for (int32_t l = 0; l <= D; ++l) {
        F.level_offset[l] = static_cast<int32_t>(pos);
        F.h_level_offset[l] = static_cast<int32_t>(hpos);
        F.c_level_offset[l] = static_cast<int32_t>(cpos);
        for (int s = 0; s < 2; ++s) {
            if (s == 1) {
                F.up_end[l] = static_cast<int32_t>(pos);
                F.h_up_end[l] = static_cast<int32_t>(hpos);
                F.c_up_end[l] = static_cast<int32_t>(cpos);
            }
            for (size_t g = 0; g < n; ++g) {
                const ExecPlan& P = G[g];
                nb[g][2 * l + s] = pos;
                hb[g][2 * l + s] = hpos;
                cb[g][2 * l + s] = cpos;
                pos += seg(P, l, P.level_offset, P.up_end, s);
                hpos += seg(P, l, P.h_level_offset, P.h_up_end, s);
                cpos += seg(P, l, P.c_level_offset, P.c_up_end, s);
            }
        }
    }
    F.level_offset[D + 1] = static_cast<int32_t>(pos);
    F.h_level_offset[D + 1] = static_cast<int32_t>(hpos);
    F.c_level_offset[D + 1] = static_cast<int32_t>(cpos);
    // node, infoset and chance-node maps of every game into the forest
    std::vector<std::vector<int32_t>> node_map(n), h_map(n), c_map(n);
    for (size_t g = 0; g < n; ++g) {
        const ExecPlan& P = G[g];
        node_map[g].resize(P.N);
        h_map[g].resize(P.Hp);
        c_map[g].resize(P.C);
        for (int32_t l = 0; l <= P.D; ++l) {
            for (int32_t x = P.level_offset[l]; x < P.level_offset[l + 1]; ++x)
                node_map[g][x] = static_cast<int32_t>(
                    x < P.up_end[l] ? nb[g][2 * l] + (x - P.level_offset[l])
                                    : nb[g][2 * l + 1] + (x - P.up_end[l]));
            for (int32_t h = P.h_level_offset[l]; h < P.h_level_offset[l + 1]; ++h)
                h_map[g][h] = static_cast<int32_t>(
                    h < P.h_up_end[l] ? hb[g][2 * l] + (h - P.h_level_offset[l])
                                      : hb[g][2 * l + 1] + (h - P.h_up_end[l]));
            for (int32_t c = P.c_level_offset[l]; c < P.c_level_offset[l + 1]; ++c)
                c_map[g][c] = static_cast<int32_t>(
                    c < P.c_up_end[l] ? cb[g][2 * l] + (c - P.c_level_offset[l])
                                      : cb[g][2 * l + 1] + (c - P.c_up_end[l]));
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
    // per-node arrays; children kept at a stride where the forest positions allow it (a node
    // whose children lie in both segments of its game's level is listed)
    F.parent.resize(N);
    F.edge.resize(N);
    F.meta.resize(N);
    F.child_begin.assign(N, 0);
    F.child_stride.assign(N, 0);
    F.payoff.resize(N);
    F.canon_of.resize(N);
    int64_t node_base = 0;
    std::vector<int32_t> kids;
    for (size_t g = 0; g < n; ++g) {
        const ExecPlan& P = G[g];
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
        }
        node_base += P.N;
    }
    // children in forest positions (in forest node order, so the child list is ordered too)
    {
        std::vector<int32_t> game_of(N), local_of(N);
        std::vector<std::vector<int32_t>> nchild(n);
        for (size_t g = 0; g < n; ++g) {
            nchild[g].assign(G[g].N, 0);
            for (int64_t x = 0; x < G[g].N; ++x) {
                game_of[node_map[g][x]] = static_cast<int32_t>(g);
                local_of[node_map[g][x]] = static_cast<int32_t>(x);
                if (G[g].parent[x] >= 0) ++nchild[g][G[g].parent[x]];
            }
        }
        for (int64_t f = 0; f < N; ++f) {
            const int32_t g = game_of[f];
            const ExecPlan& P = G[g];
            const int32_t x = local_of[f];
            if ((P.meta[x] & 3) == 0) continue;
            kids.clear();
            for (int32_t a = 0; a < nchild[g][x]; ++a) {
                const int32_t c = P.child_stride[x] != 0 ? P.child_begin[x] + a * P.child_stride[x]
                                                         : P.child_list[P.child_begin[x] + a];
                kids.push_back(node_map[g][c]);
            }
            bool regular = !kids.empty();
            int32_t d = kids.size() > 1 ? kids[1] - kids[0] : 1;
            regular = regular && d != 0;
            for (size_t a = 2; a < kids.size() && regular; ++a)
                regular = kids[a] == kids[0] + static_cast<int32_t>(a) * d;
            if (regular) {
                F.child_begin[f] = kids[0];
                F.child_stride[f] = d;
            } else {
                F.child_begin[f] = static_cast<int32_t>(F.child_list.size());
                F.child_stride[f] = 0;
                F.child_list.insert(F.child_list.end(), kids.begin(), kids.end());
                ++F.n_listed;
            }
        }
    }
    F.L = static_cast<int64_t>(F.child_list.size());
    // chance units, chance probabilities
    F.chance_nodes.resize(C);
    F.chance_base.resize(C);
    F.chance_k.resize(C);
    for (size_t g = 0; g < n; ++g) {
        const ExecPlan& P = G[g];
        for (int64_t i = 0; i < P.C; ++i) {
            const int64_t fi = c_map[g][i];
            F.chance_nodes[fi] = node_map[g][P.chance_nodes[i]];
            F.chance_base[fi] = static_cast<int32_t>(Qp + q0_base[g] + (P.chance_base[i] - P.Qp));
            F.chance_k[fi] = P.chance_k[i];
        }
        F.chance_prob.insert(F.chance_prob.end(), P.chance_prob.begin(), P.chance_prob.end());
        F.n_blocks += P.n_blocks;
    }
    // packs: tier by tier, every game's packs with their records' node, pair and edge indices
    // moved to forest positions
    for (const ExecPlan& P : G) F.n_tiers = std::max(F.n_tiers, P.n_tiers);
    F.tier_offset.assign(1, 0);
    for (int32_t t = 1; t <= F.n_tiers; ++t) {
        for (size_t g = 0; g < n; ++g) {
            const ExecPlan& P = G[g];
            if (t > P.n_tiers) continue;
            auto node = [&](int32_t x) { return x < 0 ? -1 : node_map[g][x]; };
            auto edge = [&](int32_t e) {
                return e < 0 ? -1
                       : e < P.Qp ? q_map[g][e]
                                  : static_cast<int32_t>(Qp + q0_base[g] + (e - P.Qp));
            };
            for (int32_t pi = P.tier_offset[t - 1]; pi < P.tier_offset[t]; ++pi) {
                const PackDesc& pk = P.packs[pi];
                PackDesc fp = pk;
                while (F.pack_blob.size() % 4 != 0) F.pack_blob.push_back(0);
                const int32_t base = static_cast<int32_t>(F.pack_blob.size());
                const int32_t shift = base - pk.off_root;  // a multiple of 4: alignment kept
                fp.off_root += shift;
                fp.off_mem += shift;
                fp.off_inf += shift;
                fp.off_ch += shift;
                fp.off_kid += shift;
                fp.off_node += shift;
                const int32_t end = pk.off_node + pk.n_dec;
                F.pack_blob.insert(F.pack_blob.end(), P.pack_blob.begin() + pk.off_root,
                                   P.pack_blob.begin() + end);
                int32_t* B = F.pack_blob.data();
                for (int32_t r = 0; r < pk.n_root; ++r) {
                    int32_t* w = B + fp.off_root + 4 * r;
                    w[1] = node(w[1]);
                    w[2] = edge(w[2]);
                    w[3] = node(w[3]);
                }
                for (int32_t h = 0; h < pk.n_inf; ++h) {
                    int32_t* w = B + fp.off_inf + 4 * h;
                    w[0] = q_map[g][w[0]];
                }
                for (int32_t m = 0; m < pk.n_mem; ++m) {
                    int32_t* w = B + fp.off_mem + 6 * m;
                    const int32_t k = (w[0] >> 16) & 7;
                    for (int32_t c = 0; c < k; ++c)
                        if (((w[0] >> (24 + 2 * c)) & 3) == 2) w[2 + c] = node(w[2 + c]);
                }
                for (int32_t c = 0; c < pk.n_kid; ++c) {
                    int32_t* w = B + fp.off_kid + 3 * c;
                    if (w[2] == 2) w[0] = node(w[0]);
                }
                for (int32_t d = 0; d < pk.n_dec; ++d) {
                    int32_t* w = B + fp.off_node + d;
                    w[0] = node(w[0]);
                }
                F.packs.push_back(fp);
            }
        }
        F.tier_offset.push_back(static_cast<int32_t>(F.packs.size()));
    }
    build_chunks(F);
    return CFR_OK;
}

}  // namespace cfr
