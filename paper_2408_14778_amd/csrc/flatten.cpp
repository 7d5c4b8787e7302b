// Host-side flattener (see flatten.hpp for the layout it emits).
#include "flatten.hpp"

#include <cmath>
#include <cstdio>
#include <limits>

namespace cfr {

namespace {

int fail(std::string& err, int code, const char* fmt, long long a = 0, long long b = 0) {
    char buf[256];
    std::snprintf(buf, sizeof buf, fmt, a, b);
    err = buf;
    return code;
}

// Shared validation + breadth-first ordering. Fills counts, the canonical order and
// the child-slot table; everything the two entry points need.
struct Work {
    std::vector<int64_t> child_off;  // N + 1, input-id indexed
    std::vector<int32_t> slot;       // child of (p, a) at child_off[p] + a
    std::vector<int32_t> order;      // canonical -> input
    std::vector<int32_t> level_offset;
};

int validate_and_order(const cfr_game& g, Work& w, std::string& err, int32_t max_player) {
    if (g.n_nodes < 1 || g.parent == nullptr || g.node_infoset == nullptr ||
        g.node_action == nullptr || g.payoff_u1 == nullptr)
        return fail(err, CFR_EINVAL, "game arrays must be non-null and n_nodes >= 1");
    if (g.n_nodes >= std::numeric_limits<int32_t>::max())
        return fail(err, CFR_EINVAL, "n_nodes %lld exceeds the int32 index range", g.n_nodes);
    if (g.n_infosets < 0 || (g.n_infosets > 0 && (g.infoset_player == nullptr ||
                                                  g.infoset_num_actions == nullptr)))
        return fail(err, CFR_EINVAL, "infoset arrays must be non-null");
    const int64_t n = g.n_nodes;
    const int32_t H = g.n_infosets;
    for (int32_t h = 0; h < H; ++h) {
        if (g.infoset_player[h] < 0 || g.infoset_player[h] > max_player)
            return fail(err, CFR_EINVAL,
                        "infoset %lld: player %lld is neither chance (0) nor a rational player",
                        h, g.infoset_player[h]);
        if (g.infoset_num_actions[h] < 1)
            return fail(err, CFR_EACTION, "infoset %lld has %lld actions", h,
                        g.infoset_num_actions[h]);
    }
    int64_t root = -1;
    std::vector<int64_t> nch(n, 0);
    for (int64_t v = 0; v < n; ++v) {
        const int32_t p = g.parent[v];
        if (p < 0) {
            if (root >= 0) return fail(err, CFR_ENOTTREE, "two roots: %lld and %lld", root, v);
            root = v;
        } else {
            if (p >= n || p == v) return fail(err, CFR_ENOTTREE, "node %lld: bad parent %lld", v, p);
            ++nch[p];
        }
    }
    if (root < 0) return fail(err, CFR_ENOTTREE, "no root (node with parent -1)");
    std::vector<uint8_t> used(H, 0);
    for (int64_t v = 0; v < n; ++v) {
        const int32_t h = g.node_infoset[v];
        if (nch[v] == 0) {
            if (h != -1)
                return fail(err, CFR_ENOTTREE, "node %lld has no children but infoset %lld", v, h);
        } else {
            if (h < 0 || h >= H)
                return fail(err, CFR_ENOTTREE, "decision node %lld has infoset %lld", v, h);
            if (nch[v] != g.infoset_num_actions[h])
                return fail(err, CFR_EACTION, "node %lld has %lld children, infoset needs more/less",
                            v, nch[v]);
            used[h] = 1;
        }
    }
    for (int32_t h = 0; h < H; ++h)
        if (!used[h]) return fail(err, CFR_EACTION, "infoset %lld has no node", h);

    w.child_off.assign(n + 1, 0);
    for (int64_t v = 0; v < n; ++v) w.child_off[v + 1] = w.child_off[v] + nch[v];
    w.slot.assign(w.child_off[n], -1);
    for (int64_t v = 0; v < n; ++v) {
        const int32_t p = g.parent[v];
        if (p < 0) {
            if (g.node_action[v] != -1)
                return fail(err, CFR_EACTION, "root %lld must have action -1 (has %lld)", v,
                            g.node_action[v]);
            continue;
        }
        const int32_t a = g.node_action[v];
        if (a < 0 || a >= nch[p])
            return fail(err, CFR_EACTION, "node %lld: action %lld out of range", v, a);
        int32_t& s = w.slot[w.child_off[p] + a];
        if (s >= 0) return fail(err, CFR_EACTION, "two children share parent %lld action %lld", p, a);
        s = static_cast<int32_t>(v);
    }
    // breadth-first order: a FIFO over the canonical array itself
    w.order.clear();
    w.order.reserve(n);
    w.order.push_back(static_cast<int32_t>(root));
    w.level_offset.assign(1, 0);
    size_t level_end = 1;
    w.level_offset.push_back(1);
    for (size_t i = 0; i < w.order.size(); ++i) {
        const int32_t v = w.order[i];
        for (int64_t k = w.child_off[v]; k < w.child_off[v + 1]; ++k) w.order.push_back(w.slot[k]);
        if (i + 1 == level_end && w.order.size() > level_end) {
            level_end = w.order.size();
            w.level_offset.push_back(static_cast<int32_t>(level_end));
        }
        if (w.order.size() > static_cast<size_t>(n)) break;
    }
    if (w.order.size() != static_cast<size_t>(n))
        return fail(err, CFR_ENOTTREE, "%lld of %lld nodes reachable from the root",
                    static_cast<long long>(w.order.size()), n);

    // chance probabilities
    int64_t pos = 0;
    for (int32_t h = 0; h < H; ++h) {
        if (g.infoset_player[h] != 0) continue;
        if (g.chance_prob == nullptr) return fail(err, CFR_EINVAL, "chance_prob is null");
        double sum = 0.0;
        for (int32_t a = 0; a < g.infoset_num_actions[h]; ++a) {
            const double p = g.chance_prob[pos + a];
            if (!(p >= 0.0) || !std::isfinite(p))
                return fail(err, CFR_ECHANCE, "chance infoset %lld action %lld: bad probability", h, a);
            sum += p;
        }
        if (std::fabs(sum - 1.0) > 1e-9)
            return fail(err, CFR_ECHANCE, "chance infoset %lld probabilities do not sum to 1", h);
        pos += g.infoset_num_actions[h];
    }
    for (int64_t v = 0; v < n; ++v) {
        if (nch[v] != 0) continue;
        const double u = g.payoff_u1[v];
        if (!std::isfinite(u)) return fail(err, CFR_EINVAL, "terminal %lld: payoff not finite", v);
        if (g.payoff_u2 != nullptr) {
            const double u2 = g.payoff_u2[v];
            if (!(std::fabs(u + u2) <= 1e-9 * std::fmax(1.0, std::fabs(u))))
                return fail(err, CFR_EZEROSUM, "terminal %lld: u1 + u2 != 0", v);
        }
    }
    return CFR_OK;
}

}  // namespace

int plan_sizes(const cfr_game& g, Layout& L, std::string& err, int32_t max_player) {
    Work w;
    const int rc = validate_and_order(g, w, err, max_player);
    if (rc != CFR_OK) return rc;
    L.N = g.n_nodes;
    L.D = static_cast<int32_t>(w.level_offset.size()) - 2;
    L.n_terminals = L.n_chance_nodes = L.n_members = 0;
    for (int64_t v = 0; v < g.n_nodes; ++v) {
        if (w.child_off[v + 1] == w.child_off[v]) ++L.n_terminals;
        else if (g.infoset_player[g.node_infoset[v]] == 0) ++L.n_chance_nodes;
        else ++L.n_members;
    }
    L.Hp = L.Qp = L.H0 = L.Q0 = 0;
    L.max_actions = 0;
    for (int32_t h = 0; h < g.n_infosets; ++h) {
        const int32_t k = g.infoset_num_actions[h];
        if (g.infoset_player[h] == 0) { ++L.H0; L.Q0 += k; }
        else { ++L.Hp; L.Qp += k; if (k > L.max_actions) L.max_actions = k; }
    }
    // level purity: depth of each infoset's members
    std::vector<int32_t> depth_of(g.n_infosets, -1);
    L.level_pure = true;
    for (int32_t l = 0; l + 1 < static_cast<int32_t>(w.level_offset.size()); ++l)
        for (int32_t i = w.level_offset[l]; i < w.level_offset[l + 1]; ++i) {
            const int32_t h = g.node_infoset[w.order[i]];
            if (h < 0 || g.infoset_player[h] == 0) continue;
            if (depth_of[h] < 0) depth_of[h] = l;
            else if (depth_of[h] != l) L.level_pure = false;
        }
    return CFR_OK;
}

int flatten(const cfr_game& g, Layout& L, std::string& err, bool f64, int32_t max_player) {
    Work w;
    int rc = validate_and_order(g, w, err, max_player);
    if (rc != CFR_OK) return rc;
    const int64_t n = g.n_nodes;
    const int32_t H = g.n_infosets;
    L = Layout();
    L.N = n;
    L.level_offset = w.level_offset;
    L.D = static_cast<int32_t>(L.level_offset.size()) - 2;
    L.node_id = w.order;
    std::vector<int32_t> canon(n);
    for (int64_t i = 0; i < n; ++i) canon[L.node_id[i]] = static_cast<int32_t>(i);

    // infoset numbering by first appearance
    std::vector<int32_t> rmap(H, -1), cmap(H, -1);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t h = g.node_infoset[L.node_id[i]];
        if (h < 0) continue;
        if (g.infoset_player[h] == 0) {
            if (cmap[h] < 0) { cmap[h] = static_cast<int32_t>(L.chance_id.size()); L.chance_id.push_back(h); }
        } else if (rmap[h] < 0) {
            rmap[h] = static_cast<int32_t>(L.infoset_id.size());
            L.infoset_id.push_back(h);
        }
    }
    L.Hp = static_cast<int64_t>(L.infoset_id.size());
    L.H0 = static_cast<int64_t>(L.chance_id.size());
    L.q_offset.assign(L.Hp + 1, 0);
    L.infoset_player.resize(L.Hp);
    L.max_actions = 0;
    for (int64_t h = 0; h < L.Hp; ++h) {
        const int32_t k = g.infoset_num_actions[L.infoset_id[h]];
        L.q_offset[h + 1] = L.q_offset[h] + k;
        L.infoset_player[h] = g.infoset_player[L.infoset_id[h]];
        if (k > L.max_actions) L.max_actions = k;
    }
    L.Qp = L.q_offset[L.Hp];
    L.cq_offset.assign(L.H0 + 1, 0);
    for (int64_t c = 0; c < L.H0; ++c)
        L.cq_offset[c + 1] = L.cq_offset[c] + g.infoset_num_actions[L.chance_id[c]];
    L.Q0 = L.cq_offset[L.H0];

    // input pair offsets (rational) and chance-probability offsets (chance), by input id
    std::vector<int64_t> in_qoff(H, 0), in_coff(H, 0);
    {
        int64_t q = 0, c = 0;
        for (int32_t h = 0; h < H; ++h) {
            if (g.infoset_player[h] == 0) { in_coff[h] = c; c += g.infoset_num_actions[h]; }
            else { in_qoff[h] = q; q += g.infoset_num_actions[h]; }
        }
    }
    L.q_input.resize(L.Qp);
    for (int64_t h = 0; h < L.Hp; ++h)
        for (int32_t a = 0; a < L.q_offset[h + 1] - L.q_offset[h]; ++a)
            L.q_input[L.q_offset[h] + a] = static_cast<int32_t>(in_qoff[L.infoset_id[h]] + a);
    L.chance_prob.resize(L.Q0);
    L.chance_prob64.resize(f64 ? L.Q0 : 0);
    for (int64_t c = 0; c < L.H0; ++c)
        for (int32_t a = 0; a < L.cq_offset[c + 1] - L.cq_offset[c]; ++a) {
            const double p = g.chance_prob[in_coff[L.chance_id[c]] + a];
            L.chance_prob[L.cq_offset[c] + a] = static_cast<float>(p);
            if (f64) L.chance_prob64[L.cq_offset[c] + a] = p;
        }

    // per-node arrays
    L.parent.resize(n);
    L.child_begin.resize(n + 1);
    L.node_player.resize(n);
    L.node_infoset.resize(n);
    L.node_edge.resize(n);
    L.payoff.resize(n);
    L.payoff64.assign(f64 ? n : 0, 0.0);
    int64_t next_child = 1;
    L.n_terminals = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t v = L.node_id[i];
        const int32_t p = g.parent[v];
        L.parent[i] = p < 0 ? -1 : canon[p];
        L.child_begin[i] = static_cast<int32_t>(next_child);
        const int64_t k = w.child_off[v + 1] - w.child_off[v];
        next_child += k;
        const int32_t h = g.node_infoset[v];
        if (k == 0) {
            L.node_player[i] = -1;
            L.node_infoset[i] = -1;
            L.payoff[i] = static_cast<float>(g.payoff_u1[v]);
            if (f64) L.payoff64[i] = g.payoff_u1[v];
            ++L.n_terminals;
        } else {
            L.node_player[i] = g.infoset_player[h];
            L.node_infoset[i] = g.infoset_player[h] == 0 ? cmap[h] : rmap[h];
            L.payoff[i] = 0.0f;
        }
    }
    L.child_begin[n] = static_cast<int32_t>(n);
    L.n_chance_nodes = 0;
    for (int64_t i = 0; i < n; ++i)
        if (L.node_player[i] == 0) ++L.n_chance_nodes;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t p = L.parent[i];
        if (p < 0) { L.node_edge[i] = -1; continue; }
        const int32_t a = g.node_action[L.node_id[i]];
        const int32_t hp = L.node_infoset[p];
        L.node_edge[i] = L.node_player[p] == 0
                             ? static_cast<int32_t>(L.Qp + L.cq_offset[hp] + a)
                             : L.q_offset[hp] + a;
    }

    // member lists (counting sort over canonical order keeps them ascending)
    L.member_offset.assign(L.Hp + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        if (L.node_player[i] >= 1) ++L.member_offset[L.node_infoset[i] + 1];
    for (int64_t h = 0; h < L.Hp; ++h) L.member_offset[h + 1] += L.member_offset[h];
    L.members.resize(L.member_offset[L.Hp]);
    L.n_members = static_cast<int64_t>(L.members.size());
    {
        std::vector<int32_t> fill(L.member_offset.begin(), L.member_offset.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            if (L.node_player[i] >= 1) L.members[fill[L.node_infoset[i]]++] = static_cast<int32_t>(i);
    }
    // level purity
    L.level_pure = true;
    {
        std::vector<int32_t> lvl(n);
        for (int32_t l = 0; l <= L.D; ++l)
            for (int32_t i = L.level_offset[l]; i < L.level_offset[l + 1]; ++i) lvl[i] = l;
        for (int64_t h = 0; h < L.Hp && L.level_pure; ++h)
            for (int32_t m = L.member_offset[h] + 1; m < L.member_offset[h + 1]; ++m)
                if (lvl[L.members[m]] != lvl[L.members[L.member_offset[h]]]) { L.level_pure = false; break; }
    }
    return CFR_OK;
}

}  // namespace cfr
