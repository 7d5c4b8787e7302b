// Host-side planning and the host-only layout export (cfr_host_layout_* in include/cfr.h).
// Plain C++: no HIP calls, so the planner can be built and checked on the host alone.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/cfr.h"
#include "flatten.hpp"
#include "host_plan.hpp"
#include "xplan.hpp"

namespace cfr {

// Flattens and plans every game on host threads; all must be level pure with <= 16 actions.
int plan_games(const cfr_game* games, int32_t n, std::vector<cfr::ExecPlan>& plans,
               int32_t& max_actions, std::string& err, bool packs) {
    plans.assign(n, cfr::ExecPlan());
    std::vector<int> codes(n, CFR_OK);
    std::vector<std::string> errs(n);
    std::vector<int32_t> maxa(n, 0);
    std::atomic<int32_t> next{0};
    bool deep = packs;
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto work = [&]() {
        for (int32_t g = next++; g < n; g = next++) {
            cfr::Layout L;
            int rc = cfr::flatten(games[g], L, errs[g]);
            if (rc == CFR_OK && !L.level_pure) {
                rc = CFR_ELEVEL;
                errs[g] = "an infoset spans several levels";
            }
            if (rc == CFR_OK && L.max_actions > 16) {
                rc = CFR_EINVAL;
                errs[g] = "more than 16 actions in an infoset";
            }
            if (rc == CFR_OK) rc = cfr::build_exec_plan(L, plans[g], errs[g], deep);
            maxa[g] = L.max_actions;
            codes[g] = rc;
        }
    };
    // subtree packs are instantiated for at most 4 actions per infoset, over the whole batch:
    // plan with them, and again without if a game has more actions
    for (int pass = 0; pass < 2; ++pass) {
        next = 0;
        std::vector<std::thread> pool;
        for (unsigned t = 0; t < std::min<unsigned>(hw, static_cast<unsigned>(n)); ++t)
            pool.emplace_back(work);
        for (auto& t : pool) t.join();
        max_actions = 0;
        for (int32_t g = 0; g < n; ++g) {
            if (codes[g] != CFR_OK) {
                err = "game " + std::to_string(g) + ": " + errs[g];
                return codes[g];
            }
            max_actions = std::max(max_actions, maxa[g]);
        }
        if (max_actions <= 4 || !deep) break;
        deep = false;
    }
    return CFR_OK;
}

}  // namespace cfr

struct cfr_host_layout {
    cfr::Layout L;
    cfr::ExecPlan P;
    bool has_plan = false;
    bool batch = false;  // a forest: plan arrays only
};

namespace {

// (pointer, bytes) of a named host layout array
std::pair<const void*, int64_t> host_array(const cfr::Layout& L, const std::string& n) {
    auto v = [](const auto& vec) {
        return std::pair<const void*, int64_t>(
            vec.data(), static_cast<int64_t>(vec.size() * sizeof(vec[0])));
    };
    if (n == "level_offset") return v(L.level_offset);
    if (n == "node_id") return v(L.node_id);
    if (n == "parent") return v(L.parent);
    if (n == "child_begin") return v(L.child_begin);
    if (n == "node_player") return v(L.node_player);
    if (n == "node_infoset") return v(L.node_infoset);
    if (n == "node_edge") return v(L.node_edge);
    if (n == "infoset_id") return v(L.infoset_id);
    if (n == "infoset_player") return v(L.infoset_player);
    if (n == "q_offset") return v(L.q_offset);
    if (n == "chance_id") return v(L.chance_id);
    if (n == "cq_offset") return v(L.cq_offset);
    if (n == "member_offset") return v(L.member_offset);
    if (n == "members") return v(L.members);
    if (n == "chance_prob") return v(L.chance_prob);
    if (n == "payoff") return v(L.payoff);
    if (n == "q_input") return v(L.q_input);
    return {nullptr, -1};
}

std::pair<const void*, int64_t> plan_array(const cfr::ExecPlan& P, const std::string& n) {
    auto v = [](const auto& vec) {
        return std::pair<const void*, int64_t>(
            vec.data(), static_cast<int64_t>(vec.size() * sizeof(vec[0])));
    };
    if (n == "x_canon_of") return v(P.canon_of);
    if (n == "x_parent") return v(P.parent);
    if (n == "x_edge") return v(P.edge);
    if (n == "x_meta") return v(P.meta);
    if (n == "x_child_begin") return v(P.child_begin);
    if (n == "x_child_stride") return v(P.child_stride);
    if (n == "x_child_list") return v(P.child_list);
    if (n == "x_infoset_canon") return v(P.infoset_canon);
    if (n == "x_q_offset") return v(P.q_offset);
    if (n == "x_member_offset") return v(P.member_offset);
    if (n == "x_members") return v(P.members);
    if (n == "x_h_level_offset") return v(P.h_level_offset);
    if (n == "x_chance_nodes") return v(P.chance_nodes);
    if (n == "x_c_level_offset") return v(P.c_level_offset);
    if (n == "x_q_input") return v(P.q_input);
    if (n == "x_up_end") return v(P.up_end);
    if (n == "x_h_up_end") return v(P.h_up_end);
    if (n == "x_c_up_end") return v(P.c_up_end);
    if (n == "x_packs") return v(P.packs);
    if (n == "x_pack_blob") return v(P.pack_blob);
    if (n == "x_tier_offset") return v(P.tier_offset);
    return {nullptr, -1};
}

std::pair<const void*, int64_t> any_array(const cfr_host_layout* h, const std::string& n) {
    if (n.rfind("x_", 0) == 0) {
        if (!h->has_plan) return {nullptr, -1};
        if (n == "x_level_offset") return {h->P.level_offset.data(),
                                           static_cast<int64_t>(h->P.level_offset.size() * 4)};
        return plan_array(h->P, n);
    }
    if (h->batch) return {nullptr, -1};
    return host_array(h->L, n);
}

}  // namespace

extern "C" {

int cfr_host_layout_create(const cfr_game* game, uint32_t flags, cfr_host_layout** out) {
    if (game == nullptr || out == nullptr) return cfr::set_error(CFR_EINVAL, "null argument");
    if (flags & ~static_cast<uint32_t>(CFR_FLAG_SUBTREE_PACKS))
        return cfr::set_error(CFR_EINVAL, "unknown flag bits");
    auto* h = new cfr_host_layout();
    std::string err;
    int rc = cfr::flatten(*game, h->L, err);
    if (rc != CFR_OK) {
        delete h;
        return cfr::set_error(rc, err);
    }
    if (h->L.level_pure) {
        rc = cfr::build_exec_plan(h->L, h->P, err, (flags & CFR_FLAG_SUBTREE_PACKS) != 0);
        if (rc != CFR_OK) {
            delete h;
            return cfr::set_error(rc, err);
        }
        h->has_plan = true;
    }
    *out = h;
    return CFR_OK;
}

int cfr_host_layout_create_batch(const cfr_game* games, int32_t n_games, uint32_t flags,
                                 cfr_host_layout** out) {
    if (games == nullptr || out == nullptr || n_games < 1)
        return cfr::set_error(CFR_EINVAL, "bad argument");
    if (flags & ~static_cast<uint32_t>(CFR_FLAG_SUBTREE_PACKS))
        return cfr::set_error(CFR_EINVAL, "unknown flag bits");
    std::vector<cfr::ExecPlan> plans;
    int32_t max_actions = 0;
    std::string err;
    int rc = cfr::plan_games(games, n_games, plans, max_actions, err,
                             (flags & CFR_FLAG_SUBTREE_PACKS) != 0);
    if (rc != CFR_OK) return cfr::set_error(rc, err);
    auto* h = new cfr_host_layout();
    rc = cfr::build_forest_plan(plans, h->P, err);
    if (rc != CFR_OK) {
        delete h;
        return cfr::set_error(rc, err);
    }
    h->has_plan = true;
    h->batch = true;
    *out = h;
    return CFR_OK;
}

int64_t cfr_host_layout_bytes(const cfr_host_layout* layout, const char* name) {
    if (layout == nullptr || name == nullptr) return CFR_EINVAL;
    const auto a = any_array(layout, name);
    return a.second < 0 ? CFR_EINVAL : a.second;
}

int cfr_host_layout_get(const cfr_host_layout* layout, const char* name, void* out, int64_t bytes) {
    if (layout == nullptr || name == nullptr) return cfr::set_error(CFR_EINVAL, "null argument");
    const auto a = any_array(layout, name);
    if (a.second < 0) return cfr::set_error(CFR_EINVAL, "unknown layout array");
    if (bytes != a.second || (bytes > 0 && out == nullptr)) return cfr::set_error(CFR_EINVAL, "wrong output size");
    if (bytes > 0) std::memcpy(out, a.first, static_cast<size_t>(bytes));
    return CFR_OK;
}

int cfr_host_layout_destroy(cfr_host_layout* layout) {
    delete layout;
    return CFR_OK;
}

}  // extern "C"
