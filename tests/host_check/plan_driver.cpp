// Host-only driver of the planners, built by tests/test_host_sanitized.py with the address and
// undefined-behaviour sanitizers: flattens and plans every game of a file, reads every array of
// the host layout export, and plans the file's games as one batch (with and without subtree
// packs), exercising the same host code cfr_build and cfr_build_batch run before they touch a
// GPU; and cuts every game into subtree partitions at every level with several window sizes,
// checking each partition's window against the canonical layout (parents, child ranges, the
// level-cut nodes' patched child ranges, level offsets).
//
// File format (little endian): int32 n_games; per game: int64 n_nodes, int32 parent[n],
// int32 node_infoset[n], int32 node_action[n], int32 n_infosets, int8 infoset_player[h],
// int32 infoset_num_actions[h], int64 n_chance, double chance_prob[n_chance],
// double payoff_u1[n].
#include <cstdint>
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/cfr.h"
#include "../../paper_2408_14778_amd/csrc/flatten.hpp"
#include "../../paper_2408_14778_amd/csrc/host_plan.hpp"
#include "../../paper_2408_14778_amd/csrc/partition_plan.hpp"
#include "../../paper_2408_14778_amd/csrc/xplan.hpp"

namespace {
thread_local std::string g_err;
}

namespace cfr {
int set_error(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
}  // namespace cfr

extern "C" const char* cfr_last_error(void) { return g_err.c_str(); }

namespace {

struct GameData {
    std::vector<int32_t> parent, node_infoset, node_action, nact;
    std::vector<int8_t> player;
    std::vector<double> chance, payoff;
    cfr_game g{};
};

template <class T>
bool read(FILE* f, std::vector<T>& v, int64_t n) {
    v.resize(static_cast<size_t>(n));
    return n == 0 || std::fread(v.data(), sizeof(T), static_cast<size_t>(n), f) == static_cast<size_t>(n);
}

const char* kNames[] = {"level_offset", "node_id", "parent", "child_begin", "node_player",
                        "node_infoset", "node_edge", "infoset_id", "infoset_player", "q_offset",
                        "chance_id", "cq_offset", "member_offset", "members", "chance_prob",
                        "payoff", "q_input", "x_canon_of", "x_parent", "x_edge", "x_meta",
                        "x_child_begin", "x_child_stride", "x_child_list", "x_infoset_canon",
                        "x_q_offset", "x_member_offset", "x_members", "x_h_level_offset",
                        "x_chance_nodes", "x_c_level_offset", "x_q_input", "x_up_end",
                        "x_h_up_end", "x_c_up_end", "x_packs", "x_pack_blob", "x_tier_offset",
                        "x_level_offset"};

// Reads every array a host layout exports (names it does not hold report < 0); returns the
// number read.
int read_all(cfr_host_layout* h) {
    int n = 0;
    for (const char* name : kNames) {
        const int64_t b = cfr_host_layout_bytes(h, name);
        if (b < 0) continue;
        std::vector<unsigned char> buf(static_cast<size_t>(b));
        if (cfr_host_layout_get(h, name, buf.data(), b) != CFR_OK) return -1;
        ++n;
    }
    return n;
}

// The window of every partition against the canonical layout: the local id of a canonical node
// below the cut is found by walking the partition's level ranges independently of the plan.
// Returns the number of mismatches.
int64_t check_partitions(const cfr::Layout& L, const cfr::PartPlan& P) {
    int64_t bad = 0;
    const int32_t c = P.cut, D = L.D, nl = D - c;
    if (P.base != L.level_offset[c + 1]) ++bad;
    int64_t total = 0;
    for (int32_t p = 0; p < P.parts; ++p) {
        // canonical range of the partition at each level below the cut
        std::vector<int64_t> glo(D + 2), ghi(D + 2), off(D + 2);
        glo[c] = P.a[p];
        ghi[c] = P.b[p];
        int64_t w = 0;
        for (int32_t l = c + 1; l <= D; ++l) {
            glo[l] = L.child_begin[glo[l - 1]];
            ghi[l] = L.child_begin[ghi[l - 1]];
            off[l] = w;
            w += ghi[l] - glo[l];
        }
        if (P.off[p + 1] - P.off[p] != w) ++bad;
        total += w;
        auto loc = [&](int32_t l, int64_t g) { return P.base + off[l] + (g - glo[l]); };
        const int32_t* lo = P.lo.data() + static_cast<size_t>(p) * (nl + 1);
        for (int32_t l = c + 1; l <= D; ++l)
            if (lo[l - c - 1] != loc(l, glo[l])) ++bad;
        if (lo[nl] != P.base + w) ++bad;
        const int32_t* cb = P.child_begin.data() + P.off[p] + p;
        for (int32_t l = c + 1; l <= D; ++l) {
            for (int64_t g = glo[l]; g < ghi[l]; ++g) {
                const int64_t i = loc(l, g) - P.base, o = P.off[p] + i;
                const int64_t par = L.parent[g];
                if (P.parent[o] != (l == c + 1 ? par : loc(l - 1, par))) ++bad;
                if (P.player[o] != L.node_player[g] || P.infoset[o] != L.node_infoset[g] ||
                    P.edge[o] != L.node_edge[g])
                    ++bad;
                const int64_t k = L.child_begin[g + 1] - L.child_begin[g];
                if (cb[i + 1] - cb[i] != (l < D ? k : 0)) ++bad;
                if (l < D && k > 0 && cb[i] != loc(l + 1, L.child_begin[g])) ++bad;
                if ((L.node_player[g] < 0) != (k == 0)) ++bad;
            }
        }
        for (int64_t j = 0; j <= P.b[p] - P.a[p]; ++j) {
            const int64_t v = P.a[p] + j;
            if (P.patch[P.patch_off[p] + j] != loc(c + 1, L.child_begin[v])) ++bad;
        }
    }
    if (total != P.total || P.total != L.N - P.base) ++bad;
    return bad;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: plan_driver GAMES.bin\n");
        return 2;
    }
    FILE* f = std::fopen(argv[1], "rb");
    if (f == nullptr) return 2;
    int32_t n_games = 0;
    if (std::fread(&n_games, 4, 1, f) != 1 || n_games < 1) return 2;
    std::vector<GameData> games(static_cast<size_t>(n_games));
    for (GameData& d : games) {
        int64_t n = 0, nc = 0;
        int32_t h = 0;
        bool ok = std::fread(&n, 8, 1, f) == 1 && read(f, d.parent, n) && read(f, d.node_infoset, n) &&
                  read(f, d.node_action, n) && std::fread(&h, 4, 1, f) == 1 &&
                  read(f, d.player, h) && read(f, d.nact, h) && std::fread(&nc, 8, 1, f) == 1 &&
                  read(f, d.chance, nc) && read(f, d.payoff, n);
        if (!ok) return 2;
        if (d.chance.empty()) d.chance.push_back(0.0);
        d.g.n_nodes = n;
        d.g.parent = d.parent.data();
        d.g.node_infoset = d.node_infoset.data();
        d.g.node_action = d.node_action.data();
        d.g.n_infosets = h;
        d.g.infoset_player = d.player.data();
        d.g.infoset_num_actions = d.nact.data();
        d.g.chance_prob = d.chance.data();
        d.g.payoff_u1 = d.payoff.data();
        d.g.payoff_u2 = nullptr;
    }
    std::fclose(f);
    std::vector<cfr_game> gs;
    for (size_t i = 0; i < games.size(); ++i) {
        GameData& d = games[i];
        // a game of more than two rational players: flattened with its player bound (as the
        // general-sum build does) and partitioned; the public-block plan is for two players
        int32_t max_player = 2;
        for (int8_t pl : d.player) max_player = std::max<int32_t>(max_player, pl);
        int arrays = 0;
        if (max_player == 2) {
            gs.push_back(d.g);
            cfr_host_layout* h = nullptr;
            if (cfr_host_layout_create(&d.g, CFR_FLAG_SUBTREE_PACKS, &h) != CFR_OK) {
                std::printf("game %zu: %s\n", i, cfr_last_error());
                return 1;
            }
            arrays = read_all(h);
            cfr_host_layout_destroy(h);
        }
        // the per-level tables the solver derives from a plan, with and without packs
        cfr::Layout L;
        std::string err;
        if (cfr::flatten(d.g, L, err, false, max_player) != CFR_OK) {
            std::printf("game %zu: %s\n", i, err.c_str());
            return 1;
        }
        for (bool packs : {true, false}) {
            if (!L.level_pure || max_player > 2) break;
            cfr::ExecPlan P;
            if (cfr::build_exec_plan(L, P, err, packs) != CFR_OK) return 1;
            std::vector<int64_t> dec;
            std::vector<int8_t> only;
            cfr::upper_level_stats(P, dec, only);
        }
        int parts = 0;
        for (int32_t cut = 1; cut < L.D; ++cut)
            for (int64_t window : {int64_t{1}, int64_t{64}, int64_t{1} << 40}) {
                cfr::PartPlan PP;
                if (cfr::plan_partitions(L, cut, window, PP, err) != CFR_OK) return 1;
                const int64_t bad = check_partitions(L, PP);
                if (bad != 0) {
                    std::printf("game %zu cut %d window %lld: %lld mismatches\n", i, cut,
                                static_cast<long long>(window), static_cast<long long>(bad));
                    return 1;
                }
                parts += PP.parts;
            }
        std::printf("game %zu: %lld nodes, %d arrays, %d partitions checked\n", i,
                    static_cast<long long>(d.g.n_nodes), arrays, parts);
    }
    for (uint32_t flags : {0u, static_cast<uint32_t>(CFR_FLAG_SUBTREE_PACKS)}) {
        cfr_host_layout* h = nullptr;
        const int32_t n_batch = static_cast<int32_t>(gs.size());  // the two-player games
        if (cfr_host_layout_create_batch(gs.data(), n_batch, flags, &h) != CFR_OK) {
            std::printf("batch: %s\n", cfr_last_error());
            return 1;
        }
        const int arrays = read_all(h);
        cfr_host_layout_destroy(h);
        std::vector<cfr::ExecPlan> plans;
        int32_t max_actions = 0;
        std::string err;
        if (cfr::plan_games(gs.data(), n_batch, plans, max_actions, err, flags != 0) != CFR_OK) return 1;
        cfr::ExecPlan F;
        if (cfr::build_forest_plan(plans, F, err) != CFR_OK) return 1;
        std::vector<int64_t> dec;
        std::vector<int8_t> only;
        cfr::upper_level_stats(F, dec, only);
        std::printf("batch (flags %u): %d arrays, %zu packs, %d tiers\n", flags, arrays, F.packs.size(), F.n_tiers);
    }
    std::printf("ok\n");
    return 0;
}
