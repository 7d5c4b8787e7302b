// C ABI of the library (include/cfr.h): planning, building, iterating, exports.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <cmath>
#include <cstring>
#include <thread>
#include <type_traits>
#include <utility>
#include <string>
#include <vector>

#include "../../include/cfr.h"
#include "../../include/cfr_warmstart.h"
#include "flatten.hpp"
#include "host_plan.hpp"
#include "mlp.hpp"
#include "kernels.hpp"
#include "partition.hpp"
#include "xkernels.hpp"
#include "xplan.hpp"

enum { ENGINE_NODE = 0, ENGINE_BLOCK = 1 };

struct cfr_solver {
    cfr::Dev dev{};
    cfr::Dev64 dev64{};  // fp64: the node engine's arrays in double precision (dev keeps the
                         // structure arrays, its real-valued pointers are null)
    bool fp64 = false;
    // subtree-partitioned, out-of-core solver (cfr_build_partitioned): the partitions' pinned
    // host windows (one of the two, by precision)
    std::unique_ptr<cfr::PartDev<float>> part32;
    std::unique_ptr<cfr::PartDev<double>> part64;
    bool partitioned() const { return part32 != nullptr || part64 != nullptr; }
    ~cfr_solver() {
        if (part32) part32->release();
        if (part64) part64->release();
    }
    cfr::XDev xdev{};
    int engine = ENGINE_NODE;
    int32_t n_games = 1;       // > 1: a batch (forest); canonical exports are unavailable
    bool canonical = true;     // the canonical layout arrays are on the device
    std::vector<int32_t> x_level_offset, x_h_level_offset, x_c_level_offset;
    cfr_launch_shape shape{};                    // launch shapes per bucket
    std::vector<int32_t> x_member_offset;        // host copy (chunk tables)
    std::vector<int32_t> x_k_level_offset, x_m_level_offset;
    std::vector<int32_t> up_threads, chunk_cap, chance_glog;  // per level
    std::vector<int8_t> x_meta;                                 // host copy (top-down tiles)
    std::vector<int32_t> reach_threads_l, reach_npt_l, t_level_offset;
    std::vector<int64_t> reach_units;  // upper decision nodes per level
    // upper prefixes per level (the parts outside the subtree packs) and per-level flags
    std::vector<int32_t> x_up_end, x_h_up_end, x_c_up_end, x_k_up_end, x_m_up_end;
    std::vector<int8_t> only_terminal_children;
    bool keep_nodes = false;  // the pack launches also store node values and reaches
    std::vector<int32_t> tier_offset;  // packs of each tier
    std::vector<int64_t> tier_dec;     // decision nodes of each tier
    cfr::UpdateRule rule;  // regret / average update (variant, linear weights, discounts)
    bool alternating = false;  // two passes per iteration: player 1, then player 2
    int32_t players = 0;  // general-sum game of n rational players (node engine), else 0
    bool use_graph = true;
    bool level_pure = true;
    int64_t T = 0;
    int64_t n_terminals = 0;
    int32_t max_actions = 0;
    std::vector<int32_t> level_offset;          // host copy, D + 2
    std::vector<int32_t> infoset_level_offset;  // host copy, D + 2
    hipStream_t stream = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

}  // namespace

namespace cfr {
int set_error(int code, const std::string& msg) { return set_err(code, msg); }
}  // namespace cfr

namespace {

int hip_err(hipError_t e, const char* what) {
    return set_err(CFR_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                            \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_err(e_, what); \
    } while (0)

// Bump allocator over the caller's workspace, 256-byte aligned pieces.
struct Carve {
    uintptr_t base;
    size_t off = 0;
    explicit Carve(void* p) : base(reinterpret_cast<uintptr_t>(p)) {}
    template <class T>
    T* take(int64_t count) {
        off = (off + 255) & ~size_t{255};
        T* p = reinterpret_cast<T*>(base + off);
        off += static_cast<size_t>(count > 0 ? count : 1) * sizeof(T);
        return p;
    }
};

// Sizes the device arrays depend on.
struct Sizes {
    int64_t N = 0, Hp = 0, Qp = 0, H0 = 0, Q0 = 0, M = 0, C = 0, L = 0;
    int64_t terminals = 0;
    int32_t D = 0, max_actions = 0;
    int engine = ENGINE_NODE;
    bool canonical = true;   // false for a batch: only the execution plan is on the device
    int32_t n_games = 1;
    bool packs = false;      // subtree packs (their records are on the device)
    bool fp64 = false;       // values, probabilities and state in double precision
    int32_t players = 0;     // general-sum game of n rational players (node engine), else 0
    // node engine: regret contributions may be stored per child and gathered per infoset (false:
    // always added by atomics, for the partitioned iteration's windows)
    bool gather = true;
};

// Bounds on the subtree packs of a plan over N nodes, M members, Hp infosets and C chance nodes
// with D + 1 levels: packs are cut greedily along each level of a tier, so two consecutive packs
// hold together more than 96 decision nodes and chance children (more than kPackDec = 512
// decision nodes, more than 384 pairs of at most 4 actions each, more than 128 chance nodes, or
// more than 1,024 chance children), so more than 48 nodes. Records: 4 words per root, infoset and chance node, 6 per member, 3 per chance
// child, 1 per decision node, and up to 3 words of alignment before each of 3 sections and
// after the last.
int64_t max_packs(int64_t N, int32_t D) {
    return 2 * N / 48 + int64_t{D + 1} * cfr::kMaxTiers + 1;
}
int64_t max_pack_words(int64_t N, int64_t M, int64_t Hp, int64_t C, int32_t D) {
    return 4 * N + 4 * Hp + 6 * M + 4 * C + 3 * N + N + 12 * max_packs(N, D);
}

int choose_engine(bool level_pure, int32_t max_actions, uint32_t flags) {
    if ((flags & (CFR_FLAG_NODE_ENGINE | CFR_FLAG_FP64)) != 0 || !level_pure || max_actions > 16)
        return ENGINE_NODE;
    return ENGINE_BLOCK;
}

// Lays out every device array; with base = nullptr it only measures. Canonical layout
// arrays are always present (they are exported); per-iteration state follows the engine.
size_t carve(cfr::Dev& d, cfr::Dev64& d64, cfr::XDev& x, void* base, const Sizes& z) {
    Carve c(base);
    const int64_t N = z.N, Hp = z.Hp, Qp = z.Qp, H0 = z.H0, Q0 = z.Q0, M = z.M;
    const int32_t D = z.D;
    d = cfr::Dev{};
    d64 = cfr::Dev64{};
    d.N = N; d.Hp = Hp; d.Qp = Qp; d.H0 = H0; d.Q0 = Q0; d.M = M; d.D = D;
    // payoff and value columns and reach planes: one per rational player (and chance's plane);
    // a two-player zero-sum game keeps u_1 only
    // regret contributions stored and gathered per infoset where atomics would contend: every
    // general-sum game (its kernels store them) and infosets of more than 16 members on average
    const bool store = z.gather && (z.players > 0 || M > 16 * Hp);
    const int64_t cols = z.players > 0 ? z.players : 1;
    const int64_t planes = (z.players > 0 ? z.players : 2) + 1;
    d.players = z.players;
    if (z.canonical) {
        d.parent = c.take<int32_t>(N);
        d.child_begin = c.take<int32_t>(N + 1);
        d.node_player = c.take<int8_t>(N);
        d.node_infoset = c.take<int32_t>(N);
        d.node_edge = c.take<int32_t>(N);
        d.node_id = c.take<int32_t>(N);
        d.level_offset = c.take<int32_t>(D + 2);
        d.infoset_id = c.take<int32_t>(Hp);
        d.infoset_player = c.take<int8_t>(Hp);
        d.q_offset = c.take<int32_t>(Hp + 1);
        d.chance_id = c.take<int32_t>(H0);
        d.cq_offset = c.take<int32_t>(H0 + 1);
        d.member_offset = c.take<int32_t>(Hp + 1);
        d.members = c.take<int32_t>(M);
        d.q_input = c.take<int32_t>(Qp);
        if (z.players > 0) {
            d.node_slot = c.take<int32_t>(N);
            d.slot_base = c.take<int32_t>(Hp + 1);
        }
    }
    // general-sum games store the contributions and own reaches in member order
    const int64_t n_contrib = z.players > 0 ? N + M : N;
    if (z.fp64) {
        // the node engine in double precision: structure shared with d, values here
        d.T = c.take<int64_t>(1);
        d.best = c.take<int32_t>(Hp);
        d.out2 = c.take<double>(2 * static_cast<int64_t>(z.n_games));
        d.sq_offset = d.q_offset;
        d.sq_input = d.q_input;
        d64.N = N; d64.Hp = Hp; d64.Qp = Qp; d64.H0 = H0; d64.Q0 = Q0; d64.M = M; d64.D = D;
        d64.parent = d.parent; d64.child_begin = d.child_begin; d64.node_player = d.node_player;
        d64.node_infoset = d.node_infoset; d64.node_edge = d.node_edge; d64.node_id = d.node_id;
        d64.level_offset = d.level_offset; d64.infoset_id = d.infoset_id;
        d64.infoset_player = d.infoset_player; d64.q_offset = d.q_offset;
        d64.chance_id = d.chance_id; d64.cq_offset = d.cq_offset;
        d64.member_offset = d.member_offset; d64.members = d.members; d64.q_input = d.q_input;
        d64.node_slot = d.node_slot; d64.slot_base = d.slot_base;
        d64.T = d.T; d64.best = d.best; d64.out2 = d.out2;
        d64.sq_offset = d.sq_offset; d64.sq_input = d.sq_input;
        d64.players = z.players;
        d64.payoff = c.take<double>(cols * N);
        d64.prob = c.take<double>(Qp + Q0);
        d64.R = c.take<double>(Qp);
        d64.S = c.take<double>(Qp);
        d64.value = c.take<double>(cols * N);
        d64.reach = c.take<double>(planes * N);
        d64.avgprob = c.take<double>(Qp + Q0);
        d64.br_reach = c.take<double>(N);
        d64.br_value = c.take<double>(N);
        d64.stage = c.take<double>(2 * Qp);
        d64.rtilde = c.take<double>(Qp);
        if (store) d64.contrib = c.take<double>(n_contrib);
        d64.pibar = c.take<double>(Hp);
        x = cfr::XDev{};
        return (c.off + 255) & ~size_t{255};
    }
    d.payoff = c.take<float>(cols * N);
    d.prob = c.take<float>(Qp + Q0);
    d.R = c.take<float>(Qp);
    d.S = c.take<float>(Qp);
    d.value = c.take<float>(cols * N);
    d.reach = c.take<float>(planes * N);
    d.T = c.take<int64_t>(1);
    d.avgprob = c.take<float>(Qp + Q0);
    if (z.engine == ENGINE_NODE) {
        d.br_reach = c.take<float>(N);
        d.br_value = c.take<float>(N);
        d.best = c.take<int32_t>(Hp);
    }
    d.stage = c.take<float>(2 * Qp);
    d.out2 = c.take<double>(2 * static_cast<int64_t>(z.n_games));
    d.sq_offset = d.q_offset;
    d.sq_input = d.q_input;
    x = cfr::XDev{};
    if (z.engine == ENGINE_NODE) {
        d.rtilde = c.take<float>(Qp);
        if (store) d.contrib = c.take<float>(n_contrib);
        d.pibar = c.take<float>(Hp);
    } else {
        x.N = N; x.Hp = Hp; x.Qp = Qp; x.Q0 = Q0; x.M = M; x.L = z.L; x.C = z.C;
        x.D = D; x.max_actions = z.max_actions;
        x.parent = c.take<int32_t>(N);
        x.edge = c.take<int32_t>(N);
        x.meta = c.take<int8_t>(N);
        x.parent_ek = c.take<int64_t>(N + 1);  // + 1: the top-down reads records in pairs
        x.child_begin = c.take<int32_t>(N);
        x.child_stride = c.take<int32_t>(N);
        x.child_list = c.take<int32_t>(z.L);
        x.canon_of = c.take<int32_t>(N);
        x.q_offset = c.take<int32_t>(Hp + 1);
        x.iplayer = c.take<int8_t>(Hp);
        x.member_offset = c.take<int32_t>(Hp + 1);
        x.chance_nodes = c.take<int32_t>(z.C);
        x.chance_base = c.take<int32_t>(z.C);
        x.chance_k = c.take<int32_t>(z.C);
        x.mem_rec = c.take<int4>(M);
        x.mem_kp = c.take<int8_t>(M);
        x.set_rec = c.take<int4>(Hp);
        x.tile_lo = c.take<int32_t>(N - z.terminals);
        x.tile_hi = c.take<int32_t>(N - z.terminals);
        x.chunk_first = c.take<int32_t>(Hp + D + 2);
        x.chunk_m = c.take<int32_t>(Hp + D + 2);
        x.q_input = c.take<int32_t>(Qp);
        x.payoff = c.take<float>(N);
        x.pack_done = c.take<uint32_t>(1);
        if (z.packs) {
            x.packs = c.take<cfr::PackDesc>(max_packs(N, D));
            x.pack_blob = c.take<int32_t>(max_pack_words(N, M, Hp, z.C, D));
        }
        x.prob = d.prob;
        x.R = d.R;
        x.S = d.S;
        x.value = d.value;
        x.reach = d.reach;
        x.T = d.T;
        x.br_reach = c.take<float>(2 * N);
        x.br_value = c.take<float>(2 * N);
        x.out2 = d.out2;
        d.sq_offset = x.q_offset;
        d.sq_input = x.q_input;
    }
    return (c.off + 255) & ~size_t{255};
}

int check_hip(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, what);
    return CFR_OK;
}

template <class T>
int upload(T* dst, const std::vector<T>& src, hipStream_t st) {
    if (src.empty()) return CFR_OK;
    HIP_TRY(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st),
            "upload");
    return CFR_OK;
}

void launch_one_iteration(cfr_solver* s, hipStream_t st, cfr::LaunchTimer* timer) {
    auto pass = [&](const cfr::UpdateRule& r) {
        if (s->part32)
            cfr::launch_partitioned_pass(s->dev, *s->part32, r, st);
        else if (s->part64)
            cfr::launch_partitioned_pass(s->dev64, *s->part64, r, st);
        else if (s->engine == ENGINE_BLOCK)
            cfr::launch_x_iteration(s->xdev, r, st, timer);
        else if (s->fp64)
            cfr::launch_iteration(s->dev64, s->level_offset.data(), r, st, timer);
        else
            cfr::launch_iteration(s->dev, s->level_offset.data(), r, st, timer);
    };
    if (!s->alternating) {
        pass(s->rule);
        return;
    }
    // a pass per rational player in seat order, the iteration counted by the last
    const int32_t n = s->players > 0 ? s->players : 2;
    for (int32_t i = 1; i <= n; ++i) {
        cfr::UpdateRule r = s->rule;
        r.players = 1 << (i - 1);
        r.count = i == n ? s->rule.count : 0;
        pass(r);
    }
}

int capture(cfr_solver* s) {
    hipStream_t cap;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "create capture stream");
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_err(e, "begin capture");
    }
    launch_one_iteration(s, cap, nullptr);
    e = hipStreamEndCapture(cap, &s->graph);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return hip_err(e, "end capture");
    HIP_TRY(hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0), "instantiate graph");
    return CFR_OK;
}

// Releases a solver that failed part-way through its build (graph objects included).
void discard(cfr_solver* s) {
    if (s == nullptr) return;
    if (s->exec != nullptr) (void)hipGraphExecDestroy(s->exec);
    if (s->graph != nullptr) (void)hipGraphDestroy(s->graph);
    delete s;
}

// Validates a configuration (null: the defaults); CFR_OK or an error code with a message.
int check_config(const cfr_config* c) {
    if (c == nullptr) return CFR_OK;
    if (c->variant < CFR_VANILLA || c->variant > CFR_DCFR) return set_err(CFR_EINVAL, "bad variant");
    if (c->flags & ~(CFR_FLAG_NO_GRAPH | CFR_FLAG_NODE_ENGINE | CFR_FLAG_ALTERNATING |
                     CFR_FLAG_KEEP_NODE_VALUES | CFR_FLAG_SUBTREE_PACKS | CFR_FLAG_FP64))
        return set_err(CFR_EINVAL, "unknown flag bits");
    if ((c->flags & CFR_FLAG_FP64) && (c->flags & CFR_FLAG_SUBTREE_PACKS))
        return set_err(CFR_EINVAL, "CFR_FLAG_FP64 runs on the node engine; subtree packs belong "
                                   "to the public-block engine");
    if (c->averaging < CFR_AVG_DEFAULT || c->averaging > CFR_AVG_LINEAR)
        return set_err(CFR_EINVAL, "bad averaging");
    if (c->variant == CFR_DCFR) {
        if (c->averaging != CFR_AVG_DEFAULT)
            return set_err(CFR_EINVAL, "discounted CFR weights the average by gamma: averaging "
                                       "must be CFR_AVG_DEFAULT");
        for (float v : {c->dcfr_alpha, c->dcfr_beta, c->dcfr_gamma})
            if (!std::isfinite(v) || v < -64.0f || v > 64.0f)
                return set_err(CFR_EINVAL, "discount exponents must be finite and in [-64, 64]");
    }
    return CFR_OK;
}

// The update rule a validated configuration asks for.
cfr::UpdateRule rule_of(const cfr_config& c) {
    cfr::UpdateRule u;
    u.variant = c.variant;
    u.linear = c.variant == CFR_DCFR ? 0
               : c.averaging == CFR_AVG_DEFAULT ? (c.variant == CFR_PLUS)
                                                : c.averaging;
    u.alpha = c.dcfr_alpha;
    u.beta = c.dcfr_beta;
    u.gamma = c.dcfr_gamma;
    return u;
}

// Per level, which launch computes its top-down reach (0: none, the roots and levels without
// decision nodes; 1: the single-workgroup launch of the first levels; 2: the launch of several
// small levels; 3: a launch of its own; 4: the level's bottom-up launch; 5: the subtree-pack
// launch, for a level whose decision nodes all lie in packs). For a level split between the
// per-level launches and the packs, the code names the launch of the upper part.
// Deepest level of the solver's iteration (a batch: of its forest).
int32_t launch_depth(const cfr_solver* s) {
    return s->engine == ENGINE_BLOCK ? s->xdev.D : s->dev.D;
}

std::vector<int32_t> reach_launch(const cfr_solver* s) {
    const int32_t D = launch_depth(s);
    std::vector<int32_t> r(D + 1, 3);
    r[0] = 0;
    r[D] = 0;  // the deepest level holds only terminal nodes
    if (s->engine != ENGINE_BLOCK) return r;
    const cfr::XDev& x = s->xdev;
    for (int32_t l = 1; l <= D; ++l) {
        const bool in_packs = x.up_end_host[l] < x.level_offset_host[l + 1];
        if (x.reach_units_host[l] == 0) r[l] = in_packs && l < D ? 5 : 0;
        else if (l <= x.fused_reach) r[l] = 1;
        else if (l <= x.path_reach) r[l] = 2;
    }
    if (const int32_t ld = cfr::derived_reach_level(x); ld >= 0) r[ld] = 4;
    return r;
}


// A general-sum game of n rational players as the two-player path reads it: the same tree, its
// first payoff column as u_1 and no u_2 (so no zero-sum check).
struct GameN {
    cfr_game g{};
    std::vector<double> u1;
};

int game_n(const cfr_game* game, int32_t players, const double* payoff, GameN& out) {
    if (game == nullptr || payoff == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (players < 2 || players > cfr::kMaxPlayers)
        return set_err(CFR_EINVAL, "a general-sum game has 2 to " + std::to_string(cfr::kMaxPlayers) +
                                       " rational players");
    if (game->n_nodes < 1) return set_err(CFR_EINVAL, "game arrays must be non-null and n_nodes >= 1");
    out.g = *game;
    out.u1.resize(static_cast<size_t>(game->n_nodes));
    for (int64_t v = 0; v < game->n_nodes; ++v) out.u1[v] = payoff[v * players];
    out.g.payoff_u1 = out.u1.data();
    out.g.payoff_u2 = nullptr;
    return CFR_OK;
}

// A general-sum solver runs the node engine (no subtree packs).
int check_config_n(const cfr_config* c) {
    if (const int rc = check_config(c); rc != CFR_OK) return rc;
    if (c != nullptr && (c->flags & CFR_FLAG_SUBTREE_PACKS))
        return set_err(CFR_EINVAL, "a general-sum game runs the node engine: "
                                   "CFR_FLAG_SUBTREE_PACKS does not apply");
    return CFR_OK;
}

// cfr_plan for a two-player zero-sum game (players = 0) or a general-sum game of `players`.
int plan_impl(const cfr_game* game, const cfr_config* config, int32_t players,
              cfr_plan_info* out) {
    cfr::Layout L;
    std::string err;
    const int rc = cfr::plan_sizes(*game, L, err, players > 0 ? players : 2);
    if (rc != CFR_OK) return set_err(rc, err);
    Sizes z;
    z.N = L.N; z.Hp = L.Hp; z.Qp = L.Qp; z.H0 = L.H0; z.Q0 = L.Q0; z.M = L.n_members;
    z.terminals = L.n_terminals;
    z.C = L.n_chance_nodes; z.L = L.N; z.D = L.D; z.max_actions = L.max_actions;
    z.engine = players > 0 ? ENGINE_NODE
                           : choose_engine(L.level_pure, L.max_actions, config ? config->flags : 0u);
    z.packs = z.engine == ENGINE_BLOCK && L.max_actions <= 4 && config != nullptr &&
              (config->flags & CFR_FLAG_SUBTREE_PACKS) != 0;
    z.fp64 = config != nullptr && (config->flags & CFR_FLAG_FP64) != 0;
    z.players = players;
    cfr::Dev d{};
    cfr::Dev64 d64{};
    cfr::XDev x{};
    std::memset(out, 0, sizeof *out);
    out->n_nodes = L.N;
    out->n_terminals = L.n_terminals;
    out->n_infosets = L.Hp;
    out->n_q = L.Qp;
    out->n_chance_infosets = L.H0;
    out->n_chance_q = L.Q0;
    out->max_actions = L.max_actions;
    out->depth = L.D;
    out->level_pure = L.level_pure ? 1 : 0;
    out->engine = z.engine;
    out->workspace_bytes = static_cast<int64_t>(carve(d, d64, x, nullptr, z));
    return CFR_OK;
}

}  // namespace

extern "C" {

const char* cfr_last_error(void) { return g_err.c_str(); }

int cfr_plan(const cfr_game* game, const cfr_config* config, cfr_plan_info* out) {
    if (game == nullptr || out == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (const int rc = check_config(config); rc != CFR_OK) return rc;
    return plan_impl(game, config, 0, out);
}

int cfr_plan_n(const cfr_game* game, int32_t n_players, const double* payoff,
               const cfr_config* config, cfr_plan_info* out) {
    if (out == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (const int rc = check_config_n(config); rc != CFR_OK) return rc;
    GameN gn;
    if (const int rc = game_n(game, n_players, payoff, gn); rc != CFR_OK) return rc;
    return plan_impl(&gn.g, config, n_players, out);
}

}  // extern "C"

namespace {

// Per-level bottom-up shapes from the bucket tables (the fused first levels take one chunk of
// up to kFuseThreads members), then the chunk tables, uploaded.
int apply_shapes(cfr_solver* s, hipStream_t st) {
    cfr::XDev& x = s->xdev;
    const int32_t D = x.D;
    // top-down: per level, the shape of its decision-node count, and tiles that cover the runs
    // of decision nodes (levels past the single-workgroup ones)
    s->reach_threads_l.assign(D + 1, 256);
    s->reach_npt_l.assign(D + 1, 1);
    s->t_level_offset.assign(D + 2, 0);
    std::vector<int32_t> tlo, thi;
    for (int32_t l = 0; l <= D; ++l) {
        s->t_level_offset[l] = static_cast<int32_t>(tlo.size());
        if (l < 1 + x.fused_reach || l >= D) continue;
        const int b = cfr::shape_bucket(s->reach_units[l]);
        const bool path = l <= x.path_reach;  // one node per lane, fixed workgroup size
        const int32_t threads = path ? cfr::kPathThreads : s->shape.reach_threads[b];
        const int32_t npt = path ? 1 : s->shape.reach_nodes[b];
        s->reach_threads_l[l] = threads;
        s->reach_npt_l[l] = npt;
        const int32_t cap = threads * npt;
        int32_t x0 = s->x_level_offset[l];
        const int32_t x1 = s->x_up_end[l];  // the upper prefix: packs take the rest
        while (x0 < x1) {
            while (x0 < x1 && (s->x_meta[x0] & 3) == 0) ++x0;
            int32_t e = x0;
            while (e < x1 && e - x0 < cap && (s->x_meta[e] & 3) != 0) ++e;
            if (e > x0) {
                tlo.push_back(x0);
                thi.push_back(e);
            }
            x0 = e;
        }
    }
    s->t_level_offset[D + 1] = static_cast<int32_t>(tlo.size());
    x.reach_threads_host = s->reach_threads_l.data();
    x.reach_npt_host = s->reach_npt_l.data();
    x.t_level_offset_host = s->t_level_offset.data();
    x.reach_units_host = s->reach_units.data();
    s->up_threads.assign(D + 1, 256);
    s->chunk_cap.assign(D + 1, 256);
    for (int32_t l = 0; l <= D; ++l) {
        if (l < x.fused_up) {
            s->up_threads[l] = cfr::kFuseThreads;
            s->chunk_cap[l] = cfr::kFuseThreads;
            continue;
        }
        const int b = cfr::shape_bucket(s->x_m_up_end[l] - s->x_m_level_offset[l]);
        s->up_threads[l] = s->shape.up_threads[b];
        s->chunk_cap[l] = s->shape.up_threads[b] * s->shape.up_members[b];
    }
    x.up_threads_host = s->up_threads.data();
    x.chunk_cap_host = s->chunk_cap.data();
    std::vector<int32_t> chunk_first, chunk_m;
    cfr::build_chunks(s->x_h_level_offset, s->x_member_offset, s->chunk_cap.data(), chunk_first,
                      s->x_k_level_offset, &s->x_h_up_end, &s->x_k_up_end);
    x.k_up_end_host = s->x_k_up_end.data();
    chunk_m.resize(chunk_first.size());
    for (size_t c = 0; c < chunk_first.size(); ++c) chunk_m[c] = s->x_member_offset[chunk_first[c]];
    x.k_level_offset_host = s->x_k_level_offset.data();
    int rc;
    if ((rc = upload(x.chunk_first, chunk_first, st)) || (rc = upload(x.chunk_m, chunk_m, st)) ||
        (rc = upload(x.tile_lo, tlo, st)) || (rc = upload(x.tile_hi, thi, st)))
        return rc;
    // the host vectors go out of scope
    HIP_TRY(hipStreamSynchronize(st), "chunk table upload");
    return CFR_OK;
}

// Copies the block plan to the device and fills the solver's exec view.
int upload_plan(cfr_solver* s, const cfr::ExecPlan& P, hipStream_t st) {
    cfr::XDev& x = s->xdev;
    int rc;
    // member-major and infoset records of the bottom-up pass
    std::vector<int4> mem_rec(P.M), set_rec(P.Hp);
    std::vector<int8_t> mem_kp(P.M);
    for (int64_t h = 0; h < P.Hp; ++h) {
        const int32_t k = P.q_offset[h + 1] - P.q_offset[h];
        const int8_t kp = static_cast<int8_t>(k | (P.infoset_player[h] == 2 ? 64 : 0));
        set_rec[h] = make_int4(P.q_offset[h], P.member_offset[h], P.member_offset[h + 1], kp);
        for (int32_t m = P.member_offset[h]; m < P.member_offset[h + 1]; ++m) {
            const int32_t xm = P.members[m];
            mem_rec[m] = make_int4(xm, P.q_offset[h], P.child_begin[xm], P.child_stride[xm]);
            mem_kp[m] = kp;
        }
    }
    // the k | player byte packed into the top byte of the stride word when every stride fits 24
    // signed bits (children by action lie a block apart), saving the bottom-up pass one load
    // per member
    bool fits = true;
    for (int64_t m = 0; m < P.M && fits; ++m)
        fits = mem_rec[m].w >= -(1 << 23) && mem_rec[m].w < (1 << 23);
    x.kp_packed = fits ? 1 : 0;
    if (fits)
        for (int64_t m = 0; m < P.M; ++m)
            mem_rec[m].w = static_cast<int32_t>((static_cast<uint32_t>(mem_rec[m].w) & 0xFFFFFFu) |
                                                (static_cast<uint32_t>(mem_kp[m]) << 24));
    // edge and kind in one word for the top-down launches, when every edge index fits 24 bits
    // (with the parent beside them in one 8-byte record)
    std::vector<int64_t> parent_ek(P.N);
    bool ek_fits = true;
    for (int64_t v = 0; v < P.N && ek_fits; ++v) ek_fits = P.edge[v] < (1 << 24);
    x.ek_packed = ek_fits ? 1 : 0;
    if (ek_fits)
        for (int64_t v = 0; v < P.N; ++v) {
            const uint32_t ek = (P.edge[v] < 0 ? 0u : static_cast<uint32_t>(P.edge[v])) |
                                (static_cast<uint32_t>(static_cast<uint8_t>(P.meta[v])) << 24);
            parent_ek[v] = static_cast<int64_t>((static_cast<uint64_t>(ek) << 32) |
                                                static_cast<uint32_t>(P.parent[v]));
        }
    if ((rc = upload(x.parent, P.parent, st)) || (rc = upload(x.edge, P.edge, st)) ||
        (rc = upload(x.parent_ek, parent_ek, st)) ||
        (rc = upload(x.meta, P.meta, st)) || (rc = upload(x.child_begin, P.child_begin, st)) ||
        (rc = upload(x.child_stride, P.child_stride, st)) ||
        (rc = upload(x.child_list, P.child_list, st)) || (rc = upload(x.canon_of, P.canon_of, st)) ||
        (rc = upload(x.q_offset, P.q_offset, st)) || (rc = upload(x.iplayer, P.infoset_player, st)) ||
        (rc = upload(x.member_offset, P.member_offset, st)) ||
        (rc = upload(x.mem_rec, mem_rec, st)) || (rc = upload(x.mem_kp, mem_kp, st)) ||
        (rc = upload(x.set_rec, set_rec, st)) || (rc = upload(x.chance_nodes, P.chance_nodes, st)) ||
        (rc = upload(x.chance_base, P.chance_base, st)) || (rc = upload(x.chance_k, P.chance_k, st)) ||
        (rc = upload(x.q_input, P.q_input, st)) || (rc = upload(x.payoff, P.payoff, st)))
        return rc;
    if (!P.packs.empty() && x.packs == nullptr)
        return set_err(CFR_EINVAL, "subtree packs planned without their storage");
    if (static_cast<int64_t>(P.packs.size()) > max_packs(P.N, P.D) ||
        static_cast<int64_t>(P.pack_blob.size()) > max_pack_words(P.N, P.M, P.Hp, P.C, P.D))
        return set_err(CFR_EINVAL, "subtree packs exceed their bound");
    if ((rc = upload(const_cast<cfr::PackDesc*>(x.packs), P.packs, st)) ||
        (rc = upload(const_cast<int32_t*>(x.pack_blob), P.pack_blob, st)))
        return rc;
    HIP_TRY(hipStreamSynchronize(st), "plan upload");
    x.n_tiers = P.n_tiers;
    s->tier_offset = P.tier_offset;
    s->tier_dec.assign(P.n_tiers, 0);
    for (int32_t t = 1; t <= P.n_tiers; ++t)
        for (int32_t i = P.tier_offset[t - 1]; i < P.tier_offset[t]; ++i)
            s->tier_dec[t - 1] += P.packs[i].n_dec;
    x.tier_offset_host = s->tier_offset.data();
    x.tier_dec_host = s->tier_dec.data();
    x.keep_nodes = s->keep_nodes ? 1 : 0;
    s->x_up_end = P.up_end;
    s->x_h_up_end = P.h_up_end;
    s->x_c_up_end = P.c_up_end;
    x.up_end_host = s->x_up_end.data();
    x.h_up_end_host = s->x_h_up_end.data();
    x.c_up_end_host = s->x_c_up_end.data();
    s->x_level_offset = P.level_offset;
    s->x_h_level_offset = P.h_level_offset;
    s->x_c_level_offset = P.c_level_offset;
    s->x_member_offset = P.member_offset;
    s->x_meta = P.meta;
    // upper decision nodes per level, and whether their children are all terminal
    cfr::upper_level_stats(P, s->reach_units, s->only_terminal_children);
    x.only_terminal_children_host = s->only_terminal_children.data();
    s->x_m_level_offset.resize(P.D + 2);
    for (int32_t l = 0; l <= P.D + 1; ++l) s->x_m_level_offset[l] = P.member_offset[P.h_level_offset[l]];
    s->x_m_up_end.resize(P.D + 1);
    for (int32_t l = 0; l <= P.D; ++l) s->x_m_up_end[l] = P.member_offset[P.h_up_end[l]];
    // lanes per chance node: the level's largest fan-out rounded up to a power of two, <= 64
    s->chance_glog.assign(P.D + 1, 0);
    for (int32_t l = 0; l <= P.D; ++l) {
        int32_t kmax = 1;
        for (int32_t c = P.c_level_offset[l]; c < P.c_level_offset[l + 1]; ++c)
            kmax = std::max(kmax, P.chance_k[c]);
        int g = 0;
        while (g < 6 && (1 << g) < kmax) ++g;
        s->chance_glog[l] = g;
    }
    x.m_level_offset_host = s->x_m_level_offset.data();
    x.level_offset_host = s->x_level_offset.data();
    x.h_level_offset_host = s->x_h_level_offset.data();
    x.c_level_offset_host = s->x_c_level_offset.data();
    x.chance_glog_host = s->chance_glog.data();
    x.fused_reach = cfr::fusable_reach_levels(x.level_offset_host, x.up_end_host, P.D);
    x.path_reach = cfr::path_reach_levels(s->reach_units.data(), x.fused_reach, P.D,
                                          cfr::kPathDepthBelowTop);
    // the path launch alone, from the roots, when it covers as many levels: one launch fewer
    const int32_t p0 = cfr::path_reach_levels(s->reach_units.data(), 0, P.D, cfr::kPathDepth);
    if (x.path_reach > x.fused_reach && p0 >= x.path_reach) {
        x.fused_reach = 0;
        x.path_reach = p0;
    }
    x.fused_up = cfr::fusable_up_levels(x.m_level_offset_host, s->x_m_up_end.data(),
                                        x.h_level_offset_host, x.h_up_end_host,
                                        x.c_level_offset_host, x.c_up_end_host,
                                        x.chance_glog_host, P.D, x.max_actions);
    // levels with nothing outside the packs need no single-workgroup launch
    auto upper_up = [&](int32_t l) {
        return x.h_up_end_host[l] > x.h_level_offset_host[l] ||
               x.c_up_end_host[l] > x.c_level_offset_host[l];
    };
    while (x.fused_up > 0 && !upper_up(x.fused_up - 1)) --x.fused_up;
    x.upper_bottom_up = 0;
    for (int32_t l = 0; l <= P.D; ++l) x.upper_bottom_up |= upper_up(l) ? 1 : 0;
    while (x.fused_reach > 0 && s->reach_units[x.fused_reach] == 0) --x.fused_reach;
    // the sigma ranges that the single-workgroup kernels read: pairs and chance probabilities
    // of the levels above the first one each leaves to per-level launches
    for (int e = 0; e < 2; ++e) {
        const int32_t l1 = std::min(e == 0 ? x.fused_reach : x.fused_up, P.D + 1);
        x.top_q_lo[e] = P.q_offset[P.h_level_offset[0]];
        x.top_q_hi[e] = P.q_offset[P.h_level_offset[l1]];
        const int32_t c0 = P.c_level_offset[0], c1 = P.c_level_offset[l1];
        int32_t clo = 0, chi = 0;
        for (int32_t c = c0; c < c1; ++c) {
            clo = c == c0 ? P.chance_base[c] : std::min(clo, P.chance_base[c]);
            chi = std::max(chi, P.chance_base[c] + P.chance_k[c]);
        }
        x.top_c_lo[e] = clo;
        x.top_c_hi[e] = chi;
    }
    return apply_shapes(s, st);
}

// The general-sum payoff matrix (input node-major, n columns) as the device's canonical planes:
// column i of canonical node v at i * N + v, terminals only (0 elsewhere). CFR_EINVAL for a
// payoff that is not finite at a terminal.
template <class F>
int payoff_planes(const cfr::Layout& L, int32_t players, const double* payoff, std::vector<F>& out) {
    const int64_t N = L.N;
    out.assign(static_cast<size_t>(players) * N, F(0));
    for (int64_t v = 0; v < N; ++v) {
        if (L.node_player[v] >= 0) continue;
        const int64_t in = L.node_id[v];
        for (int32_t i = 0; i < players; ++i) {
            const double u = payoff[in * players + i];
            if (!std::isfinite(u))
                return set_err(CFR_EINVAL, "terminal " + std::to_string(in) + ": payoff of player " +
                                               std::to_string(i + 1) + " not finite");
            out[static_cast<size_t>(i) * N + v] = static_cast<F>(u);
        }
    }
    return CFR_OK;
}

// The member-order slots of a general-sum game's contributions (DevT::node_slot): infoset h's
// n_h members, k_h + 1 values each, start at slot_base[h], in canonical infoset order.
void member_slots(const cfr::Layout& L, std::vector<int32_t>& node_slot,
                  std::vector<int32_t>& slot_base) {
    node_slot.assign(static_cast<size_t>(L.N), 0);
    slot_base.assign(static_cast<size_t>(L.Hp) + 1, 0);
    int64_t at = 0;
    for (int64_t h = 0; h < L.Hp; ++h) {
        const int32_t m0 = L.member_offset[h], n = L.member_offset[h + 1] - m0;
        const int32_t k = L.q_offset[h + 1] - L.q_offset[h];
        slot_base[h] = static_cast<int32_t>(at);
        for (int32_t j = 0; j < n; ++j)
            node_slot[L.members[m0 + j]] = static_cast<int32_t>(at + static_cast<int64_t>(j) * (k + 1));
        at += static_cast<int64_t>(n) * (k + 1);
    }
    slot_base[L.Hp] = static_cast<int32_t>(at);
}

// cfr_build for a two-player zero-sum game (players = 0) or a general-sum game of `players`
// with its payoff matrix (the node engine; simultaneous or, alternating, a pass per player).
int build_impl(const cfr_game* game, const cfr_config& cfg, int32_t players, const double* payoff,
               void* workspace, size_t bytes, void* stream, cfr_solver** out) {
    cfr::Layout L;
    std::string err;
    const bool fp64 = (cfg.flags & CFR_FLAG_FP64) != 0;
    int rc = cfr::flatten(*game, L, err, fp64, players > 0 ? players : 2);
    if (rc != CFR_OK) return set_err(rc, err);
    std::vector<float> pay32;
    std::vector<double> pay64;
    if (players > 0 && (rc = fp64 ? payoff_planes(L, players, payoff, pay64)
                                  : payoff_planes(L, players, payoff, pay32)) != CFR_OK)
        return rc;
    Sizes z;
    z.N = L.N; z.Hp = L.Hp; z.Qp = L.Qp; z.H0 = L.H0; z.Q0 = L.Q0; z.M = L.n_members;
    z.terminals = L.n_terminals;
    z.C = L.n_chance_nodes; z.L = L.N; z.D = L.D; z.max_actions = L.max_actions;
    z.engine = players > 0 ? ENGINE_NODE : choose_engine(L.level_pure, L.max_actions, cfg.flags);
    z.packs = z.engine == ENGINE_BLOCK && L.max_actions <= 4 && (cfg.flags & CFR_FLAG_SUBTREE_PACKS);
    z.fp64 = fp64;
    z.players = players;
    cfr::ExecPlan P;
    if (z.engine == ENGINE_BLOCK) {
        // subtree packs are instantiated for at most 4 actions per infoset
        rc = cfr::build_exec_plan(L, P, err,
                                  L.max_actions <= 4 && (cfg.flags & CFR_FLAG_SUBTREE_PACKS));
        if (rc != CFR_OK) return set_err(rc, err);
    }
    cfr::Dev d{};
    cfr::Dev64 d64{};
    cfr::XDev x{};
    const size_t need = carve(d, d64, x, nullptr, z);
    if (bytes < need)
        return set_err(CFR_ENOMEM, "workspace has " + std::to_string(bytes) + " bytes, needs " +
                                       std::to_string(need));
    carve(d, d64, x, workspace, z);

    auto* s = new cfr_solver();
    s->dev = d;
    s->dev64 = d64;
    s->fp64 = fp64;
    s->xdev = x;
    s->engine = z.engine;
    s->rule = rule_of(cfg);
    if (players > 0) s->rule.players = (1 << players) - 1;
    s->players = players;
    s->alternating = (cfg.flags & CFR_FLAG_ALTERNATING) != 0;
    s->use_graph = (cfg.flags & CFR_FLAG_NO_GRAPH) == 0;
    s->keep_nodes = (cfg.flags & CFR_FLAG_KEEP_NODE_VALUES) != 0;
    s->level_pure = L.level_pure;
    s->n_terminals = L.n_terminals;
    s->max_actions = L.max_actions;
    s->stream = static_cast<hipStream_t>(stream);
    s->level_offset = L.level_offset;
    // infosets are numbered by first appearance, so with level-pure infosets each level's
    // infosets form a contiguous id range
    s->infoset_level_offset.assign(L.D + 2, static_cast<int32_t>(L.Hp));
    {
        int32_t h = 0;
        for (int32_t l = 0; l <= L.D; ++l) {
            s->infoset_level_offset[l] = h;
            while (h < L.Hp && L.members[L.member_offset[h]] < L.level_offset[l + 1]) ++h;
        }
        s->infoset_level_offset[L.D + 1] = static_cast<int32_t>(L.Hp);
    }
    hipStream_t st = s->stream;
    std::vector<float> prob_tail(fp64 ? 0 : L.Qp + L.Q0, 0.0f);
    std::vector<double> prob_tail64(fp64 ? L.Qp + L.Q0 : 0, 0.0);
    for (int64_t i = 0; i < L.Q0; ++i) {
        if (fp64) prob_tail64[L.Qp + i] = L.chance_prob64[i];
        else prob_tail[L.Qp + i] = L.chance_prob[i];
    }
    if (fp64 && ((rc = upload(d64.payoff, players > 0 ? pay64 : L.payoff64, st)) ||
                 (rc = upload(d64.prob, prob_tail64, st)))) {
        discard(s);
        return rc;
    }
    if ((rc = upload(d.parent, L.parent, st)) || (rc = upload(d.child_begin, L.child_begin, st)) ||
        (rc = upload(d.node_player, L.node_player, st)) ||
        (rc = upload(d.node_infoset, L.node_infoset, st)) ||
        (rc = upload(d.node_edge, L.node_edge, st)) || (rc = upload(d.node_id, L.node_id, st)) ||
        (rc = upload(d.level_offset, L.level_offset, st)) ||
        (rc = upload(d.infoset_id, L.infoset_id, st)) ||
        (rc = upload(d.infoset_player, L.infoset_player, st)) ||
        (rc = upload(d.q_offset, L.q_offset, st)) || (rc = upload(d.chance_id, L.chance_id, st)) ||
        (rc = upload(d.cq_offset, L.cq_offset, st)) ||
        (rc = upload(d.member_offset, L.member_offset, st)) ||
        (rc = upload(d.members, L.members, st)) || (rc = upload(d.q_input, L.q_input, st)) ||
        (!fp64 && ((rc = upload(d.payoff, players > 0 ? pay32 : L.payoff, st)) ||
                   (rc = upload(d.prob, prob_tail, st))))) {
        discard(s);
        return rc;
    }
    std::vector<int32_t> node_slot;
    std::vector<int32_t> slot_base;
    if (players > 0) {
        member_slots(L, node_slot, slot_base);
        if ((rc = upload(d.node_slot, node_slot, st)) || (rc = upload(d.slot_base, slot_base, st))) {
            discard(s);
            return rc;
        }
    }
    if (s->engine == ENGINE_BLOCK) {
        cfr_default_launch_shape(&s->shape);
        if ((rc = upload_plan(s, P, st))) {
            discard(s);
            return rc;
        }
    }
    if (fp64) cfr::launch_reset(d64, st, true);
    else cfr::launch_reset(d, st, s->engine == ENGINE_NODE);
    if (s->engine == ENGINE_BLOCK) cfr::launch_x_reset(s->xdev, st);
    if ((rc = check_hip("reset")) != CFR_OK) {
        discard(s);
        return rc;
    }
    // host vectors are released when L and P go out of scope: wait for the copies first
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        discard(s);
        return hip_err(e, "build synchronise");
    }
    if (s->use_graph && (rc = capture(s)) != CFR_OK) {
        discard(s);
        return rc;
    }
    *out = s;
    return CFR_OK;
}

cfr_config config_or_default(const cfr_config* config) {
    cfr_config cfg{};
    cfg.variant = CFR_VANILLA;
    cfg.averaging = CFR_AVG_DEFAULT;
    if (config != nullptr) cfg = *config;
    return cfg;
}

}  // namespace

extern "C" {

int cfr_build(const cfr_game* game, const cfr_config* config, void* workspace, size_t bytes,
              void* stream, cfr_solver** out) {
    if (game == nullptr || workspace == nullptr || out == nullptr)
        return set_err(CFR_EINVAL, "null argument");
    const cfr_config cfg = config_or_default(config);
    if (const int rc = check_config(&cfg); rc != CFR_OK) return rc;
    return build_impl(game, cfg, 0, nullptr, workspace, bytes, stream, out);
}

int cfr_build_n(const cfr_game* game, int32_t n_players, const double* payoff,
                const cfr_config* config, void* workspace, size_t bytes, void* stream,
                cfr_solver** out) {
    if (workspace == nullptr || out == nullptr) return set_err(CFR_EINVAL, "null argument");
    const cfr_config cfg = config_or_default(config);
    if (const int rc = check_config_n(&cfg); rc != CFR_OK) return rc;
    GameN gn;
    if (const int rc = game_n(game, n_players, payoff, gn); rc != CFR_OK) return rc;
    return build_impl(&gn.g, cfg, n_players, payoff, workspace, bytes, stream, out);
}

}  // extern "C"

namespace {

// Flags a partitioned solver takes: the schedule and the precision (it always enqueues its
// kernels and copies directly and runs the node engine's kernels).
int check_partitioned_config(const cfr_config& c) {
    if (const int rc = check_config(&c); rc != CFR_OK) return rc;
    if (c.flags & (CFR_FLAG_SUBTREE_PACKS | CFR_FLAG_KEEP_NODE_VALUES))
        return set_err(CFR_EINVAL, "a partitioned solver takes CFR_FLAG_ALTERNATING, CFR_FLAG_FP64, "
                                   "CFR_FLAG_NO_GRAPH and CFR_FLAG_NODE_ENGINE only");
    return CFR_OK;
}

// Device sizes of a partitioned solver: the resident levels and one window, every pair.
Sizes partitioned_sizes(const cfr::Layout& L, const cfr::PartPlan& P, bool fp64) {
    Sizes z;
    z.N = P.base + P.window;
    z.Hp = L.Hp; z.Qp = L.Qp; z.H0 = L.H0; z.Q0 = L.Q0; z.M = 0;
    z.terminals = 0; z.C = 0; z.L = z.N; z.D = L.D; z.max_actions = L.max_actions;
    z.engine = ENGINE_NODE;
    z.fp64 = fp64;
    z.gather = false;
    return z;
}

}  // namespace

extern "C" {

int cfr_plan_partitioned(const cfr_game* game, const cfr_config* config, int32_t cut_level,
                         int64_t max_window_nodes, cfr_plan_info* out, int32_t* n_partitions,
                         int64_t* host_bytes) {
    if (game == nullptr || out == nullptr) return set_err(CFR_EINVAL, "null argument");
    cfr_config cfg{};
    cfg.variant = CFR_VANILLA;
    cfg.averaging = CFR_AVG_DEFAULT;
    if (config != nullptr) cfg = *config;
    if (const int rc = check_partitioned_config(cfg); rc != CFR_OK) return rc;
    const bool fp64 = (cfg.flags & CFR_FLAG_FP64) != 0;
    cfr::Layout L;
    std::string err;
    int rc = cfr::flatten(*game, L, err, fp64);
    if (rc != CFR_OK) return set_err(rc, err);
    cfr::PartPlan P;
    if ((rc = cfr::plan_partitions(L, cut_level, max_window_nodes, P, err)) != CFR_OK)
        return set_err(rc, err);
    const Sizes z = partitioned_sizes(L, P, fp64);
    cfr::Dev d{};
    cfr::Dev64 d64{};
    cfr::XDev x{};
    std::memset(out, 0, sizeof *out);
    out->n_nodes = L.N;
    out->n_terminals = L.n_terminals;
    out->n_infosets = L.Hp;
    out->n_q = L.Qp;
    out->n_chance_infosets = L.H0;
    out->n_chance_q = L.Q0;
    out->max_actions = L.max_actions;
    out->depth = L.D;
    out->level_pure = L.level_pure ? 1 : 0;
    out->engine = ENGINE_NODE;
    out->workspace_bytes = static_cast<int64_t>(carve(d, d64, x, nullptr, z));
    if (n_partitions != nullptr) *n_partitions = P.parts;
    if (host_bytes != nullptr)
        *host_bytes = P.total * (4 * 3 + 1 + (fp64 ? 8 : 4)) + (P.total + P.parts) * 4 +
                      static_cast<int64_t>(P.patch.size()) * 4;
    return CFR_OK;
}

int cfr_build_partitioned(const cfr_game* game, const cfr_config* config, int32_t cut_level,
                          int64_t max_window_nodes, void* workspace, size_t bytes, void* stream,
                          cfr_solver** out) {
    if (game == nullptr || workspace == nullptr || out == nullptr)
        return set_err(CFR_EINVAL, "null argument");
    cfr_config cfg{};
    cfg.variant = CFR_VANILLA;
    cfg.averaging = CFR_AVG_DEFAULT;
    if (config != nullptr) cfg = *config;
    if (const int rc = check_partitioned_config(cfg); rc != CFR_OK) return rc;
    const bool fp64 = (cfg.flags & CFR_FLAG_FP64) != 0;
    cfr::Layout L;
    std::string err;
    int rc = cfr::flatten(*game, L, err, fp64);
    if (rc != CFR_OK) return set_err(rc, err);
    cfr::PartPlan P;
    if ((rc = cfr::plan_partitions(L, cut_level, max_window_nodes, P, err)) != CFR_OK)
        return set_err(rc, err);
    const Sizes z = partitioned_sizes(L, P, fp64);
    cfr::Dev d{};
    cfr::Dev64 d64{};
    cfr::XDev x{};
    const size_t need = carve(d, d64, x, nullptr, z);
    if (bytes < need)
        return set_err(CFR_ENOMEM, "workspace has " + std::to_string(bytes) + " bytes, needs " +
                                       std::to_string(need));
    carve(d, d64, x, workspace, z);
    auto* s = new cfr_solver();
    s->dev = d;
    s->dev64 = d64;
    s->fp64 = fp64;
    s->engine = ENGINE_NODE;
    s->canonical = false;  // the device holds the resident levels and a window, not the tree
    s->rule = rule_of(cfg);
    s->alternating = (cfg.flags & CFR_FLAG_ALTERNATING) != 0;
    s->use_graph = false;  // each pass streams host memory through the window
    s->level_pure = L.level_pure;
    s->n_terminals = L.n_terminals;
    s->max_actions = L.max_actions;
    s->stream = static_cast<hipStream_t>(stream);
    s->level_offset = L.level_offset;
    hipStream_t st = s->stream;
    const int64_t base = P.base, Nloc = z.N;
    // the resident levels 0 .. cut keep their canonical ids; the window's ids start at base
    auto head = [&](const auto& v, int64_t n) {
        using T = typename std::decay_t<decltype(v)>::value_type;
        return std::vector<T>(v.begin(), v.begin() + n);
    };
    std::vector<float> prob_tail(fp64 ? 0 : L.Qp + L.Q0, 0.0f);
    std::vector<double> prob_tail64(fp64 ? L.Qp + L.Q0 : 0, 0.0);
    for (int64_t i = 0; i < L.Q0; ++i) {
        if (fp64) prob_tail64[L.Qp + i] = L.chance_prob64[i];
        else prob_tail[L.Qp + i] = L.chance_prob[i];
    }
    // (named: the copies must find them alive until the synchronisation below)
    const std::vector<int32_t> cb = head(L.child_begin, base + 1), par = head(L.parent, base),
                               inf = head(L.node_infoset, base), edg = head(L.node_edge, base);
    std::vector<int8_t> player(Nloc, -1);
    std::copy(L.node_player.begin(), L.node_player.begin() + base, player.begin());
    std::vector<double> pay64(fp64 ? Nloc : 0, 0.0);
    std::vector<float> pay32(fp64 ? 0 : Nloc, 0.0f);
    if (fp64) std::copy(L.payoff64.begin(), L.payoff64.begin() + base, pay64.begin());
    else std::copy(L.payoff.begin(), L.payoff.begin() + base, pay32.begin());
    if ((rc = upload(d.parent, par, st)) || (rc = upload(d.child_begin, cb, st)) ||
        (rc = upload(d.node_player, player, st)) || (rc = upload(d.node_infoset, inf, st)) ||
        (rc = upload(d.node_edge, edg, st)) ||
        (rc = upload(d.level_offset, L.level_offset, st)) ||
        (rc = upload(d.infoset_id, L.infoset_id, st)) ||
        (rc = upload(d.infoset_player, L.infoset_player, st)) ||
        (rc = upload(d.q_offset, L.q_offset, st)) || (rc = upload(d.chance_id, L.chance_id, st)) ||
        (rc = upload(d.cq_offset, L.cq_offset, st)) || (rc = upload(d.q_input, L.q_input, st))) {
        discard(s);
        return rc;
    }
    if (fp64) {
        if ((rc = upload(d64.payoff, pay64, st)) || (rc = upload(d64.prob, prob_tail64, st))) {
            discard(s);
            return rc;
        }
        s->part64 = std::make_unique<cfr::PartDev<double>>();
        s->part64->plan = std::move(P);
        s->part64->level_offset = L.level_offset;
        rc = s->part64->upload(st);
    } else {
        if ((rc = upload(d.payoff, pay32, st)) || (rc = upload(d.prob, prob_tail, st))) {
            discard(s);
            return rc;
        }
        s->part32 = std::make_unique<cfr::PartDev<float>>();
        s->part32->plan = std::move(P);
        s->part32->level_offset = L.level_offset;
        rc = s->part32->upload(st);
    }
    if (rc != 0) {
        discard(s);
        return set_err(CFR_ENOMEM, "pinned host memory for the partition windows");
    }
    if (fp64) cfr::launch_reset(d64, st, true);
    else cfr::launch_reset(d, st, true);
    if ((rc = check_hip("reset")) != CFR_OK) {
        discard(s);
        return rc;
    }
    // host vectors are released when L goes out of scope: wait for the copies first
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        discard(s);
        return hip_err(e, "build synchronise");
    }
    *out = s;
    return CFR_OK;
}

int cfr_iterate(cfr_solver* s, int32_t n) {
    if (s == nullptr || n < 0) return set_err(CFR_EINVAL, "bad solver or count");
    for (int32_t i = 0; i < n; ++i) {
        if (s->use_graph) {
            HIP_TRY(hipGraphLaunch(s->exec, s->stream), "graph launch");
        } else {
            launch_one_iteration(s, s->stream, nullptr);
            const int rc = check_hip("iteration launch");
            if (rc != CFR_OK) return rc;
        }
    }
    s->T += n;
    return CFR_OK;
}

namespace {
struct EventTimer : cfr::LaunchTimer {
    std::vector<hipEvent_t> ev;
    std::vector<int> kinds, levels;
    std::vector<int64_t> units;
    size_t used = 0;
    hipError_t err = hipSuccess;
    hipEvent_t next() {
        if (used == ev.size()) {
            hipEvent_t e;
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) err = r;
            ev.push_back(e);
        }
        return ev[used++];
    }
    void before(int kind, int level, int64_t n, hipStream_t st) override {
        kinds.push_back(kind);
        levels.push_back(level);
        units.push_back(n);
        const hipError_t r = hipEventRecord(next(), st);
        if (r != hipSuccess) err = r;
    }
    void after(int, hipStream_t st) override {
        const hipError_t r = hipEventRecord(next(), st);
        if (r != hipSuccess) err = r;
    }
    ~EventTimer() override {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};
}  // namespace

// Kernel kinds: the node engine's kinds first, then the block engine's.
const char* cfr_kernel_name(int32_t kind) {
    if (kind < cfr::K_NUM_KINDS) return cfr::kernel_kind_name(kind);
    return cfr::xkernel_kind_name(kind);
}

int cfr_iterate_timed(cfr_solver* s, int32_t n, double* kernel_ms, int64_t* kernel_launches,
                      int32_t n_kinds) {
    if (s == nullptr || n < 0 || n_kinds < 0 || (n_kinds > 0 && (kernel_ms == nullptr ||
                                                                  kernel_launches == nullptr)))
        return set_err(CFR_EINVAL, "bad argument");
    for (int32_t k = 0; k < n_kinds; ++k) {
        kernel_ms[k] = 0.0;
        kernel_launches[k] = 0;
    }
    EventTimer timer;
    for (int32_t i = 0; i < n; ++i) {
        timer.used = 0;
        timer.kinds.clear();
        timer.levels.clear();
        timer.units.clear();
        launch_one_iteration(s, s->stream, &timer);
        int rc = check_hip("timed iteration launch");
        if (rc != CFR_OK) return rc;
        if (timer.err != hipSuccess) return hip_err(timer.err, "event record");
        HIP_TRY(hipStreamSynchronize(s->stream), "timed iteration synchronise");
        for (size_t j = 0; j < timer.kinds.size(); ++j) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, timer.ev[2 * j], timer.ev[2 * j + 1]), "event time");
            const int k = timer.kinds[j];
            if (k < n_kinds) {
                kernel_ms[k] += ms;
                kernel_launches[k] += 1;
            }
        }
        s->T += 1;
    }
    return CFR_OK;
}

int cfr_iterate_profile(cfr_solver* s, int32_t n, double* launch_ms, int32_t* launch_kind,
                        int32_t* launch_level, int64_t* launch_units, int32_t max_launches,
                        int32_t* n_launches) {
    if (s == nullptr || n < 1 || n_launches == nullptr || max_launches < 0)
        return set_err(CFR_EINVAL, "bad argument");
    EventTimer timer;
    std::vector<double> acc;
    for (int32_t i = 0; i < n; ++i) {
        timer.used = 0;
        timer.kinds.clear();
        timer.levels.clear();
        timer.units.clear();
        launch_one_iteration(s, s->stream, &timer);
        int rc = check_hip("profiled iteration launch");
        if (rc != CFR_OK) return rc;
        if (timer.err != hipSuccess) return hip_err(timer.err, "event record");
        HIP_TRY(hipStreamSynchronize(s->stream), "profiled iteration synchronise");
        acc.resize(timer.kinds.size(), 0.0);
        for (size_t j = 0; j < timer.kinds.size(); ++j) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, timer.ev[2 * j], timer.ev[2 * j + 1]), "event time");
            acc[j] += ms;
        }
        s->T += 1;
    }
    *n_launches = static_cast<int32_t>(timer.kinds.size());
    for (size_t j = 0; j < timer.kinds.size() && static_cast<int32_t>(j) < max_launches; ++j) {
        if (launch_ms) launch_ms[j] = acc[j];
        if (launch_kind) launch_kind[j] = timer.kinds[j];
        if (launch_level) launch_level[j] = timer.levels[j];
        if (launch_units) launch_units[j] = timer.units[j];
    }
    return CFR_OK;
}

void cfr_default_launch_shape(cfr_launch_shape* out) {
    if (out == nullptr) return;
    for (int b = 0; b < cfr::kShapeBuckets; ++b) {
        out->up_threads[b] = 256;
        out->up_members[b] = b >= 14 ? 2 : 1;
        out->reach_threads[b] = 256;
        out->reach_nodes[b] = b >= 16 ? 2 : 1;
    }
}

int cfr_set_launch_shape(cfr_solver* s, const cfr_launch_shape* shape) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null solver");
    if (s->engine != ENGINE_BLOCK) return set_err(CFR_EINVAL, "launch shapes apply to the block engine");
    cfr_launch_shape sh;
    if (shape != nullptr) sh = *shape;
    else cfr_default_launch_shape(&sh);
    for (int b = 0; b < cfr::kShapeBuckets; ++b) {
        const int32_t ut = sh.up_threads[b], um = sh.up_members[b];
        const int32_t rt = sh.reach_threads[b], rn = sh.reach_nodes[b];
        if (!(ut == 64 || ut == 128 || ut == 256 || ut == 512) || !(um == 1 || um == 2) ||
            !(rt >= 64 && rt <= 1024 && rt % 64 == 0) || !(rn == 1 || rn == 2 || rn == 4))
            return set_err(CFR_EINVAL,
                           "bucket " + std::to_string(b) +
                               ": bottom-up threads must be 64, 128, 256 or 512 with 1 or 2 "
                               "members each; top-down threads a multiple of 64 in [64, 1024] "
                               "with 1, 2 or 4 nodes each");
    }
    HIP_TRY(hipStreamSynchronize(s->stream), "launch shape synchronise");
    s->shape = sh;
    const int rc = apply_shapes(s, s->stream);
    if (rc != CFR_OK) return rc;
    if (s->exec != nullptr) (void)hipGraphExecDestroy(s->exec);
    if (s->graph != nullptr) (void)hipGraphDestroy(s->graph);
    s->exec = nullptr;
    s->graph = nullptr;
    if (s->use_graph) return capture(s);
    return CFR_OK;
}

}  // extern "C"

namespace {

// The precision a call asks for against the solver's: the float calls serve FP32 solvers, the
// _f64 calls FP64 solvers.
int check_precision(const cfr_solver* s, bool f64) {
    if (s->fp64 == f64) return CFR_OK;
    return set_err(CFR_EINVAL, f64 ? "an _f64 call needs a solver built with CFR_FLAG_FP64"
                                   : "this solver was built with CFR_FLAG_FP64: use the _f64 call");
}

template <class F>
int strategy_out(cfr_solver* s, const cfr::DevT<F>& d, const F* src, F* out, int64_t n_q,
                 int out_on_device, const char* what) {
    if (out_on_device) {
        cfr::launch_scatter_q(d, src, out, s->stream);
        return check_hip(what);
    }
    cfr::launch_scatter_q(d, src, d.stage, s->stream);
    HIP_TRY(hipMemcpyAsync(out, d.stage, n_q * sizeof(F), hipMemcpyDeviceToHost, s->stream), what);
    HIP_TRY(hipStreamSynchronize(s->stream), what);
    return CFR_OK;
}

template <class F>
int average_strategy_t(cfr_solver* s, const cfr::DevT<F>& d, F* out, int64_t n_q,
                       int out_on_device) {
    if (out == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (n_q != d.Qp) return set_err(CFR_ESTATE, "n_q does not match the game");
    cfr::launch_average(d, s->stream);
    return strategy_out(s, d, d.avgprob, out, n_q, out_on_device, "average strategy");
}

template <class F>
int current_strategy_t(cfr_solver* s, const cfr::DevT<F>& d, F* out, int64_t n_q,
                       int out_on_device) {
    if (out == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (n_q != d.Qp) return set_err(CFR_ESTATE, "n_q does not match the game");
    return strategy_out(s, d, d.prob, out, n_q, out_on_device, "current strategy");
}

template <class F>
int get_state_t(cfr_solver* s, const cfr::DevT<F>& d, int64_t* T, F* R, F* S, int64_t n_q) {
    if (n_q != d.Qp) return set_err(CFR_ESTATE, "n_q does not match the game");
    if (T != nullptr) *T = s->T;
    const F* srcs[2] = {d.R, d.S};
    F* dsts[2] = {R, S};
    for (int k = 0; k < 2; ++k) {
        if (dsts[k] == nullptr) continue;
        cfr::launch_scatter_q(d, srcs[k], d.stage, s->stream);
        HIP_TRY(hipMemcpyAsync(dsts[k], d.stage, n_q * sizeof(F), hipMemcpyDeviceToHost,
                               s->stream), "state copy");
        HIP_TRY(hipStreamSynchronize(s->stream), "state synchronise");
    }
    return CFR_OK;
}

template <class F>
int set_state_t(cfr_solver* s, const cfr::DevT<F>& d, int64_t T, const F* R, const F* S,
                int64_t n_q) {
    if (R == nullptr || S == nullptr || T < 0)
        return set_err(CFR_EINVAL, "null argument or negative T");
    if (n_q != d.Qp) return set_err(CFR_ESTATE, "n_q does not match the game");
    const F* srcs[2] = {R, S};
    F* dsts[2] = {d.R, d.S};
    for (int k = 0; k < 2; ++k) {
        HIP_TRY(hipMemcpyAsync(d.stage, srcs[k], n_q * sizeof(F), hipMemcpyHostToDevice,
                               s->stream), "state copy");
        cfr::launch_gather_q(d, d.stage, dsts[k], s->stream);
        // the staging buffer is reused: keep the two transfers apart
        HIP_TRY(hipStreamSynchronize(s->stream), "state synchronise");
    }
    cfr::launch_regret_match(d, s->stream);
    cfr::launch_set_T(d, T, s->stream);
    HIP_TRY(hipStreamSynchronize(s->stream), "state synchronise");
    s->T = T;
    return check_hip("set state");
}

}  // namespace

extern "C" {

int cfr_average_strategy(cfr_solver* s, float* out, int64_t n_q, int out_on_device) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (const int rc = check_precision(s, false); rc != CFR_OK) return rc;
    return average_strategy_t(s, s->dev, out, n_q, out_on_device);
}

int cfr_average_strategy_f64(cfr_solver* s, double* out, int64_t n_q, int out_on_device) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (const int rc = check_precision(s, true); rc != CFR_OK) return rc;
    return average_strategy_t(s, s->dev64, out, n_q, out_on_device);
}

int cfr_current_strategy(cfr_solver* s, float* out, int64_t n_q, int out_on_device) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (const int rc = check_precision(s, false); rc != CFR_OK) return rc;
    return current_strategy_t(s, s->dev, out, n_q, out_on_device);
}

int cfr_current_strategy_f64(cfr_solver* s, double* out, int64_t n_q, int out_on_device) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (const int rc = check_precision(s, true); rc != CFR_OK) return rc;
    return current_strategy_t(s, s->dev64, out, n_q, out_on_device);
}

int cfr_exploitability(cfr_solver* s, double* expl, double br_value[2]) {
    if (s == nullptr || expl == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (s->players > 0)
        return set_err(CFR_EINVAL, "exploitability is defined for two-player zero-sum games; this "
                                   "solver holds a general-sum game");
    if (s->n_games != 1) return set_err(CFR_EINVAL, "a batch reports cfr_exploitability_batch");
    if (s->partitioned())
        return set_err(CFR_EINVAL, "a partitioned solver keeps no whole tree on the device: read its "
                                   "state (cfr_get_state) into an in-core solver of the same game");
    if (!s->level_pure) return set_err(CFR_ELEVEL, "an infoset spans several levels");
    if (s->fp64) {
        cfr::launch_average(s->dev64, s->stream);
        for (int player = 1; player <= 2; ++player)
            cfr::launch_best_response(s->dev64, s->level_offset.data(),
                                      s->infoset_level_offset.data(), player, s->stream);
    } else {
        cfr::launch_average(s->dev, s->stream);
        if (s->engine == ENGINE_BLOCK) {
            cfr::launch_x_best_response(s->xdev, s->dev.avgprob, s->stream);
        } else {
            for (int player = 1; player <= 2; ++player)
                cfr::launch_best_response(s->dev, s->level_offset.data(),
                                          s->infoset_level_offset.data(), player, s->stream);
        }
    }
    int rc = check_hip("best response launch");
    if (rc != CFR_OK) return rc;
    double br[2];
    HIP_TRY(hipMemcpyAsync(br, s->dev.out2, sizeof br, hipMemcpyDeviceToHost, s->stream), "br copy");
    HIP_TRY(hipStreamSynchronize(s->stream), "exploitability synchronise");
    *expl = 0.5 * (br[0] + br[1]);
    if (br_value != nullptr) {
        br_value[0] = br[0];
        br_value[1] = br[1];
    }
    return CFR_OK;
}

int cfr_get_state(cfr_solver* s, int64_t* T, float* R, float* S, int64_t n_q) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null solver");
    if (const int rc = check_precision(s, false); rc != CFR_OK) return rc;
    return get_state_t(s, s->dev, T, R, S, n_q);
}

int cfr_get_state_f64(cfr_solver* s, int64_t* T, double* R, double* S, int64_t n_q) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null solver");
    if (const int rc = check_precision(s, true); rc != CFR_OK) return rc;
    return get_state_t(s, s->dev64, T, R, S, n_q);
}

int cfr_set_state(cfr_solver* s, int64_t T, const float* R, const float* S, int64_t n_q) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null argument or negative T");
    if (const int rc = check_precision(s, false); rc != CFR_OK) return rc;
    return set_state_t(s, s->dev, T, R, S, n_q);
}

int cfr_set_state_f64(cfr_solver* s, int64_t T, const double* R, const double* S, int64_t n_q) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null argument or negative T");
    if (const int rc = check_precision(s, true); rc != CFR_OK) return rc;
    return set_state_t(s, s->dev64, T, R, S, n_q);
}

int64_t cfr_layout_bytes(cfr_solver* s, const char* name) {
    if (s == nullptr || name == nullptr) return CFR_EINVAL;
    const std::string n(name);
    if (s->partitioned()) return CFR_EINVAL;  // no canonical arrays on the device
    if (n == "reach_launch") return (launch_depth(s) + 1) * 4;  // batches too
    if (!s->canonical) return CFR_EINVAL;
    const cfr::Dev& d = s->dev;
    if (n == "level_offset") return (d.D + 2) * 4;
    if (n == "node_id" || n == "parent" || n == "node_infoset" || n == "node_edge") return d.N * 4;
    if (n == "child_begin") return (d.N + 1) * 4;
    if (n == "node_player") return d.N;
    if (n == "infoset_id") return d.Hp * 4;
    if (n == "infoset_player") return d.Hp;
    if (n == "q_offset" || n == "member_offset") return (d.Hp + 1) * 4;
    if (n == "chance_id") return d.H0 * 4;
    if (n == "cq_offset") return (d.H0 + 1) * 4;
    if (n == "members") return d.M * 4;
    if (n == "chance_prob") return d.Q0 * 4;
    if (n == "payoff") return d.N * 4;
    if (n == "q_input") return d.Qp * 4;
    return CFR_EINVAL;
}


int cfr_get_layout(cfr_solver* s, const char* name, void* out, int64_t bytes) {
    const int64_t need = cfr_layout_bytes(s, name);
    if (need < 0) return set_err(CFR_EINVAL, "unknown layout array");
    if (out == nullptr || bytes != need) return set_err(CFR_EINVAL, "wrong output size");
    const cfr::Dev& d = s->dev;
    const std::string n(name);
    if (n == "reach_launch") {
        const std::vector<int32_t> r = reach_launch(s);
        std::memcpy(out, r.data(), bytes);
        return CFR_OK;
    }
    const void* src = nullptr;
    if (n == "level_offset") src = d.level_offset;
    else if (n == "node_id") src = d.node_id;
    else if (n == "parent") src = d.parent;
    else if (n == "child_begin") src = d.child_begin;
    else if (n == "node_player") src = d.node_player;
    else if (n == "node_infoset") src = d.node_infoset;
    else if (n == "node_edge") src = d.node_edge;
    else if (n == "infoset_id") src = d.infoset_id;
    else if (n == "infoset_player") src = d.infoset_player;
    else if (n == "q_offset") src = d.q_offset;
    else if (n == "chance_id") src = d.chance_id;
    else if (n == "cq_offset") src = d.cq_offset;
    else if (n == "member_offset") src = d.member_offset;
    else if (n == "members") src = d.members;
    else if (n == "chance_prob") src = d.prob + d.Qp;
    else if (n == "payoff") src = d.payoff;
    else if (n == "q_input") src = d.q_input;
    if (bytes == 0) return CFR_OK;
    if (s->fp64 && (n == "chance_prob" || n == "payoff")) {
        // the FP64 solver holds these in double precision: exported rounded to float
        const int64_t count = bytes / 4;
        std::vector<double> tmp(count);
        const double* src64 = n == "payoff" ? s->dev64.payoff : s->dev64.prob + d.Qp;
        HIP_TRY(hipMemcpyAsync(tmp.data(), src64, count * sizeof(double), hipMemcpyDeviceToHost,
                               s->stream), "layout copy");
        HIP_TRY(hipStreamSynchronize(s->stream), "layout synchronise");
        float* o = static_cast<float*>(out);
        for (int64_t i = 0; i < count; ++i) o[i] = static_cast<float>(tmp[i]);
        return CFR_OK;
    }
    HIP_TRY(hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToHost, s->stream), "layout copy");
    HIP_TRY(hipStreamSynchronize(s->stream), "layout synchronise");
    return CFR_OK;
}

}  // extern "C"

namespace {

template <class F>
int node_values_t(cfr_solver* s, const F* value, const F* reach_planes, F* u1, F* reach,
                  int64_t n_nodes) {
    if (!s->canonical) return set_err(CFR_EINVAL, "node values are not exported for a batch");
    if (n_nodes != s->dev.N) return set_err(CFR_EINVAL, "n_nodes does not match the game");
    if (s->engine == ENGINE_BLOCK && s->xdev.n_tiers > 0 && !s->keep_nodes)
        return set_err(CFR_EINVAL, "the subtree packs keep node values on chip: build with "
                                   "CFR_FLAG_KEEP_NODE_VALUES to read them");
    const int64_t N = s->dev.N;
    std::vector<F> val(u1 != nullptr ? N : 0), planes(reach != nullptr ? 3 * N : 0);
    std::vector<int32_t> canon(s->engine == ENGINE_BLOCK ? N : 0);
    if (u1 != nullptr)
        HIP_TRY(hipMemcpyAsync(val.data(), value, N * sizeof(F), hipMemcpyDeviceToHost,
                               s->stream), "value copy");
    if (reach != nullptr)
        HIP_TRY(hipMemcpyAsync(planes.data(), reach_planes, 3 * N * sizeof(F),
                               hipMemcpyDeviceToHost, s->stream), "reach copy");
    if (s->engine == ENGINE_BLOCK)
        HIP_TRY(hipMemcpyAsync(canon.data(), s->xdev.canon_of, N * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s->stream), "order copy");
    HIP_TRY(hipStreamSynchronize(s->stream), "node values synchronise");
    for (int64_t x = 0; x < N; ++x) {
        const int64_t v = s->engine == ENGINE_BLOCK ? canon[x] : x;  // canonical position
        if (u1 != nullptr) u1[v] = val[x];
        if (reach != nullptr)
            for (int k = 0; k < 3; ++k) reach[3 * v + k] = planes[k * N + x];
    }
    return CFR_OK;
}

}  // namespace

extern "C" {

int cfr_get_node_values(cfr_solver* s, float* u1, float* reach, int64_t n_nodes) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null solver");
    if (s->players > 0) return set_err(CFR_EINVAL, "a general-sum solver: use cfr_get_node_values_n");
    if (const int rc = check_precision(s, false); rc != CFR_OK) return rc;
    return node_values_t(s, s->dev.value, s->dev.reach, u1, reach, n_nodes);
}

int cfr_get_node_values_f64(cfr_solver* s, double* u1, double* reach, int64_t n_nodes) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null solver");
    if (s->players > 0) return set_err(CFR_EINVAL, "a general-sum solver: use cfr_get_node_values_n");
    if (const int rc = check_precision(s, true); rc != CFR_OK) return rc;
    return node_values_t(s, s->dev64.value, s->dev64.reach, u1, reach, n_nodes);
}

int cfr_get_node_values_n(cfr_solver* s, double* values, double* reach, int64_t n_nodes) {
    if (s == nullptr) return set_err(CFR_EINVAL, "null solver");
    if (s->players <= 0)
        return set_err(CFR_EINVAL, "a two-player zero-sum solver: use cfr_get_node_values");
    if (n_nodes != s->dev.N) return set_err(CFR_EINVAL, "n_nodes does not match the game");
    const int64_t N = s->dev.N, P = s->players;
    std::vector<double> val(values != nullptr ? P * N : 0), planes(reach != nullptr ? (P + 1) * N : 0);
    auto fetch = [&](auto* src32, auto* src64, std::vector<double>& dst, int64_t count,
                     const char* what) -> int {
        if (s->fp64) {
            HIP_TRY(hipMemcpyAsync(dst.data(), src64, count * sizeof(double), hipMemcpyDeviceToHost,
                                   s->stream), what);
            return CFR_OK;
        }
        std::vector<float> tmp(count);
        HIP_TRY(hipMemcpyAsync(tmp.data(), src32, count * sizeof(float), hipMemcpyDeviceToHost,
                               s->stream), what);
        HIP_TRY(hipStreamSynchronize(s->stream), what);
        for (int64_t i = 0; i < count; ++i) dst[i] = tmp[i];
        return CFR_OK;
    };
    int rc;
    if (values != nullptr &&
        (rc = fetch(s->dev.value, s->dev64.value, val, P * N, "value copy")) != CFR_OK)
        return rc;
    if (reach != nullptr &&
        (rc = fetch(s->dev.reach, s->dev64.reach, planes, (P + 1) * N, "reach copy")) != CFR_OK)
        return rc;
    HIP_TRY(hipStreamSynchronize(s->stream), "node values synchronise");
    for (int64_t v = 0; v < N; ++v) {
        if (values != nullptr)
            for (int64_t i = 0; i < P; ++i) values[v * P + i] = val[i * N + v];
        if (reach != nullptr)
            for (int64_t k = 0; k <= P; ++k) reach[v * (P + 1) + k] = planes[k * N + v];
    }
    return CFR_OK;
}

int cfr_destroy(cfr_solver* s) {
    if (s == nullptr) return CFR_OK;
    (void)hipStreamSynchronize(s->stream);
    if (s->exec != nullptr) (void)hipGraphExecDestroy(s->exec);
    if (s->graph != nullptr) (void)hipGraphDestroy(s->graph);
    delete s;
    return CFR_OK;
}

}  // extern "C"


namespace {

}  // namespace

extern "C" {

int cfr_plan_batch(const cfr_game* games, int32_t n_games, const cfr_config* config,
                   cfr_plan_info* out) {
    if (games == nullptr || out == nullptr || n_games < 1) return set_err(CFR_EINVAL, "bad argument");
    if (const int rc = check_config(config); rc != CFR_OK) return rc;
    if (config != nullptr && (config->flags & CFR_FLAG_FP64))
        return set_err(CFR_EINVAL, "a batch runs on the public-block engine in FP32: "
                                   "CFR_FLAG_FP64 is for single games");
    Sizes z;
    z.engine = ENGINE_BLOCK;
    z.canonical = false;
    z.n_games = n_games;
    int64_t terminals = 0;
    for (int32_t g = 0; g < n_games; ++g) {
        cfr::Layout L;
        std::string err;
        const int rc = cfr::plan_sizes(games[g], L, err);
        if (rc != CFR_OK) return set_err(rc, "game " + std::to_string(g) + ": " + err);
        if (!L.level_pure) return set_err(CFR_ELEVEL, "game " + std::to_string(g) + " is not level pure");
        if (L.max_actions > 16) return set_err(CFR_EINVAL, "more than 16 actions in an infoset");
        z.N += L.N; z.Hp += L.Hp; z.Qp += L.Qp; z.H0 += L.H0; z.Q0 += L.Q0; z.M += L.n_members;
        z.C += L.n_chance_nodes; z.L += L.N;
        z.D = std::max(z.D, L.D);
        z.max_actions = std::max(z.max_actions, L.max_actions);
        terminals += L.n_terminals;
        z.terminals += L.n_terminals;
    }
    z.packs = z.max_actions <= 4 && config != nullptr && (config->flags & CFR_FLAG_SUBTREE_PACKS);
    cfr::Dev d{};
    cfr::Dev64 d64{};
    cfr::XDev x{};
    std::memset(out, 0, sizeof *out);
    out->n_nodes = z.N;
    out->n_terminals = terminals;
    out->n_infosets = z.Hp;
    out->n_q = z.Qp;
    out->n_chance_infosets = z.H0;
    out->n_chance_q = z.Q0;
    out->max_actions = z.max_actions;
    out->depth = z.D;
    out->level_pure = 1;
    out->engine = ENGINE_BLOCK;
    out->workspace_bytes = static_cast<int64_t>(carve(d, d64, x, nullptr, z));
    return CFR_OK;
}

int cfr_build_batch(const cfr_game* games, int32_t n_games, const cfr_config* config,
                    void* workspace, size_t bytes, void* stream, cfr_solver** out) {
    if (games == nullptr || workspace == nullptr || out == nullptr || n_games < 1)
        return set_err(CFR_EINVAL, "bad argument");
    cfr_config cfg{};
    cfg.variant = CFR_VANILLA;
    cfg.averaging = CFR_AVG_DEFAULT;
    if (config != nullptr) cfg = *config;
    if (const int rc = check_config(&cfg); rc != CFR_OK) return rc;
    if (cfg.flags & CFR_FLAG_FP64)
        return set_err(CFR_EINVAL, "a batch runs on the public-block engine in FP32: "
                                   "CFR_FLAG_FP64 is for single games");
    std::string err;
    std::vector<cfr::ExecPlan> plans;
    int32_t max_actions = 0;
    int rc = cfr::plan_games(games, n_games, plans, max_actions, err,
                             (cfg.flags & CFR_FLAG_SUBTREE_PACKS) != 0);
    if (rc != CFR_OK) return set_err(rc, err);
    cfr::ExecPlan F;
    rc = cfr::build_forest_plan(plans, F, err);
    if (rc != CFR_OK) return set_err(rc, err);
    plans.clear();
    plans.shrink_to_fit();
    Sizes z;
    z.N = F.N; z.Hp = F.Hp; z.Qp = F.Qp; z.Q0 = F.Q0; z.M = F.M; z.C = F.C; z.L = F.L; z.D = F.D;
    for (int8_t m : F.meta) z.terminals += (m & 3) == 0;
    z.max_actions = max_actions;
    z.engine = ENGINE_BLOCK;
    z.canonical = false;
    z.n_games = n_games;
    z.packs = max_actions <= 4 && (cfg.flags & CFR_FLAG_SUBTREE_PACKS);
    cfr::Dev d{};
    cfr::Dev64 d64{};
    cfr::XDev x{};
    // cfr_plan_batch bounds the explicit child lists by the node count, so a workspace of the
    // planned size always covers the exact need
    const size_t need = carve(d, d64, x, nullptr, z);
    if (bytes < need)
        return set_err(CFR_ENOMEM, "workspace has " + std::to_string(bytes) + " bytes, needs " +
                                       std::to_string(need));
    carve(d, d64, x, workspace, z);
    auto* s = new cfr_solver();
    s->dev = d;
    s->xdev = x;
    s->engine = ENGINE_BLOCK;
    s->n_games = n_games;
    s->canonical = false;
    s->rule = rule_of(cfg);
    s->alternating = (cfg.flags & CFR_FLAG_ALTERNATING) != 0;
    s->use_graph = (cfg.flags & CFR_FLAG_NO_GRAPH) == 0;
    s->level_pure = true;
    s->max_actions = max_actions;
    s->stream = static_cast<hipStream_t>(stream);
    hipStream_t st = s->stream;
    std::vector<float> prob_tail(F.Qp + F.Q0, 0.0f);
    std::copy(F.chance_prob.begin(), F.chance_prob.end(), prob_tail.begin() + F.Qp);
    cfr_default_launch_shape(&s->shape);
    if ((rc = upload_plan(s, F, st)) || (rc = upload(d.prob, prob_tail, st))) {
        discard(s);
        return rc;
    }
    cfr::launch_reset(d, st, false);
    cfr::launch_x_reset(s->xdev, st);
    if ((rc = check_hip("reset")) != CFR_OK) {
        discard(s);
        return rc;
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        discard(s);
        return hip_err(e, "build synchronise");
    }
    if (s->use_graph && (rc = capture(s)) != CFR_OK) {
        discard(s);
        return rc;
    }
    *out = s;
    return CFR_OK;
}

int cfr_exploitability_batch(cfr_solver* s, double* expl, double* br_values, int32_t n_games) {
    if (s == nullptr || expl == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (n_games != s->n_games) return set_err(CFR_EINVAL, "n_games does not match the batch");
    if (s->engine != ENGINE_BLOCK) return set_err(CFR_EINVAL, "not a batch solver");
    cfr::launch_average(s->dev, s->stream);
    cfr::launch_x_best_response(s->xdev, s->dev.avgprob, s->stream);
    int rc = check_hip("best response launch");
    if (rc != CFR_OK) return rc;
    std::vector<double> br(2 * static_cast<size_t>(n_games));
    HIP_TRY(hipMemcpyAsync(br.data(), s->dev.out2, br.size() * sizeof(double), hipMemcpyDeviceToHost,
                           s->stream), "br copy");
    HIP_TRY(hipStreamSynchronize(s->stream), "exploitability synchronise");
    for (int32_t g = 0; g < n_games; ++g) {
        expl[g] = 0.5 * (br[2 * g] + br[2 * g + 1]);
        if (br_values != nullptr) {
            br_values[2 * g] = br[2 * g];
            br_values[2 * g + 1] = br[2 * g + 1];
        }
    }
    return CFR_OK;
}

}  // extern "C"

extern "C" int cfr_warm_start(cfr_solver* s, const float* probs, int64_t n_q, float weight) {
    if (s == nullptr || probs == nullptr) return set_err(CFR_EINVAL, "null argument");
    if (n_q != s->dev.Qp) return set_err(CFR_ESTATE, "n_q does not match the game");
    if (!(weight >= 0.0f)) return set_err(CFR_EINVAL, "weight must be >= 0");
    cfr::launch_warm_start(s->dev.Hp, s->dev.sq_offset, s->dev.sq_input, probs, weight, s->dev.R,
                           s->dev.S, s->dev.prob, s->stream);
    cfr::launch_set_T(s->dev, 0, s->stream);
    s->T = 0;
    return check_hip("warm start");
}

