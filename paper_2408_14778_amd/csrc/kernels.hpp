// Device arrays of one solver and the launch wrappers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cfr {

// The most rational players of a general-sum game (the general-sum value kernels hold one
// register per player).
constexpr int32_t kMaxPlayers = 8;

// All pointers are device memory inside the caller's workspace, canonical order. F is the
// arithmetic type of the values, probabilities and state: float (the default path) or double
// (the FP64 path of the node engine).
template <class F>
struct DevT {
    int64_t N, Hp, Qp, H0, Q0, M;
    int32_t D;
    // rational players of a general-sum game (Section 3.1: one payoff column per player), or 0
    // for a two-player zero-sum game (u_2 = -u_1, one column). With n > 0, payoff and value hold
    // n columns (player i's at (i - 1) * N + v) and reach n + 1 planes (the players', then
    // chance's).
    int32_t players = 0;
    // structure (constant after build)
    int32_t* parent;        // N
    int32_t* child_begin;   // N + 1
    int8_t* node_player;    // N
    int32_t* node_infoset;  // N
    int32_t* node_edge;     // N
    int32_t* node_id;       // N
    int32_t* level_offset;  // D + 2
    int32_t* infoset_id;    // Hp
    int8_t* infoset_player; // Hp
    int32_t* q_offset;      // Hp + 1
    int32_t* chance_id;     // H0
    int32_t* cq_offset;     // H0 + 1
    int32_t* member_offset; // Hp + 1
    int32_t* members;       // M
    int32_t* q_input;       // Qp
    // general-sum games (players > 0): the gather pass reads each infoset's regret contributions
    // and own reaches in member order, contiguously. Infoset h owns n_h (k_h + 1) values of
    // contrib from slot_base[h]: for its j-th member v, from node_slot[v] = slot_base[h] +
    // j (k_h + 1), v's k_h action contributions, then v's own reach (unused at other nodes)
    int32_t* node_slot;     // N (players > 0)
    int32_t* slot_base;     // Hp + 1 (players > 0)
    F* payoff;              // N (players > 0: players * N)
    // iteration state
    F* prob;                // Qp + Q0: current sigma, then sigma_0
    F* R;                   // Qp cumulative regret
    F* S;                   // Qp cumulative average-strategy weight
    F* rtilde;              // Qp accumulator (zero between iterations)
    F* pibar;               // Hp accumulator (zero between iterations)
    F* contrib;             // N, the regret contribution of each player node's child, summed
                            //   per infoset by the gather pass: games whose infosets average
                            //   more than 16 members (many atomic additions to one accumulator
                            //   serialise); players > 0: N + M in the member-order slots of
                            //   node_slot; null: the value kernels add to rtilde and pibar by
                            //   atomics
    F* value;               // N  expected payoff of player 1 (terminals hold the payoff);
                            //    players > 0: players * N, one column per player
    F* reach;               // 3N (pi_1, pi_2, pi_c) planes; players > 0: (players + 1) N
    int64_t* T;             // iterations done (device copy)
    // exploitability and staging
    F* avgprob;             // Qp + Q0: average strategy, then sigma_0
    F* br_reach;            // N
    F* br_value;            // N
    int32_t* best;          // Hp
    F* stage;               // 2 * Qp (state and average-strategy transfers)
    double* out2;           // 2 best-response values
    // pair numbering of the state arrays (canonical for the node engine, exec for the
    // block engine)
    int32_t* sq_offset;     // Hp + 1
    int32_t* sq_input;      // Qp
};
using Dev = DevT<float>;
using Dev64 = DevT<double>;

// Zero R, S, accumulators and T; sigma uniform; values at terminals; root reach 1.
// node_arrays = false skips the canonical per-node state (the block engine resets its own).
template <class F>
void launch_reset(const DevT<F>& d, hipStream_t st, bool node_arrays = true);
// sigma = regret matching of R (all infosets).
template <class F>
void launch_regret_match(const DevT<F>& d, hipStream_t st);
// Kernel kinds of one iteration, for per-kernel timing.
enum KernelKind { K_REACH = 0, K_VALUE = 1, K_INFOSET = 2, K_TICK = 3, K_NUM_KINDS = 4 };
const char* kernel_kind_name(int kind);

// Optional per-launch hooks, called before and after each launch of an iteration with the
// kernel kind, the tree level it processes (-1 if none) and its number of work items.
struct LaunchTimer {
    virtual void before(int kind, int level, int64_t units, hipStream_t st) = 0;
    virtual void after(int kind, hipStream_t st) = 0;
    virtual ~LaunchTimer() = default;
};

// The cumulative-regret and average-strategy update of an iteration (Eqs.
// average_counterfactual_regrets_vector and average_strategy_profile_vector in cumulative form):
// variant 0 vanilla, 1 CFR+ (regrets clipped at zero), 2 discounted (the weighting scheme the
// paper's discussion names: exponents alpha on positive cumulative regrets, beta on the others,
// gamma on the strategy sums); linear weights iteration t's strategy by t (variants 0 and 1).
// players: the players whose infosets a pass updates (bit i - 1 player i; the others keep R, S
// and sigma); count: whether the pass ends the iteration (T += 1). The alternating schedule is a
// pass with players 1, count 0, then one with players 2, count 1.
struct UpdateRule {
    int32_t variant = 0;
    int32_t linear = 0;
    float alpha = 1.5f, beta = 0.0f, gamma = 2.0f;
    int32_t players = 3;
    int32_t count = 1;
};

// The discounted update's factors for iteration t (1-based): t^alpha / (t^alpha + 1) on positive
// cumulative regrets, t^beta / (t^beta + 1) on the others, (t / (t + 1))^gamma on the strategy
// sums; written as 1 / (1 + t^-x) so that a large t^x cannot overflow, and with the powers as
// exp2(x log2 t) (t >= 1) on the hardware's base-2 exponential and logarithm, which keeps the
// infoset update short. With y = x log2 t, a relative rounding e of y moves 1 / (1 + 2^-y) by a
// relative e y ln2 / (1 + 2^y), below e for every y >= 0 and below e |y| for y < 0, where the
// factor itself is below 2^y.
__device__ __forceinline__ void dcfr_discounts(const UpdateRule& u, float t, float& pos, float& neg,
                                               float& avg) {
    const float lt = log2f(t);
    pos = 1.0f / (1.0f + exp2f(-u.alpha * lt));
    neg = 1.0f / (1.0f + exp2f(-u.beta * lt));
    avg = exp2f(u.gamma * log2f(t / (t + 1.0f)));
}
// The same factors in double precision (the FP64 path), from the same exponents.
__device__ __forceinline__ void dcfr_discounts(const UpdateRule& u, double t, double& pos,
                                               double& neg, double& avg) {
    const double lt = log2(t);
    pos = 1.0 / (1.0 + exp2(-static_cast<double>(u.alpha) * lt));
    neg = 1.0 / (1.0 + exp2(-static_cast<double>(u.beta) * lt));
    avg = exp2(static_cast<double>(u.gamma) * log2(t / (t + 1.0)));
}

// One iteration (Section 3.2): top-down reach, bottom-up values + regrets, infoset update.
template <class F>
void launch_iteration(const DevT<F>& d, const int32_t* level_offset_host, const UpdateRule& rule,
                      hipStream_t st, LaunchTimer* timer = nullptr);
// The parts of one iteration on a node range [lo, hi) of one level (the partitioned iteration
// composes them): top-down reach, bottom-up values with the regret and own-reach accumulation;
// then the infoset pass over every infoset (and T += 1 if rule.count).
template <class F>
void launch_reach_range(const DevT<F>& d, int32_t lo, int32_t hi, hipStream_t st);
template <class F>
void launch_value_range(const DevT<F>& d, int32_t lo, int32_t hi, hipStream_t st);
template <class F>
void launch_infoset_pass(const DevT<F>& d, const UpdateRule& rule, hipStream_t st);
// Average strategy into d.avgprob (canonical order; chance tail copied at reset).
template <class F>
void launch_average(const DevT<F>& d, hipStream_t st);
// Best response of player i against d.avgprob; value lands in d.out2[i - 1].
template <class F>
void launch_best_response(const DevT<F>& d, const int32_t* level_offset_host,
                          const int32_t* infoset_level_offset_host, int player, hipStream_t st);
// dst[q_input[q]] = src[q]  (canonical -> input order)
template <class F>
void launch_scatter_q(const DevT<F>& d, const F* src, F* dst, hipStream_t st);
// dst[q] = src[q_input[q]]  (input -> canonical order)
template <class F>
void launch_gather_q(const DevT<F>& d, const F* src, F* dst, hipStream_t st);
// *T = value
template <class F>
void launch_set_T(const DevT<F>& d, int64_t value, hipStream_t st);

}  // namespace cfr
