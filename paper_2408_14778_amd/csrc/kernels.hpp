// Device arrays of one solver and the launch wrappers of the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cfr {

// All pointers are device memory inside the caller's workspace, canonical order.
struct Dev {
    int64_t N, Hp, Qp, H0, Q0, M;
    int32_t D;
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
    float* payoff;          // N
    // iteration state
    float* prob;            // Qp + Q0: current sigma, then sigma_0
    float* R;               // Qp cumulative regret
    float* S;               // Qp cumulative average-strategy weight
    float* rtilde;          // Qp accumulator (zero between iterations)
    float* pibar;           // Hp accumulator (zero between iterations)
    float* value;           // N  expected payoff of player 1 (terminals hold the payoff)
    float* reach;           // 3N (pi_1, pi_2, pi_c) planes
    int64_t* T;             // iterations done (device copy)
    // exploitability and staging
    float* avgprob;         // Qp + Q0: average strategy, then sigma_0
    float* br_reach;        // N
    float* br_value;        // N
    int32_t* best;          // Hp
    float* stage;           // 2 * Qp (state and average-strategy transfers)
    double* out2;           // 2 best-response values
    // pair numbering of the state arrays (canonical for the node engine, exec for the
    // block engine)
    int32_t* sq_offset;     // Hp + 1
    int32_t* sq_input;      // Qp
};

// Zero R, S, accumulators and T; sigma uniform; values at terminals; root reach 1.
// node_arrays = false skips the canonical per-node state (the block engine resets its own).
void launch_reset(const Dev& d, hipStream_t st, bool node_arrays = true);
// sigma = regret matching of R (all infosets).
void launch_regret_match(const Dev& d, hipStream_t st);
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

// One iteration (Section 3.2): top-down reach, bottom-up values + regrets, infoset update.
void launch_iteration(const Dev& d, const int32_t* level_offset_host, int variant, int linear,
                      hipStream_t st, LaunchTimer* timer = nullptr);
// Average strategy into d.avgprob (canonical order; chance tail copied at reset).
void launch_average(const Dev& d, hipStream_t st);
// Best response of player i against d.avgprob; value lands in d.out2[i - 1].
void launch_best_response(const Dev& d, const int32_t* level_offset_host,
                          const int32_t* infoset_level_offset_host, int player, hipStream_t st);
// dst[q_input[q]] = src[q]  (canonical -> input order)
void launch_scatter_q(const Dev& d, const float* src, float* dst, hipStream_t st);
// dst[q] = src[q_input[q]]  (input -> canonical order)
void launch_gather_q(const Dev& d, const float* src, float* dst, hipStream_t st);
// *T = value
void launch_set_T(const Dev& d, int64_t value, hipStream_t st);

}  // namespace cfr
