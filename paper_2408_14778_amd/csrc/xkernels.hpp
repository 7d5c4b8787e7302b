// Device view of the public-block execution plan and its launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace cfr {

// Timer kinds continue after the node engine's kinds.
enum XKernelKind { XK_REACH = K_NUM_KINDS, XK_UP = K_NUM_KINDS + 1 };
const char* xkernel_kind_name(int kind);

// Launch shapes: threads per workgroup for a launch of `units` work items is
// table[bucket(units)], bucket = floor(log2(units)) clamped to [0, kShapeBuckets).
constexpr int kShapeBuckets = 32;
int shape_bucket(int64_t units);

struct XDev {
    int64_t N, Hp, Qp, Q0, M, L, C;
    int32_t D, max_actions;
    const int32_t* up_block;     // host, kShapeBuckets entries (unused by the chunked bottom-up)
    const int32_t* reach_block;  // host, kShapeBuckets entries (nullptr: 256 threads)
    const int32_t* k_level_offset_host;  // D + 2: chunks of each level
    const int32_t* chunk_cap_host;       // D + 1: members per chunk (= threads) of each level
    const int32_t* m_level_offset_host;  // D + 2: first member of each level
    // host copies of the level tables (launch bounds)
    const int32_t* level_offset_host;
    const int32_t* h_level_offset_host;
    const int32_t* c_level_offset_host;
    // plan arrays (exec order)
    int32_t* parent;
    int32_t* edge;
    int8_t* meta;
    int32_t* child_begin;
    int32_t* child_stride;
    int32_t* child_list;
    int32_t* canon_of;
    int32_t* q_offset;
    int8_t* iplayer;
    int32_t* member_offset;
    int32_t* members;
    int32_t* chance_nodes;
    int32_t* chance_base;  // index into prob of the chance node's action 0
    int32_t* chance_k;
    int32_t* chunk_first;  // chunks + 1 (capacity Hp + D + 2)
    int32_t* q_input;
    float* payoff;
    // state (exec order)
    float* prob;     // Qp + Q0: sigma (exec pairs), then sigma_0
    float* R;
    float* S;
    float* value;    // N (terminals hold the payoff)
    float* reach;    // 3N planes
    int64_t* T;
    float* br_reach;
    float* br_value;
    double* out2;
};

void launch_x_reset(const XDev& x, hipStream_t st);
void launch_x_iteration(const XDev& x, int variant, int linear, hipStream_t st,
                        LaunchTimer* timer = nullptr);
void launch_x_best_response(const XDev& x, const float* avgprob, int player, hipStream_t st);
void launch_x_values_to_canonical(const XDev& x, float* dst, hipStream_t st);
void launch_x_reach_to_canonical(const XDev& x, float* dst, hipStream_t st);

}  // namespace cfr
