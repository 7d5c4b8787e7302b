// Device view of the public-block execution plan and its launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "xplan.hpp"

namespace cfr {

// Timer kinds continue after the node engine's kinds.
enum XKernelKind { XK_REACH = K_NUM_KINDS, XK_UP = K_NUM_KINDS + 1, XK_SUBTREE = K_NUM_KINDS + 2 };
const char* xkernel_kind_name(int kind);

// Launch shapes are chosen per log2 bucket of a launch's work items:
// bucket = floor(log2(units)) clamped to [0, kShapeBuckets).
constexpr int kShapeBuckets = 32;
int shape_bucket(int64_t units);

// Levels handled together by the single-workgroup kernels of the first levels.
constexpr int kFuseMax = 16;
constexpr int kFuseThreads = 1024;
// Top-down levels after those computed in one launch by walking up to the last stored level:
// levels of at most kPathNodes decision nodes, at most kPathDepthBelowTop of them below the
// single-workgroup levels, or at most kPathDepth from the roots when that covers as many
// levels as both launches (then there is no single-workgroup top-down launch); tiles of
// kPathThreads nodes.
constexpr int kPathDepth = 7;
constexpr int kPathDepthBelowTop = 5;
constexpr int64_t kPathNodes = 200000;
constexpr int kPathThreads = 256;
// Byte ranges that a single-workgroup kernel reads, touched once before its level chain (one
// byte per kWarmLine-byte line, every load in flight together), so that the chain's dependent
// loads find their lines in the L2 cache of the workgroup's XCD instead of going to memory
// one level at a time. Every entry is a valid range (unused ones repeat entry 0); lines[0]
// == 0: no ranges.
constexpr int kWarmMax = 18;
constexpr int kWarmLine = 64;
struct WarmTable {
    const uint8_t* p[kWarmMax];
    int32_t lines[kWarmMax];  // 1 .. kFuseThreads lines each
};

struct XDev {
    int64_t N, Hp, Qp, Q0, M, L, C;
    int32_t D, max_actions;
    // top-down launches (host), per level: threads per workgroup, nodes per thread, and the
    // level's tiles t_level_offset[l] .. t_level_offset[l + 1] - 1 (runs of decision nodes)
    const int32_t* reach_threads_host;  // D + 1
    const int32_t* reach_npt_host;      // D + 1
    const int32_t* t_level_offset_host; // D + 2
    const int64_t* reach_units_host;    // D + 1: decision nodes of each level
    // bottom-up shapes (host), per level: threads per workgroup and members per chunk
    // (threads x members per thread)
    const int32_t* up_threads_host;      // D + 1
    const int32_t* chunk_cap_host;       // D + 1
    const int32_t* k_level_offset_host;  // D + 2: chunks of each level
    const int32_t* m_level_offset_host;  // D + 2: first member of each level
    const int32_t* chance_glog_host;     // D + 1: log2 of lanes per chance node
    // host copies of the level tables (launch bounds)
    const int32_t* level_offset_host;
    const int32_t* h_level_offset_host;
    const int32_t* c_level_offset_host;
    // per level, the end of the upper prefix (the part outside the subtree packs) of its nodes,
    // infosets, chance nodes and bottom-up chunks (host)
    const int32_t* up_end_host;
    const int32_t* h_up_end_host;
    const int32_t* c_up_end_host;
    const int32_t* k_up_end_host;
    // subtree packs (device): descriptors and records; tiers 1 .. n_tiers, the packs of tier t
    // at tier_offset_host[t - 1] .. tier_offset_host[t] - 1 with tier_dec_host[t - 1] decision
    // nodes; keep_nodes != 0: the pack launches also store every node's value and reach
    int32_t n_tiers;
    const int32_t* tier_offset_host;
    const int64_t* tier_dec_host;
    const PackDesc* packs;
    const int32_t* pack_blob;
    uint32_t* pack_done;   // finished workgroups of the counting pack launch (0 between launches)
    int32_t keep_nodes;
    // some upper level has bottom-up work (else the last pack launch counts the iteration)
    int32_t upper_bottom_up;
    // the first levels run in one workgroup: top-down levels 1 .. fused_reach and
    // bottom-up levels fused_up - 1 .. 0 (0: none)
    int32_t fused_reach, fused_up;
    // top-down levels fused_reach + 1 .. path_reach run in one path launch (path_reach <=
    // fused_reach: none)
    int32_t path_reach;
    // per level (host): 1 if every upper decision node of the level has only terminal children
    const int8_t* only_terminal_children_host;
    // pair ranges [lo, hi) of prob that the single-workgroup kernels read (host): the infosets'
    // pairs and the chance probabilities of levels 0 .. fused_reach - 1 (entry 0) and
    // 0 .. fused_up - 1 (entry 1)
    int32_t top_q_lo[2], top_q_hi[2], top_c_lo[2], top_c_hi[2];
    // plan arrays (exec order)
    int32_t* parent;
    int32_t* edge;
    int8_t* meta;
    // per node, parent in the low 32 bits and edge | meta << 24 in the high 32 (ek_packed = 1 when
    // every edge index fits 24 bits): the per-level top-down launches read a node's parent, edge and
    // kind in one 8-byte load
    int64_t* parent_ek;
    int32_t ek_packed;
    int32_t* child_begin;
    int32_t* child_stride;
    int32_t* child_list;
    int32_t* canon_of;
    int32_t* q_offset;
    int8_t* iplayer;
    int32_t* member_offset;
    // member-major records (member m of the level-ordered member list), one 16-byte load each:
    // {node, its infoset's first pair, the node's child begin, its child stride}; and
    // k | (player 2 ? 64 : 0)
    int4* mem_rec;
    int8_t* mem_kp;
    // 1: mem_rec.w holds the child stride in its low 24 bits (signed) and the k | player byte in
    // its top byte (mem_kp is then read by the other kernels only)
    int32_t kp_packed;
    // infoset records: {first pair, first member, end of members, k | (player 2 ? 64 : 0)}
    int4* set_rec;
    int32_t* chance_nodes;
    int32_t* chance_base;  // index into prob of the chance node's action 0
    int32_t* chance_k;
    int32_t* tile_lo;      // top-down tiles: nodes tile_lo[t] .. tile_hi[t] - 1, all decision
    int32_t* tile_hi;      // nodes of one level (capacity: decision nodes)
    int32_t* chunk_first;  // chunks + 1 (capacity Hp + D + 2)
    int32_t* chunk_m;      // first member of each chunk, chunks + 1
    int32_t* q_input;
    float* payoff;
    // state (exec order)
    float* prob;     // Qp + Q0: sigma (exec pairs), then sigma_0
    float* R;
    float* S;
    float* value;    // N (terminals hold the payoff)
    float* reach;    // 3N planes: pi_1, pi_2 (every iteration), pi_c (set up once, constant)
    int64_t* T;
    float* br_reach;  // 2N: pi_{-1}, pi_{-2}
    float* br_value;  // 2N: values under player 1's, player 2's best response
    double* out2;
};

// How many first levels the single-workgroup kernels take (from the plan's level tables).
int32_t fusable_reach_levels(const int32_t* level_offset, const int32_t* up_end, int32_t D);
int32_t path_reach_levels(const int64_t* decision_nodes_per_level, int32_t fused, int32_t D,
                          int32_t max_depth);
int32_t fusable_up_levels(const int32_t* m_level_offset, const int32_t* m_up_end,
                          const int32_t* h_level_offset, const int32_t* h_up_end,
                          const int32_t* c_level_offset, const int32_t* c_up_end,
                          const int32_t* chance_glog, int32_t D, int32_t max_actions);

// The level whose top-down reach its bottom-up launch computes (from the parents' stored
// reach) instead of a top-down launch of its own, or -1.
int32_t derived_reach_level(const XDev& x);

void launch_x_reset(const XDev& x, hipStream_t st);
void launch_x_iteration(const XDev& x, const UpdateRule& rule, hipStream_t st,
                        LaunchTimer* timer = nullptr);
// Best responses of both players to sigma-bar (avgprob: exec pairs, then sigma_0); the root
// values land in out2[2 g], out2[2 g + 1].
void launch_x_best_response(const XDev& x, const float* avgprob, hipStream_t st);
void launch_x_values_to_canonical(const XDev& x, float* dst, hipStream_t st);
void launch_x_reach_to_canonical(const XDev& x, float* dst, hipStream_t st);

}  // namespace cfr
