// Execution plan: the canonical layout re-ordered into "public blocks" for the GPU.
//
// The paper's per-level sparse products (Section 3.2) touch, for each infoset, the
// nodes of its members and their children. In breadth-first order those members are
// scattered across the level (one per private deal), so every infoset reduction is a
// gather over distant cache lines. The plan groups each level's nodes into blocks:
//   (a) all members of a rational infoset share a block;
//   (b) the parents of a block's nodes share a block (so blocks form a tree);
//   (c) the children, by one action, of a block of rational-player nodes share a block.
// (a)-(c) give the finest such partition (union-find). In poker-like games a block is a
// public state: the same public history under every private deal. Nodes are ordered
// level by level, blocks in (parent block, first action, first canonical node) order,
// and nodes inside a block in canonical order. Then an infoset's members lie inside one
// block, a block's children by one action form the next block at the same offsets, and
// infosets of one level are numbered contiguously, so one thread per infoset can compute
// its members' values, its regrets and its regret-matching update with nearby reads.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "flatten.hpp"

namespace cfr {

constexpr int kChunk = 256;  // members per bottom-up workgroup (= threads per workgroup)

struct ExecPlan {
    int64_t N = 0, Hp = 0, Qp = 0, Q0 = 0, M = 0, L = 0, C = 0;
    int32_t D = 0;
    std::vector<int32_t> exec_of;        // canonical node -> exec node
    std::vector<int32_t> canon_of;       // exec node -> canonical node
    std::vector<int32_t> level_offset;   // D + 2 (same level sizes as canonical)
    // per exec node
    std::vector<int32_t> parent;         // exec parent, -1 at root
    std::vector<int32_t> edge;           // exec edge index into [sigma_exec | sigma_0], -1 at root
    std::vector<int8_t> meta;            // bits 0-1: own kind + 1 (0 terminal, 1 chance, 2 P1, 3 P2)
                                         // bits 2-3: actor into the node + 1 (0 root, 1 chance, 2 P1, 3 P2)
    std::vector<int32_t> child_begin;    // exec index of the action-0 child, or offset into child_list
    std::vector<int32_t> child_stride;   // exec distance between consecutive children; 0 = listed
    std::vector<int32_t> child_list;     // explicit children (exec), for irregular nodes
    std::vector<float> payoff;           // u_1 at terminals, 0 elsewhere
    // rational infosets in exec numbering (contiguous per level)
    std::vector<int32_t> infoset_canon;  // exec infoset -> canonical infoset
    std::vector<int8_t> infoset_player;
    std::vector<int32_t> q_offset;       // Hp + 1
    std::vector<int32_t> member_offset;  // Hp + 1
    std::vector<int32_t> members;        // exec member nodes, ascending
    std::vector<int32_t> h_level_offset; // D + 2: infosets of level l
    // chance nodes per level
    std::vector<int32_t> chance_nodes;   // exec indices, level-major
    std::vector<int32_t> c_level_offset; // D + 2
    std::vector<int32_t> chance_base;    // per chance node: index into [sigma | sigma_0] of action 0
    std::vector<int32_t> chance_k;       // per chance node: number of actions
    std::vector<float> chance_prob;      // sigma_0, Q0 entries (the tail of the probability array)
    // bottom-up work chunks: runs of whole infosets of one level with at most kChunk members
    // (an infoset with more members is a chunk of its own); chunk c covers infosets
    // chunk_first[c] .. chunk_first[c + 1] - 1; chunks of level l are k_level_offset[l] ..
    std::vector<int32_t> chunk_first;    // n_chunks + 1 (last entry = Hp)
    std::vector<int32_t> k_level_offset; // D + 2
    // pair maps
    std::vector<int32_t> q_input;        // exec pair -> input pair
    int64_t n_blocks = 0;
    int64_t n_listed = 0;                // nodes whose children are listed explicitly
};

// Requires level-pure infosets. Returns CFR_OK or an error code with a message.
int build_exec_plan(const Layout& L, ExecPlan& P, std::string& err);

// Forest of independent games, level-major: level l of the forest is level l of game 0, then
// of game 1, ...; so level 0 holds the games' roots in game order. Infosets and pairs are
// numbered per level across games; q_input maps a forest pair to its position in the
// concatenation of the games' input pair orders (game 0's pairs first).
int build_forest_plan(const std::vector<ExecPlan>& games, ExecPlan& F, std::string& err);

// Fills chunk_first / k_level_offset from h_level_offset and member_offset; level l packs at
// most members_per_chunk[l] members per chunk (default kChunk for every level).
void build_chunks(ExecPlan& P, const int32_t* members_per_chunk = nullptr);
void build_chunks(const std::vector<int32_t>& h_level_offset,
                  const std::vector<int32_t>& member_offset, const int32_t* members_per_chunk,
                  std::vector<int32_t>& chunk_first, std::vector<int32_t>& k_level_offset);

}  // namespace cfr
