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

// Subtree packs. A pack is a set of public blocks of one level together with the blocks below
// them, small enough for one workgroup to hold the reach of every decision node, the value of
// every decision node and the strategy, regrets and averages of every pair in LDS. The blocks
// are assigned in tiers: tier 1 takes the highest blocks whose whole subtree fits; tier t + 1
// the highest remaining blocks whose subtree fits once the roots of tiers 1..t count as
// leaves ("external" children, whose values those tiers produce). An iteration then runs the
// levels outside every pack (the "upper" prefix of each level) top-down, each tier from the
// highest down computing its packs' reach and storing the reach of the nodes that have
// external children, tier 1 through both sweeps and its infoset updates, each tier from 2 up
// recomputing its reach on chip and finishing its bottom-up sweep and updates, then the upper
// levels bottom-up. Each pack is described by compact records (pack_blob), read in one burst:
// children as LDS indices, terminal payoffs inline, external children by node index.
constexpr int kPackDec = 512;      // decision nodes (player and chance) of a pack
constexpr int kPackPairs = 384;    // infoset-action pairs of a pack
constexpr int kPackChance = 128;   // chance nodes of a pack
constexpr int kPackKids = 1024;    // children of a pack's chance nodes
constexpr int kPackLevels = 8;     // levels a pack spans
constexpr int kPackSubMembers = 256;  // members of an infoset in a pack
constexpr int kPackThreads = 256;     // threads of a pack workgroup
constexpr int kPackSlots = kPackDec / kPackThreads;  // member (and infoset) records per thread
constexpr int kMaxTiers = 8;

// Record layouts in pack_blob (int32 words), offsets relative to the pack's section starts:
//  root (4 words): {didx | actor << 16, parent node, edge index, node}; parent -1: the game's
//     root (reach 1); actor: 1 chance, 2 player 1, 3 player 2 (the kind of the parent)
//  member (6 words): {didx | k << 16 | p2 << 19 | boundary << 20 | kind_a << (24 + 2 a),
//     first local pair, child 0..3}; child kind 0: a decision node of the pack (its didx),
//     1: a terminal (its payoff, float bits), 2: an external child (its node index);
//     boundary: some child is external
//  infoset (4 words): {first pair (global), first local pair, first member | end member << 16,
//     k | player << 8}
//  chance (4 words): {didx | boundary << 20, k, first child record (local), 0}
//  chance child (3 words): {child (as for members), probability (float bits), kind}
//  node (1 word per didx): the decision node's exec index
// Root, infoset and chance sections start 16-byte aligned (they are read as int4).
struct PackDesc {
    int32_t tier, level0, nlv, n_dec, n_mem, n_ch, n_root, n_inf, n_pairs, n_kid;
    int32_t off_root, off_mem, off_inf, off_ch, off_kid, off_node;
    int32_t mlo[kPackLevels + 1];  // members of level level0 + i: mlo[i] .. mlo[i + 1] - 1
    int32_t clo[kPackLevels + 1];  // chance nodes, likewise
};

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
    // chunks of level l outside the packs: k_level_offset[l] .. k_up_end[l] - 1
    std::vector<int32_t> k_up_end;       // D + 1
    // upper prefix of each level (blocks outside the packs): nodes level_offset[l] ..
    // up_end[l] - 1, infosets h_level_offset[l] .. h_up_end[l] - 1, chance nodes
    // c_level_offset[l] .. c_up_end[l] - 1
    std::vector<int32_t> up_end, h_up_end, c_up_end;  // D + 1 each
    // subtree packs, tier by tier: the packs of tier t are packs[tier_offset[t - 1]] ..
    // packs[tier_offset[t] - 1], t = 1 .. n_tiers
    std::vector<PackDesc> packs;
    std::vector<int32_t> pack_blob;
    std::vector<int32_t> tier_offset;    // n_tiers + 1
    int32_t n_tiers = 0;
    // pair maps
    std::vector<int32_t> q_input;        // exec pair -> input pair
    int64_t n_blocks = 0;
    int64_t n_listed = 0;                // nodes whose children are listed explicitly
};

// Requires level-pure infosets. Returns CFR_OK or an error code with a message. deep = false:
// no subtree packs (every level entirely in the per-level launches). Packs need at most 4
// actions per infoset.
int build_exec_plan(const Layout& L, ExecPlan& P, std::string& err, bool deep = true);

// Forest of independent games, level-major: level l of the forest is level l of game 0, then
// of game 1, ...; so level 0 holds the games' roots in game order. Infosets and pairs are
// numbered per level across games; q_input maps a forest pair to its position in the
// concatenation of the games' input pair orders (game 0's pairs first).
int build_forest_plan(const std::vector<ExecPlan>& games, ExecPlan& F, std::string& err);

// Per level: the decision nodes of the upper prefix, and whether all their children are
// terminal (1) or not (0).
void upper_level_stats(const ExecPlan& P, std::vector<int64_t>& decision,
                       std::vector<int8_t>& only_terminal_children);

// Fills chunk_first / k_level_offset from h_level_offset and member_offset; level l packs at
// most members_per_chunk[l] members per chunk (default kChunk for every level).
void build_chunks(ExecPlan& P, const int32_t* members_per_chunk = nullptr);
// With h_split (per level: end of the upper infosets), no chunk straddles it and k_split
// receives each level's first chunk past it.
void build_chunks(const std::vector<int32_t>& h_level_offset,
                  const std::vector<int32_t>& member_offset, const int32_t* members_per_chunk,
                  std::vector<int32_t>& chunk_first, std::vector<int32_t>& k_level_offset,
                  const std::vector<int32_t>* h_split = nullptr,
                  std::vector<int32_t>* k_split = nullptr);

}  // namespace cfr
