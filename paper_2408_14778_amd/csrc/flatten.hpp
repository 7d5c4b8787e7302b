// Host-side flattener: the game tuple of Definition 1 (Section 2.1) into the canonical
// level-ordered index arrays that replace the constant matrices of Section 3.1.
//
// Each of those matrices has at most one nonzero per column, so each becomes an index
// array: G and the level graphs L^(l) become parent / child_begin / level_offset,
// M^(Q+,V) becomes node_edge (and the infoset member lists), M^(H+,Q+) becomes q_offset,
// M^(V,I+) becomes the player of the parent, and s^(sigma0) becomes chance_prob indexed
// through node_edge.
//
// Canonical order: breadth-first from the root, each node's children appended in action
// order. Level l+1 is therefore sorted by (canonical parent, action), every parent's
// children are contiguous, and levels are contiguous ranges. Rational infosets are
// numbered by first appearance in that order, chance infosets likewise (separately).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cfr.h"

namespace cfr {

struct Layout {
    int64_t N = 0, n_terminals = 0, n_chance_nodes = 0, n_members = 0;
    int64_t Hp = 0, Qp = 0, H0 = 0, Q0 = 0;
    int32_t D = 0, max_actions = 0;
    bool level_pure = true;

    std::vector<int32_t> level_offset;   // D + 2
    std::vector<int32_t> node_id;        // canonical -> input node
    std::vector<int32_t> parent;         // canonical parent, -1 at root
    std::vector<int32_t> child_begin;    // N + 1
    std::vector<int8_t> node_player;     // -1 terminal, 0 chance, 1 .. players
    std::vector<int32_t> node_infoset;   // rational or chance canonical id, -1 terminal
    std::vector<int32_t> node_edge;      // unified edge index into [sigma | sigma_0], -1 root
    std::vector<int32_t> infoset_id;     // canonical rational infoset -> input id
    std::vector<int8_t> infoset_player;  // 1 .. players
    std::vector<int32_t> q_offset;       // Hp + 1
    std::vector<int32_t> chance_id;      // canonical chance infoset -> input id
    std::vector<int32_t> cq_offset;      // H0 + 1
    std::vector<int32_t> member_offset;  // Hp + 1
    std::vector<int32_t> members;        // member nodes per rational infoset, ascending
    std::vector<float> chance_prob;      // Q0
    std::vector<float> payoff;           // N, u_1 at terminals, 0 elsewhere
    // the same two in double precision (filled only when flatten is asked for them)
    std::vector<double> chance_prob64;   // Q0
    std::vector<double> payoff64;        // N
    std::vector<int32_t> q_input;        // canonical pair -> input pair
};

// Validates and flattens. Returns CFR_OK or a CFR_E* code with a message in `err`. f64: also
// fill chance_prob64 and payoff64 with the input's double values. max_player: the highest
// rational player an infoset may name (2, or n for a game of n players).
int flatten(const cfr_game& g, Layout& out, std::string& err, bool f64 = false,
            int32_t max_player = 2);

// Validation and sizes only (no layout arrays kept).
int plan_sizes(const cfr_game& g, Layout& sizes, std::string& err, int32_t max_player = 2);

}  // namespace cfr
