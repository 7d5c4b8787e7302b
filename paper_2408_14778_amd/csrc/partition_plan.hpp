// Subtree-partitioned, out-of-core iteration: the host plan (no HIP), which cuts a canonical
// layout at one level into a resident top and partitions of whole subtrees, each partition's
// levels below the cut renumbered into one device window.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "flatten.hpp"

namespace cfr {

// Window layout of partition p: its nodes at levels cut + 1 .. D, level by level in canonical
// order, at local ids base .. base + n[p] - 1 (base = level_offset[cut + 1], the first id past
// the resident levels 0 .. cut, whose local ids are their canonical ids).
struct PartPlan {
    int32_t cut = 0, D = 0;
    int64_t base = 0;          // first window id
    int64_t window = 0;        // largest partition (window nodes)
    int64_t total = 0;         // window nodes of all partitions (= N - base)
    int32_t parts = 0;
    std::vector<int32_t> a, b;     // level-cut node range [a, b) of each partition
    std::vector<int64_t> off;      // first node of each partition in the host arrays (parts + 1)
    std::vector<int32_t> lo;       // per partition, local level offsets of levels cut + 1 .. D + 1
    std::vector<int64_t> patch_off;  // per partition, its level-cut child_begin patch (b - a + 1)
    // host arrays, partition-major (node arrays: off[p] + i; child_begin: off[p] + p + i)
    std::vector<int32_t> parent, child_begin, infoset, edge;
    std::vector<int8_t> player;
    std::vector<double> value0;    // the payoff at terminal nodes, 0 elsewhere
    std::vector<int32_t> patch;    // level-cut child_begin entries, local, per partition
};

// Plans the partitions of layout L cut at level `cut` (1 <= cut <= D - 1), grouping consecutive
// level-cut subtrees while their window nodes stay within max_window (a larger subtree is a
// partition of its own; terminal level-cut nodes join the current partition). CFR_OK or
// CFR_EINVAL with a message.
int plan_partitions(const Layout& L, int32_t cut, int64_t max_window, PartPlan& P, std::string& err);

}  // namespace cfr
