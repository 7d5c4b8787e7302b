// Subtree-partitioned, out-of-core iteration (host side): the plan that cuts a canonical layout
// at one level into a resident top and partitions of whole subtrees, each partition's levels
// below the cut renumbered into one device window, and the per-partition arrays held in pinned
// host memory and streamed through the window every iteration.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "partition_plan.hpp"

namespace cfr {

// Device side of a partitioned solver of real type F: the pinned host copies of the window
// arrays and the device window they are streamed into.
template <class F>
struct PartDev {
    PartPlan plan;
    // pinned host memory (hipHostMalloc), released by release()
    int32_t *h_parent = nullptr, *h_cb = nullptr, *h_infoset = nullptr, *h_edge = nullptr;
    int8_t* h_player = nullptr;
    F* h_value0 = nullptr;
    int32_t* h_patch = nullptr;
    std::vector<int32_t> level_offset;  // canonical, D + 2 (the resident levels)
    int upload(hipStream_t st);         // plan -> pinned buffers (once, at build)
    void release();
};

// One pass of the partitioned iteration on d (N = base + window local nodes; structure of the
// resident levels uploaded at build): resident top-down, then per partition its window
// streamed in, its top-down and bottom-up, and the bottom-up of its level-cut nodes; the
// resident bottom-up; the infoset pass.
template <class F>
void launch_partitioned_pass(const DevT<F>& d, const PartDev<F>& P, const UpdateRule& rule,
                             hipStream_t st);

}  // namespace cfr
