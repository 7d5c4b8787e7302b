// Device side of the subtree-partitioned, out-of-core iteration: pinned host buffers of the
// partition windows, and one pass of the iteration that streams them through the device window.
#include "partition.hpp"

#include <cstring>

namespace cfr {

namespace {

template <class T>
int pinned(T** p, int64_t n) {
    *p = nullptr;
    if (n <= 0) return 0;
    return hipHostMalloc(reinterpret_cast<void**>(p), static_cast<size_t>(n) * sizeof(T),
                         hipHostMallocDefault) == hipSuccess
               ? 0
               : -1;
}

}  // namespace

template <class F>
int PartDev<F>::upload(hipStream_t) {
    const PartPlan& P = plan;
    if (pinned(&h_parent, P.total) || pinned(&h_infoset, P.total) || pinned(&h_edge, P.total) ||
        pinned(&h_player, P.total) || pinned(&h_value0, P.total) ||
        pinned(&h_cb, P.total + P.parts) || pinned(&h_patch, static_cast<int64_t>(P.patch.size()))) {
        release();
        return -1;
    }
    if (P.total > 0) {
        std::memcpy(h_parent, P.parent.data(), P.total * sizeof(int32_t));
        std::memcpy(h_infoset, P.infoset.data(), P.total * sizeof(int32_t));
        std::memcpy(h_edge, P.edge.data(), P.total * sizeof(int32_t));
        std::memcpy(h_player, P.player.data(), P.total * sizeof(int8_t));
        for (int64_t i = 0; i < P.total; ++i) h_value0[i] = static_cast<F>(P.value0[i]);
    }
    std::memcpy(h_cb, P.child_begin.data(), (P.total + P.parts) * sizeof(int32_t));
    if (!P.patch.empty()) std::memcpy(h_patch, P.patch.data(), P.patch.size() * sizeof(int32_t));
    // the host vectors are no longer needed: the pinned copies are what each pass streams
    plan.parent = {};
    plan.infoset = {};
    plan.edge = {};
    plan.player = {};
    plan.value0 = {};
    plan.child_begin = {};
    plan.patch = {};
    return 0;
}

template <class F>
void PartDev<F>::release() {
    for (void* p : {static_cast<void*>(h_parent), static_cast<void*>(h_infoset),
                    static_cast<void*>(h_edge), static_cast<void*>(h_player),
                    static_cast<void*>(h_value0), static_cast<void*>(h_cb),
                    static_cast<void*>(h_patch)})
        if (p != nullptr) (void)hipHostFree(p);
    h_parent = h_infoset = h_edge = h_cb = h_patch = nullptr;
    h_player = nullptr;
    h_value0 = nullptr;
}

template <class F>
void launch_partitioned_pass(const DevT<F>& d, const PartDev<F>& Pd, const UpdateRule& rule,
                             hipStream_t st) {
    const PartPlan& P = Pd.plan;
    const int32_t* lo = Pd.level_offset.data();
    const int32_t cut = P.cut, D = P.D, nl = D - cut;
    const int64_t base = P.base;
    // resident top-down: levels 1 .. cut
    for (int32_t l = 1; l <= cut; ++l) launch_reach_range(d, lo[l], lo[l + 1], st);
    auto h2d = [&](void* dst, const void* src, size_t bytes) {
        if (bytes > 0) (void)hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    for (int32_t p = 0; p < P.parts; ++p) {
        const int64_t o = P.off[p], w = P.off[p + 1] - o;
        // stream the partition's window in (stream order keeps it after the previous
        // partition's kernels)
        h2d(d.parent + base, Pd.h_parent + o, w * sizeof(int32_t));
        h2d(d.child_begin + base, Pd.h_cb + o + p, (w + 1) * sizeof(int32_t));
        h2d(d.node_player + base, Pd.h_player + o, w * sizeof(int8_t));
        h2d(d.node_infoset + base, Pd.h_infoset + o, w * sizeof(int32_t));
        h2d(d.node_edge + base, Pd.h_edge + o, w * sizeof(int32_t));
        h2d(d.value + base, Pd.h_value0 + o, w * sizeof(F));
        h2d(d.child_begin + P.a[p], Pd.h_patch + P.patch_off[p],
            (P.patch_off[p + 1] - P.patch_off[p]) * sizeof(int32_t));
        const int32_t* wl = P.lo.data() + static_cast<size_t>(p) * (nl + 1);  // levels cut+1 ..
        for (int32_t i = 0; i + 1 < nl; ++i) launch_reach_range(d, wl[i], wl[i + 1], st);
        for (int32_t i = nl - 2; i >= 0; --i) launch_value_range(d, wl[i], wl[i + 1], st);
        launch_value_range(d, P.a[p], P.b[p], st);  // the partition's level-cut nodes
    }
    // resident bottom-up: levels cut - 1 .. 0
    for (int32_t l = cut - 1; l >= 0; --l) launch_value_range(d, lo[l], lo[l + 1], st);
    launch_infoset_pass(d, rule, st);
}

template struct PartDev<float>;
template struct PartDev<double>;
template void launch_partitioned_pass<float>(const DevT<float>&, const PartDev<float>&,
                                             const UpdateRule&, hipStream_t);
template void launch_partitioned_pass<double>(const DevT<double>&, const PartDev<double>&,
                                              const UpdateRule&, hipStream_t);

}  // namespace cfr
