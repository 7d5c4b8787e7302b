// Allocation-free forward pass of the warm-start network: cfr_mlp_forward_noalloc.
//
// The same three BF16 MFMA GEMMs as cfr_mlp_forward, with the two hidden activations held in a
// file-scope device array instead of the network's workspace, and the logits written straight
// to the caller's buffer. Nothing is allocated on any call. Host code never passes the array's
// name to a kernel (in host code it is only a stand-in for the symbol): its device address is
// looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/cfr_warmstart.h"
#include "mlp.hpp"
#include "mlp_net.hpp"

namespace cfr {
int set_error(int code, const std::string& msg);  // solver.cpp
}

namespace {

// Both hidden activations of one call: 2 x batch x hidden BF16 values, each block 256-aligned.
constexpr size_t kNoAllocScratchBytes = size_t{16} << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) & ~size_t{255}; }

// Device address of this device's copy of `scratch` (looked up on the first call per device).
int scratch_of_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return cfr::set_error(CFR_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return cfr::set_error(CFR_EINVAL, "device index too large");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return cfr::set_error(CFR_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                                hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CFR_OK;
}

}  // namespace

extern "C" int cfr_mlp_forward_noalloc(cfr_mlp* n, const void* x, int32_t batch, float* logits) {
    if (n == nullptr || x == nullptr || logits == nullptr || batch < 1)
        return cfr::set_error(CFR_EINVAL, "bad batch or null argument");
    const size_t act = align256(static_cast<size_t>(batch) * static_cast<size_t>(n->H) * 2);
    if (2 * act > kNoAllocScratchBytes)
        return cfr::set_error(CFR_EINVAL,
                              "batch x hidden too large for the allocation-free forward pass (2 "
                              "BF16 activations of batch x hidden must fit in 16 MiB)");
    void* base = nullptr;
    if (const int rc = scratch_of_current_device(&base); rc != CFR_OK) return rc;
    __bf16* A1 = static_cast<__bf16*>(base);
    __bf16* A2 = reinterpret_cast<__bf16*>(static_cast<unsigned char*>(base) + act);
    int64_t o[7], t[3];
    cfr::offsets(n->F, n->H, n->A, o);
    cfr::transposed_offsets(n->F, n->H, n->A, t);
    const int F = n->F, H = n->H, A = n->A;
    // the weights' transposed copies, k-contiguous, as in cfr_mlp_forward
    cfr::launch_gemm(batch, H, F, x, F, 1, n->wbT + t[0], 1, F, n->w + o[1], 1, nullptr, nullptr, A1,
                     H, n->st);
    cfr::launch_gemm(batch, H, H, A1, H, 1, n->wbT + t[1], 1, H, n->w + o[3], 1, nullptr, nullptr, A2,
                     H, n->st);
    cfr::launch_gemm(batch, A, H, A2, H, 1, n->wbT + t[2], 1, H, n->w + o[5], 0, nullptr, logits,
                     nullptr, A, n->st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return cfr::set_error(CFR_EHIP, std::string("forward launch: ") + hipGetErrorString(e));
    return CFR_OK;
}
