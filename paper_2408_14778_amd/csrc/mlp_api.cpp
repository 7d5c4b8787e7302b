// C ABI of the warm-start network (include/cfr_warmstart.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/cfr_warmstart.h"
#include "mlp.hpp"
#include "mlp_net.hpp"

namespace cfr {
int set_error(int code, const std::string& msg);  // solver.cpp
}

namespace {

using cfr::offsets;

size_t layout(cfr_mlp& n, void* base, int32_t F, int32_t H, int32_t A, int32_t maxB) {
    uintptr_t p = reinterpret_cast<uintptr_t>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t{255};
        void* r = reinterpret_cast<void*>(p + off);
        off += bytes > 0 ? bytes : 1;
        return r;
    };
    int64_t o[7];
    const int64_t P = offsets(F, H, A, o);
    n.F = F; n.H = H; n.A = A; n.maxB = maxB; n.n_params = P;
    n.w = static_cast<float*>(take(P * 4));
    n.g = static_cast<float*>(take(P * 4));
    n.m = static_cast<float*>(take(P * 4));
    n.v = static_cast<float*>(take(P * 4));
    n.wb = static_cast<__bf16*>(take(P * 2));
    n.wbT = static_cast<__bf16*>(take(P * 2));
    n.wbP = static_cast<__bf16*>(take(P * 2));
    n.A1 = static_cast<__bf16*>(take(int64_t{maxB} * H * 2));
    n.A2 = static_cast<__bf16*>(take(int64_t{maxB} * H * 2));
    n.dZ2 = static_cast<__bf16*>(take(int64_t{maxB} * H * 2));
    n.dZ1 = static_cast<__bf16*>(take(int64_t{maxB} * H * 2));
    n.dZ3 = static_cast<__bf16*>(take(int64_t{maxB} * A * 2));
    n.Z3 = static_cast<float*>(take(int64_t{maxB} * A * 4));
    n.loss = static_cast<float*>(take(4));
    // split-K partials of the weight gradients, or the column-sum partials of the bias gradients
    n.part = static_cast<float*>(
        take(std::max(int64_t{cfr::kMaxSplits} * std::max(F, H) * std::max(H, A),
                      int64_t{cfr::kColsumMaxSplits} * std::max(H, A)) * 4));
    return (off + 255) & ~size_t{255};
}

int hip_fail(hipError_t e, const char* what) {
    return cfr::set_error(CFR_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define MLP_TRY(expr, what)                              \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

void forward(cfr_mlp* n, const void* x, int32_t B) {
    int64_t o[7], t[3];
    offsets(n->F, n->H, n->A, o);
    cfr::transposed_offsets(n->F, n->H, n->A, t);
    const int F = n->F, H = n->H, A = n->A;
    // B(k, j) = W[k][j] = W^T[j][k]: the transposed copies are k-contiguous
    cfr::launch_gemm(B, H, F, x, F, 1, n->wbT + t[0], 1, F, n->w + o[1], 1, nullptr, nullptr, n->A1,
                     H, n->st);
    cfr::launch_gemm(B, H, H, n->A1, H, 1, n->wbT + t[1], 1, H, n->w + o[3], 1, nullptr, nullptr,
                     n->A2, H, n->st);
    cfr::launch_gemm(B, A, H, n->A2, H, 1, n->wbT + t[2], 1, H, n->w + o[5], 0, nullptr, n->Z3,
                     nullptr, A, n->st);
}

// Refreshes the transposed weight copies from wb.
void transpose_weights(cfr_mlp* n) {
    int64_t o[7], t[3];
    offsets(n->F, n->H, n->A, o);
    cfr::transposed_offsets(n->F, n->H, n->A, t);
    cfr::launch_transpose_bf16(n->F, n->H, n->wb + o[0], n->wbT + t[0], n->st);
    cfr::launch_transpose_bf16(n->H, n->H, n->wb + o[2], n->wbT + t[1], n->st);
    cfr::launch_transpose_bf16(n->H, n->A, n->wb + o[4], n->wbT + t[2], n->st);
    cfr::launch_pack_fragments(n->F, n->H, n->wbT + t[0], n->wbP, n->st);
    cfr::launch_pack_fragments(n->H, n->H, n->wbT + t[1], n->wbP + int64_t{n->F} * n->H, n->st);
}

}  // namespace

extern "C" {

int64_t cfr_mlp_num_params(int32_t in_features, int32_t hidden, int32_t outputs) {
    if (in_features < 1 || hidden < 1 || outputs < 1) return CFR_EINVAL;
    int64_t o[7];
    return offsets(in_features, hidden, outputs, o);
}

int64_t cfr_mlp_workspace_bytes(int32_t in_features, int32_t hidden, int32_t outputs,
                                int32_t max_batch) {
    if (in_features < 1 || hidden < 1 || outputs < 1 || max_batch < 1) return CFR_EINVAL;
    cfr_mlp n{};
    return static_cast<int64_t>(layout(n, nullptr, in_features, hidden, outputs, max_batch));
}

int cfr_mlp_create(int32_t in_features, int32_t hidden, int32_t outputs, int32_t max_batch,
                   void* workspace, size_t bytes, void* stream, cfr_mlp** out) {
    if (workspace == nullptr || out == nullptr || in_features < 1 || hidden < 1 || outputs < 1 ||
        outputs > 32 || max_batch < 1)
        return cfr::set_error(CFR_EINVAL, "bad network shape or null argument");
    auto* n = new cfr_mlp();
    const size_t need = layout(*n, workspace, in_features, hidden, outputs, max_batch);
    if (bytes < need) {
        delete n;
        return cfr::set_error(CFR_ENOMEM, "network workspace too small");
    }
    n->st = static_cast<hipStream_t>(stream);
    n->step = 0;
    *out = n;
    return CFR_OK;
}

int cfr_mlp_set_params(cfr_mlp* n, const float* params, int64_t count) {
    if (n == nullptr || params == nullptr || count != n->n_params)
        return cfr::set_error(CFR_EINVAL, "parameter count mismatch");
    MLP_TRY(hipMemcpyAsync(n->w, params, count * 4, hipMemcpyHostToDevice, n->st), "params copy");
    cfr::launch_to_bf16(count, n->w, n->wb, n->st);
    transpose_weights(n);
    std::vector<float> zeros(count, 0.0f);
    MLP_TRY(hipMemcpyAsync(n->m, zeros.data(), count * 4, hipMemcpyHostToDevice, n->st), "moments");
    MLP_TRY(hipMemcpyAsync(n->v, zeros.data(), count * 4, hipMemcpyHostToDevice, n->st), "moments");
    MLP_TRY(hipMemcpyAsync(n->g, zeros.data(), count * 4, hipMemcpyHostToDevice, n->st), "grads");
    MLP_TRY(hipStreamSynchronize(n->st), "params synchronise");
    n->step = 0;
    return CFR_OK;
}

int cfr_mlp_get_params(cfr_mlp* n, float* params, int64_t count) {
    if (n == nullptr || params == nullptr || count != n->n_params)
        return cfr::set_error(CFR_EINVAL, "parameter count mismatch");
    MLP_TRY(hipMemcpyAsync(params, n->w, count * 4, hipMemcpyDeviceToHost, n->st), "params copy");
    MLP_TRY(hipStreamSynchronize(n->st), "params synchronise");
    return CFR_OK;
}

int cfr_mlp_get_grads(cfr_mlp* n, float* grads, int64_t count) {
    if (n == nullptr || grads == nullptr || count != n->n_params)
        return cfr::set_error(CFR_EINVAL, "parameter count mismatch");
    MLP_TRY(hipMemcpyAsync(grads, n->g, count * 4, hipMemcpyDeviceToHost, n->st), "grads copy");
    MLP_TRY(hipStreamSynchronize(n->st), "grads synchronise");
    return CFR_OK;
}

int cfr_mlp_forward(cfr_mlp* n, const void* x, int32_t batch, float* logits) {
    if (n == nullptr || x == nullptr || logits == nullptr || batch < 1 || batch > n->maxB)
        return cfr::set_error(CFR_EINVAL, "bad batch or null argument");
    // the three layers in one kernel where the shape allows (the same logits, bit for bit),
    // else layer by layer through the activation buffers
    int64_t o[7], t[3];
    offsets(n->F, n->H, n->A, o);
    cfr::transposed_offsets(n->F, n->H, n->A, t);
    if (!cfr::launch_mlp_forward(batch, n->F, n->H, n->A, x, n->wbP, n->w + o[1],
                                 n->wbP + int64_t{n->F} * n->H, n->w + o[3], n->wbT + t[2],
                                 n->w + o[5], logits, n->st)) {
        forward(n, x, batch);
        MLP_TRY(hipMemcpyAsync(logits, n->Z3, int64_t{batch} * n->A * 4, hipMemcpyDeviceToDevice,
                               n->st),
                "logits copy");
    }
    MLP_TRY(hipGetLastError(), "forward launch");
    return CFR_OK;
}

int cfr_mlp_train_step(cfr_mlp* n, const void* x, const float* target, const float* mask,
                       int32_t B, float lr, float* loss) {
    if (n == nullptr || x == nullptr || target == nullptr || mask == nullptr || B < 1 || B > n->maxB)
        return cfr::set_error(CFR_EINVAL, "bad batch or null argument");
    int64_t o[7];
    offsets(n->F, n->H, n->A, o);
    const int F = n->F, H = n->H, A = n->A;
    forward(n, x, B);
    MLP_TRY(hipMemsetAsync(n->loss, 0, 4, n->st), "loss reset");
    cfr::launch_softmax_xent(B, A, n->Z3, target, mask, n->dZ3, n->loss, n->st);
    // layer 3
    cfr::launch_gemm(H, A, B, n->A2, 1, H, n->dZ3, A, 1, nullptr, 0, nullptr, n->g + o[4], nullptr,
                     A, n->st, n->part);
    cfr::launch_colsum(B, A, n->dZ3, n->g + o[5], n->st, n->part);
    cfr::launch_gemm(B, H, A, n->dZ3, A, 1, n->wb + o[4], 1, A, nullptr, 2, n->A2, nullptr, n->dZ2,
                     H, n->st);
    // layer 2
    cfr::launch_gemm(H, H, B, n->A1, 1, H, n->dZ2, H, 1, nullptr, 0, nullptr, n->g + o[2], nullptr,
                     H, n->st, n->part);
    cfr::launch_colsum(B, H, n->dZ2, n->g + o[3], n->st, n->part);
    cfr::launch_gemm(B, H, H, n->dZ2, H, 1, n->wb + o[2], 1, H, nullptr, 2, n->A1, nullptr, n->dZ1,
                     H, n->st);
    // layer 1
    cfr::launch_gemm(F, H, B, x, 1, F, n->dZ1, H, 1, nullptr, 0, nullptr, n->g + o[0], nullptr, H,
                     n->st, n->part);
    cfr::launch_colsum(B, H, n->dZ1, n->g + o[1], n->st, n->part);
    // Adam
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, static_cast<float>(n->step));
    const float c2 = 1.0f - std::pow(b2, static_cast<float>(n->step));
    cfr::launch_adam(n->n_params, n->w, n->g, n->m, n->v, n->wb, lr, b1, b2, 1e-8f, c1, c2, n->st);
    transpose_weights(n);
    MLP_TRY(hipGetLastError(), "train launch");
    if (loss != nullptr) {
        MLP_TRY(hipMemcpyAsync(loss, n->loss, 4, hipMemcpyDeviceToHost, n->st), "loss copy");
        MLP_TRY(hipStreamSynchronize(n->st), "train synchronise");
    }
    return CFR_OK;
}

int cfr_mlp_destroy(cfr_mlp* n) {
    if (n != nullptr) (void)hipStreamSynchronize(n->st);
    delete n;
    return CFR_OK;
}

int cfr_features(const int16_t* desc, const float* beliefs, int64_t n, int32_t in_features,
                 void* x, void* stream) {
    if (desc == nullptr || beliefs == nullptr || x == nullptr || n < 0 || in_features < 1)
        return cfr::set_error(CFR_EINVAL, "bad argument");
    if (n == 0) return CFR_OK;
    cfr::launch_features(n, in_features, desc, beliefs, x, static_cast<hipStream_t>(stream));
    MLP_TRY(hipGetLastError(), "features launch");
    return CFR_OK;
}

int cfr_probs_to_pairs(const float* logits, const int16_t* desc, const int64_t* q_off, int64_t n,
                       int32_t outputs, float* probs, void* stream) {
    if (logits == nullptr || desc == nullptr || q_off == nullptr || probs == nullptr || n < 0 ||
        outputs < 1 || outputs > 16)
        return cfr::set_error(CFR_EINVAL, "bad argument");
    if (n == 0) return CFR_OK;
    cfr::launch_probs_to_pairs(n, outputs, logits, desc, q_off, probs,
                               static_cast<hipStream_t>(stream));
    MLP_TRY(hipGetLastError(), "probs launch");
    return CFR_OK;
}

}  // extern "C"
