// Internal layout of a warm-start network handle (shared by the C ABI sources).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/cfr_warmstart.h"

struct cfr_mlp {
    int32_t F, H, A, maxB;
    hipStream_t st;
    int64_t n_params;
    // [W1 | b1 | W2 | b2 | W3 | b3] blocks
    float *w, *g, *m, *v;
    __bf16* wb;
    // the weight matrices transposed, [W1^T (H x F) | W2^T (H x H) | W3^T (A x H)], refreshed
    // with wb: the forward pass reads both GEMM operands along k
    __bf16* wbT;
    // W1 and W2 packed in MFMA fragment order for the fused forward pass, [W1 | W2]
    __bf16* wbP;
    // activations
    __bf16 *A1, *A2, *dZ3, *dZ2, *dZ1;
    float *Z3, *loss;
    float* part;  // split-K partials: kMaxSplits * max(F, H) * max(H, A) floats
    int64_t step;
};

namespace cfr {

// Parameter block offsets: W1, b1, W2, b2, W3, b3 and the end (the parameter count).
inline int64_t offsets(int32_t F, int32_t H, int32_t A, int64_t off[7]) {
    off[0] = 0;                       // W1
    off[1] = off[0] + int64_t{F} * H;  // b1
    off[2] = off[1] + H;               // W2
    off[3] = off[2] + int64_t{H} * H;  // b2
    off[4] = off[3] + H;               // W3
    off[5] = off[4] + int64_t{H} * A;  // b3
    off[6] = off[5] + A;
    return off[6];
}

// Offsets of W1^T, W2^T, W3^T in the transposed copy.
inline void transposed_offsets(int32_t F, int32_t H, int32_t A, int64_t t[3]) {
    (void)A;
    t[0] = 0;
    t[1] = int64_t{F} * H;
    t[2] = t[1] + int64_t{H} * H;
}

}  // namespace cfr
