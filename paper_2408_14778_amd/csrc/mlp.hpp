// Warm-start network: descriptor layout and launch wrappers (kernels in mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cfr {

// Per-infoset descriptor of a poker subgame (int16 fields).
enum DescField {
    kDPlayer = 0,   // 1 or 2
    kDOwn = 1,      // own private rank
    kDRound = 2,    // absolute betting round 0..2
    kDBoard0 = 3,   // public ranks dealt so far, -1 if none (3 slots)
    kDRaises = 6,   // raises so far in this round
    kDLast = 7,     // last action in this round: 0 none, 1 check/call, 2 pot-raise, 3 all-in
    kDCMe = 8,      // own commitment
    kDCOpp = 9,     // opponent's commitment
    kDStack = 10,   // stack
    kDMask = 11,    // legal slots: bit 0 fold, 1 call, 2 pot-raise, 3 all-in
    kDDepth = 12,   // depth in the subgame
    kDCap = 13,     // raise cap
    kDRanks = 14,   // ranks in the deck
    kDGame = 15,    // index of the game in the batch (beliefs row)
    kDescFields = 16
};
constexpr int kFeatures = 81;  // meaningful features; the input width pads with zeros
constexpr int kSlots = 4;      // action slots: fold, call, pot-raise, all-in

// Split K for long reductions: kSplitK k-values per split at least, at most kMaxSplits splits;
// the partials need kMaxSplits * M * N floats at `part` (nullptr: no split).
constexpr int kSplitK = 256;
constexpr int kMaxSplits = 32;
// Column sums (bias gradients) split the rows 32 at a time into at most this many partials of
// `cols` floats each at `part`.
constexpr int kColsumMaxSplits = 1024;
void launch_gemm(int M, int N, int K, const void* A, int64_t a_i, int64_t a_k, const void* B,
                 int64_t b_k, int64_t b_j, const float* bias, int mode, const void* gate, float* Cf,
                 void* Cb, int64_t ldc, hipStream_t st, float* part = nullptr);
void launch_softmax_xent(int B, int A, const float* Z, const float* target, const float* mask,
                         void* dZ, float* loss, hipStream_t st);
void launch_colsum(int rows, int cols, const void* G, float* out, hipStream_t st, float* part);
// The three layers in one kernel (F a multiple of 16 up to 128, H 64, 128 or 256, A <= 8, X
// 16-byte aligned): W1P, W2P the hidden layers' weights packed by launch_pack_fragments, W3T the
// last layer's transposed; false (nothing launched) for other shapes. The logits equal those of
// the three per-layer launch_gemm calls bit for bit.
bool launch_mlp_forward(int M, int F, int H, int A, const void* X, const void* W1P, const float* b1,
                        const void* W2P, const float* b2, const void* W3T, const float* b3,
                        float* Z, hipStream_t st);
// The K x H weights W, given transposed (WT, H x K), packed in MFMA B-fragment order for
// launch_mlp_forward (K a multiple of 16, H of 32; otherwise nothing is written).
void launch_pack_fragments(int K, int H, const void* WT, void* dst, hipStream_t st);
// dst = src transposed, src a rows x cols BF16 matrix
void launch_transpose_bf16(int rows, int cols, const void* src, void* dst, hipStream_t st);
void launch_adam(int64_t n, float* w, const float* g, float* m, float* v, void* wb, float lr,
                 float b1, float b2, float eps, float c1, float c2, hipStream_t st);
void launch_to_bf16(int64_t n, const float* src, void* dst, hipStream_t st);
void launch_features(int64_t n, int F, const int16_t* desc, const float* beliefs, void* X,
                     hipStream_t st);
void launch_probs_to_pairs(int64_t n, int A, const float* Z, const int16_t* desc,
                           const int64_t* q_off, float* probs, hipStream_t st);
void launch_warm_start(int64_t Hp, const int32_t* q_offset, const int32_t* q_input,
                       const float* probs, float w, float* R, float* S, float* sigma, hipStream_t st);

}  // namespace cfr
