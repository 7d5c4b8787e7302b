// Warm-start network kernels for gfx950: BF16 MFMA GEMMs with FP32 accumulation, the masked
// softmax cross-entropy, Adam, the poker-subgame feature extractor and the warm start of
// cumulative regrets from predicted strategies.
//
// The network (3 layers, ReLU) maps infoset features to a distribution over action slots;
// the warm start turns it into initial cumulative regrets R0(h, a) = w * m(h) * p(h, a),
// where m(h) is the magnitude of h's regrets after one iteration from zero. CFR from zero
// regrets remains the fallback (the caller decides, by exploitability).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp.hpp"

namespace cfr {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ int64_t gid() {
    return static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}

inline unsigned blocks_for(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

// C = epilogue(A . B) on 32 x 32 tiles, one wavefront per tile, v_mfma_f32_32x32x16_bf16.
// A(i, k) = A[i * a_i + k * a_k] (M x K), B(k, j) = B[k * b_k + j * b_j] (K x N), bf16.
// Operand fragments: lane l holds A rows i = l % 32 and B columns j = l % 32, with the 8
// k-values 8 * (l / 32) .. + 7 of the current 16-wide k step; the 32 x 32 FP32 result has
// element e of lane l at row 8 * (e / 4) + 4 * (l / 32) + e % 4, column l % 32.
// Epilogue: + bias[j] (if bias), then mode 0: store FP32; 1: relu, store BF16; 2: multiply by
// (gate[i, j] > 0) (the ReLU derivative of the layer's output), store BF16.
// Split K (weight gradients, where K is the batch): workgroup z of gridDim.z takes k in
// [z kps, (z + 1) kps) and stores its FP32 partial tile to part[z][M][N]; k_sum_splits adds the
// partials in z order (deterministic) and applies mode 0.
__global__ void __launch_bounds__(64) k_gemm(int M, int N, int K, const __bf16* __restrict__ A,
                                             int64_t a_i, int64_t a_k,
                                             const __bf16* __restrict__ B, int64_t b_k,
                                             int64_t b_j, const float* __restrict__ bias, int mode,
                                             const __bf16* __restrict__ gate, float* __restrict__ Cf,
                                             __bf16* __restrict__ Cb, int64_t ldc, int kps,
                                             float* __restrict__ part) {
    const int lane = threadIdx.x;
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    const int r = lane & 31, half = lane >> 5;
    const int ai = m0 + r, bj = n0 + r;
    const int kbeg = blockIdx.z * kps;
    const int kend = min(K, kbeg + kps);
    floatx16 acc = {};
    for (int k0 = kbeg; k0 < kend; k0 += 16) {
        bf16x8 fa, fb;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + 8 * half + j;
            const bool kin = k < kend;
            fa[j] = (kin && ai < M) ? A[ai * a_i + k * a_k] : static_cast<__bf16>(0.0f);
            fb[j] = (kin && bj < N) ? B[k * b_k + bj * b_j] : static_cast<__bf16>(0.0f);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int i = m0 + 8 * (e >> 2) + 4 * half + (e & 3);
        const int j = n0 + r;
        if (i >= M || j >= N) continue;
        if (gridDim.z > 1) {
            part[(static_cast<int64_t>(blockIdx.z) * M + i) * N + j] = acc[e];
            continue;
        }
        float v = acc[e];
        if (bias != nullptr) v += bias[j];
        const int64_t o = static_cast<int64_t>(i) * ldc + j;
        if (mode == 0) {
            Cf[o] = v;
        } else if (mode == 1) {
            Cb[o] = static_cast<__bf16>(fmaxf(v, 0.0f));
        } else {
            const float g = static_cast<float>(gate[o]);
            Cb[o] = static_cast<__bf16>(g > 0.0f ? v : 0.0f);
        }
    }
}

// Masked softmax cross-entropy per row: loss += -(1/B) sum_a mask t log p, and
// dZ[b, a] = mask (p tsum - t) / B in BF16.
__global__ void k_softmax_xent(int B, int A, const float* __restrict__ Z,
                               const float* __restrict__ target, const float* __restrict__ mask,
                               __bf16* __restrict__ dZ, float* __restrict__ loss) {
    const int64_t b = gid();
    float l = 0.0f;
    if (b < B) {
        const float* z = Z + b * A;
        const float* t = target + b * A;
        const float* mk = mask + b * A;
        float mx = -3.0e38f;
        for (int a = 0; a < A; ++a)
            if (mk[a] > 0.0f) mx = fmaxf(mx, z[a]);
        float se = 0.0f, tsum = 0.0f;
        for (int a = 0; a < A; ++a)
            if (mk[a] > 0.0f) {
                se += __expf(z[a] - mx);
                tsum += t[a];
            }
        const float lse = mx + __logf(se);
        for (int a = 0; a < A; ++a) {
            float g = 0.0f;
            if (mk[a] > 0.0f) {
                const float p = __expf(z[a] - lse);
                l -= t[a] * (z[a] - lse);
                g = (p * tsum - t[a]) / static_cast<float>(B);
            }
            dZ[b * A + a] = static_cast<__bf16>(g);
        }
        l /= static_cast<float>(B);
    }
    // wave reduction then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off, 64);
    if ((threadIdx.x & 63) == 0 && loss != nullptr) atomicAdd(loss, l);
}

// Sums split partials part[z][M][N] over z in order into C (row stride ldc), one thread per
// element.
__global__ void k_sum_splits(int M, int N, int splits, const float* __restrict__ part,
                             float* __restrict__ C, int64_t ldc) {
    const int64_t t = gid();
    if (t >= static_cast<int64_t>(M) * N) return;
    const int64_t i = t / N, j = t % N;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[(static_cast<int64_t>(z) * M + i) * N + j];
    C[i * ldc + j] = s;
}

// Column sums of a BF16 [rows x cols] matrix (bias gradients), split over rows: workgroup
// (x, y) takes 64 columns (one per lane, coalesced rows) and rows [y rps, (y + 1) rps), with
// four interleaved accumulators combined in a fixed order, into part[y][cols].
__global__ void __launch_bounds__(64) k_colsum_part(int rows, int cols, int rps,
                                                    const __bf16* __restrict__ G,
                                                    float* __restrict__ part) {
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= cols) return;
    const int r0 = blockIdx.y * rps, r1 = min(rows, r0 + rps);
    float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int i = r0;
    for (; i + 4 <= r1; i += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] += static_cast<float>(G[static_cast<int64_t>(i + u) * cols + j]);
    }
    for (; i < r1; ++i) s[0] += static_cast<float>(G[static_cast<int64_t>(i) * cols + j]);
    part[static_cast<int64_t>(blockIdx.y) * cols + j] = (s[0] + s[1]) + (s[2] + s[3]);
}

// Adam on FP32 master parameters; refreshes the BF16 copy used by the GEMMs.
__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, __bf16* __restrict__ wb,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = gid();
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb != nullptr) wb[i] = static_cast<__bf16>(wi);
}

__global__ void k_to_bf16(int64_t n, const float* __restrict__ src, __bf16* __restrict__ dst) {
    const int64_t i = gid();
    if (i < n) dst[i] = static_cast<__bf16>(src[i]);
}

// Poker-subgame features, one thread per infoset. Descriptor fields (int16): see mlp.hpp.
__global__ void k_features(int64_t n, int F, const int16_t* __restrict__ desc,
                           const float* __restrict__ beliefs, __bf16* __restrict__ X) {
    const int64_t h = gid();
    if (h >= n) return;
    const int16_t* d = desc + h * kDescFields;
    float f[kFeatures];
#pragma unroll
    for (int i = 0; i < kFeatures; ++i) f[i] = 0.0f;
    const int player = d[kDPlayer], own = d[kDOwn], rnd = d[kDRound], game = d[kDGame];
    const int ranks = d[kDRanks];
    const float stack = static_cast<float>(d[kDStack]);
    const float cme = static_cast<float>(d[kDCMe]), cop = static_cast<float>(d[kDCOpp]);
    int o = 0;
    if (own >= 0 && own < 13) f[o + own] = 1.0f;                         // own rank 0..12
    o += 13;
    f[o + (player == 1 ? 0 : 1)] = 1.0f;                                  // player
    o += 2;
    if (rnd >= 0 && rnd < 3) f[o + rnd] = 1.0f;                          // absolute round
    o += 3;
    for (int i = 0; i < 3; ++i) {                                         // board multi-hot
        const int c = d[kDBoard0 + i];
        if (c >= 0 && c < 13) f[o + c] = 1.0f;
    }
    o += 13;
    const int raises = d[kDRaises];
    if (raises >= 0 && raises < 4) f[o + raises] = 1.0f;                  // raises this round
    o += 4;
    const int last = d[kDLast];
    if (last >= 0 && last < 5) f[o + last] = 1.0f;                        // last action
    o += 5;
    f[o + 0] = cme / stack;                                               // commitments and pot
    f[o + 1] = cop / stack;
    f[o + 2] = (cme + cop) / stack;
    f[o + 3] = (cop - cme) / fmaxf(cme + cop, 1.0f);
    o += 4;
    for (int i = 0; i < 4; ++i) f[o + i] = (d[kDMask] >> i) & 1 ? 1.0f : 0.0f;  // legal slots
    o += 4;
    f[o++] = static_cast<float>(d[kDDepth]) / 16.0f;
    f[o++] = static_cast<float>(d[kDCap]) / 3.0f;
    f[o++] = logf(stack) / logf(1000.0f);
    f[o++] = static_cast<float>(ranks) / 13.0f;
    // root beliefs: the opponent's and my own range over ranks, and my win chance
    const float* bme = beliefs + (static_cast<int64_t>(game) * 2 + (player - 1)) * 13;
    const float* bop = beliefs + (static_cast<int64_t>(game) * 2 + (2 - player)) * 13;
    float below = 0.0f, above = 0.0f;
    for (int i = 0; i < 13; ++i) {
        f[o + i] = bop[i];
        f[o + 13 + i] = bme[i];
        if (i < own) below += bop[i];
        if (i > own) above += bop[i];
    }
    o += 26;
    f[o++] = below;
    f[o++] = above;
    f[o++] = 1.0f;  // bias input
    for (int i = 0; i < F; ++i) X[h * F + i] = static_cast<__bf16>(i < kFeatures ? f[i] : 0.0f);
}

// Masked softmax of logits over the legal slots, scattered to pair order: action a of infoset
// h is the a-th legal slot; probs[q_off[h] + a].
__global__ void k_probs_to_pairs(int64_t n, int A, const float* __restrict__ Z,
                                 const int16_t* __restrict__ desc, const int64_t* __restrict__ q_off,
                                 float* __restrict__ probs) {
    const int64_t h = gid();
    if (h >= n) return;
    const int mask = desc[h * kDescFields + kDMask];
    const float* z = Z + h * A;
    float mx = -3.0e38f;
    for (int s = 0; s < A; ++s)
        if ((mask >> s) & 1) mx = fmaxf(mx, z[s]);
    float se = 0.0f;
    for (int s = 0; s < A; ++s)
        if ((mask >> s) & 1) se += __expf(z[s] - mx);
    int a = 0;
    for (int s = 0; s < A; ++s)
        if ((mask >> s) & 1) probs[q_off[h] + a++] = __expf(z[s] - mx) / se;
}

// R0(h, a) = w * m(h) * p(h, a) with m(h) = sum_a max(R(h, a), 0) of the current state,
// S = 0, then regret matching. Pairs in the solver's order; p read through q_input.
__global__ void k_warm_start(int64_t Hp, const int32_t* __restrict__ q_offset,
                             const int32_t* __restrict__ q_input, const float* __restrict__ probs,
                             float w, float* __restrict__ R, float* __restrict__ S,
                             float* __restrict__ sigma) {
    const int64_t h = gid();
    if (h >= Hp) return;
    const int32_t o = q_offset[h], k = q_offset[h + 1] - o;
    float m = 0.0f;
    for (int32_t a = 0; a < k; ++a) m += fmaxf(R[o + a], 0.0f);
    float pos = 0.0f;
    for (int32_t a = 0; a < k; ++a) {
        const float r = w * m * probs[q_input[o + a]];
        R[o + a] = r;
        S[o + a] = 0.0f;
        pos += fmaxf(r, 0.0f);
    }
    for (int32_t a = 0; a < k; ++a)
        sigma[o + a] = pos > 0.0f ? fmaxf(R[o + a], 0.0f) / pos : 1.0f / static_cast<float>(k);
}

}  // namespace

void launch_gemm(int M, int N, int K, const void* A, int64_t a_i, int64_t a_k, const void* B,
                 int64_t b_k, int64_t b_j, const float* bias, int mode, const void* gate, float* Cf,
                 void* Cb, int64_t ldc, hipStream_t st, float* part) {
    // split K only for FP32 outputs without bias (weight gradients) when K is long
    int splits = 1;
    if (part != nullptr && mode == 0 && bias == nullptr && K >= 2 * kSplitK)
        splits = min(kMaxSplits, K / kSplitK);
    const int kps = ((K + splits - 1) / splits + 15) / 16 * 16;
    splits = (K + kps - 1) / kps;
    dim3 grid((N + 31) / 32, (M + 31) / 32, splits);
    hipLaunchKernelGGL(k_gemm, grid, dim3(64), 0, st, M, N, K, static_cast<const __bf16*>(A), a_i,
                       a_k, static_cast<const __bf16*>(B), b_k, b_j, bias, mode,
                       static_cast<const __bf16*>(gate), Cf, static_cast<__bf16*>(Cb), ldc, kps,
                       part);
    if (splits > 1)
        hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for(int64_t{M} * N, 256)), dim3(256), 0, st, M,
                           N, splits, part, Cf, ldc);
}

void launch_softmax_xent(int B, int A, const float* Z, const float* target, const float* mask,
                         void* dZ, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_softmax_xent, dim3(blocks_for(B, 256)), dim3(256), 0, st, B, A, Z, target,
                       mask, static_cast<__bf16*>(dZ), loss);
}

void launch_colsum(int rows, int cols, const void* G, float* out, hipStream_t st, float* part) {
    const int splits = max(1, min(kMaxSplits, rows / kSplitK));
    const int rps = (rows + splits - 1) / splits;
    hipLaunchKernelGGL(k_colsum_part, dim3((cols + 63) / 64, splits), dim3(64), 0, st, rows, cols,
                       rps, static_cast<const __bf16*>(G), part);
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for(cols, 256)), dim3(256), 0, st, 1, cols, splits,
                       part, out, int64_t{cols});
}

void launch_adam(int64_t n, float* w, const float* g, float* m, float* v, void* wb, float lr,
                 float b1, float b2, float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, w, g, m, v,
                       static_cast<__bf16*>(wb), lr, b1, b2, eps, c1, c2);
}

void launch_to_bf16(int64_t n, const float* src, void* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, src,
                       static_cast<__bf16*>(dst));
}

void launch_features(int64_t n, int F, const int16_t* desc, const float* beliefs, void* X,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_features, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, F, desc, beliefs,
                       static_cast<__bf16*>(X));
}

void launch_probs_to_pairs(int64_t n, int A, const float* Z, const int16_t* desc,
                           const int64_t* q_off, float* probs, hipStream_t st) {
    hipLaunchKernelGGL(k_probs_to_pairs, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, A, Z, desc,
                       q_off, probs);
}

void launch_warm_start(int64_t Hp, const int32_t* q_offset, const int32_t* q_input,
                       const float* probs, float w, float* R, float* S, float* sigma, hipStream_t st) {
    hipLaunchKernelGGL(k_warm_start, dim3(blocks_for(Hp, 256)), dim3(256), 0, st, Hp, q_offset,
                       q_input, probs, w, R, S, sigma);
}

}  // namespace cfr
