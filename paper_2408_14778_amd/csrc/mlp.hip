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

// The same product on TM x TM output tiles (TM = 128 or 64) staged through LDS, for operands of
// at least 64 rows and columns. Workgroup of 256 threads = 4 wavefronts in 2 x 2, each a
// TM/2 x TM/2 quarter (TM/64 x TM/64 MFMA tiles of 32 x 32); the K loop steps by 32, two
// 16-wide MFMA steps per slice. Both operands sit in LDS k-contiguous (A as [m][k], B transposed
// as [n][k]) with rows padded to 40 elements (80 bytes: eight lanes reading or writing 16 bytes
// each cover the 32 banks once), so every fragment read and every slice write is a 16-byte LDS
// access. The next slice is loaded from memory into registers while the current one is
// multiplied (two LDS buffers, one barrier per slice). An operand is loaded along k when it is
// k-contiguous (AKC / BKC: 16-byte loads of 8-element granules) and otherwise one element per k
// with the wavefront's lanes on consecutive rows (each load instruction reads one contiguous run
// of the row dimension). The loads are branch-free: addresses are clamped into the operand and
// out-of-range values replaced by zero, so that the loads of the next slice stay in flight
// while the current one is multiplied. Epilogue and split K as in k_gemm.
constexpr int kTK = 32, kTPad = 40;

__device__ __forceinline__ uint32_t bf16_bits(__bf16 x) {
    return __builtin_bit_cast(unsigned short, x);
}

// EPT bf16 values of one thread's share of a slice, packed two to a 32-bit word.
template <int EPT>
struct Slice {
    uint4 w[EPT / 8];
};

// One operand's slice (TM rows: m, or n for B; kTK k-values) into registers. x_r, x_k: the
// operand's strides along its rows and along k; r0: the tile's first row; k0: the slice's first
// k; rows and kend bound the operand. KC: k-contiguous (x_k == 1, x_r and kend multiples of 8,
// 16-byte aligned base); otherwise x_r == 1.
template <int TM, bool KC>
__device__ __forceinline__ void load_slice(const __bf16* __restrict__ X, int64_t x_r, int64_t x_k,
                                           int r0, int rows, int k0, int kend, int tid,
                                           Slice<TM / 8>& sl) {
    constexpr int EPT = TM / 8;           // elements per thread
    constexpr int TPR = kTK / EPT;        // threads per row (k-contiguous mapping)
    if constexpr (KC) {
        const int r = r0 + tid / TPR, k = k0 + EPT * (tid % TPR);
        const __bf16* row = X + static_cast<int64_t>(min(r, rows - 1)) * x_r;
#pragma unroll
        for (int g = 0; g < EPT / 8; ++g) {
            const int kg = k + 8 * g;
            const uint4 v = *reinterpret_cast<const uint4*>(row + min(kg, kend - 8));
            const bool ok = r < rows && kg < kend;
            sl.w[g].x = ok ? v.x : 0u;
            sl.w[g].y = ok ? v.y : 0u;
            sl.w[g].z = ok ? v.z : 0u;
            sl.w[g].w = ok ? v.w : 0u;
        }
    } else {
        // one row per thread, EPT consecutive k; consecutive lanes take consecutive rows
        const int r = r0 + tid % TM, k = k0 + EPT * (tid / TM);
        const __bf16* col = X + min(r, rows - 1);
        uint32_t h[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const uint32_t v = bf16_bits(col[static_cast<int64_t>(min(k + e, kend - 1)) * x_k]);
            h[e] = (r < rows && k + e < kend) ? v : 0u;
        }
#pragma unroll
        for (int q = 0; q < EPT / 8; ++q) {
            sl.w[q].x = h[8 * q + 0] | (h[8 * q + 1] << 16);
            sl.w[q].y = h[8 * q + 2] | (h[8 * q + 3] << 16);
            sl.w[q].z = h[8 * q + 4] | (h[8 * q + 5] << 16);
            sl.w[q].w = h[8 * q + 6] | (h[8 * q + 7] << 16);
        }
    }
}

// Writes a slice loaded by load_slice into the LDS tile T[row][k] (row stride kTPad).
template <int TM, bool KC>
__device__ __forceinline__ void store_slice(__bf16 (*T)[kTPad], int tid, const Slice<TM / 8>& sl) {
    constexpr int EPT = TM / 8, TPR = kTK / EPT;
    const int r = KC ? tid / TPR : tid % TM;
    const int k = KC ? EPT * (tid % TPR) : EPT * (tid / TM);
    uint4* d = reinterpret_cast<uint4*>(&T[r][k]);
#pragma unroll
    for (int q = 0; q < EPT / 8; ++q) d[q] = sl.w[q];
}

template <int TM, bool AKC, bool BKC>
__global__ void __launch_bounds__(256) k_gemm_tile(int M, int N, int K, const __bf16* __restrict__ A,
                                                   int64_t a_i, int64_t a_k,
                                                   const __bf16* __restrict__ B, int64_t b_k,
                                                   int64_t b_j, const float* __restrict__ bias,
                                                   int mode, const __bf16* __restrict__ gate,
                                                   float* __restrict__ Cf, __bf16* __restrict__ Cb,
                                                   int64_t ldc, int kps, float* __restrict__ part) {
    constexpr int NT = TM / 64;  // MFMA tiles per wavefront along each dimension
    __shared__ __attribute__((aligned(16))) __bf16 As[2][TM][kTPad];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][TM][kTPad];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
    const int kbeg = blockIdx.z * kps, kend = min(K, kbeg + kps);
    // B is addressed as [n][k]: its row stride is b_j, its k stride b_k
    Slice<TM / 8> sa, sb;
    load_slice<TM, AKC>(A, a_i, a_k, m0, M, kbeg, kend, tid, sa);
    load_slice<TM, BKC>(B, b_j, b_k, n0, N, kbeg, kend, tid, sb);
    store_slice<TM, AKC>(As[0], tid, sa);
    store_slice<TM, BKC>(Bs[0], tid, sb);
    __syncthreads();
    floatx16 acc[NT][NT] = {};
    const int r = lane & 31, half = lane >> 5;
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += kTK) {
        // the last slice reloads itself (in range, unused): no branch around the loads
        const int kn = k0 + kTK < kend ? k0 + kTK : k0;
        load_slice<TM, AKC>(A, a_i, a_k, m0, M, kn, kend, tid, sa);
        load_slice<TM, BKC>(B, b_j, b_k, n0, N, kn, kend, tid, sb);
#pragma unroll
        for (int ks = 0; ks < kTK / 16; ++ks) {
            bf16x8 fa[NT], fb[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                fa[t] = *reinterpret_cast<const bf16x8*>(
                    &As[buf][wm * (TM / 2) + t * 32 + r][ks * 16 + 8 * half]);
                fb[t] = *reinterpret_cast<const bf16x8*>(
                    &Bs[buf][wn * (TM / 2) + t * 32 + r][ks * 16 + 8 * half]);
            }
#pragma unroll
            for (int tm = 0; tm < NT; ++tm)
#pragma unroll
                for (int tn = 0; tn < NT; ++tn)
                    acc[tm][tn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[tm], fb[tn],
                                                                          acc[tm][tn], 0, 0, 0);
        }
        // unconditional (the other buffer was last read before the previous barrier), so that
        // the loads above are issued before the multiplies rather than sunk into a branch
        store_slice<TM, AKC>(As[buf ^ 1], tid, sa);
        store_slice<TM, BKC>(Bs[buf ^ 1], tid, sb);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int tm = 0; tm < NT; ++tm)
#pragma unroll
        for (int tn = 0; tn < NT; ++tn)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int i = m0 + wm * (TM / 2) + tm * 32 + 8 * (e >> 2) + 4 * half + (e & 3);
                const int j = n0 + wn * (TM / 2) + tn * 32 + r;
                if (i >= M || j >= N) continue;
                const float a = acc[tm][tn][e];
                if (gridDim.z > 1) {
                    part[(static_cast<int64_t>(blockIdx.z) * M + i) * N + j] = a;
                    continue;
                }
                float v = a;
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

// Products with at most kNarrow output columns and a k-contiguous A (the action-slot layer):
// half a wavefront per row, lane l taking k = c + 8 l' .. + 7 of every 256-wide chunk c (l' =
// l % 32: one 16-byte load per lane, so the half-wavefront reads one contiguous 512-byte run of
// the row), each lane accumulating all N columns in FP32, then a butterfly over the 32 lanes in
// a fixed order. B is staged once per workgroup in LDS as FP32, ordered [chunk][e][lane][n] so
// that for each e the 32 lanes read consecutive N-float groups (no bank conflicts). Each
// wavefront takes kNarrowRows rows: the loads of all of them are issued before the first
// multiply. Epilogue as k_gemm (no split K). Needs ceil(K / 256) * 256 * N <= kNarrowLds, a row
// stride a multiple of 8 and a 16-byte aligned A.
constexpr int kNarrow = 8;
constexpr int kNarrowRows = 8;
constexpr int kNarrowLds = 8192;

__global__ void __launch_bounds__(256) k_gemm_narrow(int M, int N, int K,
                                                     const __bf16* __restrict__ A, int64_t a_i,
                                                     const __bf16* __restrict__ B, int64_t b_k,
                                                     int64_t b_j, const float* __restrict__ bias,
                                                     int mode, const __bf16* __restrict__ gate,
                                                     float* __restrict__ Cf,
                                                     __bf16* __restrict__ Cb, int64_t ldc) {
    extern __shared__ float Wl[];
    const int Kp = (K + 255) / 256 * 256;
    for (int t = threadIdx.x; t < Kp * N; t += blockDim.x) {
        const int n = t % N, q = t / N;
        const int l = q % 32, e = (q / 32) % 8, c = q / 256;
        const int k = 256 * c + 8 * l + e;
        Wl[t] = k < K ? static_cast<float>(B[static_cast<int64_t>(k) * b_k + n * b_j]) : 0.0f;
    }
    __syncthreads();
    constexpr int P = kNarrowRows / 2;  // row pairs per wavefront
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l = lane & 31, half = lane >> 5;
    const int base = (blockIdx.x * 4 + wave) * kNarrowRows + half;
    float acc[P][kNarrow];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int n = 0; n < kNarrow; ++n) acc[p][n] = 0.0f;
#pragma unroll 1
    for (int c = 0; c < K; c += 256) {
        const int k = c + 8 * l;
        uint4 xw[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int i = min(base + 2 * p, M - 1);
            const uint4 v = *reinterpret_cast<const uint4*>(A + static_cast<int64_t>(i) * a_i +
                                                            min(k, K - 8));
            const bool ok = k < K;  // K is a multiple of 8
            xw[p].x = ok ? v.x : 0u;
            xw[p].y = ok ? v.y : 0u;
            xw[p].z = ok ? v.z : 0u;
            xw[p].w = ok ? v.w : 0u;
        }
        const float* wl = Wl + (c / 256) * 256 * N;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float w[kNarrow];
#pragma unroll
            for (int n = 0; n < kNarrow; ++n) w[n] = n < N ? wl[(e * 32 + l) * N + n] : 0.0f;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const uint32_t wd = e / 2 == 0 ? xw[p].x : e / 2 == 1 ? xw[p].y
                                    : e / 2 == 2 ? xw[p].z : xw[p].w;
                const float x = static_cast<float>(__builtin_bit_cast(
                    __bf16, static_cast<unsigned short>(wd >> (16 * (e % 2)))));
#pragma unroll
                for (int n = 0; n < kNarrow; ++n) acc[p][n] = fmaf(x, w[n], acc[p][n]);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int n = 0; n < kNarrow; ++n)
            for (int off = 16; off > 0; off >>= 1) acc[p][n] += __shfl_xor(acc[p][n], off, 32);
    if (l != 0) return;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int i = base + 2 * p;
        if (i >= M) break;
#pragma unroll
        for (int n = 0; n < kNarrow; ++n) {
            if (n >= N) break;
            float v = acc[p][n];
            if (bias != nullptr) v += bias[n];
            const int64_t o = static_cast<int64_t>(i) * ldc + n;
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
}

// The whole forward pass in one kernel (inference): one wavefront per 32 rows, its rows' input,
// then its hidden activations, in a private LDS region; the hidden layers' weights come from
// BF16 copies packed in MFMA fragment order (L2-resident), one coalesced kilobyte per B
// fragment, the last layer's from its transposed copy.
// Layer 1: A fragments from the staged input rows, H / 32 output tiles of 32 x 32 in FP32
// accumulators; bias and ReLU, rounded to BF16 into LDS (over the input, which is no longer
// needed). Layer 2: the same from the first hidden layer, written back over it. Layer 3 as
// k_gemm_narrow does it, from LDS, FP32 logits to memory. Every element is computed as by the
// per-layer kernels (k_gemm_tile, k_gemm_narrow), bit for bit: the same BF16 operands, FP32
// accumulation over k in the same 16-wide MFMA steps, the same rounding of the hidden layers,
// the same order of the last layer's sums. F: a multiple of 16 up to kFusedMaxF; A <= kNarrow.
constexpr int kFusedMaxF = 128;

// One layer of a wavefront's 32 rows: acc[t] = sum over k-steps of A(k) . B_t(k), A fragments
// at a[k] (LDS), K a multiple of 16. B: the layer's weights packed in fragment order (see
// launch_pack_fragments): fragment (t, k-step s) is 64 lanes x 8 consecutive elements at
// wp[((t * K / 16 + s) * 64 + lane) * 8], so that each load instruction reads one contiguous
// kilobyte. The B fragments of the next k-step are loaded before the multiplies of the
// current one.
template <int NT>
__device__ __forceinline__ void wave_layer(const __bf16* a, const __bf16* __restrict__ wp, int K,
                                           int lane, floatx16 (&acc)[NT]) {
    const int KS = K / 16;
    const __bf16* w = wp + lane * 8;
    bf16x8 fb[NT], nb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        acc[t] = floatx16{};
        fb[t] = *reinterpret_cast<const bf16x8*>(w + static_cast<int64_t>(t) * KS * 512);
    }
#pragma unroll 1
    for (int s = 0; s < KS; ++s) {
        const int sn = s + 1 < KS ? s + 1 : s;  // the last step reloads itself, unused
#pragma unroll
        for (int t = 0; t < NT; ++t)
            nb[t] = *reinterpret_cast<const bf16x8*>(w + (static_cast<int64_t>(t) * KS + sn) * 512);
        const bf16x8 fa = *reinterpret_cast<const bf16x8*>(a + 16 * s);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb[t], acc[t], 0, 0, 0);
            fb[t] = nb[t];
        }
    }
}

template <int H>
__global__ void __launch_bounds__(64, 2) k_mlp_forward(int M, int F, int A,
                                                    const __bf16* __restrict__ X,
                                                    const __bf16* __restrict__ W1P,
                                                    const float* __restrict__ b1,
                                                    const __bf16* __restrict__ W2P,
                                                    const float* __restrict__ b2,
                                                    const __bf16* __restrict__ W3T,
                                                    const float* __restrict__ b3,
                                                    float* __restrict__ Z) {
    constexpr int LD = H + 8;  // row stride of the LDS tile (elements): 16-byte aligned rows
    constexpr int NT = H / 32;
    __shared__ __attribute__((aligned(16))) __bf16 T[32][LD];
    const int lane = threadIdx.x, r = lane & 31, half = lane >> 5;
    const int m0 = blockIdx.x * 32;
    // stage the 32 input rows (zero past M): 8-element granules, 16-byte loads
    const int gpr = F / 8;  // granules per row
    for (int q = lane; q < 32 * gpr; q += 64) {
        const int row = q / gpr, c = 8 * (q % gpr);
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (m0 + row < M) v = *reinterpret_cast<const uint4*>(X + static_cast<int64_t>(m0 + row) * F + c);
        *reinterpret_cast<uint4*>(&T[row][c]) = v;
    }
    __syncthreads();
    floatx16 acc[NT];
    // layer 1: [32 x F] . W1 -> [32 x H]
    wave_layer<NT>(&T[r][8 * half], W1P, F, lane, acc);
    __syncthreads();  // every lane's reads of the input rows are done before they are overwritten
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = t * 32 + r;
        const float bias = b1[col];
#pragma unroll
        for (int e = 0; e < 16; ++e)
            T[8 * (e >> 2) + 4 * half + (e & 3)][col] =
                static_cast<__bf16>(fmaxf(acc[t][e] + bias, 0.0f));
    }
    __syncthreads();
    // layer 2: [32 x H] . W2 -> [32 x H]
    wave_layer<NT>(&T[r][8 * half], W2P, H, lane, acc);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int col = t * 32 + r;
        const float bias = b2[col];
#pragma unroll
        for (int e = 0; e < 16; ++e)
            T[8 * (e >> 2) + 4 * half + (e & 3)][col] =
                static_cast<__bf16>(fmaxf(acc[t][e] + bias, 0.0f));
    }
    __syncthreads();
    // layer 3: [32 x H] . W3 -> [32 x A], A <= kNarrow, in the order of k_gemm_narrow: half a
    // wavefront per row, lane l' taking k = 8 l' .. + 7 (zero past H), FMAs over e in order,
    // then the butterfly over the 32 lanes
    float w[8][kNarrow];
#pragma unroll
    for (int e = 0; e < 8; ++e)
#pragma unroll
        for (int n = 0; n < kNarrow; ++n)
            w[e][n] = (n < A && 8 * r + e < H)
                          ? static_cast<float>(W3T[static_cast<int64_t>(n) * H + 8 * r + e])
                          : 0.0f;
#pragma unroll 1
    for (int p = 0; p < 16; ++p) {
        const int row = 2 * p + half;
        float x[8];
        if (8 * r < H) {
            const uint4 v = *reinterpret_cast<const uint4*>(&T[row][8 * r]);
            const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 8; ++e)
                x[e] = static_cast<float>(__builtin_bit_cast(
                    __bf16, static_cast<unsigned short>(wd[e / 2] >> (16 * (e % 2)))));
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) x[e] = 0.0f;
        }
        float z[kNarrow];
#pragma unroll
        for (int n = 0; n < kNarrow; ++n) z[n] = 0.0f;
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
            for (int n = 0; n < kNarrow; ++n) z[n] = fmaf(x[e], w[e][n], z[n]);
#pragma unroll
        for (int n = 0; n < kNarrow; ++n)
            for (int off = 16; off > 0; off >>= 1) z[n] += __shfl_xor(z[n], off, 32);
        if (r == 0 && m0 + row < M) {
#pragma unroll
            for (int n = 0; n < kNarrow; ++n)
                if (n < A) Z[static_cast<int64_t>(m0 + row) * A + n] = z[n] + b3[n];
        }
    }
}

// Packs the K x H weight matrix W (given transposed, WT[j][k]) in MFMA fragment order: element
// j8 of lane l of fragment (t, s) is W[16 s + 8 (l / 32) + j8][32 t + l % 32].
__global__ void k_pack_fragments(int K, int H, const __bf16* __restrict__ WT,
                                 __bf16* __restrict__ dst) {
    const int64_t i = gid();
    if (i >= static_cast<int64_t>(K) * H) return;
    const int j8 = static_cast<int>(i % 8), l = static_cast<int>((i / 8) % 64);
    const int64_t f = i / 512;
    const int KS = K / 16, s = static_cast<int>(f % KS), t = static_cast<int>(f / KS);
    dst[i] = WT[static_cast<int64_t>(32 * t + l % 32) * K + 16 * s + 8 * (l / 32) + j8];
}

// dst[c][r] = src[r][c] for a rows x cols BF16 matrix (the transposed weight copies).
__global__ void k_transpose_bf16(int rows, int cols, const __bf16* __restrict__ src,
                                 __bf16* __restrict__ dst) {
    const int64_t t = gid();
    if (t >= static_cast<int64_t>(rows) * cols) return;
    const int64_t r = t / cols, c = t % cols;
    dst[c * rows + r] = src[t];
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

// Sums `splits` partials part[z][cols] per column: one wavefront per column, lane l adding
// partials l, l + 64, ... in order, then a butterfly over the 64 lanes in a fixed order.
__global__ void __launch_bounds__(256) k_sum_cols(int cols, int splits,
                                                  const float* __restrict__ part,
                                                  float* __restrict__ out) {
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c >= cols) return;
    float s = 0.0f;
    for (int z = lane; z < splits; z += 64) s += part[static_cast<int64_t>(z) * cols + c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[c] = s;
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
    const auto* a = static_cast<const __bf16*>(A);
    const auto* b = static_cast<const __bf16*>(B);
    const auto* g = static_cast<const __bf16*>(gate);
    auto* cb = static_cast<__bf16*>(Cb);
    // a few output columns from a k-contiguous A: half a wavefront per row
    const int Kp = (K + 255) / 256 * 256;
    if (N <= kNarrow && a_k == 1 && a_i % 8 == 0 && K % 8 == 0 && Kp * N <= kNarrowLds &&
        (reinterpret_cast<uintptr_t>(a) % 16) == 0 &&
        (part == nullptr || mode != 0 || bias != nullptr || K < 2 * kSplitK)) {
        const int rows_per_wg = 4 * kNarrowRows;
        hipLaunchKernelGGL(k_gemm_narrow, dim3((M + rows_per_wg - 1) / rows_per_wg), dim3(256),
                           static_cast<size_t>(Kp) * N * sizeof(float), st, M, N, K, a, a_i, b, b_k,
                           b_j, bias, mode, g, Cf, cb, ldc);
        return;
    }
    // LDS tiles where both output dimensions fill them and each operand is k-contiguous (rows
    // of 8-element granules, 16-byte aligned) or row-contiguous; the other skinny products stay
    // on one wavefront per 32 x 32 tile
    auto aligned16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) % 16) == 0; };
    const bool akc = a_k == 1 && a_i % 8 == 0 && K % 8 == 0 && aligned16(a);
    const bool bkc = b_k == 1 && b_j % 8 == 0 && K % 8 == 0 && aligned16(b);
    const bool tiled = M >= 64 && N >= 64 && K >= kTK && (akc || a_i == 1) && (bkc || b_j == 1);
    const int step = tiled ? kTK : 16;
    // split K only for FP32 outputs without bias (weight gradients) when K is long
    int splits = 1;
    if (part != nullptr && mode == 0 && bias == nullptr && K >= 2 * kSplitK)
        splits = min(kMaxSplits, K / kSplitK);
    const int kps = ((K + splits - 1) / splits + step - 1) / step * step;
    splits = (K + kps - 1) / kps;
    if (tiled) {
        // 128 x 128 tiles when they alone give the chip a few workgroups per CU, else 64 x 64
        const int64_t big = int64_t{(N + 127) / 128} * ((M + 127) / 128) * splits;
        const int tm = big >= 512 ? 128 : 64;
        dim3 grid((N + tm - 1) / tm, (M + tm - 1) / tm, splits);
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, grid, dim3(256), 0, st, M, N, K, a, a_i, a_k, b, b_k, b_j,
                               bias, mode, g, Cf, cb, ldc, kps, part);
        };
        if (tm == 128) {
            if (akc && bkc) go(k_gemm_tile<128, true, true>);
            else if (akc) go(k_gemm_tile<128, true, false>);
            else if (bkc) go(k_gemm_tile<128, false, true>);
            else go(k_gemm_tile<128, false, false>);
        } else {
            if (akc && bkc) go(k_gemm_tile<64, true, true>);
            else if (akc) go(k_gemm_tile<64, true, false>);
            else if (bkc) go(k_gemm_tile<64, false, true>);
            else go(k_gemm_tile<64, false, false>);
        }
    } else {
        dim3 grid((N + 31) / 32, (M + 31) / 32, splits);
        hipLaunchKernelGGL(k_gemm, grid, dim3(64), 0, st, M, N, K, a, a_i, a_k, b, b_k, b_j, bias,
                           mode, g, Cf, cb, ldc, kps, part);
    }
    if (splits > 1)
        hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for(int64_t{M} * N, 256)), dim3(256), 0, st, M,
                           N, splits, part, Cf, ldc);
}

void launch_softmax_xent(int B, int A, const float* Z, const float* target, const float* mask,
                         void* dZ, float* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_softmax_xent, dim3(blocks_for(B, 256)), dim3(256), 0, st, B, A, Z, target,
                       mask, static_cast<__bf16*>(dZ), loss);
}

bool launch_mlp_forward(int M, int F, int H, int A, const void* X, const void* W1P, const float* b1,
                        const void* W2P, const float* b2, const void* W3T, const float* b3,
                        float* Z, hipStream_t st) {
    if (F % 16 != 0 || F > kFusedMaxF || A > kNarrow ||
        (reinterpret_cast<uintptr_t>(X) % 16) != 0)
        return false;
    const auto* x = static_cast<const __bf16*>(X);
    const auto* w1 = static_cast<const __bf16*>(W1P);
    const auto* w2 = static_cast<const __bf16*>(W2P);
    const auto* w3 = static_cast<const __bf16*>(W3T);
    const dim3 grid((M + 31) / 32);
    switch (H) {
        case 64:
            hipLaunchKernelGGL(k_mlp_forward<64>, grid, dim3(64), 0, st, M, F, A, x, w1, b1, w2, b2,
                               w3, b3, Z);
            return true;
        case 128:
            hipLaunchKernelGGL(k_mlp_forward<128>, grid, dim3(64), 0, st, M, F, A, x, w1, b1, w2,
                               b2, w3, b3, Z);
            return true;
        case 256:
            hipLaunchKernelGGL(k_mlp_forward<256>, grid, dim3(64), 0, st, M, F, A, x, w1, b1, w2,
                               b2, w3, b3, Z);
            return true;
        default:
            return false;
    }
}

void launch_pack_fragments(int K, int H, const void* WT, void* dst, hipStream_t st) {
    const int64_t n = int64_t{K} * H;
    if (n > 0 && K % 16 == 0 && H % 32 == 0)
        hipLaunchKernelGGL(k_pack_fragments, dim3(blocks_for(n, 256)), dim3(256), 0, st, K, H,
                           static_cast<const __bf16*>(WT), static_cast<__bf16*>(dst));
}

void launch_transpose_bf16(int rows, int cols, const void* src, void* dst, hipStream_t st) {
    const int64_t n = int64_t{rows} * cols;
    if (n > 0)
        hipLaunchKernelGGL(k_transpose_bf16, dim3(blocks_for(n, 256)), dim3(256), 0, st, rows, cols,
                           static_cast<const __bf16*>(src), static_cast<__bf16*>(dst));
}

void launch_colsum(int rows, int cols, const void* G, float* out, hipStream_t st, float* part) {
    // 32 rows per split, at most kColsumMaxSplits partials
    const int splits = max(1, min(kColsumMaxSplits, rows / 32));
    const int rps = (rows + splits - 1) / splits;
    hipLaunchKernelGGL(k_colsum_part, dim3((cols + 63) / 64, splits), dim3(64), 0, st, rows, cols,
                       rps, static_cast<const __bf16*>(G), part);
    hipLaunchKernelGGL(k_sum_cols, dim3((cols + 3) / 4), dim3(256), 0, st, cols, splits, part, out);
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
