// gfx950 kernels over the public-block execution plan (xplan.hpp).
//
// An iteration (Section 3.2) is one top-down launch per level for the reach
// probabilities (Eq. excepted_reach_probabilities_matrix_recurrence and its own-reach
// twin) and one bottom-up launch per level that, per chunk of whole infosets, finishes
// each infoset: its members' expected payoffs (Eq. expected_payoffs_matrix_recurrence), the
// instantaneous counterfactual regrets in their multiplied-out form (Eq.
// instantaneous_counterfactual_regret), the player reach of Eq. (player_reach_probability),
// and the cumulative regret / average / regret-matching update (Eqs.
// average_counterfactual_regrets_vector, average_strategy_profile_vector,
// next_strategy_profile). All members of an infoset sit in one public block, so a chunk
// reads a compact slice; nothing is accumulated with atomics and the result does not depend
// on scheduling or on the launch shape. Chance nodes are reduced by lane groups. The first,
// tiny levels of each direction run in one workgroup with barriers between levels.
//
// The passes are bound by HBM traffic and by the latency of dependent loads (the level
// structure forces node -> child -> value chains), so the kernels keep those chains short
// (member-major copies of the per-member operands, pair operands loaded before they are
// needed) and give each thread several independent nodes or members.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "xkernels.hpp"

namespace cfr {

namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

inline unsigned blocks_of(int64_t n, int threads) {
    return static_cast<unsigned>((n + threads - 1) / threads);
}

__device__ __forceinline__ int64_t gid() {
    return static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}

// The hardware hands workgroup b to XCD b % 8 (each XCD has its own L2). Renumber so that each
// XCD takes one contiguous run of tiles: neighbouring tiles share cache lines (a parent block,
// the edges of a child range), and that sharing then stays inside one L2.
__device__ __forceinline__ uint32_t xcd_tile() {
    constexpr uint32_t kXcds = 8;
    const uint32_t g = gridDim.x, b = blockIdx.x;
    const uint32_t q = g / kXcds, r = g % kXcds;
    const uint32_t xcd = b % kXcds, j = b / kXcds;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + j;
}

__device__ __forceinline__ int32_t child_of(const int32_t* __restrict__ child_begin,
                                            const int32_t* __restrict__ child_stride,
                                            const int32_t* __restrict__ child_list, int32_t x,
                                            int32_t a) {
    const int32_t st = child_stride[x];
    const int32_t cb = child_begin[x];
    return st != 0 ? cb + a * st : child_list[cb + a];
}

// A 16-byte record read once per iteration, loaded with the non-temporal hint. The member and
// infoset records of the bottom-up pass and the parent and edge words of the top-down pass are
// streamed once per iteration; with the hint they stop displacing, from the caches, the values,
// reaches and strategies that the next launches read again (the large-game iteration: 247.7 to
// 224-226 us). The same hint on the reaches, the children's values or the regret and strategy
// sums made it slower: those lines are read again.
__device__ __forceinline__ int4 nt_load4(const int4* p) {
    typedef int v4 __attribute__((ext_vector_type(4)));
    const v4 v = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
    return make_int4(v.x, v.y, v.z, v.w);
}

// A member record's child stride and k | player byte: with packed records (XDev::kp_packed) the
// stride is the low 24 bits of the last word (signed) and the byte its top 8 bits; otherwise the
// word is the stride and the byte comes from mem_kp.
__device__ __forceinline__ int32_t rec_stride(int32_t w, int32_t packed) {
    return packed ? static_cast<int32_t>(static_cast<uint32_t>(w) << 8) >> 8 : w;
}
__device__ __forceinline__ int rec_kp(int32_t w, int32_t packed, const int8_t* mem_kp, int32_t m) {
    return packed ? static_cast<int>(static_cast<uint32_t>(w) >> 24) : mem_kp[m];
}

// ---- top-down (reach)

// Reach of NPT nodes x = first + u * stride: the factor of whoever acted into the node (meta
// bits 2-3) is multiplied by the edge probability (sigma or sigma_0). Terminal nodes need no
// reach. All loads of the NPT nodes are issued before any of them is used, and a node's parent
// and edge are loaded together with its kind (with parent_ek, all three in one 8-byte word). The chance plane depends on sigma_0 alone: FULL
// computes all three planes (once, when the solver is set up); otherwise only the two player
// planes are written, a chance edge copies them and the chance plane is left as it is.
template <int NPT, bool FULL>
__device__ __forceinline__ void reach_nodes(int64_t first, int64_t stride, int64_t hi, int64_t N,
                                            const int32_t* __restrict__ parent,
                                            const int32_t* __restrict__ edge,
                                            const int8_t* __restrict__ meta,
                                            const float* __restrict__ prob,
                                            float* __restrict__ reach,
                                            const int64_t* __restrict__ parent_ek = nullptr) {
    int64_t xs[NPT];
    int kind[NPT];
    int32_t p[NPT], e[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        xs[u] = first + u * stride;
        kind[u] = 0;
        p[u] = e[u] = 0;
        if (xs[u] < hi) {  // every node below the root has a parent and an edge
            if (parent_ek != nullptr) {  // parent low; edge in bits 32-55, the kind byte on top
                const uint64_t w =
                    static_cast<uint64_t>(__builtin_nontemporal_load(&parent_ek[xs[u]]));
                p[u] = static_cast<int32_t>(static_cast<uint32_t>(w));
                kind[u] = static_cast<int>(w >> 56);
                e[u] = static_cast<int32_t>((w >> 32) & 0xFFFFFFu);
            } else {
                p[u] = __builtin_nontemporal_load(&parent[xs[u]]);
                kind[u] = meta[xs[u]];
                e[u] = edge[xs[u]];
            }
        }
    }
    float r1[NPT], r2[NPT], rc[NPT], s[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        r1[u] = r2[u] = rc[u] = s[u] = 0.0f;
        if (kind[u] & 3) {
            r1[u] = reach[p[u]];
            r2[u] = reach[N + p[u]];
            if (FULL) rc[u] = reach[2 * N + p[u]];
            if (FULL || (kind[u] >> 2) != 1) s[u] = prob[e[u]];
        }
    }
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        if ((kind[u] & 3) == 0) continue;
        const int actor = kind[u] >> 2;  // 1 chance, 2 player 1, 3 player 2
        if (actor == 2) r1[u] *= s[u];
        else if (actor == 3) r2[u] *= s[u];
        else rc[u] *= s[u];
        reach[xs[u]] = r1[u];
        reach[N + xs[u]] = r2[u];
        if (FULL) reach[2 * N + xs[u]] = rc[u];
    }
}

// One level: workgroup b takes tile t0 + b, a run of at most blockDim * NPT decision nodes
// (terminal nodes, which need no reach, take no lanes); each thread takes NPT of them blockDim
// apart (every load coalesced across the wavefront).
template <int NPT>
__global__ void __launch_bounds__(1024) k_x_reach(int32_t t0, int64_t N,
                                                  const int32_t* __restrict__ tile_lo,
                                                  const int32_t* __restrict__ tile_hi,
                                                  const int32_t* __restrict__ parent,
                                                  const int32_t* __restrict__ edge,
                                                  const int8_t* __restrict__ meta,
                                                  const float* __restrict__ prob,
                                                  float* __restrict__ reach,
                                                  const int64_t* __restrict__ parent_ek) {
    const int32_t t = t0 + static_cast<int32_t>(xcd_tile());
    const int32_t lo = tile_lo[t], hi = tile_hi[t];
    reach_nodes<NPT, false>(lo + static_cast<int64_t>(threadIdx.x), blockDim.x, hi, N, parent, edge,
                            meta, prob, reach, parent_ek);
}

// One level as k_x_reach, with the records read two nodes at a time: thread i takes the pairs of
// nodes (b + 2j, b + 2j + 1), j = i + u * blockDim, from b = lo rounded down to even, and loads
// both nodes' {parent, edge | kind << 24} records in one 16-byte load (the record array holds
// N + 1 entries, so the pair at N - 1 stays in bounds). Nodes outside [lo, hi) are neither
// computed nor stored. A tile of at most blockDim * NPT nodes spans at most blockDim * NPT / 2 + 1
// pairs: NPT / 2 + 1 pair slots per thread. The arithmetic is reach_nodes' (bit-identical).
template <int NPT>
__global__ void __launch_bounds__(1024) k_x_reach_pairs(int32_t t0, int64_t N,
                                                        const int32_t* __restrict__ tile_lo,
                                                        const int32_t* __restrict__ tile_hi,
                                                        const float* __restrict__ prob,
                                                        float* __restrict__ reach,
                                                        const int64_t* __restrict__ parent_ek) {
    typedef long long v2i64 __attribute__((ext_vector_type(2)));
    constexpr int NP = NPT / 2 + 1;
    const int32_t t = t0 + static_cast<int32_t>(xcd_tile());
    const int64_t lo = tile_lo[t], hi = tile_hi[t];
    const int64_t base = lo & ~int64_t{1};
    const int64_t npairs = (hi - base + 1) >> 1;
    int64_t xs[2 * NP];
    int kind[2 * NP];
    int32_t p[2 * NP], e[2 * NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        const int64_t pj = static_cast<int64_t>(threadIdx.x) + static_cast<int64_t>(u) * blockDim.x;
        xs[2 * u] = base + 2 * pj;
        xs[2 * u + 1] = base + 2 * pj + 1;
        uint64_t w[2] = {0, 0};
        if (pj < npairs) {
            const v2i64 r = __builtin_nontemporal_load(
                reinterpret_cast<const v2i64*>(parent_ek + base + 2 * pj));
            w[0] = static_cast<uint64_t>(r.x);
            w[1] = static_cast<uint64_t>(r.y);
        }
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int64_t x = xs[2 * u + v];
            const bool in = x >= lo && x < hi;
            p[2 * u + v] = static_cast<int32_t>(static_cast<uint32_t>(w[v]));
            kind[2 * u + v] = in ? static_cast<int>(w[v] >> 56) : 0;
            e[2 * u + v] = static_cast<int32_t>((w[v] >> 32) & 0xFFFFFFu);
        }
    }
    float r1[2 * NP], r2[2 * NP], s[2 * NP];
#pragma unroll
    for (int u = 0; u < 2 * NP; ++u) {
        r1[u] = r2[u] = s[u] = 0.0f;
        if (kind[u] & 3) {
            r1[u] = reach[p[u]];
            r2[u] = reach[N + p[u]];
            if ((kind[u] >> 2) != 1) s[u] = prob[e[u]];
        }
    }
#pragma unroll
    for (int u = 0; u < 2 * NP; ++u) {
        if ((kind[u] & 3) == 0) continue;
        const int actor = kind[u] >> 2;  // 1 chance, 2 player 1, 3 player 2
        if (actor == 2) r1[u] *= s[u];
        else if (actor == 3) r2[u] *= s[u];
        reach[xs[u]] = r1[u];
        reach[N + xs[u]] = r2[u];
    }
}

// Several small levels in one launch without a barrier between them: the node of each lane
// (tiles as in k_x_reach, one node per lane) walks up through its ancestors to the first stored
// level (nodes below `stop`), at most kPathDepth steps, collecting the edge probabilities and
// actors, then multiplies them onto the ancestor's reach from the top down, in the order the
// level-by-level pass uses.
__global__ void __launch_bounds__(256) k_x_reach_path(int32_t t0, int32_t stop, int64_t N,
                                                      const int32_t* __restrict__ tile_lo,
                                                      const int32_t* __restrict__ tile_hi,
                                                      const int32_t* __restrict__ parent,
                                                      const int32_t* __restrict__ edge,
                                                      const int8_t* __restrict__ meta,
                                                      const float* __restrict__ prob,
                                                      float* __restrict__ reach) {
    const int32_t t = t0 + static_cast<int32_t>(xcd_tile());
    const int32_t x = tile_lo[t] + static_cast<int32_t>(threadIdx.x);
    if (x >= tile_hi[t] || (meta[x] & 3) == 0) return;
    float s[kPathDepth];
    int actor[kPathDepth];
    int n = 0;
    int32_t y = x;
    while (y >= stop && n < kPathDepth) {
        actor[n] = (meta[y] >> 2) & 3;
        s[n] = actor[n] == 1 ? 1.0f : prob[edge[y]];
        y = parent[y];
        ++n;
    }
    float r1 = reach[y], r2 = reach[N + y];
    for (int i = n - 1; i >= 0; --i) {
        if (actor[i] == 2) r1 *= s[i];
        else if (actor[i] == 3) r2 *= s[i];
    }
    reach[x] = r1;
    reach[N + x] = r2;
}

// All three planes of one level's nodes lo .. hi - 1 (grid-stride), the chance plane included:
// run level by level when the solver is set up.
__global__ void __launch_bounds__(256) k_x_reach_full(int32_t lo, int32_t hi, int64_t N,
                                                      const int32_t* __restrict__ parent,
                                                      const int32_t* __restrict__ edge,
                                                      const int8_t* __restrict__ meta,
                                                      const float* __restrict__ prob,
                                                      float* __restrict__ reach) {
    for (int64_t x = lo + gid(); x < hi; x += static_cast<int64_t>(gridDim.x) * blockDim.x)
        reach_nodes<1, true>(x, 1, hi, N, parent, edge, meta, prob, reach);
}

// The levels one single-workgroup kernel takes, in the order it takes them; entry i covers
// nodes (top-down) or chunks (bottom-up) lo[i] .. hi[i] - 1 and chance nodes clo[i] .. chi[i] - 1.
struct LevelTable {
    int32_t n;
    int32_t lo[kFuseMax], hi[kFuseMax];
    int32_t clo[kFuseMax], chi[kFuseMax];
    int32_t glog[kFuseMax];  // log2 lanes per chance node (bottom-up)
};

// Touches the table's lines: each of the workgroup's kFuseThreads threads loads one byte of
// its line (or of the range's last line) in every range, all loads issued before the first
// wait. The bytes themselves are not needed.
__device__ __forceinline__ void warm_lines(const WarmTable& w, int tid) {
    if (w.lines[0] == 0) return;
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < kWarmMax; ++r) {
        const int32_t i = tid < w.lines[r] ? tid : w.lines[r] - 1;
        acc ^= w.p[r][static_cast<int64_t>(i) * kWarmLine];
    }
    asm volatile("" ::"v"(acc));
}

// The first top-down levels in one workgroup: a barrier between levels instead of a launch.
__global__ void __launch_bounds__(kFuseThreads) k_x_reach_top(LevelTable t, WarmTable w, int64_t N,
                                                              const int32_t* __restrict__ parent,
                                                              const int32_t* __restrict__ edge,
                                                              const int8_t* __restrict__ meta,
                                                              const float* __restrict__ prob,
                                                              float* __restrict__ reach) {
    warm_lines(w, threadIdx.x);
    for (int32_t i = 0; i < t.n; ++i) {
        reach_nodes<2, false>(t.lo[i] + threadIdx.x, kFuseThreads, t.hi[i], N, parent, edge, meta,
                              prob, reach);
        __syncthreads();
    }
}

// ---- bottom-up (values, regrets, average, regret matching)

struct UpArgs {
    int64_t N;
    const int32_t* chunk_first;
    const int32_t* chunk_m;
    const int32_t* child_begin;
    const int32_t* child_stride;
    const int32_t* child_list;
    const int4* mem_rec;
    const int8_t* mem_kp;
    const int4* set_rec;
    const int32_t* chance_nodes;
    const int32_t* chance_base;
    const int32_t* chance_k;
    float* prob;
    float* value;
    float* reach;
    float* R;
    float* S;
    int64_t* T;
    UpdateRule rule;
    // derive_reach != 0 (the deepest decision level, whose children are all terminal): the
    // level had no top-down launch; a member's player planes are its parent's times its edge
    // probability on the factor of whoever acted (the top-down products), computed and stored
    // here
    int32_t derive_reach;
    int32_t kp_packed;  // member records carry the k | player byte (XDev::kp_packed)
    const int32_t* parent;
    const int32_t* edge;
    const int8_t* meta;
};

// The three reach planes of member node x: loaded, or (derive_reach) the player planes computed
// from the parent's as the top-down pass would and stored (the chance plane is constant).
__device__ __forceinline__ void member_reach(const UpArgs& a, int32_t x, float& r1, float& r2,
                                             float& rc) {
    rc = a.reach[2 * a.N + x];
    if (!a.derive_reach) {
        r1 = a.reach[x];
        r2 = a.reach[a.N + x];
        return;
    }
    const int kind = a.meta[x];
    const int32_t p = a.parent[x], e = a.edge[x];
    r1 = a.reach[p];
    r2 = a.reach[a.N + p];
    const int actor = kind >> 2;  // 1 chance, 2 player 1, 3 player 2
    const float s = actor != 1 ? a.prob[e] : 1.0f;
    if (actor == 2) r1 *= s;
    else if (actor == 3) r2 *= s;
    a.reach[x] = r1;
    a.reach[a.N + x] = r2;
}

// Chance node ci (if ok) on a group of 2^glog lanes: lane l sums children l, l + 2^glog, ...,
// then a butterfly over the group (a fixed order). Every lane of the wavefront must call it
// with the same glog.
__device__ __forceinline__ void chance_group(const UpArgs& a, int32_t ci, bool ok, int lane,
                                             int glog) {
    float v = 0.0f;
    int32_t x = 0;
    if (ok) {
        x = a.chance_nodes[ci];
        const int32_t base = a.chance_base[ci], k = a.chance_k[ci];
        const int32_t cb = a.child_begin[x], st = a.child_stride[x];
        for (int32_t c = lane; c < k; c += 1 << glog)
            v = fmaf(a.prob[base + c], a.value[st != 0 ? cb + c * st : a.child_list[cb + c]], v);
    }
    for (int off = (1 << glog) >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (ok && lane == 0) a.value[x] = v;
}

// Phase 2 of a chunk for one infoset h (pair operands pr = R, ps = S, pp = sigma already
// loaded): sums its members' LDS slots slo .. shi - 1 in member order, then the regret update
// (vanilla, CFR+ clipped, or discounted), the average-strategy update S += w pi-bar sigma
// (discounted: then scaled) and regret matching into sigma, written to Ro, So, Po (the
// infoset's first pair, in memory or in LDS); t is the 1-based iteration.
template <int KMAX>
__device__ __forceinline__ void update_infoset(const UpArgs& a, float* Ro, float* So, float* Po,
                                               int32_t k, int player, int32_t slo, int32_t shi,
                                               const float* pr, const float* ps, const float* pp,
                                               float (*s_con)[KMAX], const float* s_own, float t) {
    if (!((a.rule.players >> (player - 1)) & 1)) return;  // not this pass's player
    float racc[KMAX];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) racc[j] = 0.0f;
    float own = 0.0f;
    // member order; unrolled so that several members' slots are read at once
#pragma unroll 4
    for (int32_t sl = slo; sl < shi; ++sl) {
#pragma unroll
        for (int j = 0; j < KMAX; ++j) racc[j] += s_con[sl][j];
        own += s_own[sl];
    }
    const float sgn = player == 1 ? 1.0f : -1.0f;
    const bool disc = a.rule.variant == 2;
    float wt = a.rule.linear ? t : 1.0f;
    float d_pos = 1.0f, d_neg = 1.0f, d_avg = 1.0f;
    if (disc) {
        wt = 1.0f;
        dcfr_discounts(a.rule, t, d_pos, d_neg, d_avg);
    }
    float pos_sum = 0.0f;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        if (j < k) {
            float r = fmaf(sgn, racc[j], pr[j]);
            if (a.rule.variant == 1) r = fmaxf(r, 0.0f);
            else if (disc) r *= r > 0.0f ? d_pos : d_neg;
            Ro[j] = r;
            const float sn = fmaf(wt * own, pp[j], ps[j]);
            So[j] = disc ? sn * d_avg : sn;
            racc[j] = r;
            pos_sum += fmaxf(r, 0.0f);
        }
    }
    if (pos_sum > 0.0f) {
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) Po[j] = fmaxf(racc[j], 0.0f) / pos_sum;
    } else {
        const float unif = 1.0f / static_cast<float>(k);
#pragma unroll
        for (int j = 0; j < KMAX; ++j)
            if (j < k) Po[j] = unif;
    }
}

template <int KMAX>
__device__ __forceinline__ void load_pairs(const UpArgs& a, int32_t o, int32_t k, float* pr,
                                           float* ps, float* pp) {
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        pr[j] = ps[j] = pp[j] = 0.0f;
        if (j < k) {
            pr[j] = a.R[o + j];
            ps[j] = a.S[o + j];
            pp[j] = a.prob[o + j];
        }
    }
}

// One chunk: whole infosets of one level with at most CH * MPT members in total (or one
// larger infoset). Phase 1, MPT members per thread, all their loads issued first: child
// values (gather by stride), the member's value, its regret contributions cf * (w_a - v) and
// its own reach, into the member's LDS slot. Phase 2, one thread per infoset (a chunk of
// single-member infosets has up to CH * MPT of them: threads stride): sums its members'
// slots in member order (deterministic, independent of the shape), then update_infoset. The
// pair operands of each thread's first infoset are loaded before phase 1. An infoset with
// more members than the chunk holds is accumulated per thread (CH slots). Every thread of the
// workgroup must call it; it holds one barrier.
template <int KMAX, int CH, int MPT>
__device__ __forceinline__ void up_chunk(const UpArgs& a, int32_t c, float (*s_con)[KMAX],
                                         float* s_own, int tid) {
    constexpr int CAP = CH * MPT;
    constexpr bool kPrefetch = KMAX <= 4;
    const int32_t h0 = a.chunk_first[c], h1 = a.chunk_first[c + 1];
    const int32_t m0 = a.chunk_m[c], m1 = a.chunk_m[c + 1];
    const int32_t nm = m1 - m0, nh = h1 - h0;
    const bool big = nm > CAP;
    int32_t o = 0, k = 0, slo = 0, shi = 0;
    int player = 1;
    float pr[KMAX], ps[KMAX], pp[KMAX];
    if (tid < nh) {
        const int4 hr = nt_load4(&a.set_rec[h0 + tid]);
        o = hr.x;
        slo = hr.y - m0;
        shi = hr.z - m0;
        k = hr.w & 31;
        player = (hr.w & 64) ? 2 : 1;
        if (kPrefetch) load_pairs<KMAX>(a, o, k, pr, ps, pp);
    }
    if (!big) {
        int32_t x[MPT], q[MPT], cb[MPT], st[MPT], kp[MPT];
#pragma unroll
        for (int u = 0; u < MPT; ++u) {
            const int32_t mi = tid + u * CH;
            x[u] = q[u] = cb[u] = st[u] = kp[u] = 0;
            if (mi < nm) {
                const int32_t m = m0 + mi;
                const int4 r = nt_load4(&a.mem_rec[m]);
                x[u] = r.x;
                q[u] = r.y;
                cb[u] = r.z;
                st[u] = rec_stride(r.w, a.kp_packed);
                kp[u] = rec_kp(r.w, a.kp_packed, a.mem_kp, m);
            }
        }
        float w[MPT][KMAX], sg[MPT][KMAX], r1[MPT], r2[MPT], rc[MPT];
#pragma unroll
        for (int u = 0; u < MPT; ++u) {
            r1[u] = r2[u] = rc[u] = 0.0f;
            const int kk = kp[u] & 31;
            if (kk > 0) member_reach(a, x[u], r1[u], r2[u], rc[u]);
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                w[u][j] = sg[u][j] = 0.0f;
                if (j < kk) {
                    const int32_t ch = st[u] != 0 ? cb[u] + j * st[u] : a.child_list[cb[u] + j];
                    w[u][j] = a.value[ch];
                    sg[u][j] = a.prob[q[u] + j];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < MPT; ++u) {
            const int32_t mi = tid + u * CH;
            if (mi >= nm) continue;
            float v = 0.0f;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) v = fmaf(sg[u][j], w[u][j], v);
            a.value[x[u]] = v;
            const bool p2 = (kp[u] & 64) != 0;
            const float cf = (p2 ? r1[u] : r2[u]) * rc[u];
#pragma unroll
            for (int j = 0; j < KMAX; ++j) s_con[mi][j] = cf * (w[u][j] - v);
            s_own[mi] = p2 ? r2[u] : r1[u];
        }
    } else {
        float con[KMAX];
        float own = 0.0f;
#pragma unroll
        for (int j = 0; j < KMAX; ++j) con[j] = 0.0f;
#pragma unroll 1
        for (int32_t mi = tid; mi < nm; mi += CH) {
            const int32_t m = m0 + mi;
            const int4 r = a.mem_rec[m];
            const int32_t xm = r.x, qm = r.y, cbm = r.z, stm = rec_stride(r.w, a.kp_packed);
            const int kpm = rec_kp(r.w, a.kp_packed, a.mem_kp, m);
            const int kk = kpm & 31;
            float w[KMAX];
            float v = 0.0f;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                w[j] = 0.0f;
                if (j < kk) {
                    w[j] = a.value[stm != 0 ? cbm + j * stm : a.child_list[cbm + j]];
                    v = fmaf(a.prob[qm + j], w[j], v);
                }
            }
            a.value[xm] = v;
            float r1, r2, rc;
            member_reach(a, xm, r1, r2, rc);
            const bool p2 = (kpm & 64) != 0;
            const float cf = (p2 ? r1 : r2) * rc;
            own += p2 ? r2 : r1;
#pragma unroll
            for (int j = 0; j < KMAX; ++j)
                if (j < kk) con[j] = fmaf(cf, w[j] - v, con[j]);
        }
#pragma unroll
        for (int j = 0; j < KMAX; ++j) s_con[tid][j] = con[j];
        s_own[tid] = own;
    }
    __syncthreads();
    if (big) {
        if (tid == 0) {
            if (!kPrefetch) load_pairs<KMAX>(a, o, k, pr, ps, pp);
            update_infoset<KMAX>(a, a.R + o, a.S + o, a.prob + o, k, player, 0,
                                 nm < CH ? nm : CH, pr, ps, pp, s_con, s_own,
                                 static_cast<float>(*a.T + 1));
        }
        return;
    }
    // nh <= nm <= CH * MPT: each thread has at most MPT infosets
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
        const int32_t li = tid + u * CH;
        if (li >= nh) break;
        const int32_t h = h0 + li;
        if (u > 0) {  // the first infoset's operands were loaded before phase 1
            const int4 hr = a.set_rec[h];
            o = hr.x;
            slo = hr.y - m0;
            shi = hr.z - m0;
            k = hr.w & 31;
            player = (hr.w & 64) ? 2 : 1;
        }
        if (u > 0 || !kPrefetch) load_pairs<KMAX>(a, o, k, pr, ps, pp);
        update_infoset<KMAX>(a, a.R + o, a.S + o, a.prob + o, k, player, slo, shi, pr, ps, pp,
                             s_con, s_own, static_cast<float>(*a.T + 1));
    }
}

// Bottom-up of one level: workgroups [0, nk) take the level's chunks, the rest its chance
// nodes, CH >> glog of them per workgroup.
template <int KMAX, int CH, int MPT>
__global__ void __launch_bounds__(CH) k_x_up_level(UpArgs a, int32_t klo, int32_t nk, int32_t clo,
                                                   int32_t nc, int glog) {
    __shared__ float s_con[CH * MPT][KMAX];
    __shared__ float s_own[CH * MPT];
    const int32_t b = static_cast<int32_t>(xcd_tile());
    if (b < nk) {
        up_chunk<KMAX, CH, MPT>(a, klo + b, s_con, s_own, threadIdx.x);
        return;
    }
    const int32_t i = (b - nk) * (CH >> glog) + static_cast<int32_t>(threadIdx.x >> glog);
    chance_group(a, clo + i, i < nc, threadIdx.x & ((1 << glog) - 1), glog);
}

// The shallowest levels, deepest first, in one workgroup (each level's chance nodes fit one
// pass of the workgroup); then the iteration is counted (every read of T came before).
__global__ void __launch_bounds__(kFuseThreads) k_x_up_top(UpArgs a, LevelTable t, WarmTable w) {
    __shared__ float s_con[kFuseThreads][4];
    __shared__ float s_own[kFuseThreads];
    const int tid = threadIdx.x;
    warm_lines(w, tid);
    for (int32_t i = 0; i < t.n; ++i) {
        const int g = t.glog[i];
        const int32_t ci = t.clo[i] + (tid >> g);
        chance_group(a, ci, ci < t.chi[i], tid & ((1 << g) - 1), g);
        for (int32_t c = t.lo[i]; c < t.hi[i]; ++c) {
            up_chunk<4, kFuseThreads, 1>(a, c, s_con, s_own, tid);
            __syncthreads();
        }
        __syncthreads();
    }
    if (tid == 0 && a.rule.count) *a.T += 1;
}

// ---- subtree packs (xplan.hpp): one workgroup per pack, both sweeps on chip
//
// The pack's decision nodes are numbered 0 .. n_dec - 1 (didx); LDS holds their reach planes and
// values and the pack's pairs (sigma, and R and S where the launch updates them). Each thread
// keeps its members' records in registers (member m in slot m / T of thread m % T). The
// arithmetic is that of the per-level kernels in the same order: a child's reach is its
// parent's times the edge probability on the actor's factor; a member's value is sum_a
// sigma(a) w_a in action order; its regret contributions cf (w_a - v) and own reach go to its
// slot, and each infoset sums its slots in member order before update_infoset. Modes: 0 both
// sweeps (tier 1), 1 top-down only (tiers >= 2: store the reach of the members and chance
// nodes that have external children), 2 bottom-up (tiers >= 2: reach again on chip, then the
// values, with the external children's values from memory, and the updates).

struct PackArgs {
    const PackDesc* packs;
    const int32_t* blob;
    int32_t first;  // the launch takes packs first .. first + gridDim.x - 1
    int32_t mode;
    int32_t keep;   // also store every decision node's value and reach
    int32_t count;  // the launch ends the iteration: its last workgroup counts it (T += 1)
    uint32_t* done; // workgroups of the launch that have finished (zero between launches)
};

__device__ __forceinline__ float as_float(int32_t w) { return __int_as_float(w); }

template <int T>
__global__ void __launch_bounds__(T) k_x_pack(UpArgs a, PackArgs pa) {
    constexpr int S = kPackSlots;
    constexpr int kDescWords = sizeof(PackDesc) / 4;
    __shared__ float s_val[kPackDec];
    __shared__ float s_rch[3][kPackDec];
    __shared__ float s_sig[kPackPairs];
    __shared__ float s_R[kPackPairs];
    __shared__ float s_S[kPackPairs];
    __shared__ float s_con[kPackDec][4];  // per member of the level being finished
    __shared__ float s_own[kPackDec];
    __shared__ int4 s_ch[kPackChance];
    __shared__ int32_t s_kw[kPackKids];   // child: decision index, or value bits
    __shared__ float s_kp[kPackKids];     // probability, sign bit set for a decision child
    __shared__ int32_t s_desc[kDescWords];
    __shared__ float s_t;
    const int tid = threadIdx.x;
    const int64_t N = a.N;
    const int mode = pa.mode;
    const bool bottom_up = mode != 1;
    {
        const int32_t* d = reinterpret_cast<const int32_t*>(pa.packs + pa.first + xcd_tile());
        for (int w = tid; w < kDescWords; w += T) s_desc[w] = d[w];
        if (tid == 0) s_t = static_cast<float>(*a.T + 1);  // read before this workgroup counts
    }
    __syncthreads();
    const PackDesc& pk = *reinterpret_cast<const PackDesc*>(s_desc);
    const int32_t* __restrict__ B = pa.blob;
    const int32_t n_mem = pk.n_mem, n_inf = pk.n_inf, nlv = pk.nlv;

    // every record the sweeps need, all loads in flight together: members and infosets into
    // registers (record m in slot m / T of thread m % T), chance nodes and their children into
    // LDS
    int32_t rec[S][6];
    int4 inf[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int32_t m = tid + j * T;
#pragma unroll
        for (int w = 0; w < 6; ++w) rec[j][w] = m < n_mem ? B[pk.off_mem + 6 * m + w] : 0;
        inf[j] = m < n_inf ? *reinterpret_cast<const int4*>(B + pk.off_inf + 4 * m)
                           : make_int4(0, 0, 0, 0);
    }
    // (unrolled, so that every load is issued before the first wait)
    constexpr int KU = kPackKids / T, CU = (kPackChance + T - 1) / T, RU = kPackDec / T;
    const int32_t n_kid = pk.n_kid, n_ch = pk.n_ch, n_root = pk.n_root;
    int32_t kwv[KU], kpv[KU], kkv[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
        const int32_t c = tid + u * T;
        kwv[u] = kpv[u] = kkv[u] = 0;
        if (c < n_kid) {
            const int32_t* kw = B + pk.off_kid + 3 * c;
            kwv[u] = kw[0];
            kpv[u] = kw[1];
            kkv[u] = kw[2];
        }
    }
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        const int32_t c = tid + u * T;
        if (c < n_ch) s_ch[c] = *reinterpret_cast<const int4*>(B + pk.off_ch + 4 * c);
    }
    int4 root[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
        const int32_t i = tid + u * T;
        root[u] = i < n_root ? *reinterpret_cast<const int4*>(B + pk.off_root + 4 * i)
                             : make_int4(0, -1, 0, 0);
    }
    // second round: external children's values (bottom-up), the roots' parents' reach and
    // edge probabilities, the pairs
#pragma unroll
    for (int u = 0; u < KU; ++u) {
        if (kkv[u] == 2 && bottom_up) {  // an external child: its value, as a constant
            kwv[u] = __float_as_int(a.value[kwv[u]]);
            kkv[u] = 1;
        }
    }
    // pairs: sigma (and R, S for the updates)
#pragma unroll
    for (int j = 0; j < S; ++j) {
        if (tid + j * T >= n_inf) continue;
        const int k = inf[j].w & 255;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= k) continue;
            s_sig[inf[j].y + c] = a.prob[inf[j].x + c];
            if (bottom_up) {
                s_R[inf[j].y + c] = a.R[inf[j].x + c];
                s_S[inf[j].y + c] = a.S[inf[j].x + c];
            }
        }
    }
    // roots: reach from their parents' stored reach (the game's root: 1)
#pragma unroll
    for (int u = 0; u < RU; ++u) {
        if (tid + u * T >= n_root) continue;
        const int4 r = root[u];
        float r1 = 1.0f, r2 = 1.0f, rc = 1.0f;
        if (r.y >= 0) {
            r1 = a.reach[r.y];
            r2 = a.reach[N + r.y];
            rc = a.reach[2 * N + r.y];
            const float s = a.prob[r.z];
            const int actor = (r.x >> 16) & 3;  // 1 chance, 2 player 1, 3 player 2
            if (actor == 2) r1 *= s;
            else if (actor == 3) r2 *= s;
            else rc *= s;
        }
        const int d = r.x & 0xffff;
        s_rch[0][d] = r1;
        s_rch[1][d] = r2;
        s_rch[2][d] = rc;
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) {
        const int32_t c = tid + u * T;
        if (c >= n_kid) continue;
        s_kw[c] = kwv[u];
        // probabilities are >= 0: the sign bit marks a child that is a decision node of the pack
        s_kp[c] = kkv[u] == 0 ? -as_float(kpv[u]) : as_float(kpv[u]);
    }
    // bottom-up: the members' external children's values, read once and held as constants
    if (mode == 2) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (tid + j * T >= n_mem || !((rec[j][0] >> 20) & 1)) continue;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (((rec[j][0] >> (24 + 2 * c)) & 3) == 2) {
                    rec[j][2 + c] = __float_as_int(a.value[rec[j][2 + c]]);
                    rec[j][0] ^= 3 << (24 + 2 * c);  // kind 2 -> kind 1 (a constant)
                }
        }
    }
    __syncthreads();

    // top-down: each decision node of level d gives its decision children their reach
    for (int32_t d = 0; d + 1 < nlv; ++d) {
        const int32_t m0 = pk.mlo[d], m1 = pk.mlo[d + 1];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int32_t m = tid + j * T;
            if (m < m0 || m >= m1) continue;
            const int32_t w0 = rec[j][0];
            const int dd = w0 & 0xffff, k = (w0 >> 16) & 7;
            const bool p2 = (w0 >> 19) & 1;
            const float r1 = s_rch[0][dd], r2 = s_rch[1][dd], rc = s_rch[2][dd];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (c >= k || ((w0 >> (24 + 2 * c)) & 3) != 0) continue;
                const int cd = rec[j][2 + c];
                const float s = s_sig[rec[j][1] + c];
                s_rch[0][cd] = p2 ? r1 : r1 * s;
                s_rch[1][cd] = p2 ? r2 * s : r2;
                s_rch[2][cd] = rc;
            }
        }
        for (int32_t ci = pk.clo[d] + tid; ci < pk.clo[d + 1]; ci += T) {
            const int4 r = s_ch[ci];
            const int dd = r.x & 0xffff;
            const float r1 = s_rch[0][dd], r2 = s_rch[1][dd], rc = s_rch[2][dd];
#pragma unroll 4
            for (int32_t c = r.z; c < r.z + r.y; ++c) {
                const float p = s_kp[c];
                if (!signbit(p)) continue;
                const int cd = s_kw[c];
                s_rch[0][cd] = r1;
                s_rch[1][cd] = r2;
                s_rch[2][cd] = rc * fabsf(p);
            }
        }
        __syncthreads();
    }
    if (mode == 1) {
        // the reach of the nodes with external children, for the lower tiers' roots
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (tid + j * T >= n_mem || !((rec[j][0] >> 20) & 1)) continue;
            const int dd = rec[j][0] & 0xffff;
            const int32_t x = B[pk.off_node + dd];
            a.reach[x] = s_rch[0][dd];
            a.reach[N + x] = s_rch[1][dd];
            a.reach[2 * N + x] = s_rch[2][dd];
        }
        for (int32_t ci = tid; ci < pk.n_ch; ci += T) {
            const int32_t w0 = s_ch[ci].x;
            if (!((w0 >> 20) & 1)) continue;
            const int dd = w0 & 0xffff;
            const int32_t x = B[pk.off_node + dd];
            a.reach[x] = s_rch[0][dd];
            a.reach[N + x] = s_rch[1][dd];
            a.reach[2 * N + x] = s_rch[2][dd];
        }
        return;
    }

    // bottom-up values, deepest level first: chance nodes, then members
    const float t = s_t;
    for (int32_t d = nlv - 1; d >= 0; --d) {
        for (int32_t ci = pk.clo[d] + tid; ci < pk.clo[d + 1]; ci += T) {
            const int4 r = s_ch[ci];
            float v = 0.0f;
#pragma unroll 4
            for (int32_t c = r.z; c < r.z + r.y; ++c) {
                const float p = s_kp[c];
                v = fmaf(fabsf(p), signbit(p) ? s_val[s_kw[c]] : as_float(s_kw[c]), v);
            }
            s_val[r.x & 0xffff] = v;
        }
        // the level's members: values, and their regret contributions and own reach into the
        // member's slot (slot = member index in the pack)
        const int32_t m0 = pk.mlo[d], m1 = pk.mlo[d + 1];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int32_t m = tid + j * T;
            if (m < m0 || m >= m1) continue;
            const int32_t w0 = rec[j][0];
            const int dd = w0 & 0xffff, k = (w0 >> 16) & 7;
            float w[4], v = 0.0f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                w[c] = 0.0f;
                if (c >= k) continue;
                const int kind = (w0 >> (24 + 2 * c)) & 3;
                w[c] = kind == 0 ? s_val[rec[j][2 + c]] : as_float(rec[j][2 + c]);
                v = fmaf(s_sig[rec[j][1] + c], w[c], v);
            }
            s_val[dd] = v;
            const bool p2 = (w0 >> 19) & 1;
            const float cf = (p2 ? s_rch[0][dd] : s_rch[1][dd]) * s_rch[2][dd];
#pragma unroll
            for (int c = 0; c < 4; ++c) s_con[m][c] = cf * (w[c] - v);
            s_own[m] = p2 ? s_rch[1][dd] : s_rch[0][dd];
        }
        __syncthreads();
    }
    // every infoset of the pack at once (their updates read only their own members' slots and
    // pairs, which no value below needs any more): sums in member order, then the update; the
    // updated pairs stay in LDS until the end, so no barrier waits on stores
#pragma unroll
    for (int j = 0; j < S; ++j) {
        if (tid + j * T >= n_inf) continue;
        const int4 r = inf[j];
        const int32_t k = r.w & 255;
        const int player = (r.w >> 8) & 3;
        float pr[4], ps[4], pp[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            pr[c] = ps[c] = pp[c] = 0.0f;
            if (c < k) {
                pr[c] = s_R[r.y + c];
                ps[c] = s_S[r.y + c];
                pp[c] = s_sig[r.y + c];
            }
        }
        update_infoset<4>(a, s_R + r.y, s_S + r.y, s_sig + r.y, k, player, r.z & 0xffff,
                          r.z >> 16, pr, ps, pp, s_con, s_own, t);
    }
    __syncthreads();
    // the updated pairs; the roots' values for the parents' bottom-up; every decision node's
    // value and reach when they are kept for inspection
#pragma unroll
    for (int j = 0; j < S; ++j) {
        if (tid + j * T >= n_inf) continue;
        const int4 r = inf[j];
        const int k = r.w & 255;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= k) continue;
            a.R[r.x + c] = s_R[r.y + c];
            a.S[r.x + c] = s_S[r.y + c];
            a.prob[r.x + c] = s_sig[r.y + c];
        }
    }
#pragma unroll
    for (int u = 0; u < RU; ++u)
        if (tid + u * T < n_root) a.value[root[u].w] = s_val[root[u].x & 0xffff];
    if (pa.keep)
        for (int32_t dd = tid; dd < pk.n_dec; dd += T) {
            const int32_t x = B[pk.off_node + dd];
            a.value[x] = s_val[dd];
            a.reach[x] = s_rch[0][dd];
            a.reach[N + x] = s_rch[1][dd];
            a.reach[2 * N + x] = s_rch[2][dd];
        }
    // the launch's last workgroup counts the iteration: every workgroup read T at its start
    if (pa.count && tid == 0) {
        __threadfence();
        if (atomicAdd(pa.done, 1u) == gridDim.x - 1) {
            *a.T += 1;
            *pa.done = 0;
        }
    }
}

__global__ void k_x_reset_nodes(int64_t N, int32_t n_roots, const int8_t* __restrict__ meta,
                                const float* __restrict__ payoff, float* __restrict__ value,
                                float* __restrict__ reach) {
    const int64_t x = gid();
    if (x >= N) return;
    value[x] = (meta[x] & 3) == 0 ? payoff[x] : 0.0f;
    if (x < n_roots) {
        reach[x] = 1.0f;
        reach[N + x] = 1.0f;
        reach[2 * N + x] = 1.0f;
    }
}

// ---- best response over the plan (Section 2.2), both players in one sweep
//
// Planes: br_reach[p N + x] = pi_{-i}(x) for i = p + 1 (chance and the other player's average
// strategy); br_value[p N + x] = the value of x to player i when i best responds. Terminal
// entries of br_value (+u_1, -u_1) and the roots' reach are written when the solver is built
// and never again.

__global__ void k_x_br_setup(int64_t N, int32_t n_roots, const int8_t* __restrict__ meta,
                             const float* __restrict__ payoff, float* __restrict__ br_value,
                             float* __restrict__ br_reach) {
    const int64_t x = gid();
    if (x >= N) return;
    if ((meta[x] & 3) == 0) {
        br_value[x] = payoff[x];
        br_value[N + x] = -payoff[x];
    }
    if (x < n_roots) {
        br_reach[x] = 1.0f;
        br_reach[N + x] = 1.0f;
    }
}

// pi_{-1} takes chance and player-2 edges, pi_{-2} chance and player-1 edges (sigma-bar).
__global__ void k_x_br_reach(int32_t lo, int32_t hi, int64_t N, const int32_t* __restrict__ parent,
                             const int32_t* __restrict__ edge, const int8_t* __restrict__ meta,
                             const float* __restrict__ avgprob, float* __restrict__ br_reach) {
    constexpr int NPT = 2;
    const int64_t first = lo + static_cast<int64_t>(blockIdx.x) * blockDim.x * NPT + threadIdx.x;
    int64_t xs[NPT];
    int kind[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        xs[u] = first + u * static_cast<int64_t>(blockDim.x);
        kind[u] = xs[u] < hi ? meta[xs[u]] : 0;
    }
    int32_t p[NPT], e[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        p[u] = e[u] = 0;
        if (kind[u] & 3) {
            p[u] = parent[xs[u]];
            e[u] = edge[xs[u]];
        }
    }
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        if ((kind[u] & 3) == 0) continue;
        const int actor = kind[u] >> 2;  // 1 chance, 2 player 1, 3 player 2
        const float s = avgprob[e[u]];
        float r0 = br_reach[p[u]], r1 = br_reach[N + p[u]];
        if (actor != 2) r0 *= s;  // chance or player 2 moved: pi_{-1}
        if (actor != 3) r1 *= s;  // chance or player 1 moved: pi_{-2}
        br_reach[xs[u]] = r0;
        br_reach[N + xs[u]] = r1;
    }
}

struct BrArgs {
    int64_t N;
    const int32_t* chunk_first;
    const int32_t* chunk_m;
    const int4* mem_rec;
    const int8_t* mem_kp;
    const int4* set_rec;
    const int32_t* child_begin;
    const int32_t* child_stride;
    const int32_t* child_list;
    const int32_t* chance_nodes;
    const int32_t* chance_base;
    const int32_t* chance_k;
    const float* avgprob;
    const float* br_reach;
    float* br_value;
    int32_t kp_packed;  // member records carry the k | player byte (XDev::kp_packed)
};

// One level. Chunks (one thread per member): the acting player i's plane takes, per infoset,
// a* = argmax_a sum_m pi_{-i}(m) V_i(child(m, a)) (member order, lowest index on ties) and
// V_i(m) = V_i(child(m, a*)); the other player's plane takes the expectation under sigma-bar.
// Chance nodes (groups of 2^glog lanes) take expectations in both planes.
template <int KMAX, int CH>
__global__ void __launch_bounds__(CH) k_x_br_level(BrArgs a, int32_t klo, int32_t nk, int32_t clo,
                                                   int32_t nc, int glog) {
    __shared__ float s_con[CH][KMAX];
    __shared__ int32_t s_sel[CH];
    const int tid = threadIdx.x;
    const int64_t N = a.N;
    if (static_cast<int32_t>(blockIdx.x) >= nk) {
        const int32_t i = (blockIdx.x - nk) * (CH >> glog) + (tid >> glog);
        const int lane = tid & ((1 << glog) - 1);
        const bool ok = i < nc;
        float v0 = 0.0f, v1 = 0.0f;
        int32_t x = 0;
        if (ok) {
            x = a.chance_nodes[clo + i];
            const int32_t base = a.chance_base[clo + i], k = a.chance_k[clo + i];
            const int32_t cb = a.child_begin[x], st = a.child_stride[x];
            for (int32_t c = lane; c < k; c += 1 << glog) {
                const int32_t ch = st != 0 ? cb + c * st : a.child_list[cb + c];
                const float pr = a.avgprob[base + c];
                v0 = fmaf(pr, a.br_value[ch], v0);
                v1 = fmaf(pr, a.br_value[N + ch], v1);
            }
        }
        for (int off = (1 << glog) >> 1; off > 0; off >>= 1) {
            v0 += __shfl_xor(v0, off, 64);
            v1 += __shfl_xor(v1, off, 64);
        }
        if (ok && lane == 0) {
            a.br_value[x] = v0;
            a.br_value[N + x] = v1;
        }
        return;
    }
    const int32_t c = klo + blockIdx.x;
    const int32_t h0 = a.chunk_first[c], h1 = a.chunk_first[c + 1];
    const int32_t m0 = a.chunk_m[c], m1 = a.chunk_m[c + 1];
    const int32_t nm = m1 - m0;
    const bool big = nm > CH;
    float wr[KMAX];
    int32_t x = 0, resp = 0;
    if (!big) {
        const bool ok = tid < nm;
        float con[KMAX];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) wr[j] = con[j] = 0.0f;
        if (ok) {
            const int32_t m = m0 + tid;
            const int4 r = a.mem_rec[m];
            x = r.x;
            const int32_t q = r.y, cb = r.z, st = rec_stride(r.w, a.kp_packed);
            const int kp = rec_kp(r.w, a.kp_packed, a.mem_kp, m);
            const int k = kp & 31;
            resp = (kp & 64) ? 1 : 0;
            const float pr = a.br_reach[resp * N + x];
            float vo = 0.0f;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < k) {
                    const int32_t ch = st != 0 ? cb + j * st : a.child_list[cb + j];
                    wr[j] = a.br_value[resp * N + ch];
                    vo = fmaf(a.avgprob[q + j], a.br_value[(1 - resp) * N + ch], vo);
                    con[j] = pr * wr[j];
                }
            }
            a.br_value[(1 - resp) * N + x] = vo;
        }
#pragma unroll
        for (int j = 0; j < KMAX; ++j) s_con[tid][j] = con[j];
    } else {
        float con[KMAX];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) con[j] = 0.0f;
        for (int32_t mi = tid; mi < nm; mi += CH) {
            const int32_t m = m0 + mi;
            const int4 r = a.mem_rec[m];
            const int32_t xm = r.x, q = r.y, cb = r.z, st = rec_stride(r.w, a.kp_packed);
            const int kp = rec_kp(r.w, a.kp_packed, a.mem_kp, m);
            const int k = kp & 31;
            const int rp = (kp & 64) ? 1 : 0;
            const float pr = a.br_reach[rp * N + xm];
            float vo = 0.0f;
#pragma unroll
            for (int j = 0; j < KMAX; ++j) {
                if (j < k) {
                    const int32_t ch = st != 0 ? cb + j * st : a.child_list[cb + j];
                    con[j] = fmaf(pr, a.br_value[rp * N + ch], con[j]);
                    vo = fmaf(a.avgprob[q + j], a.br_value[(1 - rp) * N + ch], vo);
                }
            }
            a.br_value[(1 - rp) * N + xm] = vo;
        }
#pragma unroll
        for (int j = 0; j < KMAX; ++j) s_con[tid][j] = con[j];
    }
    __syncthreads();
    if (tid < h1 - h0) {
        const int4 hr = a.set_rec[h0 + tid];
        const int32_t slo = big ? 0 : hr.y - m0;
        const int32_t shi = big ? (nm < CH ? nm : CH) : hr.z - m0;
        const int k = hr.w & 31;
        float tot[KMAX];
#pragma unroll
        for (int j = 0; j < KMAX; ++j) tot[j] = 0.0f;
        for (int32_t sl = slo; sl < shi; ++sl) {
#pragma unroll
            for (int j = 0; j < KMAX; ++j) tot[j] += s_con[sl][j];
        }
        int32_t best = 0;
        float best_v = tot[0];
#pragma unroll
        for (int j = 1; j < KMAX; ++j) {
            if (j < k && tot[j] > best_v) {
                best_v = tot[j];
                best = j;
            }
        }
        if (big) s_sel[0] = best;
        else
            for (int32_t sl = slo; sl < shi; ++sl) s_sel[sl] = best;
    }
    __syncthreads();
    if (!big) {
        if (tid < nm) {
            const int32_t b = s_sel[tid];
            float v = wr[0];
#pragma unroll
            for (int j = 1; j < KMAX; ++j)
                if (j == b) v = wr[j];
            a.br_value[resp * N + x] = v;
        }
    } else {
        const int32_t b = s_sel[0];
        for (int32_t mi = tid; mi < nm; mi += CH) {
            const int32_t m = m0 + mi;
            const int4 r = a.mem_rec[m];
            const int32_t xm = r.x, cb = r.z, st = rec_stride(r.w, a.kp_packed);
            const int rp = (rec_kp(r.w, a.kp_packed, a.mem_kp, m) & 64) ? 1 : 0;
            const int32_t ch = st != 0 ? cb + b * st : a.child_list[cb + b];
            a.br_value[rp * N + xm] = a.br_value[rp * N + ch];
        }
    }
}

__global__ void k_x_tick(int64_t* T) {
    if (gid() == 0) *T += 1;
}

// Best-response values of every root (level 0, in game order): out[2 g + p] = plane p.
__global__ void k_x_store_roots(int32_t n_roots, int64_t N, const float* __restrict__ br_value,
                                double* out) {
    const int64_t g = gid();
    if (g >= n_roots) return;
    out[2 * g] = static_cast<double>(br_value[g]);
    out[2 * g + 1] = static_cast<double>(br_value[N + g]);
}

__global__ void k_x_permute_values(int64_t N, const int32_t* __restrict__ canon_of,
                                   const float* __restrict__ src, float* __restrict__ dst) {
    const int64_t x = gid();
    if (x < N) dst[canon_of[x]] = src[x];
}

}  // namespace

int shape_bucket(int64_t units) {
    int b = 0;
    while (b + 1 < kShapeBuckets && (int64_t{1} << (b + 1)) <= units) ++b;
    return b;
}

const char* xkernel_kind_name(int kind) {
    switch (kind) {
        case XK_REACH: return "block_reach";
        case XK_UP: return "block_up";
        case XK_SUBTREE: return "block_subtree";
        default: return "";
    }
}

__global__ void k_x_zero_u32(uint32_t* p) {
    if (gid() == 0) *p = 0;
}

void launch_x_reset(const XDev& x, hipStream_t st) {
    hipLaunchKernelGGL(k_x_zero_u32, dim3(1), dim3(64), 0, st, x.pack_done);
    hipLaunchKernelGGL(k_x_reset_nodes, dim3(blocks_for(x.N)), dim3(kBlock), 0, st, x.N,
                       x.level_offset_host[1], x.meta, x.payoff, x.value, x.reach);
    hipLaunchKernelGGL(k_x_br_setup, dim3(blocks_for(x.N)), dim3(kBlock), 0, st, x.N,
                       x.level_offset_host[1], x.meta, x.payoff, x.br_value, x.br_reach);
    // the chance plane of every upper node, level by level (constant from here on)
    for (int32_t l = 1; l < x.D; ++l) {
        const int32_t lo = x.level_offset_host[l], hi = x.up_end_host[l];
        if (hi <= lo) continue;
        const unsigned grid = std::min<unsigned>(blocks_for(hi - lo), 4096u);
        hipLaunchKernelGGL(k_x_reach_full, dim3(grid), dim3(kBlock), 0, st, lo, hi, x.N, x.parent,
                           x.edge, x.meta, x.prob, x.reach);
    }
}

namespace {

UpArgs up_args(const XDev& x, const UpdateRule& rule) {
    UpArgs a;
    a.N = x.N;
    a.chunk_first = x.chunk_first;
    a.chunk_m = x.chunk_m;
    a.child_begin = x.child_begin;
    a.child_stride = x.child_stride;
    a.child_list = x.child_list;
    a.mem_rec = x.mem_rec;
    a.mem_kp = x.mem_kp;
    a.set_rec = x.set_rec;
    a.chance_nodes = x.chance_nodes;
    a.chance_base = x.chance_base;
    a.chance_k = x.chance_k;
    a.prob = x.prob;
    a.value = x.value;
    a.reach = x.reach;
    a.R = x.R;
    a.S = x.S;
    a.T = x.T;
    a.rule = rule;
    a.derive_reach = 0;
    a.kp_packed = x.kp_packed;
    a.parent = x.parent;
    a.edge = x.edge;
    a.meta = x.meta;
    return a;
}

template <int KMAX, int CH, int MPT>
void launch_up_level(const XDev& x, const UpArgs& a, int32_t l, hipStream_t st) {
    // the level's chunks and chance nodes outside the subtree packs
    const int32_t klo = x.k_level_offset_host[l], nk = x.k_up_end_host[l] - klo;
    const int32_t clo = x.c_level_offset_host[l], nc = x.c_up_end_host[l] - clo;
    const int glog = x.chance_glog_host[l];
    const int32_t per = CH >> glog;
    const int32_t grid = nk + (nc + per - 1) / per;
    if (grid == 0) return;
    hipLaunchKernelGGL((k_x_up_level<KMAX, CH, MPT>), dim3(grid), dim3(CH), 0, st, a, klo, nk, clo,
                       nc, glog);
}

template <int KMAX, int MPT>
void launch_up_threads(const XDev& x, const UpArgs& a, int32_t l, hipStream_t st) {
    switch (x.up_threads_host[l]) {
        case 64: launch_up_level<KMAX, 64, MPT>(x, a, l, st); break;
        case 128: launch_up_level<KMAX, 128, MPT>(x, a, l, st); break;
        case 512: launch_up_level<KMAX, 512, MPT>(x, a, l, st); break;
        default: launch_up_level<KMAX, 256, MPT>(x, a, l, st); break;
    }
}

template <int KMAX>
void launch_up(const XDev& x, const UpArgs& a, int32_t l, hipStream_t st) {
    if (x.chunk_cap_host[l] > x.up_threads_host[l]) launch_up_threads<KMAX, 2>(x, a, l, st);
    else launch_up_threads<KMAX, 1>(x, a, l, st);
}

void launch_reach_level(const XDev& x, int32_t l, hipStream_t st) {
    const int32_t t0 = x.t_level_offset_host[l], nt = x.t_level_offset_host[l + 1] - t0;
    if (nt == 0) return;
    const int64_t* ek = x.ek_packed ? x.parent_ek : nullptr;
    const int threads = x.reach_threads_host[l];
    if (ek != nullptr && x.reach_npt_host[l] == 2) {
        hipLaunchKernelGGL(k_x_reach_pairs<2>, dim3(nt), dim3(threads), 0, st, t0, x.N, x.tile_lo,
                           x.tile_hi, x.prob, x.reach, ek);
        return;
    }
    switch (x.reach_npt_host[l]) {
        case 2:
            hipLaunchKernelGGL(k_x_reach<2>, dim3(nt), dim3(threads), 0, st, t0, x.N, x.tile_lo,
                               x.tile_hi, x.parent, x.edge, x.meta, x.prob, x.reach, ek);
            break;
        case 4:
            hipLaunchKernelGGL(k_x_reach<4>, dim3(nt), dim3(threads), 0, st, t0, x.N, x.tile_lo,
                               x.tile_hi, x.parent, x.edge, x.meta, x.prob, x.reach, ek);
            break;
        default:
            hipLaunchKernelGGL(k_x_reach<1>, dim3(nt), dim3(threads), 0, st, t0, x.N, x.tile_lo,
                               x.tile_hi, x.parent, x.edge, x.meta, x.prob, x.reach, ek);
            break;
    }
}

}  // namespace

int32_t fusable_reach_levels(const int32_t* level_offset, const int32_t* up_end, int32_t D) {
    int32_t k = 0;
    while (1 + k < D && k < kFuseMax && up_end[k + 1] - level_offset[k + 1] <= 2 * kFuseThreads)
        ++k;
    return k;
}

int32_t path_reach_levels(const int64_t* units, int32_t fused, int32_t D, int32_t max_depth) {
    // levels fused + 1 .. l with at most kPathNodes decision nodes each and at most max_depth
    // (<= kPathDepth) levels below the last stored one
    const int32_t depth = max_depth < kPathDepth ? max_depth : kPathDepth;
    int32_t l = fused;
    while (l + 1 < D && l + 1 - fused <= depth && units[l + 1] <= kPathNodes) ++l;
    return l;
}

int32_t fusable_up_levels(const int32_t* m_level_offset, const int32_t* m_up_end,
                          const int32_t* h_level_offset, const int32_t* h_up_end,
                          const int32_t* c_level_offset, const int32_t* c_up_end,
                          const int32_t* chance_glog, int32_t D, int32_t max_actions) {
    if (max_actions > 4) return 0;
    int32_t k = 0;
    while (k <= D && k < kFuseMax && m_up_end[k] - m_level_offset[k] <= kFuseThreads &&
           h_up_end[k] - h_level_offset[k] <= kFuseThreads &&
           (static_cast<int64_t>(c_up_end[k] - c_level_offset[k]) << chance_glog[k]) <=
               kFuseThreads)
        ++k;
    return k;
}

namespace {

// Adds elements [lo, hi) of an array of elem-byte elements to a warm table (empty: skipped;
// clipped to kFuseThreads lines).
template <typename E>
void warm_add(WarmTable& w, int& n, const E* base, int64_t lo, int64_t hi) {
    if (hi <= lo || n == kWarmMax) return;
    const int64_t bytes = (hi - lo) * static_cast<int64_t>(sizeof(E));
    w.p[n] = reinterpret_cast<const uint8_t*>(base + lo);
    w.lines[n] = static_cast<int32_t>(std::min<int64_t>((bytes + kWarmLine - 1) / kWarmLine,
                                                        kFuseThreads));
    ++n;
}

void warm_fill(WarmTable& w, int n) {
    for (int r = n; r < kWarmMax; ++r) {
        w.p[r] = n > 0 ? w.p[0] : nullptr;
        w.lines[r] = n > 0 ? w.lines[0] : 0;
    }
}

// What k_x_reach_top reads: parent, edge and kind of levels 1 .. fr, the player reach planes of
// levels 0 .. fr - 1 and sigma at those levels' pairs.
WarmTable reach_warm(const XDev& x, int32_t fr) {
    WarmTable w{};
    int n = 0;
    const int32_t* lo = x.level_offset_host;
    warm_add(w, n, x.reach, lo[0], lo[fr]);
    warm_add(w, n, x.reach + x.N, lo[0], lo[fr]);
    warm_add(w, n, x.parent, lo[1], lo[1 + fr]);
    warm_add(w, n, x.edge, lo[1], lo[1 + fr]);
    warm_add(w, n, x.meta, lo[1], lo[1 + fr]);
    warm_add(w, n, x.prob, x.top_q_lo[0], x.top_q_hi[0]);
    warm_fill(w, n);
    return w;
}

// What k_x_up_top reads at levels 0 .. fu - 1: chunk, member and infoset records, chance
// tables, child offsets, the three reach planes, the children's values (one level deeper)
// and the infosets' regrets, average and sigma, and the chance probabilities.
WarmTable up_warm(const XDev& x, int32_t fu) {
    WarmTable w{};
    int n = 0;
    const int32_t* lo = x.level_offset_host;
    const int32_t l1 = std::min(fu + 1, x.D + 1);
    warm_add(w, n, x.value, lo[0], lo[l1]);
    warm_add(w, n, x.chunk_first, x.k_level_offset_host[0], x.k_level_offset_host[fu] + 1);
    warm_add(w, n, x.chunk_m, x.k_level_offset_host[0], x.k_level_offset_host[fu] + 1);
    warm_add(w, n, x.mem_rec, x.m_level_offset_host[0], x.m_level_offset_host[fu]);
    warm_add(w, n, x.mem_kp, x.m_level_offset_host[0], x.m_level_offset_host[fu]);
    warm_add(w, n, x.set_rec, x.h_level_offset_host[0], x.h_level_offset_host[fu]);
    warm_add(w, n, x.chance_nodes, x.c_level_offset_host[0], x.c_level_offset_host[fu]);
    warm_add(w, n, x.chance_base, x.c_level_offset_host[0], x.c_level_offset_host[fu]);
    warm_add(w, n, x.chance_k, x.c_level_offset_host[0], x.c_level_offset_host[fu]);
    warm_add(w, n, x.child_begin, lo[0], lo[fu]);
    warm_add(w, n, x.child_stride, lo[0], lo[fu]);
    warm_add(w, n, x.reach, lo[0], lo[fu]);
    warm_add(w, n, x.reach + x.N, lo[0], lo[fu]);
    warm_add(w, n, x.reach + 2 * x.N, lo[0], lo[fu]);
    warm_add(w, n, x.R, x.top_q_lo[1], x.top_q_hi[1]);
    warm_add(w, n, x.S, x.top_q_lo[1], x.top_q_hi[1]);
    warm_add(w, n, x.prob, x.top_q_lo[1], x.top_q_hi[1]);
    warm_add(w, n, x.prob, x.top_c_lo[1], x.top_c_hi[1]);
    warm_fill(w, n);
    return w;
}

}  // namespace

int32_t derived_reach_level(const XDev& x) {
    // the deepest level with upper decision nodes, when their children are all terminal (no
    // pack starts below them), it has a launch of its own on both sweeps and no upper chance
    // nodes
    int32_t ld = x.D - 1;
    while (ld >= 1 && x.reach_units_host[ld] == 0) --ld;
    const int32_t top = x.path_reach > x.fused_reach ? x.path_reach : x.fused_reach;
    const bool ok = ld >= 1 + top && ld >= x.fused_up && x.only_terminal_children_host[ld] &&
                    x.c_up_end_host[ld] == x.c_level_offset_host[ld];
    return ok ? ld : -1;
}

void launch_x_iteration(const XDev& x, const UpdateRule& rule, hipStream_t st, LaunchTimer* timer) {
    auto pre = [&](int k, int l, int64_t n) { if (timer) timer->before(k, l, n, st); };
    auto post = [&](int k) { if (timer) timer->after(k, st); };
    const int32_t* lo = x.level_offset_host;
    // top-down: the first small levels in one workgroup, then a launch per level
    const int32_t fr = x.fused_reach;
    if (fr > 0) {
        LevelTable t{};
        t.n = fr;
        int64_t units = 0;
        for (int32_t i = 0; i < fr; ++i) {  // entry i is level 1 + i, its upper prefix
            t.lo[i] = lo[1 + i];
            t.hi[i] = x.up_end_host[1 + i];
            units += x.reach_units_host[1 + i];
        }
        if (units > 0) {
            pre(XK_REACH, -1, units);
            hipLaunchKernelGGL(k_x_reach_top, dim3(1), dim3(kFuseThreads), 0, st, t,
                               reach_warm(x, fr), x.N, x.parent, x.edge, x.meta, x.prob, x.reach);
            post(XK_REACH);
        }
    }
    const int32_t fp = x.path_reach;
    if (fp > fr) {
        const int32_t t0 = x.t_level_offset_host[1 + fr], nt = x.t_level_offset_host[fp + 1] - t0;
        if (nt > 0) {
            int64_t units = 0;
            for (int32_t l = 1 + fr; l <= fp; ++l) units += x.reach_units_host[l];
            pre(XK_REACH, -2, units);
            hipLaunchKernelGGL(k_x_reach_path, dim3(nt), dim3(kPathThreads), 0, st, t0, lo[1 + fr],
                               x.N, x.tile_lo, x.tile_hi, x.parent, x.edge, x.meta, x.prob, x.reach);
            post(XK_REACH);
        }
    }
    const int32_t ld = derived_reach_level(x);
    const bool derive = ld >= 0;
    for (int32_t l = 1 + (fp > fr ? fp : fr); l < x.D; ++l) {
        if (x.t_level_offset_host[l + 1] == x.t_level_offset_host[l]) continue;
        if (derive && l == ld) continue;
        pre(XK_REACH, l, x.reach_units_host[l]);
        launch_reach_level(x, l, st);
        post(XK_REACH);
    }
    const UpArgs a = up_args(x, rule);
    // the subtree packs, tier by tier: top-down from the highest tier, tier 1 through both
    // sweeps, bottom-up from tier 2 (one workgroup per pack)
    // with no upper level to finish bottom-up, the last pack launch counts the iteration
    const bool pack_counts = rule.count && !x.upper_bottom_up && x.n_tiers >= 1;
    auto pack_launch = [&](int32_t t, int mode, bool count) {
        const int32_t p0 = x.tier_offset_host[t - 1], np = x.tier_offset_host[t] - p0;
        PackArgs pa{x.packs, x.pack_blob, p0, mode, x.keep_nodes, count ? 1 : 0, x.pack_done};
        pre(XK_SUBTREE, -10 * mode - t, x.tier_dec_host[t - 1]);
        hipLaunchKernelGGL(k_x_pack<kPackThreads>, dim3(np), dim3(kPackThreads), 0, st, a, pa);
        post(XK_SUBTREE);
    };
    for (int32_t t = x.n_tiers; t >= 2; --t) pack_launch(t, 1, false);
    if (x.n_tiers >= 1) pack_launch(1, 0, pack_counts && x.n_tiers == 1);
    for (int32_t t = 2; t <= x.n_tiers; ++t) pack_launch(t, 2, pack_counts && t == x.n_tiers);
    // bottom-up: a launch per deep level, then the shallow levels in one workgroup (upper
    // prefixes only)
    UpArgs ad = a;
    ad.derive_reach = 1;
    const int32_t fu = x.fused_up;
    for (int32_t l = x.D; l >= fu; --l) {
        const int32_t nunits = x.h_up_end_host[l] - x.h_level_offset_host[l] +
                               x.c_up_end_host[l] - x.c_level_offset_host[l];
        if (nunits == 0) continue;
        const UpArgs& al = derive && l == ld ? ad : a;
        pre(XK_UP, l, x.m_level_offset_host[l + 1] - x.m_level_offset_host[l]);
        if (x.max_actions <= 4) launch_up<4>(x, al, l, st);
        else launch_up<16>(x, al, l, st);
        post(XK_UP);
    }
    if (fu > 0) {
        LevelTable t{};
        t.n = fu;
        for (int32_t i = 0; i < fu; ++i) {  // entry i is level fu - 1 - i
            const int32_t l = fu - 1 - i;
            t.lo[i] = x.k_level_offset_host[l];
            t.hi[i] = x.k_up_end_host[l];
            t.clo[i] = x.c_level_offset_host[l];
            t.chi[i] = x.c_up_end_host[l];
            t.glog[i] = x.chance_glog_host[l];
        }
        pre(XK_UP, -1, x.m_level_offset_host[fu] - x.m_level_offset_host[0]);
        hipLaunchKernelGGL(k_x_up_top, dim3(1), dim3(kFuseThreads), 0, st, a, t, up_warm(x, fu));
        post(XK_UP);
    } else if (rule.count && !pack_counts) {
        // the linear-averaging weight of every launch above read T: count the iteration last
        hipLaunchKernelGGL(k_x_tick, dim3(1), dim3(64), 0, st, x.T);
    }
}

namespace {

template <int KMAX, int CH>
void launch_br_level(const XDev& x, const BrArgs& a, int32_t l, hipStream_t st) {
    const int32_t klo = x.k_level_offset_host[l], nk = x.k_level_offset_host[l + 1] - klo;
    const int32_t clo = x.c_level_offset_host[l], nc = x.c_level_offset_host[l + 1] - clo;
    const int glog = x.chance_glog_host[l];
    const int32_t per = CH >> glog;
    const int32_t grid = nk + (nc + per - 1) / per;
    if (grid == 0) return;
    hipLaunchKernelGGL((k_x_br_level<KMAX, CH>), dim3(grid), dim3(CH), 0, st, a, klo, nk, clo, nc,
                       glog);
}

template <int KMAX>
void launch_br_cap(const XDev& x, const BrArgs& a, int32_t l, hipStream_t st) {
    switch (x.chunk_cap_host[l]) {  // one thread per member of a chunk
        case 64: launch_br_level<KMAX, 64>(x, a, l, st); break;
        case 128: launch_br_level<KMAX, 128>(x, a, l, st); break;
        case 256: launch_br_level<KMAX, 256>(x, a, l, st); break;
        case 512: launch_br_level<KMAX, 512>(x, a, l, st); break;
        default: launch_br_level<KMAX, 1024>(x, a, l, st); break;
    }
}

}  // namespace

void launch_x_best_response(const XDev& x, const float* avgprob, hipStream_t st) {
    const int32_t* lo = x.level_offset_host;
    for (int32_t l = 1; l < x.D; ++l)
        hipLaunchKernelGGL(k_x_br_reach, dim3(blocks_of(lo[l + 1] - lo[l], 2 * kBlock)), dim3(kBlock),
                           0, st, lo[l], lo[l + 1], x.N, x.parent, x.edge, x.meta, avgprob,
                           x.br_reach);
    BrArgs a;
    a.N = x.N;
    a.chunk_first = x.chunk_first;
    a.chunk_m = x.chunk_m;
    a.mem_rec = x.mem_rec;
    a.mem_kp = x.mem_kp;
    a.kp_packed = x.kp_packed;
    a.set_rec = x.set_rec;
    a.child_begin = x.child_begin;
    a.child_stride = x.child_stride;
    a.child_list = x.child_list;
    a.chance_nodes = x.chance_nodes;
    a.chance_base = x.chance_base;
    a.chance_k = x.chance_k;
    a.avgprob = avgprob;
    a.br_reach = x.br_reach;
    a.br_value = x.br_value;
    for (int32_t l = x.D; l >= 0; --l) {
        if (x.max_actions <= 4) launch_br_cap<4>(x, a, l, st);
        else launch_br_cap<16>(x, a, l, st);
    }
    const int32_t n_roots = lo[1];
    hipLaunchKernelGGL(k_x_store_roots, dim3(blocks_for(n_roots)), dim3(kBlock), 0, st, n_roots, x.N,
                       x.br_value, x.out2);
}

void launch_x_values_to_canonical(const XDev& x, float* dst, hipStream_t st) {
    hipLaunchKernelGGL(k_x_permute_values, dim3(blocks_for(x.N)), dim3(kBlock), 0, st, x.N,
                       x.canon_of, x.value, dst);
}

void launch_x_reach_to_canonical(const XDev& x, float* dst, hipStream_t st) {
    for (int k = 0; k < 3; ++k)
        hipLaunchKernelGGL(k_x_permute_values, dim3(blocks_for(x.N)), dim3(kBlock), 0, st, x.N,
                           x.canon_of, x.reach + k * x.N, dst + k * x.N);
}

}  // namespace cfr
