// gfx950 kernels over the public-block execution plan (xplan.hpp).
//
// An iteration (Section 3.2) is one top-down launch per level for the reach
// probabilities (Eq. excepted_reach_probabilities_matrix_recurrence and its own-reach
// twin) and one bottom-up launch per level that, per unit of work, finishes a whole
// infoset: its members' expected payoffs (Eq. expected_payoffs_matrix_recurrence), the
// instantaneous counterfactual regrets in their multiplied-out form (Eq.
// instantaneous_counterfactual_regret), the player reach of Eq. (player_reach_probability),
// and the cumulative regret / average / regret-matching update (Eqs.
// average_counterfactual_regrets_vector, average_strategy_profile_vector,
// next_strategy_profile). All members of an infoset sit in one public block, so the unit
// reads a compact, coalesced slice; nothing is accumulated with atomics and the result
// does not depend on scheduling. Chance nodes are units of their own.
#include <hip/hip_runtime.h>

#include "xkernels.hpp"

namespace cfr {

namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

inline int pick(const int32_t* table, int64_t units) {
    return table != nullptr ? table[shape_bucket(units)] : kBlock;
}

inline unsigned blocks_of(int64_t n, int threads) {
    return static_cast<unsigned>((n + threads - 1) / threads);
}

__device__ __forceinline__ int64_t gid() {
    return static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ int32_t child_of(const int32_t* __restrict__ child_begin,
                                            const int32_t* __restrict__ child_stride,
                                            const int32_t* __restrict__ child_list, int32_t x,
                                            int32_t a) {
    const int32_t st = child_stride[x];
    const int32_t cb = child_begin[x];
    return st != 0 ? cb + a * st : child_list[cb + a];
}

// Reach of one level: the factor of whoever acted into the node (meta bits 2-3) is
// multiplied by the edge probability (sigma or sigma_0).
__global__ void k_x_reach(int32_t lo, int32_t hi, int64_t N, const int32_t* __restrict__ parent,
                          const int32_t* __restrict__ edge, const int8_t* __restrict__ meta,
                          const float* __restrict__ prob, float* __restrict__ reach) {
    const int64_t x = lo + gid();
    if (x >= hi) return;
    const int m = meta[x];
    if ((m & 3) == 0) return;  // terminal: no reach needed
    const int actor = m >> 2;  // 1 chance, 2 player 1, 3 player 2
    const int32_t p = parent[x];
    const float s = prob[edge[x]];
    float r1 = reach[p], r2 = reach[N + p], rc = reach[2 * N + p];
    if (actor == 2) r1 *= s;
    else if (actor == 3) r2 *= s;
    else rc *= s;
    reach[x] = r1;
    reach[N + x] = r2;
    reach[2 * N + x] = rc;
}

// Bottom-up of one level, member-parallel. Workgroup b < n_chunks takes chunk b: whole
// infosets with at most CH members in total, one thread per member (or one infoset with more
// members, each thread striding over them). Phase 1: each member's child values (gather by
// stride), its value, its regret contributions cf * (w_a - v) and own reach, into LDS.
// Phase 2: one thread per infoset sums its members' slots in member order (deterministic)
// and applies the regret update, the average-strategy update and regret matching.
// Workgroups past the chunks take the level's chance nodes, one thread each.
template <int KMAX, int CH>
__global__ void __launch_bounds__(CH) k_x_up_chunk(
    int32_t chunk_lo, int32_t n_chunks, int32_t clo, int32_t nc, int64_t N,
    const int32_t* __restrict__ chunk_first, const int32_t* __restrict__ child_begin,
    const int32_t* __restrict__ child_stride, const int32_t* __restrict__ child_list,
    const int32_t* __restrict__ q_offset, const int8_t* __restrict__ iplayer,
    const int32_t* __restrict__ member_offset, const int32_t* __restrict__ members,
    const int32_t* __restrict__ chance_nodes, const int32_t* __restrict__ chance_base,
    const int32_t* __restrict__ chance_k, float* __restrict__ prob, float* __restrict__ value,
    const float* __restrict__ reach, float* __restrict__ R, float* __restrict__ S,
    const int64_t* __restrict__ T, int variant, int linear) {
    __shared__ float s_con[CH][KMAX];
    __shared__ float s_own[CH];
    __shared__ int32_t s_owner[CH];
    const int tid = threadIdx.x;
    const int32_t b = blockIdx.x;
    if (b >= n_chunks) {
        const int64_t i = static_cast<int64_t>(b - n_chunks) * CH + tid;
        if (i >= nc) return;
        const int32_t ci = clo + static_cast<int32_t>(i);
        const int32_t x = chance_nodes[ci];
        const int32_t base = chance_base[ci], k = chance_k[ci];
        float v = 0.0f;
        for (int32_t a = 0; a < k; ++a)
            v = fmaf(prob[base + a], value[child_of(child_begin, child_stride, child_list, x, a)], v);
        value[x] = v;
        return;
    }
    const int32_t c = chunk_lo + b;
    const int32_t h0 = chunk_first[c], h1 = chunk_first[c + 1];
    const int32_t m0 = member_offset[h0], m1 = member_offset[h1];
    const int32_t nm = m1 - m0;
    const bool big = nm > CH;
    if (!big) {
        for (int32_t i = tid; i < h1 - h0; i += CH)
            for (int32_t m = member_offset[h0 + i]; m < member_offset[h0 + i + 1]; ++m)
                s_owner[m - m0] = i;
        __syncthreads();
    }
    // phase 1
    {
        float con[KMAX];
        float own = 0.0f;
#pragma unroll
        for (int a = 0; a < KMAX; ++a) con[a] = 0.0f;
        for (int32_t mi = tid; mi < nm; mi += CH) {
            const int32_t h = big ? h0 : h0 + s_owner[mi];
            const int player = iplayer[h];
            const int32_t o = q_offset[h];
            const int32_t k = q_offset[h + 1] - o;
            const int32_t x = members[m0 + mi];
            const int32_t st = child_stride[x];
            const int32_t cb = child_begin[x];
            float w[KMAX], sg[KMAX];
            float v = 0.0f;
#pragma unroll
            for (int a = 0; a < KMAX; ++a) {
                if (a < k) {
                    const int32_t ch = st != 0 ? cb + a * st : child_list[cb + a];
                    w[a] = value[ch];
                    sg[a] = prob[o + a];
                    v = fmaf(sg[a], w[a], v);
                } else {
                    w[a] = 0.0f;
                    sg[a] = 0.0f;
                }
            }
            value[x] = v;
            const float r1 = reach[x], r2 = reach[N + x], rc = reach[2 * N + x];
            const float cf = (player == 1 ? r2 : r1) * rc;
            own += player == 1 ? r1 : r2;
#pragma unroll
            for (int a = 0; a < KMAX; ++a)
                if (a < k) con[a] = fmaf(cf, w[a] - v, con[a]);
        }
#pragma unroll
        for (int a = 0; a < KMAX; ++a) s_con[tid][a] = con[a];
        s_own[tid] = own;
    }
    __syncthreads();
    // phase 2
    const int32_t nh = h1 - h0;
    if (tid >= nh) return;
    const int32_t h = h0 + tid;
    const int32_t slo = big ? 0 : member_offset[h] - m0;
    const int32_t shi = big ? (nm < CH ? nm : CH) : member_offset[h + 1] - m0;
    const int player = iplayer[h];
    const int32_t o = q_offset[h];
    const int32_t k = q_offset[h + 1] - o;
    float racc[KMAX];
#pragma unroll
    for (int a = 0; a < KMAX; ++a) racc[a] = 0.0f;
    float own = 0.0f;
    for (int32_t sl = slo; sl < shi; ++sl) {
#pragma unroll
        for (int a = 0; a < KMAX; ++a) racc[a] += s_con[sl][a];
        own += s_own[sl];
    }
    const float sgn = player == 1 ? 1.0f : -1.0f;
    const float wt = linear ? static_cast<float>(*T + 1) : 1.0f;
    float pos_sum = 0.0f;
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
        if (a < k) {
            const float sig = prob[o + a];
            float r = fmaf(sgn, racc[a], R[o + a]);
            if (variant == 1) r = fmaxf(r, 0.0f);
            R[o + a] = r;
            S[o + a] = fmaf(wt * own, sig, S[o + a]);
            racc[a] = r;
            pos_sum += fmaxf(r, 0.0f);
        }
    }
    if (pos_sum > 0.0f) {
#pragma unroll
        for (int a = 0; a < KMAX; ++a)
            if (a < k) prob[o + a] = fmaxf(racc[a], 0.0f) / pos_sum;
    } else {
        const float unif = 1.0f / static_cast<float>(k);
#pragma unroll
        for (int a = 0; a < KMAX; ++a)
            if (a < k) prob[o + a] = unif;
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

// ---- best response over the plan (Section 2.2)

__global__ void k_x_br_init(int64_t N, int32_t n_roots, const int8_t* __restrict__ meta,
                            const float* __restrict__ payoff, float sgn,
                            float* __restrict__ br_value, float* __restrict__ br_reach) {
    const int64_t x = gid();
    if (x >= N) return;
    br_value[x] = (meta[x] & 3) == 0 ? sgn * payoff[x] : 0.0f;
    if (x < n_roots) br_reach[x] = 1.0f;
}

// pi_{-i}: chance and opponent edge probabilities only.
__global__ void k_x_br_reach(int32_t lo, int32_t hi, int player, const int32_t* __restrict__ parent,
                             const int32_t* __restrict__ edge, const int8_t* __restrict__ meta,
                             const float* __restrict__ avgprob, float* __restrict__ br_reach) {
    const int64_t x = lo + gid();
    if (x >= hi) return;
    const int m = meta[x];
    if ((m & 3) == 0) return;
    const int actor = (m >> 2) - 1;  // 0 chance, 1, 2
    const float f = actor == player ? 1.0f : avgprob[edge[x]];
    br_reach[x] = br_reach[parent[x]] * f;
}

// Responder's infosets: a* = argmax_a sum_m pi_{-i}(m) V(child(m, a)) (lowest index on ties)
// and V(m) = V(child(m, a*)); other infosets and chance nodes take expectations.
__global__ void k_x_br_up(int32_t hlo, int32_t nh, int32_t clo, int32_t nc, int player,
                          const int32_t* __restrict__ child_begin,
                          const int32_t* __restrict__ child_stride,
                          const int32_t* __restrict__ child_list,
                          const int32_t* __restrict__ q_offset, const int8_t* __restrict__ iplayer,
                          const int32_t* __restrict__ member_offset,
                          const int32_t* __restrict__ members,
                          const int32_t* __restrict__ chance_nodes,
                          const int32_t* __restrict__ chance_base,
                          const int32_t* __restrict__ chance_k, const float* __restrict__ avgprob,
                          const float* __restrict__ br_reach, float* __restrict__ br_value) {
    const int64_t u = gid();
    if (u >= static_cast<int64_t>(nh) + nc) return;
    if (u >= nh) {
        const int32_t ci = clo + static_cast<int32_t>(u - nh);
        const int32_t x = chance_nodes[ci];
        const int32_t base = chance_base[ci], k = chance_k[ci];
        float v = 0.0f;
        for (int32_t a = 0; a < k; ++a)
            v = fmaf(avgprob[base + a],
                     br_value[child_of(child_begin, child_stride, child_list, x, a)], v);
        br_value[x] = v;
        return;
    }
    const int32_t h = hlo + static_cast<int32_t>(u);
    const int32_t o = q_offset[h];
    const int32_t k = q_offset[h + 1] - o;
    const int32_t m0 = member_offset[h], m1 = member_offset[h + 1];
    if (iplayer[h] == player) {
        int32_t best = 0;
        float best_v = 0.0f;
        for (int32_t a = 0; a < k; ++a) {
            float tot = 0.0f;
            for (int32_t mi = m0; mi < m1; ++mi) {
                const int32_t x = members[mi];
                tot = fmaf(br_reach[x],
                           br_value[child_of(child_begin, child_stride, child_list, x, a)], tot);
            }
            if (a == 0 || tot > best_v) {
                best_v = tot;
                best = a;
            }
        }
        for (int32_t mi = m0; mi < m1; ++mi) {
            const int32_t x = members[mi];
            br_value[x] = br_value[child_of(child_begin, child_stride, child_list, x, best)];
        }
    } else {
        for (int32_t mi = m0; mi < m1; ++mi) {
            const int32_t x = members[mi];
            float v = 0.0f;
            for (int32_t a = 0; a < k; ++a)
                v = fmaf(avgprob[o + a],
                         br_value[child_of(child_begin, child_stride, child_list, x, a)], v);
            br_value[x] = v;
        }
    }
}

__global__ void k_x_tick(int64_t* T) {
    if (gid() == 0) *T += 1;
}

// Best-response value of every root (level 0, in game order) into out[g * 2 + player - 1].
__global__ void k_x_store_roots(int32_t n_roots, int player, const float* __restrict__ br_value,
                                double* out) {
    const int64_t g = gid();
    if (g < n_roots) out[2 * g + player - 1] = static_cast<double>(br_value[g]);
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
        default: return "";
    }
}

void launch_x_reset(const XDev& x, hipStream_t st) {
    hipLaunchKernelGGL(k_x_reset_nodes, dim3(blocks_for(x.N)), dim3(kBlock), 0, st, x.N,
                       x.level_offset_host[1], x.meta, x.payoff, x.value, x.reach);
}

template <int KMAX, int CH>
static void launch_up_chunk(const XDev& x, int32_t l, int variant, int linear, hipStream_t st) {
    const int32_t klo = x.k_level_offset_host[l], nk = x.k_level_offset_host[l + 1] - klo;
    const int32_t clo = x.c_level_offset_host[l], nc = x.c_level_offset_host[l + 1] - clo;
    const int32_t grid = nk + (nc + CH - 1) / CH;
    if (grid == 0) return;
    hipLaunchKernelGGL((k_x_up_chunk<KMAX, CH>), dim3(grid), dim3(CH), 0, st, klo, nk, clo, nc, x.N,
                       x.chunk_first, x.child_begin, x.child_stride, x.child_list, x.q_offset,
                       x.iplayer, x.member_offset, x.members, x.chance_nodes, x.chance_base,
                       x.chance_k, x.prob, x.value, x.reach, x.R, x.S, x.T, variant, linear);
}

template <int KMAX>
static void launch_up_chunk_cap(const XDev& x, int32_t l, int variant, int linear, hipStream_t st) {
    switch (x.chunk_cap_host != nullptr ? x.chunk_cap_host[l] : 256) {
        case 64: launch_up_chunk<KMAX, 64>(x, l, variant, linear, st); break;
        case 128: launch_up_chunk<KMAX, 128>(x, l, variant, linear, st); break;
        case 512: launch_up_chunk<KMAX, 512>(x, l, variant, linear, st); break;
        default: launch_up_chunk<KMAX, 256>(x, l, variant, linear, st); break;
    }
}

void launch_x_iteration(const XDev& x, int variant, int linear, hipStream_t st, LaunchTimer* timer) {
    auto pre = [&](int k, int l, int64_t n) { if (timer) timer->before(k, l, n, st); };
    auto post = [&](int k) { if (timer) timer->after(k, st); };
    const int32_t* lo = x.level_offset_host;
    for (int32_t l = 1; l < x.D; ++l) {
        const int64_t units = lo[l + 1] - lo[l];
        const int threads = pick(x.reach_block, units);
        pre(XK_REACH, l, units);
        hipLaunchKernelGGL(k_x_reach, dim3(blocks_of(units, threads)), dim3(threads), 0, st, lo[l],
                           lo[l + 1], x.N, x.parent, x.edge, x.meta, x.prob, x.reach);
        post(XK_REACH);
    }
    for (int32_t l = x.D; l >= 0; --l) {
        const int32_t nunits = x.h_level_offset_host[l + 1] - x.h_level_offset_host[l] +
                               x.c_level_offset_host[l + 1] - x.c_level_offset_host[l];
        if (nunits == 0) continue;
        pre(XK_UP, l, x.m_level_offset_host[l + 1] - x.m_level_offset_host[l]);
        if (x.max_actions <= 4) launch_up_chunk_cap<4>(x, l, variant, linear, st);
        else launch_up_chunk_cap<16>(x, l, variant, linear, st);
        post(XK_UP);
    }
    // the linear-averaging weight of every launch above read T: count the iteration last
    hipLaunchKernelGGL(k_x_tick, dim3(1), dim3(64), 0, st, x.T);
}

void launch_x_best_response(const XDev& x, const float* avgprob, int player, hipStream_t st) {
    const float sgn = player == 1 ? 1.0f : -1.0f;
    hipLaunchKernelGGL(k_x_br_init, dim3(blocks_for(x.N)), dim3(kBlock), 0, st, x.N,
                       x.level_offset_host[1], x.meta, x.payoff, sgn, x.br_value, x.br_reach);
    const int32_t* lo = x.level_offset_host;
    for (int32_t l = 1; l < x.D; ++l)
        hipLaunchKernelGGL(k_x_br_reach, dim3(blocks_for(lo[l + 1] - lo[l])), dim3(kBlock), 0, st,
                           lo[l], lo[l + 1], player, x.parent, x.edge, x.meta, avgprob, x.br_reach);
    for (int32_t l = x.D; l >= 0; --l) {
        const int32_t hlo = x.h_level_offset_host[l], nh = x.h_level_offset_host[l + 1] - hlo;
        const int32_t clo = x.c_level_offset_host[l], nc = x.c_level_offset_host[l + 1] - clo;
        if (nh + nc == 0) continue;
        hipLaunchKernelGGL(k_x_br_up, dim3(blocks_for(static_cast<int64_t>(nh) + nc)), dim3(kBlock),
                           0, st, hlo, nh, clo, nc, player, x.child_begin, x.child_stride,
                           x.child_list, x.q_offset, x.iplayer, x.member_offset, x.members,
                           x.chance_nodes, x.chance_base, x.chance_k, avgprob, x.br_reach,
                           x.br_value);
    }
    const int32_t n_roots = x.level_offset_host[1];
    hipLaunchKernelGGL(k_x_store_roots, dim3(blocks_for(n_roots)), dim3(kBlock), 0, st, n_roots,
                       player, x.br_value, x.out2);
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
