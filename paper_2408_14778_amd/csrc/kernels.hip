// gfx950 kernels of one CFR iteration over the canonical level-ordered layout.
//
// Section 3.2 casts an iteration as per-level sparse products: the expected payoffs
// run bottom-up (Eq. expected_payoffs_matrix_recurrence), the excepted and own reach
// probabilities top-down (Eq. excepted_reach_probabilities_matrix_recurrence), each
// level touching only its own nodes. Here each sparse product is one launch over the
// level's contiguous node range; the matrices are index arrays (one nonzero per
// column), and the node -> infoset-action reductions are fused into the bottom-up pass.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cfr {

namespace {

constexpr int kBlock = 256;
// Levels of at most this many nodes run the general-sum values one wavefront per node, and of at
// most kWideTop nodes (a root dealing many private types, the levels just below it) a
// workgroup of 1024 per node.
constexpr int32_t kWideNodes = 4096;
constexpr int32_t kWideTop = 16;

inline unsigned blocks_for(int64_t n) {
    return static_cast<unsigned>((n + kBlock - 1) / kBlock);
}

__device__ __forceinline__ int64_t gid() {
    return static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}

// Arithmetic of both real types: fp32 (the default path) and fp64.
__device__ __forceinline__ float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float pos_(float a) { return fmaxf(a, 0.0f); }
__device__ __forceinline__ double pos_(double a) { return fmax(a, 0.0); }

// Regret matching of one infoset (Eq. next_strategy_profile): positive parts over their
// sum, or uniform when the sum is exactly 0.
template <class F>
__device__ __forceinline__ void regret_match(const F* R, F* sigma, int32_t o, int32_t k) {
    F sum = F(0);
    for (int32_t a = 0; a < k; ++a) sum += pos_(R[o + a]);
    if (sum > F(0)) {
        for (int32_t a = 0; a < k; ++a) sigma[o + a] = pos_(R[o + a]) / sum;
    } else {
        const F u = F(1) / static_cast<F>(k);
        for (int32_t a = 0; a < k; ++a) sigma[o + a] = u;
    }
}

template <class F>
__global__ void k_reset_q(int64_t Qp, F* R, F* S, F* rtilde) {
    const int64_t q = gid();
    if (q >= Qp) return;
    R[q] = F(0);
    S[q] = F(0);
    rtilde[q] = F(0);
}

template <class F>
__global__ void k_reset_h(int64_t Hp, F* pibar) {
    const int64_t h = gid();
    if (h < Hp) pibar[h] = F(0);
}

template <class F>
__global__ void k_reset_nodes(int64_t N, const int8_t* node_player, const F* payoff, F* value,
                              F* reach) {
    const int64_t v = gid();
    if (v >= N) return;
    value[v] = node_player[v] < 0 ? payoff[v] : F(0);
    if (v == 0) {
        reach[0] = F(1);
        reach[N] = F(1);
        reach[2 * N] = F(1);
    }
}

template <class F>
__global__ void k_copy_tail(int64_t Q0, const F* src, F* dst) {
    const int64_t i = gid();
    if (i < Q0) dst[i] = src[i];
}

template <class F>
__global__ void k_regret_match(int64_t Hp, const int32_t* q_offset, const F* R, F* sigma) {
    const int64_t h = gid();
    if (h >= Hp) return;
    const int32_t o = q_offset[h];
    regret_match(R, sigma, o, q_offset[h + 1] - o);
}

__global__ void k_set_T(int64_t* T, int64_t value) {
    if (gid() == 0) *T = value;
}

__global__ void k_tick(int64_t* T) {
    if (gid() == 0) *T += 1;
}

// Top-down reach of one level (Eq. excepted_reach_probabilities_matrix_recurrence and its
// own-reach twin): a decision node takes its parent's (pi_1, pi_2, pi_c) and multiplies the
// factor of whoever acted at the parent by the edge probability s_v = sigma or sigma_0.
// Terminal nodes need no reach.
template <class F>
__global__ void k_reach_level(int32_t lo, int32_t hi, int64_t N, const int32_t* __restrict__ parent,
                              const int8_t* __restrict__ node_player,
                              const int32_t* __restrict__ node_edge, const F* __restrict__ prob,
                              F* __restrict__ reach) {
    const int64_t v = lo + gid();
    if (v >= hi) return;
    if (node_player[v] < 0) return;
    const int32_t p = parent[v];
    const F s = prob[node_edge[v]];
    const int8_t who = node_player[p];  // 0 chance, 1, 2
    F r1 = reach[p], r2 = reach[N + p], rc = reach[2 * N + p];
    if (who == 1) r1 *= s;
    else if (who == 2) r2 *= s;
    else rc *= s;
    reach[v] = r1;
    reach[N + v] = r2;
    reach[2 * N + v] = rc;
}

// Bottom-up values of one level (Eq. expected_payoffs_matrix_recurrence) fused with the
// node -> infoset-action terms: for a node d of player i with value u and children values w_a,
// the contribution sgn_i * pi_{-i}(d) * (w_a - u) to r~(h, a) (the multiplied-out form of
// Eq. instantaneous_counterfactual_regret, with u_2 = -u_1) and pi_i(d) to pibar(h) (Eq.
// player_reach_probability, own-reach reading). kStore: the contribution is stored at the
// child's slot and a gather pass sums it per infoset in member order (no atomics; pibar is
// summed from the reach planes there); otherwise both are added to the per-pair and
// per-infoset accumulators by atomics (the partitioned iteration, whose windows are overwritten
// partition by partition, accumulates across them this way).
template <class F, bool kStore>
__global__ void k_value_level(int32_t lo, int32_t hi, int64_t N,
                              const int32_t* __restrict__ child_begin,
                              const int8_t* __restrict__ node_player,
                              const int32_t* __restrict__ node_infoset,
                              const int32_t* __restrict__ node_edge,
                              const F* __restrict__ prob, F* __restrict__ value,
                              const F* __restrict__ reach, F* __restrict__ rtilde,
                              F* __restrict__ pibar, F* __restrict__ contrib) {
    const int64_t p = lo + gid();
    if (p >= hi) return;
    const int8_t who = node_player[p];
    if (who < 0) return;
    const int32_t c0 = child_begin[p], c1 = child_begin[p + 1];
    // a player node's reaches (and infoset) first: their loads overlap the children's
    F r1 = F(0), r2 = F(0), rc = F(0);
    int32_t h = 0;
    if (who > 0) {
        r1 = reach[p];
        r2 = reach[N + p];
        rc = reach[2 * N + p];
        if (!kStore) h = node_infoset[p];
    }
    F u = F(0);
    for (int32_t c = c0; c < c1; ++c) u = fma_(prob[node_edge[c]], value[c], u);
    value[p] = u;
    if (who == 0) return;
    const F cf = (who == 1 ? r2 : r1) * rc;
    const F w = who == 1 ? cf : -cf;
    if (kStore) {
        for (int32_t c = c0; c < c1; ++c) contrib[c] = w * (value[c] - u);
        return;
    }
    for (int32_t c = c0; c < c1; ++c)
        unsafeAtomicAdd(&rtilde[node_edge[c]], w * (value[c] - u));
    unsafeAtomicAdd(&pibar[h], who == 1 ? r1 : r2);
}

// ---- general-sum games of P rational players (Section 3.1: the payoff matrix and the
// expected-payoff recurrence carry one column per rational player)

// Values and reach planes at reset: every player's payoff column at terminals, 0 elsewhere;
// every reach plane 1 at the root (canonical node 0).
template <class F>
__global__ void k_reset_nodes_n(int64_t N, int32_t P, const int8_t* node_player, const F* payoff,
                                F* value, F* reach) {
    const int64_t v = gid();
    if (v >= N) return;
    const bool term = node_player[v] < 0;
    for (int32_t i = 0; i < P; ++i) value[i * N + v] = term ? payoff[i * N + v] : F(0);
    if (v == 0)
        for (int32_t k = 0; k <= P; ++k) reach[k * N] = F(1);
}

// Top-down reach of one level: a decision node copies its parent's P + 1 planes and multiplies
// the plane of whoever acted at the parent (plane P for chance) by the edge probability.
template <class F>
__global__ void k_reach_level_n(int32_t lo, int32_t hi, int64_t N, int32_t P,
                                const int32_t* __restrict__ parent,
                                const int8_t* __restrict__ node_player,
                                const int32_t* __restrict__ node_edge, const F* __restrict__ prob,
                                F* __restrict__ reach) {
    const int64_t v = lo + gid();
    if (v >= hi) return;
    if (node_player[v] < 0) return;
    const int32_t p = parent[v];
    const F s = prob[node_edge[v]];
    const int8_t who = node_player[p];  // 0 chance, 1 .. P
    const int32_t acted = who == 0 ? P : who - 1;
    for (int32_t k = 0; k <= P; ++k) {
        const F r = reach[k * N + p];
        reach[k * N + v] = k == acted ? r * s : r;
    }
}

// Bottom-up values of one level: every player's column u_i = sum_a s_a w_a[i]; at a node d of
// player i, each child's regret contribution pi_{-i}(d) (w_a[i] - u_i), with pi_{-i} = pi_c times
// the other players' planes in player order, then d's own reach pi_i(d), are stored at d's
// member-order slot (node_slot: one short contiguous run per node; no atomics: an infoset of a
// general-sum game can have many members, whose additions to one accumulator would serialise);
// k_gather_slots sums them per infoset.
template <class F>
__global__ void k_value_level_n(int32_t lo, int32_t hi, int64_t N, int32_t P,
                                const int32_t* __restrict__ child_begin,
                                const int8_t* __restrict__ node_player,
                                const int32_t* __restrict__ node_edge, const F* __restrict__ prob,
                                const int32_t* __restrict__ node_slot, F* __restrict__ value,
                                const F* __restrict__ reach, F* __restrict__ contrib) {
    const int64_t p = lo + gid();
    if (p >= hi) return;
    const int8_t who = node_player[p];
    if (who < 0) return;
    const int32_t c0 = child_begin[p], c1 = child_begin[p + 1];
    // a player node's reaches and slot first: their loads overlap the children's
    const int32_t me = who - 1;
    F cf = F(0), own_r = F(0);
    int32_t at = 0;
    if (who > 0) {
        cf = reach[P * N + p];
        for (int32_t j = 0; j < P; ++j)
            if (j != me) cf *= reach[j * N + p];
        own_r = reach[me * N + p];
        at = node_slot[p];
    }
    // every player's column in one walk over the children (each sum in child order)
    F u[kMaxPlayers];
#pragma unroll
    for (int i = 0; i < kMaxPlayers; ++i) u[i] = F(0);
    for (int32_t c = c0; c < c1; ++c) {
        const F s = prob[node_edge[c]];
#pragma unroll
        for (int i = 0; i < kMaxPlayers; ++i)
            if (i < P) u[i] = fma_(s, value[i * N + c], u[i]);
    }
    F own_u = F(0);
#pragma unroll
    for (int i = 0; i < kMaxPlayers; ++i) {
        if (i < P) value[i * N + p] = u[i];
        if (i == me) own_u = u[i];
    }
    if (who == 0) return;
    F* slot = contrib + at;
    for (int32_t c = c0; c < c1; ++c) slot[c - c0] = cf * (value[me * N + c] - own_u);
    slot[c1 - c0] = own_r;
}

// k_value_level_n for a level of few nodes, W wavefronts per node: thread t takes children
// t, t + 64 W, ..., summing every player's column in the one walk over them; the partial sums
// are added by a fixed butterfly in each wavefront, then over the wavefronts in order (a node
// with a wide fan-out, such as a root dealing thousands of private-type combinations, would
// otherwise walk its children on one thread). W = 1: a workgroup of 256 holds four nodes, one
// per wavefront; W > 1: the workgroup is the node's (grid = the level's node count).
template <class F, int W>
__global__ void __launch_bounds__(W == 1 ? 256 : 64 * W)
    k_value_wide_n(int32_t lo, int32_t hi, int64_t N, int32_t P,
                   const int32_t* __restrict__ child_begin, const int8_t* __restrict__ node_player,
                   const int32_t* __restrict__ node_edge, const F* __restrict__ prob,
                   const int32_t* __restrict__ node_slot, F* __restrict__ value,
                   const F* __restrict__ reach, F* __restrict__ contrib) {
    constexpr int kT = 64 * W;  // threads per node
    const int tid = W == 1 ? static_cast<int>(threadIdx.x & 63) : static_cast<int>(threadIdx.x);
    const int64_t p = W == 1 ? lo + ((static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6)
                             : lo + static_cast<int64_t>(blockIdx.x);
    if (p >= hi) return;  // whole wavefronts (W = 1) or the whole workgroup (W > 1) leave together
    const int8_t who = node_player[p];
    if (who < 0) return;
    const int32_t c0 = child_begin[p], c1 = child_begin[p + 1];
    F u[kMaxPlayers];
#pragma unroll
    for (int i = 0; i < kMaxPlayers; ++i) u[i] = F(0);
    for (int32_t c = c0 + tid; c < c1; c += kT) {
        const F s = prob[node_edge[c]];
#pragma unroll
        for (int i = 0; i < kMaxPlayers; ++i)
            if (i < P) u[i] = fma_(s, value[i * N + c], u[i]);
    }
#pragma unroll
    for (int i = 0; i < kMaxPlayers; ++i)
        if (i < P)
            for (int off = 32; off > 0; off >>= 1) u[i] += __shfl_xor(u[i], off, 64);
    F own_u = F(0);
    if constexpr (W == 1) {
        if (tid == 0)
            for (int32_t i = 0; i < P; ++i) value[i * N + p] = u[i];
#pragma unroll
        for (int i = 0; i < kMaxPlayers; ++i)
            if (i == who - 1) own_u = u[i];
    } else {
        __shared__ F s_part[W][kMaxPlayers];
        __shared__ F s_u[kMaxPlayers];
        const int wave = tid >> 6;
        if ((tid & 63) == 0)
#pragma unroll
            for (int i = 0; i < kMaxPlayers; ++i) s_part[wave][i] = u[i];
        __syncthreads();
        if (tid < P) {
            F sum = F(0);
#pragma unroll
            for (int w = 0; w < W; ++w) sum += s_part[w][tid];
            value[tid * N + p] = sum;
            s_u[tid] = sum;
        }
        __syncthreads();
        if (who > 0) own_u = s_u[who - 1];
    }
    if (who == 0) return;
    const int32_t me = who - 1;
    F cf = reach[P * N + p];
    for (int32_t j = 0; j < P; ++j)
        if (j != me) cf *= reach[j * N + p];
    F* slot = contrib + node_slot[p];
    for (int32_t c = c0 + tid; c < c1; c += kT) slot[c - c0] = cf * (value[me * N + c] - own_u);
    if (tid == 0) slot[c1 - c0] = reach[me * N + p];
}

// Per infoset of a general-sum game, one workgroup of W wavefronts sums its members' slots
// (node_slot: k + 1 values per member, the infoset's members contiguous): r~(h, a) = the sum of
// the members' action-a contributions, pibar(h) = the sum of their own reaches (Eq.
// player_reach_probability, own-reach reading). Thread t takes members t, t + 64 W, ..., up to
// kGatherActions of the k + 1 sums at once; the partial sums are added by a fixed butterfly in
// each wavefront, then over the wavefronts in order, so the result does not depend on
// scheduling. Written over the accumulators the infoset update reads (and clears). Grid: one
// workgroup per infoset.
constexpr int kGatherActions = 4;

template <class F, int W>
__global__ void __launch_bounds__(64 * W) k_gather_slots(int64_t Hp,
                                                        const int32_t* __restrict__ q_offset,
                                                        const int32_t* __restrict__ member_offset,
                                                        const int32_t* __restrict__ slot_base,
                                                        const F* __restrict__ contrib,
                                                        F* __restrict__ rtilde,
                                                        F* __restrict__ pibar) {
    constexpr int kT = 64 * W, KB = kGatherActions;
    __shared__ F s_part[W][KB];
    const int64_t h = blockIdx.x;
    if (h >= Hp) return;  // the whole workgroup leaves together
    const int tid = threadIdx.x, wave = tid >> 6;
    const int32_t o = q_offset[h], k = q_offset[h + 1] - o;
    const int32_t n = member_offset[h + 1] - member_offset[h];
    const F* slots = contrib + slot_base[h];
    for (int32_t r0 = 0; r0 <= k; r0 += KB) {  // sums 0 .. k
        F acc[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = F(0);
        for (int32_t m = tid; m < n; m += kT)
#pragma unroll
            for (int j = 0; j < KB; ++j)
                if (r0 + j <= k) acc[j] += slots[m * (k + 1) + r0 + j];
#pragma unroll
        for (int j = 0; j < KB; ++j)
            for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off, 64);
        if ((tid & 63) == 0)
#pragma unroll
            for (int j = 0; j < KB; ++j) s_part[wave][j] = acc[j];
        __syncthreads();
        if (tid < KB && r0 + tid <= k) {
            F sum = F(0);
#pragma unroll
            for (int w = 0; w < W; ++w) sum += s_part[w][tid];
            if (r0 + tid < k) rtilde[o + r0 + tid] = sum;
            else pibar[h] = sum;
        }
        __syncthreads();  // s_part is reused by the next sums
    }
}

// The two-player node engine's gather (contributions at each child's slot, k_value_level with
// kStore). Per infoset, one workgroup of W wavefronts: r~(h, a) = the sum over the members d of
// their action-a child's contribution, and pibar(h) = the sum of the members' own reaches (Eq.
// player_reach_probability, own-reach reading). Thread t takes members t, t + 64 W, ... in member
// order, each member's node and child offset loaded once for up to kGatherActions actions; the
// partial sums are added by a fixed butterfly in each wavefront, then over the wavefronts in
// order, so the result does not depend on scheduling. An infoset of more actions walks its
// members once per kGatherActions. Written over the accumulators the infoset update reads (and
// clears). Grid: one workgroup per infoset.
template <class F, int W>
__global__ void __launch_bounds__(64 * W) k_gather_n(int64_t Hp, int64_t N,
                                                     const int32_t* __restrict__ q_offset,
                                                     const int32_t* __restrict__ member_offset,
                                                     const int32_t* __restrict__ members,
                                                     const int32_t* __restrict__ child_begin,
                                                     const int8_t* __restrict__ infoset_player,
                                                     const F* __restrict__ reach,
                                                     const F* __restrict__ contrib,
                                                     F* __restrict__ rtilde, F* __restrict__ pibar) {
    constexpr int kT = 64 * W, KB = kGatherActions;
    __shared__ F s_part[W][KB + 1];
    const int64_t h = blockIdx.x;
    if (h >= Hp) return;  // the whole workgroup leaves together
    const int tid = threadIdx.x, wave = tid >> 6;
    const int32_t o = q_offset[h], k = q_offset[h + 1] - o;
    const int32_t m0 = member_offset[h], m1 = member_offset[h + 1];
    const int64_t own_plane = static_cast<int64_t>(infoset_player[h] - 1) * N;
    // the first walk also sums the own reaches (slot KB), so it runs even for k = 0
    for (int32_t a0 = 0; a0 == 0 || a0 < k; a0 += KB) {
        F acc[KB + 1];
#pragma unroll
        for (int j = 0; j <= KB; ++j) acc[j] = F(0);
        for (int32_t m = m0 + tid; m < m1; m += kT) {
            const int32_t x = members[m];
            const int32_t cb = child_begin[x] + a0;
            if (a0 == 0) acc[KB] += reach[own_plane + x];
#pragma unroll
            for (int j = 0; j < KB; ++j)
                if (a0 + j < k) acc[j] += contrib[cb + j];
        }
#pragma unroll
        for (int j = 0; j <= KB; ++j)
            for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off, 64);
        if ((tid & 63) == 0)
#pragma unroll
            for (int j = 0; j <= KB; ++j) s_part[wave][j] = acc[j];
        __syncthreads();
        if (tid <= KB) {
            F sum = F(0);
#pragma unroll
            for (int w = 0; w < W; ++w) sum += s_part[w][tid];
            if (tid < KB && a0 + tid < k) rtilde[o + a0 + tid] = sum;
            if (tid == KB && a0 == 0) pibar[h] = sum;
        }
        __syncthreads();  // s_part is reused by the next walk
    }
}

// Infoset pass: regret update (vanilla R += r~, CFR+ R = max(R + r~, 0), discounted
// R = (R + r~) * d+ or d-; Eq. average_counterfactual_regrets_vector in cumulative form),
// average-strategy accumulation S += w_T * pibar * sigma (discounted: then S *= d_avg; Eq.
// average_strategy_profile_vector in cumulative form), then regret matching for the next
// strategy, for the infosets of the pass's players. Clears the accumulators of all.
template <class F>
__global__ void k_infoset_update(int64_t Hp, const int32_t* __restrict__ q_offset,
                                 const int8_t* __restrict__ infoset_player,
                                 F* __restrict__ R, F* __restrict__ S,
                                 F* __restrict__ sigma, F* __restrict__ rtilde,
                                 F* __restrict__ pibar, const int64_t* __restrict__ T,
                                 UpdateRule rule) {
    const int64_t h = gid();
    if (h >= Hp) return;
    const int32_t o = q_offset[h], k = q_offset[h + 1] - o;
    const F t = static_cast<F>(*T + 1);
    F wt = rule.linear ? t : F(1);
    F d_pos = F(1), d_neg = F(1), d_avg = F(1);
    if (rule.variant == 2) {
        wt = F(1);
        dcfr_discounts(rule, t, d_pos, d_neg, d_avg);
    }
    const F pb = pibar[h];
    pibar[h] = F(0);
    if (!((rule.players >> (infoset_player[h] - 1)) & 1)) {
        for (int32_t a = 0; a < k; ++a) rtilde[o + a] = F(0);
        return;
    }
    for (int32_t a = 0; a < k; ++a) {
        const int32_t q = o + a;
        F r = R[q] + rtilde[q];
        if (rule.variant == 1) r = pos_(r);
        else if (rule.variant == 2) r *= r > F(0) ? d_pos : d_neg;
        R[q] = r;
        const F sn = fma_(wt * pb, sigma[q], S[q]);
        S[q] = rule.variant == 2 ? sn * d_avg : sn;
        rtilde[q] = F(0);
    }
    regret_match(R, sigma, o, k);
}

// Average strategy: S normalised per infoset, uniform where its sum is 0.
template <class F>
__global__ void k_average(int64_t Hp, const int32_t* __restrict__ q_offset,
                          const F* __restrict__ S, F* __restrict__ avg) {
    const int64_t h = gid();
    if (h >= Hp) return;
    const int32_t o = q_offset[h], k = q_offset[h + 1] - o;
    F sum = F(0);
    for (int32_t a = 0; a < k; ++a) sum += S[o + a];
    if (sum > F(0)) {
        for (int32_t a = 0; a < k; ++a) avg[o + a] = S[o + a] / sum;
    } else {
        const F u = F(1) / static_cast<F>(k);
        for (int32_t a = 0; a < k; ++a) avg[o + a] = u;
    }
}

// ---- best response (Section 2.2): the responder i maximises, everyone else plays avgprob

template <class F>
__global__ void k_br_terminal(int64_t N, const int8_t* __restrict__ node_player,
                              const F* __restrict__ payoff, F sgn, F* __restrict__ br_value,
                              F* __restrict__ br_reach) {
    const int64_t v = gid();
    if (v >= N) return;
    br_value[v] = node_player[v] < 0 ? sgn * payoff[v] : F(0);
    if (v == 0) br_reach[0] = F(1);
}

// pi_{-i}: product of chance and opponent edge probabilities (decision nodes only).
template <class F>
__global__ void k_br_reach_level(int32_t lo, int32_t hi, int player,
                                 const int32_t* __restrict__ parent,
                                 const int8_t* __restrict__ node_player,
                                 const int32_t* __restrict__ node_edge,
                                 const F* __restrict__ avgprob, F* __restrict__ br_reach) {
    const int64_t v = lo + gid();
    if (v >= hi) return;
    if (node_player[v] < 0) return;
    const int32_t p = parent[v];
    const F f = node_player[p] == player ? F(1) : avgprob[node_edge[v]];
    br_reach[v] = br_reach[p] * f;
}

// a*(h) = argmax_a sum_{d in h} pi_{-i}(d) V(child(d, a)), lowest index on ties.
template <class F>
__global__ void k_br_choose(int32_t hlo, int32_t hhi, int player,
                            const int8_t* __restrict__ infoset_player,
                            const int32_t* __restrict__ q_offset,
                            const int32_t* __restrict__ member_offset,
                            const int32_t* __restrict__ members,
                            const int32_t* __restrict__ child_begin,
                            const F* __restrict__ br_reach, const F* __restrict__ br_value,
                            int32_t* __restrict__ best) {
    const int64_t h = hlo + gid();
    if (h >= hhi) return;
    if (infoset_player[h] != player) return;
    const int32_t k = q_offset[h + 1] - q_offset[h];
    const int32_t m0 = member_offset[h], m1 = member_offset[h + 1];
    int32_t a_star = 0;
    F v_star = F(0);
    for (int32_t a = 0; a < k; ++a) {
        F tot = F(0);
        for (int32_t m = m0; m < m1; ++m) {
            const int32_t d = members[m];
            tot = fma_(br_reach[d], br_value[child_begin[d] + a], tot);
        }
        if (a == 0 || tot > v_star) {
            v_star = tot;
            a_star = a;
        }
    }
    best[h] = a_star;
}

template <class F>
__global__ void k_br_value_level(int32_t lo, int32_t hi, int player,
                                 const int32_t* __restrict__ child_begin,
                                 const int8_t* __restrict__ node_player,
                                 const int32_t* __restrict__ node_infoset,
                                 const int32_t* __restrict__ node_edge,
                                 const F* __restrict__ avgprob, const int32_t* __restrict__ best,
                                 F* __restrict__ br_value) {
    const int64_t p = lo + gid();
    if (p >= hi) return;
    const int8_t who = node_player[p];
    if (who < 0) return;
    const int32_t c0 = child_begin[p], c1 = child_begin[p + 1];
    if (who == player) {
        br_value[p] = br_value[c0 + best[node_infoset[p]]];
        return;
    }
    F u = F(0);
    for (int32_t c = c0; c < c1; ++c) u = fma_(avgprob[node_edge[c]], br_value[c], u);
    br_value[p] = u;
}

template <class F>
__global__ void k_br_store(const F* __restrict__ br_value, double* out) {
    if (gid() == 0) *out = static_cast<double>(br_value[0]);
}

template <class F>
__global__ void k_scatter_q(int64_t Qp, const int32_t* __restrict__ q_input,
                            const F* __restrict__ src, F* __restrict__ dst) {
    const int64_t q = gid();
    if (q < Qp) dst[q_input[q]] = src[q];
}

template <class F>
__global__ void k_gather_q(int64_t Qp, const int32_t* __restrict__ q_input,
                           const F* __restrict__ src, F* __restrict__ dst) {
    const int64_t q = gid();
    if (q < Qp) dst[q] = src[q_input[q]];
}

}  // namespace

template <class F>
void launch_reset(const DevT<F>& d, hipStream_t st, bool node_arrays) {
    if (d.Qp > 0) hipLaunchKernelGGL(k_reset_q<F>, dim3(blocks_for(d.Qp)), dim3(kBlock), 0, st,
                                     d.Qp, d.R, d.S, node_arrays ? d.rtilde : d.stage);
    if (d.Hp > 0 && node_arrays)
        hipLaunchKernelGGL(k_reset_h<F>, dim3(blocks_for(d.Hp)), dim3(kBlock), 0, st, d.Hp,
                           d.pibar);
    if (node_arrays && d.players > 0)
        hipLaunchKernelGGL(k_reset_nodes_n<F>, dim3(blocks_for(d.N)), dim3(kBlock), 0, st, d.N,
                           d.players, d.node_player, d.payoff, d.value, d.reach);
    else if (node_arrays)
        hipLaunchKernelGGL(k_reset_nodes<F>, dim3(blocks_for(d.N)), dim3(kBlock), 0, st, d.N,
                           d.node_player, d.payoff, d.value, d.reach);
    if (d.Q0 > 0)
        hipLaunchKernelGGL(k_copy_tail<F>, dim3(blocks_for(d.Q0)), dim3(kBlock), 0, st, d.Q0,
                           d.prob + d.Qp, d.avgprob + d.Qp);
    hipLaunchKernelGGL(k_set_T, dim3(1), dim3(64), 0, st, d.T, int64_t{0});
    launch_regret_match(d, st);
}

template <class F>
void launch_regret_match(const DevT<F>& d, hipStream_t st) {
    if (d.Hp > 0)
        hipLaunchKernelGGL(k_regret_match<F>, dim3(blocks_for(d.Hp)), dim3(kBlock), 0, st, d.Hp,
                           d.sq_offset, d.R, d.prob);
}

template <class F>
void launch_set_T(const DevT<F>& d, int64_t value, hipStream_t st) {
    hipLaunchKernelGGL(k_set_T, dim3(1), dim3(64), 0, st, d.T, value);
}

const char* kernel_kind_name(int kind) {
    switch (kind) {
        case K_REACH: return "reach_level";
        case K_VALUE: return "value_level";
        case K_INFOSET: return "infoset_update";
        case K_TICK: return "tick";
        default: return "";
    }
}

// With stored contributions (d.contrib): the per-infoset sums of the children's regret
// contributions and of the members' own reaches (k_gather_n, a wavefront per infoset), before
// the infoset update.
template <class F, int W>
void launch_gather_w(const DevT<F>& d, hipStream_t st) {
    if (d.players > 0)
        hipLaunchKernelGGL((k_gather_slots<F, W>), dim3(static_cast<unsigned>(d.Hp)), dim3(64 * W),
                           0, st, d.Hp, d.q_offset, d.member_offset, d.slot_base, d.contrib,
                           d.rtilde, d.pibar);
    else
        hipLaunchKernelGGL((k_gather_n<F, W>), dim3(static_cast<unsigned>(d.Hp)), dim3(64 * W), 0,
                           st, d.Hp, d.N, d.q_offset, d.member_offset, d.members, d.child_begin,
                           d.infoset_player, d.reach, d.contrib, d.rtilde, d.pibar);
}

// The wavefronts per infoset follow the mean member count (one pass of the workgroup over the
// members of an average infoset, at most four wavefronts).
template <class F>
void launch_gather(const DevT<F>& d, hipStream_t st) {
    if (d.contrib == nullptr || d.Hp <= 0) return;
    const int64_t mean = (d.M + d.Hp - 1) / d.Hp;
    if (mean <= 64) launch_gather_w<F, 1>(d, st);
    else if (mean <= 128) launch_gather_w<F, 2>(d, st);
    else launch_gather_w<F, 4>(d, st);
}

template <class F>
void launch_iteration(const DevT<F>& d, const int32_t* lo, const UpdateRule& rule, hipStream_t st,
                      LaunchTimer* timer) {
    auto pre = [&](int k, int l, int64_t n) { if (timer) timer->before(k, l, n, st); };
    auto post = [&](int k) { if (timer) timer->after(k, st); };
    // top-down: levels 1 .. D-1 (level D holds terminals only)
    for (int32_t l = 1; l < d.D; ++l) {
        const int32_t a = lo[l], b = lo[l + 1];
        pre(K_REACH, l, b - a);
        launch_reach_range(d, a, b, st);
        post(K_REACH);
    }
    // bottom-up: levels D-1 .. 0
    for (int32_t l = d.D - 1; l >= 0; --l) {
        const int32_t a = lo[l], b = lo[l + 1];
        pre(K_VALUE, l, b - a);
        launch_value_range(d, a, b, st);
        post(K_VALUE);
    }
    if (d.Hp > 0) {
        pre(K_INFOSET, -1, d.Hp);
        launch_gather(d, st);
        hipLaunchKernelGGL(k_infoset_update<F>, dim3(blocks_for(d.Hp)), dim3(kBlock), 0, st, d.Hp,
                           d.q_offset, d.infoset_player, d.R, d.S, d.prob, d.rtilde, d.pibar, d.T,
                           rule);
        post(K_INFOSET);
    }
    if (rule.count) {
        pre(K_TICK, -1, 1);
        hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, d.T);
        post(K_TICK);
    }
}

template <class F>
void launch_reach_range(const DevT<F>& d, int32_t lo, int32_t hi, hipStream_t st) {
    if (hi <= lo) return;
    if (d.players > 0)
        hipLaunchKernelGGL(k_reach_level_n<F>, dim3(blocks_for(hi - lo)), dim3(kBlock), 0, st, lo,
                           hi, d.N, d.players, d.parent, d.node_player, d.node_edge, d.prob,
                           d.reach);
    else
        hipLaunchKernelGGL(k_reach_level<F>, dim3(blocks_for(hi - lo)), dim3(kBlock), 0, st, lo, hi,
                           d.N, d.parent, d.node_player, d.node_edge, d.prob, d.reach);
}

template <class F>
void launch_value_range(const DevT<F>& d, int32_t lo, int32_t hi, hipStream_t st) {
    if (hi <= lo) return;
    if (d.players > 0 && hi - lo <= kWideTop)
        hipLaunchKernelGGL((k_value_wide_n<F, 16>), dim3(static_cast<unsigned>(hi - lo)), dim3(1024),
                           0, st, lo, hi, d.N, d.players, d.child_begin, d.node_player,
                           d.node_edge, d.prob, d.node_slot, d.value, d.reach, d.contrib);
    else if (d.players > 0 && hi - lo <= kWideNodes)
        hipLaunchKernelGGL((k_value_wide_n<F, 1>), dim3(static_cast<unsigned>((hi - lo + 3) / 4)),
                           dim3(256), 0, st, lo, hi, d.N, d.players, d.child_begin, d.node_player,
                           d.node_edge, d.prob, d.node_slot, d.value, d.reach, d.contrib);
    else if (d.players > 0)
        hipLaunchKernelGGL(k_value_level_n<F>, dim3(blocks_for(hi - lo)), dim3(kBlock), 0, st, lo,
                           hi, d.N, d.players, d.child_begin, d.node_player, d.node_edge, d.prob,
                           d.node_slot, d.value, d.reach, d.contrib);
    else if (d.contrib != nullptr)
        hipLaunchKernelGGL((k_value_level<F, true>), dim3(blocks_for(hi - lo)), dim3(kBlock), 0, st,
                           lo, hi, d.N, d.child_begin, d.node_player, d.node_infoset, d.node_edge,
                           d.prob, d.value, d.reach, d.rtilde, d.pibar, d.contrib);
    else
        hipLaunchKernelGGL((k_value_level<F, false>), dim3(blocks_for(hi - lo)), dim3(kBlock), 0,
                           st, lo, hi, d.N, d.child_begin, d.node_player, d.node_infoset,
                           d.node_edge, d.prob, d.value, d.reach, d.rtilde, d.pibar, d.contrib);
}

template <class F>
void launch_infoset_pass(const DevT<F>& d, const UpdateRule& rule, hipStream_t st) {
    launch_gather(d, st);
    if (d.Hp > 0)
        hipLaunchKernelGGL(k_infoset_update<F>, dim3(blocks_for(d.Hp)), dim3(kBlock), 0, st, d.Hp,
                           d.q_offset, d.infoset_player, d.R, d.S, d.prob, d.rtilde, d.pibar, d.T,
                           rule);
    if (rule.count) hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, d.T);
}

template <class F>
void launch_average(const DevT<F>& d, hipStream_t st) {
    if (d.Hp > 0)
        hipLaunchKernelGGL(k_average<F>, dim3(blocks_for(d.Hp)), dim3(kBlock), 0, st, d.Hp,
                           d.sq_offset, d.S, d.avgprob);
}

template <class F>
void launch_best_response(const DevT<F>& d, const int32_t* lo, const int32_t* hlo, int player,
                          hipStream_t st) {
    const F sgn = player == 1 ? F(1) : F(-1);
    hipLaunchKernelGGL(k_br_terminal<F>, dim3(blocks_for(d.N)), dim3(kBlock), 0, st, d.N,
                       d.node_player, d.payoff, sgn, d.br_value, d.br_reach);
    for (int32_t l = 1; l < d.D; ++l) {
        const int32_t a = lo[l], b = lo[l + 1];
        hipLaunchKernelGGL(k_br_reach_level<F>, dim3(blocks_for(b - a)), dim3(kBlock), 0, st, a,
                           b, player, d.parent, d.node_player, d.node_edge, d.avgprob,
                           d.br_reach);
    }
    for (int32_t l = d.D - 1; l >= 0; --l) {
        const int32_t ha = hlo[l], hb = hlo[l + 1];
        if (hb > ha)
            hipLaunchKernelGGL(k_br_choose<F>, dim3(blocks_for(hb - ha)), dim3(kBlock), 0, st, ha,
                               hb, player, d.infoset_player, d.q_offset, d.member_offset,
                               d.members, d.child_begin, d.br_reach, d.br_value, d.best);
        const int32_t a = lo[l], b = lo[l + 1];
        hipLaunchKernelGGL(k_br_value_level<F>, dim3(blocks_for(b - a)), dim3(kBlock), 0, st, a,
                           b, player, d.child_begin, d.node_player, d.node_infoset, d.node_edge,
                           d.avgprob, d.best, d.br_value);
    }
    hipLaunchKernelGGL(k_br_store<F>, dim3(1), dim3(64), 0, st, d.br_value,
                       d.out2 + (player - 1));
}

template <class F>
void launch_scatter_q(const DevT<F>& d, const F* src, F* dst, hipStream_t st) {
    if (d.Qp > 0)
        hipLaunchKernelGGL(k_scatter_q<F>, dim3(blocks_for(d.Qp)), dim3(kBlock), 0, st, d.Qp,
                           d.sq_input, src, dst);
}

template <class F>
void launch_gather_q(const DevT<F>& d, const F* src, F* dst, hipStream_t st) {
    if (d.Qp > 0)
        hipLaunchKernelGGL(k_gather_q<F>, dim3(blocks_for(d.Qp)), dim3(kBlock), 0, st, d.Qp,
                           d.sq_input, src, dst);
}

#define CFR_INSTANTIATE(F)                                                                     \
    template void launch_reset<F>(const DevT<F>&, hipStream_t, bool);                          \
    template void launch_regret_match<F>(const DevT<F>&, hipStream_t);                         \
    template void launch_set_T<F>(const DevT<F>&, int64_t, hipStream_t);                       \
    template void launch_iteration<F>(const DevT<F>&, const int32_t*, const UpdateRule&,       \
                                      hipStream_t, LaunchTimer*);                              \
    template void launch_average<F>(const DevT<F>&, hipStream_t);                              \
    template void launch_reach_range<F>(const DevT<F>&, int32_t, int32_t, hipStream_t);        \
    template void launch_value_range<F>(const DevT<F>&, int32_t, int32_t, hipStream_t);        \
    template void launch_infoset_pass<F>(const DevT<F>&, const UpdateRule&, hipStream_t);      \
    template void launch_best_response<F>(const DevT<F>&, const int32_t*, const int32_t*, int, \
                                          hipStream_t);                                        \
    template void launch_scatter_q<F>(const DevT<F>&, const F*, F*, hipStream_t);              \
    template void launch_gather_q<F>(const DevT<F>&, const F*, F*, hipStream_t);
CFR_INSTANTIATE(float)
CFR_INSTANTIATE(double)
#undef CFR_INSTANTIATE

}  // namespace cfr
