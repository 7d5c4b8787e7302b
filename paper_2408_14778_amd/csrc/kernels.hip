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

inline unsigned blocks_for(int64_t n) {
    return static_cast<unsigned>((n + kBlock - 1) / kBlock);
}

__device__ __forceinline__ int64_t gid() {
    return static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}

// Regret matching of one infoset (Eq. next_strategy_profile): positive parts over their
// sum, or uniform when the sum is exactly 0.
__device__ __forceinline__ void regret_match(const float* R, float* sigma, int32_t o, int32_t k) {
    float sum = 0.0f;
    for (int32_t a = 0; a < k; ++a) sum += fmaxf(R[o + a], 0.0f);
    if (sum > 0.0f) {
        for (int32_t a = 0; a < k; ++a) sigma[o + a] = fmaxf(R[o + a], 0.0f) / sum;
    } else {
        const float u = 1.0f / static_cast<float>(k);
        for (int32_t a = 0; a < k; ++a) sigma[o + a] = u;
    }
}

__global__ void k_reset_q(int64_t Qp, float* R, float* S, float* rtilde) {
    const int64_t q = gid();
    if (q >= Qp) return;
    R[q] = 0.0f;
    S[q] = 0.0f;
    rtilde[q] = 0.0f;
}

__global__ void k_reset_h(int64_t Hp, float* pibar) {
    const int64_t h = gid();
    if (h < Hp) pibar[h] = 0.0f;
}

__global__ void k_reset_nodes(int64_t N, const int8_t* node_player, const float* payoff,
                              float* value, float* reach) {
    const int64_t v = gid();
    if (v >= N) return;
    value[v] = node_player[v] < 0 ? payoff[v] : 0.0f;
    if (v == 0) {
        reach[0] = 1.0f;
        reach[N] = 1.0f;
        reach[2 * N] = 1.0f;
    }
}

__global__ void k_copy_tail(int64_t Q0, const float* src, float* dst) {
    const int64_t i = gid();
    if (i < Q0) dst[i] = src[i];
}

__global__ void k_regret_match(int64_t Hp, const int32_t* q_offset, const float* R, float* sigma) {
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
__global__ void k_reach_level(int32_t lo, int32_t hi, int64_t N, const int32_t* __restrict__ parent,
                              const int8_t* __restrict__ node_player,
                              const int32_t* __restrict__ node_edge, const float* __restrict__ prob,
                              float* __restrict__ reach) {
    const int64_t v = lo + gid();
    if (v >= hi) return;
    if (node_player[v] < 0) return;
    const int32_t p = parent[v];
    const float s = prob[node_edge[v]];
    const int8_t who = node_player[p];  // 0 chance, 1, 2
    float r1 = reach[p], r2 = reach[N + p], rc = reach[2 * N + p];
    if (who == 1) r1 *= s;
    else if (who == 2) r2 *= s;
    else rc *= s;
    reach[v] = r1;
    reach[N + v] = r2;
    reach[2 * N + v] = rc;
}

// Bottom-up values of one level (Eq. expected_payoffs_matrix_recurrence) fused with the
// node -> infoset-action reductions: for a node d of player i with value u and children
// values w_a, r~(h, a) += sgn_i * pi_{-i}(d) * (w_a - u) (the multiplied-out form of
// Eq. instantaneous_counterfactual_regret, with u_2 = -u_1) and pibar(h) += pi_i(d)
// (Eq. player_reach_probability, own-reach reading).
__global__ void k_value_level(int32_t lo, int32_t hi, int64_t N,
                              const int32_t* __restrict__ child_begin,
                              const int8_t* __restrict__ node_player,
                              const int32_t* __restrict__ node_infoset,
                              const int32_t* __restrict__ node_edge,
                              const float* __restrict__ prob, float* __restrict__ value,
                              const float* __restrict__ reach, float* __restrict__ rtilde,
                              float* __restrict__ pibar) {
    const int64_t p = lo + gid();
    if (p >= hi) return;
    const int8_t who = node_player[p];
    if (who < 0) return;
    const int32_t c0 = child_begin[p], c1 = child_begin[p + 1];
    float u = 0.0f;
    for (int32_t c = c0; c < c1; ++c) u = fmaf(prob[node_edge[c]], value[c], u);
    value[p] = u;
    if (who == 0) return;
    const float r1 = reach[p], r2 = reach[N + p], rc = reach[2 * N + p];
    const float cf = (who == 1 ? r2 : r1) * rc;
    const float w = who == 1 ? cf : -cf;
    for (int32_t c = c0; c < c1; ++c)
        unsafeAtomicAdd(&rtilde[node_edge[c]], w * (value[c] - u));
    unsafeAtomicAdd(&pibar[node_infoset[p]], who == 1 ? r1 : r2);
}

// Infoset pass: regret update (vanilla R += r~, CFR+ R = max(R + r~, 0), discounted
// R = (R + r~) * d+ or d-; Eq. average_counterfactual_regrets_vector in cumulative form),
// average-strategy accumulation S += w_T * pibar * sigma (discounted: then S *= d_avg; Eq.
// average_strategy_profile_vector in cumulative form), then regret matching for the next
// strategy, for the infosets of the pass's players. Clears the accumulators of all.
__global__ void k_infoset_update(int64_t Hp, const int32_t* __restrict__ q_offset,
                                 const int8_t* __restrict__ infoset_player,
                                 float* __restrict__ R, float* __restrict__ S,
                                 float* __restrict__ sigma, float* __restrict__ rtilde,
                                 float* __restrict__ pibar, const int64_t* __restrict__ T,
                                 UpdateRule rule) {
    const int64_t h = gid();
    if (h >= Hp) return;
    const int32_t o = q_offset[h], k = q_offset[h + 1] - o;
    const float t = static_cast<float>(*T + 1);
    float wt = rule.linear ? t : 1.0f;
    float d_pos = 1.0f, d_neg = 1.0f, d_avg = 1.0f;
    if (rule.variant == 2) {
        wt = 1.0f;
        dcfr_discounts(rule, t, d_pos, d_neg, d_avg);
    }
    const float pb = pibar[h];
    pibar[h] = 0.0f;
    if (!((rule.players >> (infoset_player[h] - 1)) & 1)) {
        for (int32_t a = 0; a < k; ++a) rtilde[o + a] = 0.0f;
        return;
    }
    for (int32_t a = 0; a < k; ++a) {
        const int32_t q = o + a;
        float r = R[q] + rtilde[q];
        if (rule.variant == 1) r = fmaxf(r, 0.0f);
        else if (rule.variant == 2) r *= r > 0.0f ? d_pos : d_neg;
        R[q] = r;
        const float sn = fmaf(wt * pb, sigma[q], S[q]);
        S[q] = rule.variant == 2 ? sn * d_avg : sn;
        rtilde[q] = 0.0f;
    }
    regret_match(R, sigma, o, k);
}

// Average strategy: S normalised per infoset, uniform where its sum is 0.
__global__ void k_average(int64_t Hp, const int32_t* __restrict__ q_offset,
                          const float* __restrict__ S, float* __restrict__ avg) {
    const int64_t h = gid();
    if (h >= Hp) return;
    const int32_t o = q_offset[h], k = q_offset[h + 1] - o;
    float sum = 0.0f;
    for (int32_t a = 0; a < k; ++a) sum += S[o + a];
    if (sum > 0.0f) {
        for (int32_t a = 0; a < k; ++a) avg[o + a] = S[o + a] / sum;
    } else {
        const float u = 1.0f / static_cast<float>(k);
        for (int32_t a = 0; a < k; ++a) avg[o + a] = u;
    }
}

// ---- best response (Section 2.2): the responder i maximises, everyone else plays avgprob

__global__ void k_br_terminal(int64_t N, const int8_t* __restrict__ node_player,
                              const float* __restrict__ payoff, float sgn, float* __restrict__ br_value,
                              float* __restrict__ br_reach) {
    const int64_t v = gid();
    if (v >= N) return;
    br_value[v] = node_player[v] < 0 ? sgn * payoff[v] : 0.0f;
    if (v == 0) br_reach[0] = 1.0f;
}

// pi_{-i}: product of chance and opponent edge probabilities (decision nodes only).
__global__ void k_br_reach_level(int32_t lo, int32_t hi, int player,
                                 const int32_t* __restrict__ parent,
                                 const int8_t* __restrict__ node_player,
                                 const int32_t* __restrict__ node_edge,
                                 const float* __restrict__ avgprob, float* __restrict__ br_reach) {
    const int64_t v = lo + gid();
    if (v >= hi) return;
    if (node_player[v] < 0) return;
    const int32_t p = parent[v];
    const float f = node_player[p] == player ? 1.0f : avgprob[node_edge[v]];
    br_reach[v] = br_reach[p] * f;
}

// a*(h) = argmax_a sum_{d in h} pi_{-i}(d) V(child(d, a)), lowest index on ties.
__global__ void k_br_choose(int32_t hlo, int32_t hhi, int player,
                            const int8_t* __restrict__ infoset_player,
                            const int32_t* __restrict__ q_offset,
                            const int32_t* __restrict__ member_offset,
                            const int32_t* __restrict__ members,
                            const int32_t* __restrict__ child_begin,
                            const float* __restrict__ br_reach, const float* __restrict__ br_value,
                            int32_t* __restrict__ best) {
    const int64_t h = hlo + gid();
    if (h >= hhi) return;
    if (infoset_player[h] != player) return;
    const int32_t k = q_offset[h + 1] - q_offset[h];
    const int32_t m0 = member_offset[h], m1 = member_offset[h + 1];
    int32_t a_star = 0;
    float v_star = 0.0f;
    for (int32_t a = 0; a < k; ++a) {
        float tot = 0.0f;
        for (int32_t m = m0; m < m1; ++m) {
            const int32_t d = members[m];
            tot = fmaf(br_reach[d], br_value[child_begin[d] + a], tot);
        }
        if (a == 0 || tot > v_star) {
            v_star = tot;
            a_star = a;
        }
    }
    best[h] = a_star;
}

__global__ void k_br_value_level(int32_t lo, int32_t hi, int player,
                                 const int32_t* __restrict__ child_begin,
                                 const int8_t* __restrict__ node_player,
                                 const int32_t* __restrict__ node_infoset,
                                 const int32_t* __restrict__ node_edge,
                                 const float* __restrict__ avgprob, const int32_t* __restrict__ best,
                                 float* __restrict__ br_value) {
    const int64_t p = lo + gid();
    if (p >= hi) return;
    const int8_t who = node_player[p];
    if (who < 0) return;
    const int32_t c0 = child_begin[p], c1 = child_begin[p + 1];
    if (who == player) {
        br_value[p] = br_value[c0 + best[node_infoset[p]]];
        return;
    }
    float u = 0.0f;
    for (int32_t c = c0; c < c1; ++c) u = fmaf(avgprob[node_edge[c]], br_value[c], u);
    br_value[p] = u;
}

__global__ void k_br_store(const float* __restrict__ br_value, double* out) {
    if (gid() == 0) *out = static_cast<double>(br_value[0]);
}

__global__ void k_scatter_q(int64_t Qp, const int32_t* __restrict__ q_input,
                            const float* __restrict__ src, float* __restrict__ dst) {
    const int64_t q = gid();
    if (q < Qp) dst[q_input[q]] = src[q];
}

__global__ void k_gather_q(int64_t Qp, const int32_t* __restrict__ q_input,
                           const float* __restrict__ src, float* __restrict__ dst) {
    const int64_t q = gid();
    if (q < Qp) dst[q] = src[q_input[q]];
}

}  // namespace

void launch_reset(const Dev& d, hipStream_t st, bool node_arrays) {
    if (d.Qp > 0) hipLaunchKernelGGL(k_reset_q, dim3(blocks_for(d.Qp)), dim3(kBlock), 0, st, d.Qp,
                                     d.R, d.S, node_arrays ? d.rtilde : d.stage);
    if (d.Hp > 0 && node_arrays)
        hipLaunchKernelGGL(k_reset_h, dim3(blocks_for(d.Hp)), dim3(kBlock), 0, st, d.Hp, d.pibar);
    if (node_arrays)
        hipLaunchKernelGGL(k_reset_nodes, dim3(blocks_for(d.N)), dim3(kBlock), 0, st, d.N,
                           d.node_player, d.payoff, d.value, d.reach);
    if (d.Q0 > 0)
        hipLaunchKernelGGL(k_copy_tail, dim3(blocks_for(d.Q0)), dim3(kBlock), 0, st, d.Q0,
                           d.prob + d.Qp, d.avgprob + d.Qp);
    hipLaunchKernelGGL(k_set_T, dim3(1), dim3(64), 0, st, d.T, int64_t{0});
    launch_regret_match(d, st);
}

void launch_regret_match(const Dev& d, hipStream_t st) {
    if (d.Hp > 0)
        hipLaunchKernelGGL(k_regret_match, dim3(blocks_for(d.Hp)), dim3(kBlock), 0, st, d.Hp,
                           d.sq_offset, d.R, d.prob);
}

void launch_set_T(const Dev& d, int64_t value, hipStream_t st) {
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

void launch_iteration(const Dev& d, const int32_t* lo, const UpdateRule& rule, hipStream_t st,
                      LaunchTimer* timer) {
    auto pre = [&](int k, int l, int64_t n) { if (timer) timer->before(k, l, n, st); };
    auto post = [&](int k) { if (timer) timer->after(k, st); };
    // top-down: levels 1 .. D-1 (level D holds terminals only)
    for (int32_t l = 1; l < d.D; ++l) {
        const int32_t a = lo[l], b = lo[l + 1];
        pre(K_REACH, l, b - a);
        hipLaunchKernelGGL(k_reach_level, dim3(blocks_for(b - a)), dim3(kBlock), 0, st, a, b, d.N,
                           d.parent, d.node_player, d.node_edge, d.prob, d.reach);
        post(K_REACH);
    }
    // bottom-up: levels D-1 .. 0
    for (int32_t l = d.D - 1; l >= 0; --l) {
        const int32_t a = lo[l], b = lo[l + 1];
        pre(K_VALUE, l, b - a);
        hipLaunchKernelGGL(k_value_level, dim3(blocks_for(b - a)), dim3(kBlock), 0, st, a, b, d.N,
                           d.child_begin, d.node_player, d.node_infoset, d.node_edge, d.prob,
                           d.value, d.reach, d.rtilde, d.pibar);
        post(K_VALUE);
    }
    if (d.Hp > 0) {
        pre(K_INFOSET, -1, d.Hp);
        hipLaunchKernelGGL(k_infoset_update, dim3(blocks_for(d.Hp)), dim3(kBlock), 0, st, d.Hp,
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

void launch_average(const Dev& d, hipStream_t st) {
    if (d.Hp > 0)
        hipLaunchKernelGGL(k_average, dim3(blocks_for(d.Hp)), dim3(kBlock), 0, st, d.Hp, d.sq_offset,
                           d.S, d.avgprob);
}

void launch_best_response(const Dev& d, const int32_t* lo, const int32_t* hlo, int player,
                          hipStream_t st) {
    const float sgn = player == 1 ? 1.0f : -1.0f;
    hipLaunchKernelGGL(k_br_terminal, dim3(blocks_for(d.N)), dim3(kBlock), 0, st, d.N,
                       d.node_player, d.payoff, sgn, d.br_value, d.br_reach);
    for (int32_t l = 1; l < d.D; ++l) {
        const int32_t a = lo[l], b = lo[l + 1];
        hipLaunchKernelGGL(k_br_reach_level, dim3(blocks_for(b - a)), dim3(kBlock), 0, st, a, b,
                           player, d.parent, d.node_player, d.node_edge, d.avgprob, d.br_reach);
    }
    for (int32_t l = d.D - 1; l >= 0; --l) {
        const int32_t ha = hlo[l], hb = hlo[l + 1];
        if (hb > ha)
            hipLaunchKernelGGL(k_br_choose, dim3(blocks_for(hb - ha)), dim3(kBlock), 0, st, ha, hb,
                               player, d.infoset_player, d.q_offset, d.member_offset, d.members,
                               d.child_begin, d.br_reach, d.br_value, d.best);
        const int32_t a = lo[l], b = lo[l + 1];
        hipLaunchKernelGGL(k_br_value_level, dim3(blocks_for(b - a)), dim3(kBlock), 0, st, a, b,
                           player, d.child_begin, d.node_player, d.node_infoset, d.node_edge,
                           d.avgprob, d.best, d.br_value);
    }
    hipLaunchKernelGGL(k_br_store, dim3(1), dim3(64), 0, st, d.br_value, d.out2 + (player - 1));
}

void launch_scatter_q(const Dev& d, const float* src, float* dst, hipStream_t st) {
    if (d.Qp > 0)
        hipLaunchKernelGGL(k_scatter_q, dim3(blocks_for(d.Qp)), dim3(kBlock), 0, st, d.Qp,
                           d.sq_input, src, dst);
}

void launch_gather_q(const Dev& d, const float* src, float* dst, hipStream_t st) {
    if (d.Qp > 0)
        hipLaunchKernelGGL(k_gather_q, dim3(blocks_for(d.Qp)), dim3(kBlock), 0, st, d.Qp,
                           d.sq_input, src, dst);
}

}  // namespace cfr
