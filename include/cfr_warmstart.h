/*
 * cfr_warmstart.h - learned warm start of CFR on MI355X (gfx950).
 *
 * Not part of the paper's method (which starts from uniform strategies, Section 3.1): a
 * three-layer perceptron maps infoset features to a distribution over action slots, and the
 * warm start turns it into initial cumulative regrets. Weights are BF16 on MFMA with FP32
 * accumulation; FP32 master weights are updated by Adam. Plain CFR from zero regrets remains
 * the fallback, and exploitability (cfr_exploitability*) judges the result.
 *
 * Conventions as in cfr.h: CFR_OK or a negative code, message in cfr_last_error(); the caller
 * owns the device workspace and the stream; "device" pointers are device memory.
 */
#ifndef CFR_MI355X_WARMSTART_H
#define CFR_MI355X_WARMSTART_H

#include "cfr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cfr_mlp cfr_mlp;

/* Parameters, FP32, in the order W1 [in x hidden], b1 [hidden], W2 [hidden x hidden], b2,
 * W3 [hidden x outputs], b3 [outputs], matrices row-major (input index first). */
int64_t cfr_mlp_num_params(int32_t in_features, int32_t hidden, int32_t outputs);
/* Device bytes for a network training on batches of at most max_batch rows. */
int64_t cfr_mlp_workspace_bytes(int32_t in_features, int32_t hidden, int32_t outputs,
                                int32_t max_batch);
int cfr_mlp_create(int32_t in_features, int32_t hidden, int32_t outputs, int32_t max_batch,
                   void* workspace, size_t bytes, void* stream, cfr_mlp** out);
/* Host FP32 parameters in and out (set also resets Adam's moments and step). */
int cfr_mlp_set_params(cfr_mlp* net, const float* params, int64_t n);
int cfr_mlp_get_params(cfr_mlp* net, float* params, int64_t n);
/* logits [batch x outputs] (device FP32) = network(x [batch x in_features], device BF16). */
int cfr_mlp_forward(cfr_mlp* net, const void* x, int32_t batch, float* logits);
/* One Adam step on the masked softmax cross-entropy -(1/B) sum mask * target * log p, p the
 * softmax of the logits over slots with mask > 0. target and mask: device FP32 [batch x
 * outputs]. Writes the batch loss to *loss (host) and keeps the gradient for cfr_mlp_get_grads.
 * Synchronises. */
int cfr_mlp_train_step(cfr_mlp* net, const void* x, const float* target, const float* mask,
                       int32_t batch, float lr, float* loss);
int cfr_mlp_get_grads(cfr_mlp* net, float* grads, int64_t n);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the forward pass of cfr_mlp_forward, same kernels
 * and the same logits bit for bit, with the two hidden activations in a file-scope device
 * array of 16 MiB (one per GPU the library runs on, held until the process ends) instead of
 * the network's workspace, and the logits written directly to `logits` (device FP32
 * [batch x outputs]). batch x hidden may be at most 4,194,304 (CFR_EINVAL otherwise; e.g.
 * 16,384 rows at hidden 256). No call allocates or frees memory; the array's address is
 * looked up once per device, on the first call with that device current (call with the
 * device of the network's stream current). Enqueued on the network's stream. Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams, other threads,
 * other networks) race and must be ordered by the caller. */
int cfr_mlp_forward_noalloc(cfr_mlp* net, const void* x, int32_t batch, float* logits);
int cfr_mlp_destroy(cfr_mlp* net);

/* Feature extractor for poker subgames: n descriptors (16 int16 fields each: player, own
 * rank, round, 3 board ranks, raises, last action, own and opponent commitment, stack, legal
 * slot mask, depth, raise cap, ranks, game index) and per-game root beliefs [games x 2 x 13]
 * (player 1's then player 2's range over ranks) -> x [n x in_features] BF16. Device pointers. */
int cfr_features(const int16_t* desc, const float* beliefs, int64_t n, int32_t in_features,
                 void* x, void* stream);
/* Masked softmax of logits [n x outputs] over each descriptor's legal slots, written to pair
 * order: the a-th legal slot of infoset i goes to probs[q_off[i] + a]. Device pointers. */
int cfr_probs_to_pairs(const float* logits, const int16_t* desc, const int64_t* q_off, int64_t n,
                       int32_t outputs, float* probs, void* stream);
/* Warm start: with the solver's current cumulative regrets R (typically after one iteration
 * from zero), set R(h, a) = weight * m(h) * probs[q] with m(h) = sum_a max(R(h, a), 0) and q the
 * caller's pair index, S = 0, T = 0, sigma = regret matching of R. probs: device, n_q entries,
 * the solver's input pair order. Enqueued on the solver's stream. */
int cfr_warm_start(cfr_solver* s, const float* probs, int64_t n_q, float weight);

#ifdef __cplusplus
}
#endif
#endif /* CFR_MI355X_WARMSTART_H */
