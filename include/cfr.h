/*
 * cfr.h - C ABI of the MI355X (gfx950) counterfactual regret minimisation library.
 *
 * One CFR iteration over a finite two-player zero-sum extensive-form game,
 * computed level by level over a flattened tree (Kim, "GPU-Accelerated
 * Counterfactual Regret Minimization", Section 3). The calls follow the
 * paper's statement of the problem: the game is the tuple of Definition 1
 * (Section 2.1); an iteration computes the expected payoffs of Eq.
 * (expected_payoff), the excepted and player reach probabilities of Eqs.
 * (excepted_reach_probability, player_reach_probability), the instantaneous
 * counterfactual regrets of Eq. (instantaneous_counterfactual_regret), the
 * average strategy of Eq. (average_strategy_profile) and the next strategy of
 * Eq. (next_strategy_profile); exploitability judges the average strategy
 * against the Nash condition of Section 2.2.
 *
 * Conventions for every call
 *  - Return value: CFR_OK (0) or a negative CFR_E* code; the thread-local
 *    message of the last failure is cfr_last_error(). No exception crosses
 *    the ABI. Errors of asynchronous GPU work surface at the next call that
 *    synchronises (average strategy to host, state export, exploitability).
 *  - Host arrays passed in are borrowed for the duration of the call and
 *    copied; the library keeps no pointer to them.
 *  - Device memory: the caller owns the workspace (cfr_plan reports its
 *    size); the solver lives inside it and owns only host metadata, events and
 *    the captured iteration graph. The workspace must stay allocated until
 *    cfr_destroy returns.
 *  - Streams: all GPU work of a solver is ordered on the hipStream_t given to
 *    cfr_build (may be the null stream).
 *  - Infoset-action pairs ("q") are numbered as in the input: rational-player
 *    infosets in increasing input id, actions in index order (the set Q_+ of
 *    Section 2.1).
 */
#ifndef CFR_MI355X_H
#define CFR_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CFR_OK 0
#define CFR_EINVAL (-1)   /* null pointer, bad size or bad enum value */
#define CFR_ENOTTREE (-2) /* no unique root, a cycle, an unreachable node, or a terminal/decision mismatch */
#define CFR_EACTION (-3)  /* f_a is not a bijection onto A(h), or an infoset is inconsistent */
#define CFR_ECHANCE (-4)  /* a chance probability < 0, or one chance infoset not summing to 1 (+-1e-9) */
#define CFR_EZEROSUM (-5) /* payoff_u1 + payoff_u2 != 0 at a terminal */
#define CFR_ELEVEL (-6)   /* an infoset spans several depths (exploitability needs level-pure infosets) */
#define CFR_ENOMEM (-7)   /* workspace too small */
#define CFR_ESTATE (-8)   /* state size mismatch */
#define CFR_EHIP (-9)     /* HIP runtime error; the message carries hipGetErrorString */

/* The game tuple <T, H, f_h, A, f_a, I, f_i, sigma_0, u> of Definition 1 (Section 2.1).
 * Node and infoset ids are arbitrary; the library canonicalises them. */
typedef struct cfr_game {
    int64_t n_nodes;
    const int32_t* parent;              /* [n_nodes] parent function f_Pa; -1 at the root */
    const int32_t* node_infoset;        /* [n_nodes] f_h; -1 at terminal nodes */
    const int32_t* node_action;         /* [n_nodes] index of the edge into the node within
                                           A(f_h(parent)), 0..|A|-1; -1 at the root */
    int32_t n_infosets;
    const int8_t* infoset_player;       /* [n_infosets] f_i: 0 chance, 1 or 2 */
    const int32_t* infoset_num_actions; /* [n_infosets] |A(h)| */
    const double* chance_prob;          /* sigma_0: chance infosets in increasing id order,
                                           |A(h)| probabilities each, in action order */
    const double* payoff_u1;            /* [n_nodes] u(t, 1); read at terminals only */
    const double* payoff_u2;            /* optional [n_nodes] u(t, 2), checked for zero sum */
} cfr_game;

/* Regret update of iteration t (1-based), r~ its instantaneous regrets:
 *   CFR_VANILLA  R += r~                                  (Eq. average_counterfactual_regret,
 *                                                          as a sum)
 *   CFR_PLUS     R = max(R + r~, 0)
 *   CFR_DCFR     R = (R + r~) * t^a / (t^a + 1) where R + r~ > 0, else (R + r~) * t^b / (t^b + 1);
 *                and the strategy sums S = (S + pibar * sigma) * (t / (t + 1))^g
 * The discounted variant is the weighting scheme the paper's discussion (Section 5) says
 * applies by altering the average-regret and average-strategy equations; a, b, g are
 * cfr_config.dcfr_alpha, dcfr_beta, dcfr_gamma. */
enum { CFR_VANILLA = 0, CFR_PLUS = 1, CFR_DCFR = 2 };
enum { CFR_AVG_DEFAULT = -1, CFR_AVG_UNIFORM = 0, CFR_AVG_LINEAR = 1 };
/* Averaging weight of iteration t (1-based): 1 (uniform, Eq. average_strategy_profile) or t
 * (linear). DEFAULT = uniform for vanilla, linear for CFR+; CFR_DCFR takes DEFAULT only (its
 * gamma discount sets the weights). */

#define CFR_FLAG_NO_GRAPH 1u    /* enqueue kernels directly instead of replaying a captured graph */
#define CFR_FLAG_NODE_ENGINE 2u  /* use the breadth-first node engine even where the public-block
                                    engine applies (level-pure infosets, at most 16 actions) */
#define CFR_FLAG_ALTERNATING 4u  /* alternating updates (the schedule of the cited CFR+ work): an
                                    iteration is a pass that updates player 1's infosets, then a
                                    pass, under player 1's new strategy, that updates player 2's,
                                    both with the same t; default: both players in one pass. */
#define CFR_FLAG_KEEP_NODE_VALUES 8u /* the subtree-pack launch (which keeps the values and reaches
                                    of the nodes below its first level on chip) also stores them,
                                    so that cfr_get_node_values can read every node; without it
                                    cfr_get_node_values returns CFR_EINVAL for a game with packs. */
#define CFR_FLAG_SUBTREE_PACKS 16u /* the public-block engine with subtree packs (below): the
                                    highest blocks whose subtrees fit one workgroup's LDS, tier by
                                    tier, run in pack launches instead of the per-level launches
                                    (at most 4 actions per infoset; otherwise ignored). */
#define CFR_FLAG_FP64 32u          /* values, probabilities, reaches, R and S in double precision
                                    (the paper's 64-bit GPU variant, Section 4.1): the node engine
                                    with every kernel instantiated for double, payoffs and chance
                                    probabilities taken from the input's doubles. Strategies, state
                                    and node values are read and written with the _f64 calls (their
                                    float twins return CFR_EINVAL on such a solver, and the _f64
                                    calls on an FP32 one); exploitability as usual. Not with
                                    CFR_FLAG_SUBTREE_PACKS, nor for a batch (CFR_EINVAL).
                                    Other flag bits: CFR_EINVAL */

typedef struct cfr_config {
    int32_t variant;   /* CFR_VANILLA, CFR_PLUS or CFR_DCFR */
    int32_t averaging; /* CFR_AVG_* */
    uint32_t flags;    /* CFR_FLAG_* */
    float dcfr_alpha;  /* CFR_DCFR only: exponents, finite and in [-64, 64] (EINVAL otherwise); */
    float dcfr_beta;   /* the weighting work recommends 1.5, 0 and 2; 1, 1, 1 is linear CFR */
    float dcfr_gamma;
    int32_t reserved[2];
} cfr_config;

/* Sizes of the game in the columns of the paper's game-properties table (Appendix). */
typedef struct cfr_plan_info {
    int64_t n_nodes;
    int64_t n_terminals;
    int64_t n_infosets;        /* rational-player infosets H_+ */
    int64_t n_q;               /* infoset-action pairs Q_+ */
    int64_t n_chance_infosets;
    int64_t n_chance_q;
    int32_t max_actions;
    int32_t depth;             /* D: deepest level */
    int32_t level_pure;        /* 1 if every infoset lies on one level */
    int32_t engine;            /* 0: breadth-first node engine, 1: public-block engine */
    int64_t workspace_bytes;   /* device bytes cfr_build needs */
} cfr_plan_info;

typedef struct cfr_solver cfr_solver;

/* Validate the game (see the error codes) and report its sizes and the workspace size. */
int cfr_plan(const cfr_game* game, const cfr_config* config, cfr_plan_info* out);

/* Flatten the game into the canonical level-ordered layout on the host, copy it into
 * `workspace` (device memory of at least `bytes`), set T = 0, R = S = 0 and sigma uniform
 * (Section 3.1, initial strategy), and capture the iteration. `stream` is a hipStream_t. */
int cfr_build(const cfr_game* game, const cfr_config* config, void* workspace, size_t bytes,
              void* stream, cfr_solver** out);

/* Enqueue n iterations (Section 3.2) on the solver's stream; does not synchronise. */
int cfr_iterate(cfr_solver* s, int32_t n);

/* Run n iterations with direct launches and a pair of hipEvents around every kernel launch on
 * the solver's stream (synchronises). kernel_ms[k] receives the summed event time of kernel
 * kind k over the n iterations and kernel_launches[k] its launch count, for k < n_kinds;
 * cfr_kernel_name(k) names kind k (empty string past the last kind). The results of the
 * iterations are the same as cfr_iterate's. */
int cfr_iterate_timed(cfr_solver* s, int32_t n, double* kernel_ms, int64_t* kernel_launches,
                      int32_t n_kinds);
const char* cfr_kernel_name(int32_t kind);

/* Like cfr_iterate_timed but per launch: after n iterations, for each of the *n_launches
 * launches of one iteration (in launch order, up to max_launches are written), the summed
 * event time over the n iterations, its kernel kind (cfr_kernel_name), the tree level it
 * processes (-1: the single-workgroup launch of the first levels; -2: the launch that takes
 * several small top-down levels at once) and its number of work items. Synchronises. */
int cfr_iterate_profile(cfr_solver* s, int32_t n, double* launch_ms, int32_t* launch_kind,
                        int32_t* launch_level, int64_t* launch_units, int32_t max_launches,
                        int32_t* n_launches);

/* Launch shapes of the public-block engine, per bucket b = min(floor(log2 u), 31) of a
 * launch's work items u (top-down: the level's decision nodes; bottom-up: the level's infoset
 * members). The single-workgroup launches of the first levels and the multi-level top-down
 * launch have fixed shapes.
 * A top-down launch uses reach_threads[b] threads per workgroup (a multiple of 64 in
 * [64, 1024]), each thread taking reach_nodes[b] nodes (1, 2 or 4). The bottom-up launch packs
 * whole infosets into chunks of at most up_threads[b] * up_members[b] members, one workgroup of
 * up_threads[b] threads (64, 128, 256 or 512) per chunk, each thread taking up_members[b]
 * members (1 or 2). The results do not depend on the shape (each infoset sums its members'
 * contributions in member order), except for an infoset larger than a chunk. */
typedef struct cfr_launch_shape {
    int32_t up_threads[32];
    int32_t up_members[32];
    int32_t reach_threads[32];
    int32_t reach_nodes[32];
} cfr_launch_shape;

/* Fills `out` with the library's default shapes. */
void cfr_default_launch_shape(cfr_launch_shape* out);

/* Sets the launch shapes (NULL: the defaults) and re-captures the iteration graph.
 * CFR_EINVAL for a value outside the ranges above, or for the node engine. */
int cfr_set_launch_shape(cfr_solver* s, const cfr_launch_shape* shape);

/* Average strategy sigma-bar = S / sum_a S per infoset, uniform where that sum is 0
 * (Eq. average_strategy_profile), written to out[q] for the n_q pairs in input order.
 * out_on_device != 0: `out` is device memory, the call enqueues and returns;
 * otherwise `out` is host memory and the call synchronises. */
int cfr_average_strategy(cfr_solver* s, float* out, int64_t n_q, int out_on_device);

/* Current strategy sigma^(T+1) = regret matching of R (Eq. next_strategy_profile): the
 * strategy the next iteration will play, in input pair order. Same memory convention as
 * cfr_average_strategy. */
int cfr_current_strategy(cfr_solver* s, float* out, int64_t n_q, int out_on_device);

/* The same two for a solver built with CFR_FLAG_FP64, in double precision. */
int cfr_average_strategy_f64(cfr_solver* s, double* out, int64_t n_q, int out_on_device);
int cfr_current_strategy_f64(cfr_solver* s, double* out, int64_t n_q, int out_on_device);

/* Best-response values of both players against the average strategy and the
 * exploitability (BR_1 + BR_2) / 2 (Section 2.2). Synchronises. Needs level-pure
 * infosets (CFR_ELEVEL otherwise). br_value may be NULL. */
int cfr_exploitability(cfr_solver* s, double* expl, double br_value[2]);

/* Solver state in input pair order: T (iterations done), cumulative regrets R and
 * cumulative average-strategy weights S (R / T is the average regret of Eq.
 * average_counterfactual_regret). Host arrays; both calls synchronise. */
int cfr_get_state(cfr_solver* s, int64_t* T, float* R, float* S, int64_t n_q);
int cfr_set_state(cfr_solver* s, int64_t T, const float* R, const float* S, int64_t n_q);
/* The same for a solver built with CFR_FLAG_FP64, in double precision. */
int cfr_get_state_f64(cfr_solver* s, int64_t* T, double* R, double* S, int64_t n_q);
int cfr_set_state_f64(cfr_solver* s, int64_t T, const double* R, const double* S, int64_t n_q);

/* Canonical layout export for checking (host copy, synchronises). `name` is one of
 * level_offset, node_id, parent, child_begin, node_player, node_infoset, node_edge,
 * infoset_id, infoset_player, q_offset, chance_id, cq_offset, member_offset, members,
 * chance_prob, payoff, q_input; or reach_launch: int32 per level 0 .. D, which launch of an
 * iteration computes the level's reach (0: none, the roots and levels without decision nodes;
 * 1: the single-workgroup launch of the first levels; 2: the launch that walks several small
 * levels up to the last stored one; 3: a launch of its own; 4: the
 * level's bottom-up launch, from the parents' reach; for a batch, the levels of its forest).
 * cfr_layout_bytes returns the size (< 0 for an unknown name, or for a batch any name but
 * reach_launch). */
int64_t cfr_layout_bytes(cfr_solver* s, const char* name);
int cfr_get_layout(cfr_solver* s, const char* name, void* out, int64_t bytes);

/* Per-node values of the last iteration in canonical node order (host, synchronises):
 * u1[v] = expected payoff of player 1 (Eq. expected_payoff) and reach[3 * v + k] =
 * product of player 1's (k = 0), player 2's (k = 1) and chance's (k = 2) edge
 * probabilities from the root, for decision nodes (terminal entries are unspecified).
 * Either pointer may be NULL. */
int cfr_get_node_values(cfr_solver* s, float* u1, float* reach, int64_t n_nodes);
/* The same for a solver built with CFR_FLAG_FP64, in double precision. */
int cfr_get_node_values_f64(cfr_solver* s, double* u1, double* reach, int64_t n_nodes);

/* General-sum games of n rational players (Section 3.1 writes the payoff matrix and the
 * expected-payoff recurrence with one column per rational player of I+; Table tab:properties
 * of the appendix lists a three-player game). `game` describes the tree, the infosets and
 * chance as for cfr_plan, with infoset_player in 0 (chance) .. n_players; its payoff_u1 and
 * payoff_u2 are ignored. payoff (host, n_nodes * n_players doubles, node-major in input node
 * order): u(t, i) at payoff[t * n_players + (i - 1)], read at terminals only and required
 * finite there. 2 <= n_players <= 8. The solver runs the node engine (FP32, or FP64 with
 * CFR_FLAG_FP64) with every player's infosets updated in one pass (CFR_FLAG_ALTERNATING: a
 * pass per player in seat order, each under the strategies the earlier passes produced, the
 * iteration counted by the last): at a node d of player i in
 * infoset h the regret r~(h, a) gathers pi_{-i}(d) (w_a[i] - u[i]), pi_{-i} the product of
 * chance's and the other players' reaches, and u the node's payoff vector. No step adds by
 * atomics, so the results do not depend on scheduling: the same game, configuration and state
 * give the same bits on every run. cfr_iterate,
 * cfr_get_state / cfr_set_state, cfr_average_strategy, cfr_current_strategy (and their _f64
 * forms), cfr_get_layout and cfr_destroy apply unchanged. cfr_exploitability returns
 * CFR_EINVAL (Section 2.2 defines it for two-player zero-sum games), as do cfr_get_node_values
 * and cfr_set_launch_shape. Config: CFR_FLAG_SUBTREE_PACKS gives CFR_EINVAL. Errors: those of cfr_plan / cfr_build, CFR_EINVAL for n_players out of range, a
 * null payoff or a payoff that is not finite at a terminal. Workspace ownership as in
 * cfr_build. */
int cfr_plan_n(const cfr_game* game, int32_t n_players, const double* payoff,
               const cfr_config* config, cfr_plan_info* out);
int cfr_build_n(const cfr_game* game, int32_t n_players, const double* payoff,
                const cfr_config* config, void* workspace, size_t bytes, void* stream,
                cfr_solver** out);
/* Per-node payoff vectors and reaches of the last iteration of a general-sum solver, canonical
 * node order, in double precision whatever the solver's: values[v * n + (i - 1)] = u(v, i), the
 * expected payoff of player i at node v (a terminal's payoff), and reach[v * (n + 1) + k] =
 * player k + 1's reach for k < n, chance's for k = n (host, synchronises; either may be NULL).
 * CFR_EINVAL for a two-player zero-sum solver or n_nodes that does not match. */
int cfr_get_node_values_n(cfr_solver* s, double* values, double* reach, int64_t n_nodes);

/* Subtree-partitioned, out-of-core iteration (the memory relief the paper's discussion, Section 5,
 * proposes: the iteration computed over root-to-leaf partitions of the tree instead of all of it
 * at once). Levels 0 .. cut_level stay resident on the device; the subtrees hanging from the
 * level-cut nodes are grouped, in canonical order, into partitions of at most max_window_nodes
 * nodes below the cut (a larger subtree is a partition of its own), kept in pinned host memory
 * and streamed through one device window every iteration: the resident top-down pass, then per
 * partition its window copied in, its top-down and bottom-up passes (values, regrets and own
 * reaches added into the resident per-pair accumulators) and the bottom-up of its level-cut
 * nodes; the resident bottom-up; the infoset update. The arithmetic is the node engine's (FP32,
 * or FP64 with CFR_FLAG_FP64); device memory holds the resident levels, one window and the
 * per-pair state. cut_level in 1 .. depth - 1, max_window_nodes >= 1 (CFR_EINVAL otherwise);
 * flags: CFR_FLAG_ALTERNATING, CFR_FLAG_FP64 (CFR_FLAG_NO_GRAPH and CFR_FLAG_NODE_ENGINE are
 * implied; others CFR_EINVAL).
 * cfr_plan_partitioned reports the sizes as cfr_plan does (workspace_bytes: this solver's device
 * workspace), the number of partitions and the pinned host bytes the build allocates (either
 * pointer may be NULL). The solver takes cfr_iterate, cfr_iterate_timed (no per-kernel times),
 * the strategy and state calls (float or _f64 by precision) and cfr_destroy; cfr_exploitability,
 * cfr_get_node_values and the layout exports return CFR_EINVAL (the device never holds the whole
 * tree: move the state into an in-core solver of the same game to evaluate it). */
int cfr_plan_partitioned(const cfr_game* game, const cfr_config* config, int32_t cut_level,
                         int64_t max_window_nodes, cfr_plan_info* out, int32_t* n_partitions,
                         int64_t* host_bytes);
int cfr_build_partitioned(const cfr_game* game, const cfr_config* config, int32_t cut_level,
                          int64_t max_window_nodes, void* workspace, size_t bytes, void* stream,
                          cfr_solver** out);

/* Host-only flattening, for checking the canonical layout without a GPU: build the layout
 * of `game` on the host (validation as in cfr_plan), then read arrays by the names listed for
 * cfr_get_layout. For level-pure games the public-block execution plan is built too (with
 * subtree packs if flags holds CFR_FLAG_SUBTREE_PACKS; flags: 0 or that flag, else
 * CFR_EINVAL) and its arrays are readable as x_canon_of, x_parent, x_edge, x_meta, x_child_begin, x_child_stride,
 * x_child_list, x_infoset_canon, x_q_offset, x_member_offset, x_members, x_h_level_offset,
 * x_chance_nodes, x_c_level_offset, x_q_input; and the subtree packs: x_up_end, x_h_up_end,
 * x_c_up_end (per level, the end of the nodes, infosets and chance nodes that the per-level
 * launches take; the rest of the level is in packs), x_tier_offset (int32, tiers + 1 entries:
 * the packs of tier t are t_o[t - 1] .. t_o[t] - 1), x_packs (per pack, int32: tier, first
 * level, levels, decision nodes, members, chance nodes, roots, infosets, pairs, chance
 * children, then the offsets of its root, member, infoset, chance, chance-child and node
 * records in x_pack_blob, then 9 entries each of the per-level member and chance-node ranges) and x_pack_blob (the records: roots 4 words {decision
 * index | actor << 16, parent node, edge, node}; members 6 {decision index | k << 16 | player
 * 2 << 19 | external children << 20 | child kinds << 24 (2 bits each: 0 in the pack, 1
 * terminal payoff, 2 external node), first local pair, 4 children}; infosets 4 {first pair,
 * first local pair, first member | end member << 16, k | player << 8}; chance nodes 4
 * {decision index | external children << 20, k, first child record}; chance children 3
 * {child, probability, kind}; nodes 1 per decision index). The handle owns host memory
 * only. */
typedef struct cfr_host_layout cfr_host_layout;
int cfr_host_layout_create(const cfr_game* game, uint32_t flags, cfr_host_layout** out);
int64_t cfr_host_layout_bytes(const cfr_host_layout* layout, const char* name);
int cfr_host_layout_get(const cfr_host_layout* layout, const char* name, void* out, int64_t bytes);
int cfr_host_layout_destroy(cfr_host_layout* layout);
/* Host-only plan of a batch (the forest cfr_build_batch lays out, with the same validation and
 * errors as cfr_plan_batch): only the plan arrays (x_* names, and x_level_offset) are readable.
 * flags: 0 or CFR_FLAG_SUBTREE_PACKS (CFR_EINVAL otherwise). */
int cfr_host_layout_create_batch(const cfr_game* games, int32_t n_games, uint32_t flags,
                                 cfr_host_layout** out);

/* Batched solving: n_games independent games (e.g. the subgames of a larger game) solved
 * together. They are laid out as one forest, level-major (level l holds level l of every game,
 * in game order) over the public-block plan, so each level of every game is processed by one
 * launch and one iteration of all games is one graph replay. All games must have level-pure
 * infosets and at most 16 actions per infoset (CFR_ELEVEL / CFR_EINVAL otherwise). The batch
 * solver accepts cfr_iterate, cfr_iterate_timed, cfr_average_strategy, cfr_current_strategy,
 * cfr_get_state, cfr_set_state and cfr_destroy; infoset-action pairs are numbered by
 * concatenating the games' input pair orders (game 0 first). */
int cfr_plan_batch(const cfr_game* games, int32_t n_games, const cfr_config* config,
                   cfr_plan_info* out);
int cfr_build_batch(const cfr_game* games, int32_t n_games, const cfr_config* config,
                    void* workspace, size_t bytes, void* stream, cfr_solver** out);
/* Per-game exploitability (BR_1 + BR_2) / 2 of the average strategy (Section 2.2), for
 * n_games entries; br_values (optional) receives 2 * n_games values, player 1 then player 2
 * for each game. Synchronises. */
int cfr_exploitability_batch(cfr_solver* s, double* expl, double* br_values, int32_t n_games);

/* Release host resources; the caller then frees the workspace. */
int cfr_destroy(cfr_solver* s);

const char* cfr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CFR_MI355X_H */
