/*
 * econ_mi355x.h -- C ABI of the gfx950 (MI355X) batched-economy library.
 *
 * The library advances E independent EconoJax economies (Ponse et al.,
 * "EconoJax: A Fast & Scalable Economic Simulation in JAX", AAMAS 2025), each
 * with n_e population agents and one government agent, and runs the shared
 * population policy network and its PPO learner on the GPU.
 *
 * Conventions (all entry points):
 *   - Every call returns an int: EJ_OK (0) or a negative EJ_E* code.  No C++
 *     exception crosses the ABI.  ej_strerror() names a code;
 *     ej_last_hip_error() returns the hipError_t behind the last EJ_EHIP of
 *     the calling thread.
 *   - Arrays named d_* are DEVICE pointers owned by the caller; the library
 *     never frees them and never keeps them beyond the call.  Arrays named h_*
 *     are host pointers.  State and scratch owned by a handle live inside it
 *     and are freed by the matching destroy call.  Parameters, weights and
 *     observations move in 16-byte vector loads and stores: d_params, d_work,
 *     d_obs (of the economy step, the policy and ej_ppo_batch.obs), d_grads
 *     and d_workspace must be 16-byte aligned (hipMalloc and torch
 *     allocations are; so is every observation row, D_stride being a
 *     multiple of 8), and a misaligned one returns EJ_EINVAL.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it; only calls documented as
 *     synchronous (get/set state, status) wait for it.
 *   - Per-agent arrays use "rows": the agents of economy e are rows
 *     row0[e] .. row0[e] + n_e - 1, with row0 the prefix sum of the
 *     populations (economy-major, agent-minor).  M = total rows.
 *   - Handles are not thread-safe; calls on one handle must be serialised.
 */
#ifndef ECON_MI355X_H
#define ECON_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EJ_OK 0
#define EJ_EINVAL (-1)       /* bad argument or configuration */
#define EJ_ENOMEM (-2)       /* device or host allocation failed */
#define EJ_EHIP (-3)         /* a HIP runtime call failed; see ej_last_hip_error() */
#define EJ_EUNSUPPORTED (-4) /* configuration outside the limits below */
#define EJ_ESCRATCH (-5)     /* request larger than EJ_PPO_STATIC_SCRATCH_BYTES */

#define EJ_MAX_N 1024 /* agents per economy */
#define EJ_MAX_R 16   /* resource types */
#define EJ_MAX_P 128  /* price levels */
#define EJ_MAX_K 16   /* tax brackets */
#define EJ_MAX_X 32   /* order lifetime in steps */
#define EJ_GOV_LEVELS 21 /* tax levels 0 %, 5 %, ..., 100 % */
#define EJ_SKILL_NORMAL 1 /* skill_mode bits (the multi-agent variant, Sec. 5) */
#define EJ_SKILL_GROWTH 2

/* Observation feature-group scales (float multipliers applied before the
 * bf16 rounding of the population observation). */
typedef struct ej_obs_scales {
    float coin, labor, orders, res, skill, rate, phase, price, count;
} ej_obs_scales;

/* Economy parameters.  Sec. 3 of the paper ("Population Agents",
 * "Government Agent", "Setting tax rates") and Table 2 define them.
 *   E            number of economies
 *   N            largest population (every n_e <= N <= EJ_MAX_N)
 *   R, P         resource types, price levels (prices[0..P-1], strictly increasing)
 *   X            order lifetime: an order takes part in X clearings (Table 2: 30)
 *   max_orders   live-order limit per agent (Table 2: 15)
 *   P_tax, K     tax period in steps (Table 2: 100); number of brackets
 *                (K = 0 disables taxes: the free market); cutoffs[0..K-2]
 *   T            episode length (Table 2: 1000); economies reset automatically
 *   R_kappa, R_d crafting needs R_kappa units of each of R_d types
 *   kappa_c      crafting pays (SC * kappa_c) coin, SC the crafting skill
 *   start_coin   coin at reset (Table 2: 15)
 *   labor_*      labor per action in units of 1/20 (Table 2: 20, 20, 1)
 *   allow_noop   NOOP allowed (Table 2: true)
 *   skill_mode   0: skills Pareto(4) clipped to 5, fixed within an episode.
 *                The multi-agent variant of Sec. 5: EJ_SKILL_NORMAL draws them
 *                near 1 with spread 1 (the sum of twelve uniforms minus six,
 *                plus 1, clipped to [0, 5]); EJ_SKILL_GROWTH raises a skill
 *                by 0.5 % times (1 - skill / 5) each time it is used (gather
 *                of that resource, craft), rounded down in Q16
 *   eta, omega   utility curvature (Eq. (1), 0.27) and equality weight (Eq. (4), 1)
 *   seed         key of the counter-based generator for skills, gathering
 *                luck and order tie keys */
typedef struct ej_env_config {
    int32_t E, N, R, P, X, max_orders, P_tax, K, T;
    int32_t R_kappa, R_d, kappa_c, start_coin;
    int32_t labor_gather, labor_craft, labor_trade;
    int32_t allow_noop;
    int32_t skill_mode; /* EJ_SKILL_NORMAL | EJ_SKILL_GROWTH (the Sec. 5 variant); 0: Pareto skills, fixed */
    double eta, omega;
    uint64_t seed;
    int32_t prices[EJ_MAX_P];
    int32_t cutoffs[EJ_MAX_K];
    ej_obs_scales scales;
} ej_env_config;

/* Sizes derived from a configuration (filled by ej_env_dims). */
typedef struct ej_env_dims_t {
    int64_t M;          /* total agent rows */
    int32_t A;          /* population actions: 2 + R + 2 R P (Sec. 5 counts 30 and 86) */
    int32_t mask_words; /* ceil(A / 32) uint32 words of action-mask bits per row */
    int32_t D;          /* population observation features: 7 + 7 R + K */
    int32_t D_stride;   /* bf16 elements per observation row (D rounded up to 8) */
    int32_t D_gov;      /* government observation floats: 3 (3 + R) + K + 1 + 4 R */
    int32_t K;          /* government action entries per economy */
    int32_t E;          /* economies */
    int32_t D_metrics;  /* doubles per economy in ej_env_episode_metrics: 5 R + 9 */
} ej_env_dims_t;

typedef struct ej_env ej_env;

/* Host-side view of the state of every economy, in a representation-neutral
 * form (every pointer is a HOST array supplied by the caller):
 *   t[E], ep[E]                    step within the episode, episode index
 *   rates[E * K]                   current tax levels (0..20)
 *   coin_inv, coin_esc, labor, snap, sc  [M]  coin in inventory / escrow,
 *                                  labor (1/20 units), coin at the start of the
 *                                  tax period, crafting skill (Q16.16)
 *   res_inv, res_esc, sg           [R * M]  resources in inventory / escrow,
 *                                  gathering skill (Q16.16), resource-major
 *   orders                         [X * M]  live order of each (slot, row):
 *                                  -1, or side + 2 (r + R p); side 0 = buy.
 *                                  Slot s holds the order placed at the step
 *                                  t0 with t0 mod X == s. */
typedef struct ej_state_view {
    int32_t *t, *ep, *rates;
    int32_t *coin_inv, *coin_esc, *labor, *snap, *sc;
    int32_t *res_inv, *res_esc, *sg;
    int32_t *orders;
} ej_state_view;

const char* ej_strerror(int code);
int ej_last_hip_error(void);

/* Validates `cfg`, allocates the device state of E economies and places
 * them at the reset state of episode 0 (synchronously).  h_n_per_env (host,
 * [E], nullable) gives uneven populations; NULL means n_e = N for all.
 * Errors: EJ_EINVAL (inconsistent values), EJ_EUNSUPPORTED (limits above,
 * or R*2*P*X > 8192 order-book buckets), EJ_ENOMEM, EJ_EHIP. */
int ej_env_create(const ej_env_config* cfg, const int32_t* h_n_per_env, ej_env** out);
int ej_env_destroy(ej_env* env);
int ej_env_dims(const ej_env* env, ej_env_dims_t* out);
/* Row offsets row0[0..E] (host copy owned by the handle, valid until destroy). */
const int32_t* ej_env_row_offsets(const ej_env* env);

/* Resets every economy to step 0 of `episode`: coin = start_coin, empty
 * inventories, escrow and book; skills drawn from Pareto(alpha = 4, x_m = 1)
 * clipped to 5 (Sec. 4 "Experimental details" initialises skills with a
 * Pareto distribution), keyed (seed, economy, episode, agent). */
int ej_env_reset(ej_env* env, int32_t episode, void* stream);

/* One step of every economy (Sec. 3; Eqs. (1)-(5)):
 *   d_act     [M] int32 population actions: 0 NOOP, 1..R gather r-1, R+1 craft,
 *             R+2 + r P + p buy (r, p), R+2 + R P + r P + p sell (r, p).
 *             Actions outside the step-start action mask become NOOP (no labor)
 *             and are counted (ej_env_status).
 *   d_gov     [E * K] int32 government levels 0..20, read at the first step of a
 *             tax period (t mod P_tax == 0); out-of-range levels keep the old rate.
 *             NULL when ej_env_set_gov_draw enabled the step's own draw.
 *   d_rew     [M] float  u(t+1) - u(t) (Eq. (1), Eq. (2)), difference in fp64
 *   d_gov_rew [E] float  change of Eq * Prod (Eqs. (3)-(5))
 *   d_done    [M] uint8  1 when the step ended the episode (the economy then
 *             restarts at the next episode before the call returns)
 *   d_obs     [M * D_stride] bf16 bits, nullable: the observation after the step
 *   d_mask    [M * mask_words] uint32, nullable: the action mask after the step
 * One workgroup per economy; all inputs are read before any state changes. */
int ej_env_step(ej_env* env, const int32_t* d_act, const int32_t* d_gov, float* d_rew, float* d_gov_rew,
                uint8_t* d_done, uint16_t* d_obs, uint32_t* d_mask, void* stream);

/* ej_env_step restricted to economies [e_begin, e_end): the arrays keep the
 * layout of the whole batch (rows of economy e start at row offset e) and
 * only the range's rows and economies are read and written, so that disjoint
 * ranges may run concurrently on different streams (one workgroup per
 * economy; the persistent launch applies to whole-batch calls only). */
int ej_env_step_range(ej_env* env, int32_t e_begin, int32_t e_end, const int32_t* d_act, const int32_t* d_gov,
                      float* d_rew, float* d_gov_rew, uint8_t* d_done, uint16_t* d_obs, uint32_t* d_mask,
                      void* stream);

/* Launch shape of ej_env_step.  mode 0: one workgroup per economy (one
 * launch per step).  mode 1: `workgroups` persistent workgroups (0: two per
 * compute unit) take economies from a work queue, largest populations first;
 * the queue resets itself at the end of every launch, so the call can be
 * captured in a graph and replayed.  Results are identical in both modes. */
int ej_env_set_launch(ej_env* env, int32_t mode, int32_t workgroups);

/* Agents per wavefront of ej_env_step: 64 (default), 32 or 16.  Wave w of
 * an economy's workgroup takes agents w * apw .. w * apw + apw - 1 and the
 * lanes beyond apw stay idle, so a smaller value spreads an economy over
 * more waves (ceil(n / apw) waves; at most 16).  Results are identical for
 * every value.  EJ_EUNSUPPORTED when N needs more than 16 waves. */
int ej_env_set_agents_per_wave(ej_env* env, int32_t agents_per_wave);

/* Episode statistics, the measures the paper reports at the end of an
 * episode (Sec. 4 results; Figs. 2, 3 and 6): enabled = 1 makes every
 * following step count, per economy, the actions taken by category and the
 * trades and their prices per resource, and at each episode end write the
 * economy's record.  Allocates the counters on first use (counts start at
 * the next step); 0 stops counting.  Rewards and state are unchanged. */
int ej_env_enable_metrics(ej_env* env, int32_t enabled);

/* Record of the last completed episode of every economy -> d_out
 * [E * (5 R + 9)] doubles, economy-major:
 *   [0] index of that episode (-1: none completed since enabling)
 *   [1] productivity Prod = sum_i C_i at its end (Eq. (5))
 *   [2] equality 1 - gini(C)
 *   [3] government utility Eq * Prod (Eqs. (3), (4))
 *   [4] mean and [5] lower median over the population of the episode
 *       return, the sum of an agent's rewards = its utility at the end
 *       minus its utility at the reset state (Eq. (2))
 *   [6 + j] actions of category j: 0 NOOP, 1 + r gather r, 1 + R craft,
 *       2 + R + r buy r, 2 + 2R + r sell r, 2 + 3R rejected (became NOOP)
 *   [9 + 3R + r] trades of resource r, [9 + 4R + r] the sum of their prices
 * EJ_EINVAL unless ej_env_enable_metrics was called. */
int ej_env_episode_metrics(ej_env* env, double* d_out, void* stream);

/* Government levels drawn by the step itself (ej_env_step with d_gov = NULL):
 * uniform over 0..20, exactly the levels ej_env_random_actions(env, seed, ...)
 * would write for the same step, drawn only where a tax period starts (the
 * only steps that read them; Sec. 3 "Setting tax rates").  For workloads whose
 * government acts at random; saves a launch per step.  enabled = 0 turns it
 * off (then d_gov is required again). */
int ej_env_set_gov_draw(ej_env* env, int32_t enabled, uint64_t seed);

/* Observation of the current state.  d_obs / d_mask as in ej_env_step (both
 * required); d_gov_obs [E * D_gov] float, nullable: per-feature mean, std and
 * lower median over the population of (coin, period income, labor, each
 * resource inventory), the tax levels, the period phase and the market
 * statistics (best bid, best ask, #bids, #asks per resource).  Sec. 3
 * "Action masking" and the Fig. 1 caption (government sees population
 * statistics); Appendix A (market statistics). */
int ej_env_observe(ej_env* env, uint16_t* d_obs, uint32_t* d_mask, float* d_gov_obs, void* stream);

/* Synthetic workload actions for the current step of every economy: uniform
 * over the A population actions, keyed (act_seed, economy, episode, step,
 * agent), and uniform government levels over 0..20.  d_act may be NULL
 * (government levels only). */
int ej_env_random_actions(ej_env* env, uint64_t act_seed, int32_t* d_act, int32_t* d_gov, void* stream);

/* Synchronous copies of the whole state to / from host arrays (checkpoint
 * and resume; parity checks).  set_state requires a state reachable by the
 * rules: orders with t - X < t0 < t and an uncrossed book per resource. */
int ej_env_get_state(ej_env* env, const ej_state_view* h_view, void* stream);
int ej_env_set_state(ej_env* env, const ej_state_view* h_view, void* stream);

/* Synchronous: number of population actions and government levels rejected
 * since create (summed over economies). */
int ej_env_status(ej_env* env, int64_t* h_invalid_actions, int64_t* h_invalid_gov, void* stream);

/* ------------------------------------------------------------------------
 * Shared population policy (Sec. 4 "Experimental details": all population
 * agents share one policy and one value network; Sec. 3 "Action masking").
 * Network: D -> H -> H -> (A logits, 1 value), ReLU, bf16 operands with fp32
 * accumulation.  Parameters are one flat fp32 vector (row-major W[in][out]
 * followed by its bias, for W1, b1, W2, b2, W3, b3; W3 has A + 1 columns,
 * the last one the value head).  The kernels read a bf16 "work" copy in
 * their own chunked layout, refreshed by ej_mlp_sync_weights.
 * Supported: D_stride a multiple of 8 in [D, 128] (above 64 only with
 * H >= 128 and 64-row tiles), H in {64, 128, 256, 512}, A + 1 <= 1024.
 * ------------------------------------------------------------------------ */
typedef struct ej_mlp_desc {
    int32_t D, D_stride, H, A;
    int32_t tile_rows; /* rows per workgroup of the policy forward: 0 (default, 64), 64, or 128
                          (H <= 256 only); chosen by the autotuner */
} ej_mlp_desc;

typedef struct ej_mlp_layout_t {
    int64_t n_params;                 /* fp32 parameter count */
    int64_t n_work;                   /* bf16 work-copy element count */
    int64_t W1, b1, W2, b2, W3, b3;   /* element offsets in the parameter vector */
    int64_t params_stride, work_stride; /* distance between stacked weight sets (grouped calls) */
} ej_mlp_layout_t;

int ej_mlp_layout(const ej_mlp_desc* m, ej_mlp_layout_t* out);

/* d_params [n_params] fp32 -> d_work [n_work] bf16 (round to nearest even). */
int ej_mlp_sync_weights(const ej_mlp_desc* m, const float* d_params, uint16_t* d_work, void* stream);

/* Policy forward over M rows: d_obs [M * D_stride] bf16 bits (as written by
 * ej_env_step / ej_env_observe), d_mask [M * ceil(A/32)] action-mask bits.
 * Writes the sampled action d_act [M], its log-probability d_logp [M], the
 * value d_val [M] and the entropy of the masked distribution d_ent [M];
 * d_logits [M * A] (nullable) receives the raw logits (debugging and tests).
 * Sampling is exact for the masked softmax: the logits are taken in chunks
 * of 128 actions, a chunk is chosen by weighted reservoir with one uniform
 * and the action inside it by inverse CDF with a second one (the chunk's
 * actions walked in action order); the uniforms of row r, chunk c come from
 * the counter-based generator keyed (seed, row_base + r, ctr', c / 2) with
 * ctr' = ctr + *d_ctr_base (d_ctr_base: nullable device uint64_t, read when
 * the kernel runs, so that a captured graph replayed many times draws fresh
 * uniforms after each ej_counter_add).  row_base >= 0 numbers the rows when
 * the pointers address a slice of a larger batch: slices drawn separately
 * give exactly the results of one call over the whole batch.  Logits are
 * never written to memory unless d_logits is given.  A row whose mask allows
 * no action gets action 0, log-probability 0 and entropy 0. */
int ej_policy_forward(const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work, const uint16_t* d_obs,
                      const uint32_t* d_mask, int64_t M, int64_t row_base, uint64_t seed, uint64_t ctr,
                      const uint64_t* d_ctr_base, int32_t* d_act, float* d_logp, float* d_val, float* d_ent,
                      float* d_logits, void* stream);

/* Per-agent weight sets (Sec. 5, methods 2 and 3: independent policies,
 * iPPO, and individual policies with a shared value network, MAPPO): G sets
 * stacked params_stride fp32 / work_stride bf16 elements apart (the strides
 * of ej_mlp_layout), set g serving the rows q * row_stride + g, q <
 * rows_per_group -- with economies of N agents each, set g = agent index g of
 * every economy (G = N, row_stride = N, rows_per_group = E).  One launch
 * covers every set (a grouped GEMM: each workgroup takes 64 rows of one set).
 * Outputs and sampling as ej_policy_forward, the uniforms keyed by the global
 * row, so a row draws the same uniforms as in the shared layout.
 * row_stride >= G. */
int ej_policy_forward_grouped(const ej_mlp_desc* m, int32_t groups, const float* d_params, const uint16_t* d_work,
                              const uint16_t* d_obs, const uint32_t* d_mask, int64_t rows_per_group,
                              int64_t row_stride, uint64_t seed, uint64_t ctr, const uint64_t* d_ctr_base,
                              int32_t* d_act, float* d_logp, float* d_val, float* d_ent, float* d_logits,
                              void* stream);

/* ej_mlp_sync_weights for G stacked sets (strides of ej_mlp_layout). */
int ej_mlp_sync_weights_grouped(const ej_mlp_desc* m, int32_t groups, const float* d_params, uint16_t* d_work,
                                void* stream);

/* *d_counter += inc on the stream (one tiny kernel; usable inside a graph). */
int ej_counter_add(uint64_t* d_counter, uint64_t inc, void* stream);

/* ------------------------------------------------------------------------
 * PPO learner (Table 2: clipped surrogate, clipped value loss, entropy
 * bonus, GAE; Sec. 4: population agents share the network).
 * ------------------------------------------------------------------------ */

/* Generalised advantage estimation over a rollout of T steps and M rows
 * (all arrays [T * M], time-major): d_done[t] = 1 when step t ended an
 * episode; d_last_val [M] is the value of the state after the last step.
 * adv_t = delta_t + gamma lam (1 - done_t) adv_{t+1},
 * delta_t = r_t + gamma (1 - done_t) V_{t+1} - V_t; ret = adv + V. fp32. */
int ej_gae(const float* d_rew, const float* d_val, const uint8_t* d_done, const float* d_last_val, int32_t T,
           int64_t M, float gamma, float lam, float* d_adv, float* d_ret, void* stream);

/* A minibatch of the rollout storage (every array indexed by the sample
 * index s in [0, M_total), device pointers): observation rows and mask
 * words as written by the environment, the action taken, its log-probability
 * and the value at collection time, the advantage and the return.  Row j of
 * the epoch is the sample (perm_a * j + perm_c) mod M_total (perm_a coprime
 * with M_total makes this a permutation); the minibatch is epoch rows
 * [row_begin, row_begin + rows). */
typedef struct ej_ppo_batch {
    const uint16_t* obs;
    const uint32_t* mask;
    const int32_t* act;
    const float* logp_old;
    const float* val_old;
    const float* adv;
    const float* ret;
    int64_t M_total, perm_a, perm_c, row_begin, rows;
    /* the samples s of the batch sit at storage index s * row_stride + row_offset
     * (row_stride <= 0 reads as 1): one agent's own samples of a rollout stored
     * for every agent (per-agent weight sets: row_stride = N, row_offset = agent) */
    int64_t row_stride, row_offset;
    /* nullable: the batch's samples packed by ej_ppo_pack (record s = sample
     * s).  When given, ej_ppo_backward reads each minibatch row's observation,
     * mask words and five scalars from its record, one cache-line-aligned
     * block, instead of from the seven arrays (which it still needs for the
     * advantage statistics); the results are identical.  Population backward
     * only: the government's ignores it. */
    const void* records;
} ej_ppo_batch;

/* clip epsilon (0.2), value clip (10), value coefficient c_v (0.25),
 * entropy coefficient c_e (0.1, annealed by the caller) */
typedef struct ej_ppo_hparams {
    float clip, vclip, vf_coef, ent_coef;
} ej_ppo_hparams;

/* Bytes of device scratch ej_ppo_backward needs for a minibatch of `rows`. */
int ej_ppo_workspace_size(const ej_mlp_desc* m, int64_t rows, int64_t* bytes);

/* Per-sample records of an update's samples (Table 2: every update runs
 * several epochs of minibatches over one rollout, each row a scattered
 * sample).  ej_ppo_record_bytes gives the record size for the network m (a
 * multiple of 128 bytes: the observation row, padded to 16 bytes, the mask
 * words, then action, old log-probability, old value, advantage and return,
 * 4 bytes each).  ej_ppo_pack writes record s for every sample s in
 * [0, b->M_total) of the batch (storage index s * row_stride + row_offset of
 * each array; perm_*, row_begin, rows and records are ignored) to d_records
 * [M_total * record_bytes] (16-byte aligned, caller-owned).  Pack once after
 * the advantages are computed and pass the records in ej_ppo_batch for every
 * minibatch of the update. */
int ej_ppo_record_bytes(const ej_mlp_desc* m, int64_t* bytes);
int ej_ppo_pack(const ej_mlp_desc* m, const ej_ppo_batch* b, void* d_records, void* stream);

/* Loss and gradient of one PPO minibatch with respect to every parameter:
 *   L = mean(-min(rho A, clip(rho, 1 - eps, 1 + eps) A))
 *     + c_v mean(1/2 max((V - R)^2, (V_old + clip(V - V_old, -vclip, vclip) - R)^2))
 *     - c_e mean(H),
 * rho = exp(log pi(a) - logp_old), A the advantage normalised over the
 * minibatch (population std + 1e-8), H the entropy of the masked policy.
 * The forward pass is recomputed from the stored observations (activations
 * of the rollout are never stored).  d_grads [n_params] is overwritten (not
 * accumulated); d_loss [5] receives the mean surrogate, value and entropy
 * terms, the clipped fraction, and the minibatch loss L itself.  d_workspace: caller-owned device scratch of at
 * least ej_ppo_workspace_size bytes.  Deterministic: the weight gradients
 * are reduced over a fixed split in a fixed order.  The taken action must be
 * allowed by its row's mask; a row whose mask allows no action adds nothing
 * to L or the gradients (it still counts in the means and the advantage
 * statistics). */
int ej_ppo_backward(const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work, const ej_ppo_batch* b,
                    const ej_ppo_hparams* hp, void* d_workspace, int64_t workspace_bytes, float* d_grads,
                    float* d_loss, void* stream);

/* ------------------------------------------------------------------------
 * Government policy (Sec. 3 "Government Agent", "Setting tax rates"; Sec. 4:
 * trained with PPO at the same time as the population).  The same network
 * as the population's (ej_mlp_desc with D = D_gov features, D_stride =
 * D_gov rounded up to 8, H <= 256, A = 21 K) on the economy's government
 * observation, with K independent categorical heads over the 21 tax levels
 * (bracket k: logits 21 k .. 21 k + 20) and the value as the last output;
 * K <= 12.  log pi(levels) is the sum of the heads' log-probabilities and
 * the entropy the sum of the heads' entropies.  Weights, layout and
 * ej_mlp_sync_weights as for the population.
 * ------------------------------------------------------------------------ */

/* One row per economy: d_gov_obs [E * D_gov] fp32 (ej_env_observe), each
 * feature multiplied by d_scale [D_gov] and rounded to bf16 (these rows go to
 * d_obs_bf16 [E * D_stride] when given, for the learner).  Writes the levels
 * d_levels [E * K] (0..20, the input of ej_env_step), their log-probability
 * d_logp [E], the value d_val [E] and the entropy d_ent [E]; d_logits
 * [E * 21 K] nullable (tests).  Level k of economy e is the inverse CDF of
 * head k in level order at the uniform of word k % 4 of the counter-based
 * generator keyed (seed, government sampling; e, ctr + *d_ctr_base, k / 4). */
int ej_gov_policy_forward(const ej_mlp_desc* m, int32_t K, const float* d_params, const uint16_t* d_work,
                          const float* d_gov_obs, const float* d_scale, int64_t E, uint64_t seed, uint64_t ctr,
                          const uint64_t* d_ctr_base, int32_t* d_levels, float* d_logp, float* d_val, float* d_ent,
                          uint16_t* d_obs_bf16, float* d_logits, void* stream);

/* Bytes of device scratch ej_gov_ppo_backward needs for `rows` rows. */
int ej_gov_ppo_workspace_size(const ej_mlp_desc* m, int32_t K, int64_t rows, int64_t* bytes);

/* The government's PPO minibatch loss and gradient, as ej_ppo_backward
 * (Table 2 settings, advantages normalised over the minibatch): b->obs the
 * bf16 rows written by ej_gov_policy_forward, b->act [M_total * K] the
 * levels taken, b->mask unused (NULL); d_grads overwritten; d_loss [5] as
 * for the population.  Deterministic. */
int ej_gov_ppo_backward(const ej_mlp_desc* m, int32_t K, const float* d_params, const uint16_t* d_work,
                        const ej_ppo_batch* b, const ej_ppo_hparams* hp, void* d_workspace, int64_t workspace_bytes,
                        float* d_grads, float* d_loss, void* stream);

/* d_out[e] = sum over t in [t_begin, t_end) of d_x[t * E + e] (fp32, in time
 * order): the government's reward of a tax period from the per-step rewards
 * [T * E] of ej_rollout_buffers.d_gov_rew. */
int ej_sum_steps(const float* d_x, int32_t t_begin, int32_t t_end, int64_t E, float* d_out, void* stream);

/* ------------------------------------------------------------------------
 * Rollout graph and autotuner (the batching forms around the kernels).
 * ------------------------------------------------------------------------ */

/* Storage of a T-step rollout (Table 2: rollout length), every array a
 * device pointer owned by the caller, time-major:
 *   d_obs  [(T + 1) * M * D_stride] bf16 bits: d_obs[0] holds the
 *          observation of the current state (ej_env_observe) before the first
 *          launch; step t writes the observation after it to d_obs[t + 1]
 *   d_mask [(T + 1) * M * mask_words], likewise
 *   d_act, d_logp, d_val, d_ent, d_rew [T * M]; d_done [T * M] uint8
 *   d_gov_rew [T * E]  the government's reward of every step
 *   d_last_val [M]     value of the state after the last step
 *   d_adv, d_ret [T * M] nullable together: GAE(gamma, lam) when given
 *   d_tmp [3 * M] fp32 scratch (the last-value forward's discarded outputs)
 *   d_ctr [1] uint64  sampling counter, advanced by T + 1 per launch */
typedef struct ej_rollout_buffers {
    uint16_t* d_obs;
    uint32_t* d_mask;
    int32_t* d_act;
    float *d_logp, *d_val, *d_ent, *d_rew;
    uint8_t* d_done;
    float* d_gov_rew;
    float* d_last_val;
    float *d_adv, *d_ret;
    float* d_tmp;
    uint64_t* d_ctr;
} ej_rollout_buffers;

/* T steps; economies split into `groups` contiguous ranges whose policy ->
 * step chains run on their own streams inside the graph (one group's policy
 * overlaps another's economy step); sampler seed; GAE gamma, lam;
 * last_value = 0 skips the last-value forward and GAE; carry = 1 ends every
 * launch by copying slot T of d_obs and d_mask to slot 0, so that launches
 * follow each other without the caller (slot 0 of the stored rollout is then
 * overwritten: a learner that reads the storage keeps carry = 0 and copies
 * after its update). */
typedef struct ej_rollout_config {
    int32_t T, groups, last_value, carry;
    uint64_t seed;
    float gamma, lam;
} ej_rollout_config;

typedef struct ej_rollout ej_rollout;

/* Captures the whole rollout -- T x (policy forward of every group, economy
 * step of its economies), then the last-value forward, GAE and the counter
 * advance -- as one HIP graph (stream capture on streams the library
 * creates), instantiates it, and returns the handle.  Nothing runs at
 * capture.  The economy's government must draw its own levels
 * (ej_env_set_gov_draw) and its launch shape is the one set at capture.
 * The graph keeps every pointer: env, the weights and the buffers must
 * outlive the handle.  Replays give exactly the storage of the same calls
 * launched one by one (same seeds, same counters). */
int ej_rollout_capture(ej_env* env, const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work,
                       const ej_rollout_config* cfg, const ej_rollout_buffers* bufs, ej_rollout** out);

/* Replays the captured rollout on `stream` (asynchronous). */
int ej_rollout_launch(ej_rollout* r, void* stream);

/* The same rollout from one launch per kernel (no graph), for comparison. */
int ej_rollout_launch_plain(ej_rollout* r, void* stream);

int ej_rollout_destroy(ej_rollout* r);

/* Result of ej_autotune: the chosen economy-step launch (mode and
 * persistent workgroups as in ej_env_set_launch; agents per wavefront) and
 * policy row tile, with their mean times per launch in milliseconds. */
typedef struct ej_autotune_result {
    int32_t env_mode, env_workgroups, agents_per_wave, policy_tile_rows;
    float env_ms, policy_ms;
    int32_t candidates; /* launch shapes timed */
} ej_autotune_result;

/* Times the launch shapes of the rollout kernels with HIP events on
 * `stream` (reps launches each after one warm-up launch) and applies the
 * fastest: for the economy step, one workgroup per economy or a persistent
 * launch with 1, 2 or 4 workgroups per compute unit, each at 64, 32 and 16
 * agents per wavefront; for the policy forward, 64- or 128-row tiles
 * (H <= 256), written to m->tile_rows.  The buffers are a rollout step's
 * (as ej_env_step and ej_policy_forward take them; d_gov nullable when the
 * step draws its own levels).  Everything a trial step changes -- the
 * economy state, rejection counters and cached utilities, and the d_obs,
 * d_mask, d_act, d_rew, d_gov_rew and d_done buffers -- is restored before
 * the call returns, so tuning changes no result.  m may be NULL (economy
 * only).  Allocates temporary device copies; synchronous. */
int ej_autotune(ej_env* env, ej_mlp_desc* m, const float* d_params, const uint16_t* d_work, uint16_t* d_obs,
                uint32_t* d_mask, int32_t* d_act, const int32_t* d_gov, float* d_logp, float* d_val, float* d_ent,
                float* d_rew, float* d_gov_rew, uint8_t* d_done, int32_t reps, ej_autotune_result* out,
                void* stream);

/* Allocation-free ej_ppo_backward, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results as ej_ppo_backward,
 * without the caller workspace: the workspace is a static device array of
 * EJ_PPO_STATIC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends (its address is looked up once per device, on
 * the first call there).  A minibatch whose ej_ppo_workspace_size exceeds it
 * returns EJ_ESCRATCH before anything is launched (at 35 -> 256 -> 256 ->
 * 125 + 1 that is about 3 800 rows).  The call itself allocates nothing.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (different streams, threads or handles) race and must be
 * serialised by the caller. */
#define EJ_PPO_STATIC_SCRATCH_BYTES (64u << 20)
int ej_ppo_backward_static(const ej_mlp_desc* m, const float* d_params, const uint16_t* d_work,
                           const ej_ppo_batch* b, const ej_ppo_hparams* hp, float* d_grads, float* d_loss,
                           void* stream);

/* Adam (Kingma & Ba) with bias correction on n fp32 parameters; `step` is
 * the 1-based update count. */
int ej_adam(float* d_params, const float* d_grads, float* d_m, float* d_v, int64_t n, int32_t step, float lr,
            float beta1, float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ECON_MI355X_H */
