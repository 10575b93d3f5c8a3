/*
 * pbit.h -- C ABI of the MI355X-native self-adaptive Ising machine (SAIM).
 *
 * The library samples the Lagrangian of a constrained binary problem with a
 * software probabilistic-bit (p-bit) Ising machine on one gfx950 GPU and
 * adapts the Lagrange multipliers between annealing runs (Delacour,
 * "Self-Adaptive Ising Machines for Constrained Optimization", Algorithm 1,
 * Sec. III).
 *
 * Conventions shared by every entry point
 *  - Problems are stated in maximisation form: maximise profit(x) subject to
 *    weight * x <= capacity, x in {0,1}^n (the paper minimises f = -profit,
 *    Sec. II Eq. primal_problem; Sec. IV-A and IV-B give the QKP and MKP forms).
 *  - All settings are in the paper's normalised units (Sec. IV-A: profits are
 *    divided by max|profit|, constraint data by max(|weight|, |capacity|)).
 *    Rationals are passed as (numerator, denominator) pairs.
 *  - Host arrays passed in are read during the call and may be freed after it.
 *  - All device memory is owned by the caller: the library never allocates
 *    device memory and never creates streams.  An instance borrows its
 *    workspace (pbit_workspace_bytes bytes, 256-byte aligned) until
 *    pbit_destroy_instance.
 *  - Every call returns a pbit_status; nothing throws or aborts.  On failure
 *    pbit_last_error() returns a message for the calling thread.  Argument
 *    and range errors are detected synchronously; asynchronous device errors
 *    surface at the next call that synchronises (PBIT_EDEVICE), after which the
 *    instance only accepts pbit_destroy_instance.
 *  - An instance may be used from one host thread at a time.  Calls on one
 *    instance must be ordered on one stream (or synchronised by the caller).
 *  - The library is built for gfx950 only; a call on another device returns
 *    PBIT_EDEVICE.
 */
#ifndef PBIT_H
#define PBIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *pbit_stream; /* a hipStream_t; NULL = default stream */

typedef enum {
    PBIT_OK = 0,
    PBIT_NOFEAS = 1,      /* no feasible sample yet: not an error */
    PBIT_EINVAL = -1,     /* malformed argument */
    PBIT_ERANGE = -2,     /* instance or settings exceed the exact integer bounds */
    PBIT_EWORKSPACE = -3, /* workspace missing, too small or misaligned */
    PBIT_EDEVICE = -4,    /* HIP error, or device is not gfx950 */
    PBIT_ESTATE = -5      /* instance unusable after a device error */
} pbit_status;

typedef enum { PBIT_QKP = 0, PBIT_MKP = 1 } pbit_kind;

/* Problem (Sec. IV-A quadratic knapsack, Sec. IV-B multidimensional knapsack).
 *  QKP: profit is n*n row-major and symmetric; the diagonal holds the item
 *       values h_i, the off-diagonal the pair values W_ij (each pair counts
 *       once in the objective); |entries| <= 127.
 *  MKP: profit is a length-n vector of item values.
 *  weight is m*n row-major (non-negative), capacity has m entries (non-negative).
 *  density_num/den is the nominal pair density d used by the penalty rule
 *  P = alpha d N (Sec. III-A); it is ignored for MKP, whose d is 2/(N+1)
 *  (Sec. IV-B).  N counts slack spins. */
typedef struct {
    int32_t kind;
    int32_t n, m;
    const int32_t *profit;
    const int32_t *weight;
    const int64_t *capacity;
    int32_t density_num, density_den;
} pbit_problem;

/* Sampler settings (Sec. III-B and Table 1).
 *  replicas     R independent chains per round; they share lambda.
 *  sweeps       T Monte-Carlo sweeps per annealing run (>= 1, and
 *               T * ceil(N_ext / 4) <= 2^32 so that the Philox counter word
 *               t * ceil(N_ext / 4) + i / 4 never wraps; PBIT_ERANGE otherwise).
 *  beta         beta_max of the linear schedule beta_t = beta_max t/(T-1).
 *  eta          multiplier step size (Algorithm 1); lambda += eta * mean_r g_r / s_g.
 *  p_q          256*P directly, or -1 for the rule P = alpha d N.
 *  alpha        the rule's constant.
 *  seed         Philox4x32-10 key.
 *  instance_id  last Philox counter word.
 *  fixed_beta   nonzero: every sweep runs at beta_max (test mode).
 *  eta_decay_rounds  H >= 0: the step after round k (0-based) is
 *               eta_k = eta H / (H + k), a diminishing step (sum eta_k diverges,
 *               sum eta_k^2 converges: the step-size conditions under which the
 *               surrogate subgradient ascent of Sec. III-A converges); 0 keeps
 *               eta constant as in Algorithm 1.  At most 2^20; k is capped where
 *               the step's 64-bit denominator would overflow (beyond 10^9
 *               rounds for every instance the bounds admit).
 *  pt_slots     L > 0: parallel tempering as the Ising machine (Sec. III-B: the
 *               machine inside Algorithm 1 is interchangeable) instead of
 *               annealing: replicas form chains of L (replica c L + j starts at
 *               ladder position j), held at the fixed ladder
 *               beta_j = beta_max (j + 1) / L on the beta grid; after sweep t the
 *               replicas at positions tau, tau + 1 (tau = t mod 2, 4, ...) swap
 *               positions when j = floor(256 (beta_tau - beta_tau+1)(L_a - L_b))
 *               >= 0 or u24 < round(2^24 exp(j / 256)) (Metropolis on the grid;
 *               u24 from Philox(t, k | 2^31, c L + tau, instance_id)).  Each
 *               chain's sample is its replica at position L - 1: the residual
 *               sums, the best record and the multiplier step use those R / L
 *               samples.  Quadratic instances only; L divides 64 and R;
 *               beta_max > 0 and no fixed-beta mode (PBIT_EINVAL otherwise).
 *               The multiplier range may be narrowed so that every energy
 *               difference stays exact in 64 bits (PBIT_ERANGE if below 1). */
typedef struct {
    int32_t replicas, sweeps;
    int32_t beta_num, beta_den;
    int32_t eta_num, eta_den;
    int32_t p_q;
    int32_t alpha_num, alpha_den;
    uint64_t seed;
    uint32_t instance_id;
    int32_t fixed_beta;
    int32_t eta_decay_rounds;
    int32_t pt_slots;
} pbit_params;

/* Host-side description of a compiled instance (no device needed). */
typedef struct {
    int32_t n, m, n_ext, n_pad;  /* original bits, constraints, spins with slack, padded */
    int32_t words;               /* 32-bit words per replica state (bits of n_ext spins) */
    int64_t s_f, s_g;            /* normalisation scales */
    int64_t p_q;                 /* 256 * P */
    int32_t shift;               /* beta grid shift S */
    int32_t lq_max;              /* |lambda_q| bound (lambda on the 2^-8 grid) */
    int32_t variant;             /* 0 quadratic field kernel, 1 linear, 2 linear with 64-bit dots */
    int32_t reserved;
    size_t workspace_bytes;
    /* layout of the buffer filled by pbit_round_outputs (byte offsets) */
    size_t out_x, out_g, out_profit, out_feasible, out_G, out_lambda, out_round, out_sat, out_slot, out_bytes;
} pbit_plan_info;

/* Compiles the instance on the host and describes it.  Defines the encoding of
 * Sec. IV-A (slack bits Q_k = floor(log2 b_k + 1), zero-padded profits) and the
 * exact integer scales.  Returns PBIT_EINVAL / PBIT_ERANGE as
 * pbit_create_instance would. */
pbit_status pbit_plan(const pbit_problem *prob, const pbit_params *par, pbit_plan_info *out);

/* Workspace size in bytes for (prob, par); 0 if the pair is invalid. */
size_t pbit_workspace_bytes(const pbit_problem *prob, const pbit_params *par);

typedef struct pbit_instance pbit_instance; /* opaque */

/* Uploads the compiled instance into dev_ws (device memory owned by the caller,
 * 256-byte aligned, at least pbit_workspace_bytes) with copies ordered on
 * stream, sets lambda = 0 and the round counter to 0 (Algorithm 1 start).
 * The instance runs on the device that is current at this call.
 * Errors: PBIT_EINVAL (null or malformed arguments), PBIT_ERANGE (integer
 * bounds), PBIT_EWORKSPACE (dev_ws null, misaligned or ws_bytes too small),
 * PBIT_EDEVICE (HIP failure or device not gfx950).  *out is set only on OK. */
pbit_status pbit_create_instance(const pbit_problem *prob, const pbit_params *par, void *dev_ws,
                                 size_t ws_bytes, pbit_stream stream, pbit_instance **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): pbit_create_instance
 * with the workspace taken from a static device array of the library
 * (pbit_static_workspace_bytes() = 16 MiB per device, resident from the first
 * such call on a device until the process ends) instead of a caller buffer.
 * Allocates no device memory and calls no allocating library routine; the
 * host-side handle is created as for pbit_create_instance.  Every other entry
 * point works on the returned instance unchanged; pbit_round_outputs still
 * writes into the caller's buffer.
 * One device has one static workspace: while an instance made by this call is
 * live on a device, a second call on that device returns PBIT_ESTATE, and
 * pbit_destroy_instance releases it.  The array keeps the last instance's
 * contents; creation overwrites every byte the kernels read before writing.
 * Work of a destroyed static instance that is still queued on another stream
 * races with the next static instance on that device: order the two streams.
 * Errors: as pbit_create_instance, and PBIT_EWORKSPACE when the instance needs
 * more than pbit_static_workspace_bytes(), PBIT_ESTATE as above. */
pbit_status pbit_create_instance_static(const pbit_problem *prob, const pbit_params *par, pbit_stream stream,
                                        pbit_instance **out);

/* Size of the static per-device workspace used by pbit_create_instance_static. */
size_t pbit_static_workspace_bytes(void);

/* One annealing run of every replica (Sec. III-B; Algorithm 1 "minimise L_k"):
 * each replica starts at x = 0 and performs T sequential Gibbs sweeps of the
 * p-bit update (Eq. Ii_eq, Eq. mi_eq) with beta rising linearly; its last
 * state is its sample.  The round epilogue then scores every sample on the
 * original bits (feasible iff weight*x <= capacity, profit per Sec. IV-A),
 * keeps the best feasible sample over all rounds (largest profit, ties to the
 * earliest round, then the lowest replica), sums the residuals g = A x - b
 * over replicas for the multiplier step, and advances the round counter.
 * Asynchronous on stream. */
pbit_status pbit_sample_round(pbit_instance *inst, pbit_stream stream);

/* Multiplier step of Algorithm 1 with the replica mean of the residuals:
 * lambda_n += eta * (sum_r g_r) / (R s_g), accumulated exactly on a 2^-32 grid
 * and rounded (half away from zero) to the 2^-8 grid the fields use; the
 * accumulator saturates at +-lq_max/256.  Uses the sums of the last
 * pbit_sample_round.  Asynchronous on stream. */
pbit_status pbit_update_lambda(pbit_instance *inst, pbit_stream stream);

/* Sets lambda_q (m int32 values on the 2^-8 grid, host memory) for the next
 * round, e.g. a predicted starting point instead of Algorithm 1's lambda_0 = 0.
 * Values are clamped to +-lq_max.  Copy ordered on stream. */
pbit_status pbit_set_lambda(pbit_instance *inst, const int32_t *lambda_q, pbit_stream stream);

/* Copies the current lambda_q (m values; lambda_n = lambda_q / 256, the
 * multipliers of Eq. Lagrange_energy that Algorithm 1 carries from one
 * iteration to the next) to host memory; synchronises stream.
 * Errors: PBIT_EINVAL (null pointer), PBIT_ESTATE, PBIT_EDEVICE. */
pbit_status pbit_get_lambda(pbit_instance *inst, int32_t *lambda_q, pbit_stream stream);

/* Best feasible sample so far: Algorithm 1 keeps every feasible sample of
 * every iteration and returns the one of lowest objective (here: largest
 * profit; ties to the earliest round, then the lowest replica), scored on the
 * original bits as in Sec. IV-A.  Outputs: profit, the n original bits (host
 * bytes 0/1), the round and replica it came from.  Synchronises stream.
 * Returns PBIT_NOFEAS (outputs untouched) when no feasible sample exists yet.
 * Any pointer may be NULL.  Errors: PBIT_ESTATE, PBIT_EDEVICE. */
pbit_status pbit_best_feasible(pbit_instance *inst, int64_t *profit, uint8_t *x, int32_t *round,
                               int32_t *replica, pbit_stream stream);

/* Copies the last round's per-replica results into dev_out (caller-owned
 * device memory of at least pbit_plan_info.out_bytes), ordered on stream.
 * These are the quantities of one iteration of Algorithm 1: the samples x_k,
 * their constraint residuals g(x_k) (whose replica sum drives the multiplier
 * step), their objective and feasibility (Sec. IV-A), and the multipliers for
 * the next iteration.  Errors: PBIT_EWORKSPACE (dev_out null or too small),
 * PBIT_ESTATE, PBIT_EDEVICE.  Layout (byte offsets from pbit_plan_info):
 *   out_x        uint32 [R][words]  final states, bit i of word i/32 = spin i
 *   out_g        int32  [R][m]      residuals A_ext x - b
 *   out_profit   int64  [R]         profit of the original bits
 *   out_feasible int32  [R]         1 if weight*x <= capacity
 *   out_G        int64  [m]         sum of residuals over replicas
 *   out_lambda   int32  [m]         lambda_q in force for the next round
 *   out_round    int32  [1]         rounds completed
 *   out_sat      uint32 [1]         bit k set once lambda_k has been held at
 *                                   +-lq_max by a step or a set (sticky): from
 *                                   then on it no longer follows Algorithm 1
 *   out_slot     int32  [R]         parallel tempering: final ladder position of
 *                                   each replica (L - 1: the chain's sample);
 *                                   zero without it */
pbit_status pbit_round_outputs(pbit_instance *inst, void *dev_out, size_t bytes, pbit_stream stream);

/* Releases host-side state; the workspace may be reused afterwards.  Does not
 * synchronise: the caller must not free the workspace while work is queued. */
pbit_status pbit_destroy_instance(pbit_instance *inst);

/* Describes a created instance (as pbit_plan does for its inputs). */
pbit_status pbit_instance_info(const pbit_instance *inst, pbit_plan_info *out);

/* Launch layout of the single-instance sampling kernel: waves_per_block is the
 * number of 64-replica waves per workgroup (quadratic kernel 1 or 4, linear
 * kernel 1..4; 0 = the default for the replica count).  lds_resident selects,
 * for the linear kernel, whether the per-site field constants and coefficient
 * rows are staged in LDS (1), read from global memory (0), or staged whenever
 * they fit (-1, the default); ignored by the quadratic kernel.  split selects
 * workgroups of one visiting wave plus three waves that precompute its random
 * draws and thresholds (and, for the quadratic kernel, its J slabs) (1), for
 * the quadratic kernel the same with six such waves, two per SIMD (2), plain
 * workgroups (0), or the split form whenever the replicas leave CUs idle and
 * it fits LDS (-1, the default; quadratic: six producers).  Every layout gives bit-identical results;
 * only the speed differs.  Host only, takes effect at the next
 * pbit_sample_round.  PBIT_ERANGE if lds_resident = 1 or split = 1 does not
 * fit the 160 KB of LDS. */
pbit_status pbit_set_tiling(pbit_instance *inst, int32_t waves_per_block, int32_t lds_resident, int32_t split);

/* ---- Batched execution --------------------------------------------------
 * A batch runs many independent instances, of either kind and of uneven
 * sizes, each with its own parameters (Tables 2-5 solve every instance on its
 * own, so batching changes no result).  One round of the batch is one
 * persistent kernel launch per body family (quadratic, linear): workgroups of
 * 256 replicas take work items (instance, replica tile) from the family's
 * queue, sorted by decreasing estimated cost, through an atomic counter; then
 * the round epilogue and the multiplier step run for every instance that
 * still has rounds in its budget.  Every member
 * produces exactly what a single instance created from the same problem and
 * parameters produces.  Multi-knapsack members whose constraint count has no
 * compiled batch body (1-6, 8, 10, 16, 30 and 32 do) are padded with empty
 * constraints (zero weights, zero capacity), which changes no sample; their
 * lambda and residual vectors then carry the extra zero entries. */
typedef struct pbit_batch pbit_batch; /* opaque */

/* Workspace bytes for a batch of count instances; 0 if any pair is invalid. */
size_t pbit_batch_workspace_bytes(const pbit_problem *probs, const pbit_params *params, int32_t count);

/* Launch layout of a batch (every layout gives the same results; the
 * autotuner picks one per batch shape by timing):
 *  blocks_quad    persistent workgroups of the quadratic family (0: as many
 *                 as can be resident, one per CU times the occupancy);
 *  blocks_linear  the same for the linear family;
 *  split_percent  a linear member whose plain 256-replica chain is longer than
 *                 split_percent/100 of the average linear load per CU runs as
 *                 split tiles (one visiting and three producer waves per 64
 *                 replicas, when its constants fit LDS); 0: none; -1: 200;
 *  split_members  set by pbit_batch_layout_used: members run split (ignored
 *                 on input). */
typedef struct {
    int32_t blocks_quad, blocks_linear, split_percent, split_members;
} pbit_batch_layout;

/* Creates a batch in dev_ws (caller-owned device memory, 256-byte aligned, at
 * least pbit_batch_workspace_bytes).  rounds[i] is member i's round budget
 * (NULL: unlimited); a member whose budget is spent is skipped by later rounds.
 * layout NULL: {0, 0, -1}.
 * Errors as pbit_create_instance (the message names the failing member), and
 * PBIT_EINVAL for negative grid sizes or split_percent < -1. */
pbit_status pbit_create_batch(const pbit_problem *probs, const pbit_params *params, int32_t count,
                              const int32_t *rounds, const pbit_batch_layout *layout, void *dev_ws,
                              size_t ws_bytes, pbit_stream stream, pbit_batch **out);

/* The layout a batch runs with (grids after the caps, the split rule in
 * force and how many members it splits). */
pbit_status pbit_batch_layout_used(const pbit_batch *batch, pbit_batch_layout *out);

/* One round (annealing runs and epilogue) of every member with budget left.
 * Asynchronous on stream. */
pbit_status pbit_batch_sample_round(pbit_batch *batch, pbit_stream stream);

/* The multiplier step of every member with budget left; uses one unit of
 * its budget.  Asynchronous on stream. */
pbit_status pbit_batch_update_lambda(pbit_batch *batch, pbit_stream stream);

/* rounds x (sample_round + update_lambda).  use_graph != 0 records the four
 * launches of a round once as a HIP graph and replays it; the results are
 * those of the direct launches.  Asynchronous on stream. */
pbit_status pbit_batch_run(pbit_batch *batch, int32_t rounds, int32_t use_graph, pbit_stream stream);

/* Member i as an instance handle owned by the batch (do not destroy it):
 * pbit_get_lambda, pbit_set_lambda, pbit_best_feasible, pbit_round_outputs
 * and pbit_instance_info apply to it; pbit_sample_round and
 * pbit_update_lambda on it run that member alone. */
pbit_status pbit_batch_member(pbit_batch *batch, int32_t index, pbit_instance **member);

/* Copies the remaining round budgets (count values) to host memory;
 * synchronises stream. */
pbit_status pbit_batch_rounds_left(pbit_batch *batch, int32_t *rounds_left, pbit_stream stream);

/* Work-queue description: items and persistent workgroups per round. */
pbit_status pbit_batch_shape(const pbit_batch *batch, int32_t *items, int32_t *blocks, size_t *lds_bytes);

/* Sets every member's lambda_q from lambda_q (device memory, int32
 * [count][32], member i's values at i*32 + k; entries beyond a member's m are
 * ignored), clamped to +-lq_max, e.g. the learned starting point written by
 * pbit_net_to_lambda.  Asynchronous on stream. */
pbit_status pbit_batch_set_lambdas(pbit_batch *batch, const int32_t *lambda_q, pbit_stream stream);

/* Writes one 176-byte record per member to dev_out (device memory), ordered
 * on stream: int64 best feasible profit; int32 its round, 1 if any feasible
 * sample exists, rounds done, feasible samples in the last round, the
 * multiplier saturation mask (out_sat of pbit_round_outputs), one zero
 * word; int32 lambda_q[32] (zero beyond m); int64 sum of the profits of the
 * last round's feasible samples; int64 sum over the last round's samples of
 * |g|^2 (squared residuals with slack, the penalty term of Eq.
 * penalty_energy in data units).  Together with the feasible count these give
 * the mean objective of the feasible samples that the accuracy metric of
 * Sec. IV-A averages, without copying every sample to the host. */
pbit_status pbit_batch_snapshot(pbit_batch *batch, void *dev_out, pbit_stream stream);

/* Releases the batch, its members and its graph.  Does not synchronise. */
pbit_status pbit_destroy_batch(pbit_batch *batch);

/* ---- Learned starting multipliers ---------------------------------------
 * A set encoder predicts lambda_0 for each constraint of an instance, to start
 * Algorithm 1 near the value its multipliers settle to (the paper starts from
 * lambda_0 = 0).  One set per (instance, constraint k), one element per
 * original variable i with features (bf16, 16 per element, five used)
 *   rho_i/(s_f n), n a_ki/b_k, n mean_k' a_k'i/b_k', h_i/s_f,
 *   clamp(ln(e_ki / rho_bar_k), -8, 8)
 * where rho_i = h_i + sum_j W_ij and e_ki = (h_i + sum_j W_ij / 2) / a_ki (+8
 * for a_ki = 0, -8 for e_ki <= 0), and a context of nine values per set (bf16,
 * 16 stored): log(N_ext)/8, d, P/N_ext, beta_max/50, M/32, kind, and of the
 * greedy fill of constraint k alone (decreasing e_ki, ties by index, up to the
 * first item that does not fit) that item's e / rho_bar_k (0 if all fit),
 * b_k / sum_i a_ki and the items taken before it / n.
 * Network: phi = Linear(16,128)-ReLU-Linear(128,128)-ReLU per element, mean over
 * the set, head = Linear(144,128)-ReLU-Linear(128,1) on [pooled, context] -> t.
 * lambda_q,k = round_half_away(t * scale_k), scale_k = 256 rho_bar_k s_g / s_f,
 * rho_bar_k = sum_i (h_i + sum_j W_ij / 2) / sum_i a_ki.
 * Parameters: pbit_net_param_count() floats in the order W1[128][16], b1,
 * W2[128][128], b2, W3[128][144], b3, w4[128], b4 (row = output unit).
 * Weights and stored activations are bf16, accumulation fp32 (matrix cores
 * for the per-element layers).  All device buffers are caller-owned. */
int32_t pbit_net_param_count(void);

/* Device workspace for the activations of one forward/backward pair.  Its
 * layout (each part at the next 256-byte boundary, in this order) lets a
 * caller inspect them after pbit_net_forward / pbit_net_backward:
 *   H1 bf16 [rows][128], H2 bf16 [rows][128]   per-element activations
 *   Z  bf16 [sets][144]                        pooled mean of H2 over the set's
 *                                              n rows, then the 16 context values
 *   G1 bf16 [sets][128]                        head hidden layer
 *   dP fp32 [sets][128]                        loss gradient w.r.t. the pooled mean
 *   then per-group partial gradients (internal). */
size_t pbit_net_workspace_bytes(int32_t sets, int32_t rows);

/* Host: packs the sets of count instances.  Always writes *sets and *rows (a
 * size query when x is NULL).  Otherwise fills, in host memory:
 *   x        bf16 [rows][16]  set s occupies rows set_rows[s] .. (32-aligned),
 *                             its first set_n[s] rows are its elements, the
 *                             rest zero
 *   ctx      bf16 [sets][16]
 *   set_rows int32 [sets + 1]
 *   set_n    int32 [sets]     (= n of the instance)
 *   scale    double [sets]    lambda_q = t * scale
 *   dest     int32 [sets]     member * 32 + k (index into a [count][32] array)
 * Sets are ordered by member, then constraint.  Errors as pbit_plan. */
pbit_status pbit_net_pack(const pbit_problem *probs, const pbit_params *params, int32_t count, int32_t *sets,
                          int32_t *rows, uint16_t *x, uint16_t *ctx, int32_t *set_rows, int32_t *set_n,
                          double *scale, int32_t *dest);

/* bf16 copy of fp32 parameters (device).  Asynchronous on stream. */
pbit_status pbit_net_cast(const float *w, uint16_t *w_bf16, pbit_stream stream);

/* Forward pass of all sets: t[sets] (device fp32).  The packed arrays are the
 * device copies of pbit_net_pack's output; w_bf16 and x 16-byte aligned; ws
 * (256-byte aligned, pbit_net_workspace_bytes) keeps the activations for
 * pbit_net_backward.  Asynchronous on stream. */
pbit_status pbit_net_forward(const uint16_t *w_bf16, const uint16_t *x, const uint16_t *ctx,
                             const int32_t *set_rows, const int32_t *set_n, int32_t sets, int32_t rows, void *ws,
                             size_t ws_bytes, float *t, pbit_stream stream);

/* Gradient (device fp32, pbit_net_param_count values) of the mean Huber loss
 * (delta 1) of t - y over the sets, and the loss itself (device fp32 [1]),
 * from the activations of the preceding pbit_net_forward on the same ws.
 * Deterministic.  Asynchronous on stream. */
pbit_status pbit_net_backward(const uint16_t *w_bf16, const uint16_t *x, const int32_t *set_rows,
                              const int32_t *set_n, int32_t sets, int32_t rows, const float *t, const float *y,
                              void *ws, size_t ws_bytes, float *grad, float *loss, pbit_stream stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step counts
 * from 1) on fp32 master weights w with moments m, v; refreshes w_bf16. */
pbit_status pbit_net_adam_step(float *w, float *m, float *v, const float *grad, uint16_t *w_bf16, int32_t step,
                               float lr, pbit_stream stream);

/* lambda_q[dest[s]] = round_half_away(t[s] * scale[s]) (float64, clamped to
 * +-2^30), all device memory; feeds pbit_batch_set_lambdas. */
pbit_status pbit_net_to_lambda(const float *t, const double *scale, const int32_t *dest, int32_t sets,
                               int32_t *lambda_q, pbit_stream stream);

/* Thread-local message describing the last failing call on this thread. */
const char *pbit_last_error(void);

/* Threshold table the sampler uses: theta[j + 2304] = round(2^24 (1 + tanh(j/256))/2),
 * j = -2304..2304, written to host memory (4609 entries).  Host only. */
pbit_status pbit_theta_table(int32_t *theta);

/* Replica-exchange table of the parallel-tempering machine (pt_slots):
 * x[i] = round(2^24 exp((i - 4608)/256)), i = 0..4608, the Metropolis
 * acceptance exp(j/256) on the 2^-8 grid; written to host memory (4609
 * entries).  Host only. */
pbit_status pbit_exchange_table(int32_t *x);

#ifdef __cplusplus
}
#endif
#endif
