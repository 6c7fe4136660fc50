/*
 * asdual.h - C ABI of the Active Set dual bound for ReLU networks on MI355X.
 *
 * Method: De Palma, Behl, Bunel, Torr, Kumar, "Scaling the Convex Barrier
 * with Sparse Dual Algorithms" (JMLR 2024, arXiv:2101.05844).
 *
 * The library computes lower bounds on c^T x_hat_n over an l_inf input box
 * for a feed-forward ReLU network (Sec. 2, problem eq:noncvx_pb) by
 * maximising the dual of the Anderson-type relaxation (Sec. 2.2,
 * eq:primal-anderson) restricted to an active set of multipliers
 * (Sec. 4.1, eq:dual-active-set), with Algorithm 1 (Active Set) initialised by
 * Algorithm 3 (the Big-M dual, App. B).  Any non-negative dual assignment
 * gives a valid bound (weak duality, Sec. 3); the returned value is the dual
 * objective at the final duals, evaluated in FP64.
 *
 * Conventions
 *  - All arrays passed as pointers are DEVICE memory (HIP), unless a comment
 *    says "host".  They are borrowed: the caller owns them and keeps them
 *    alive until the stream-ordered call that uses them has completed.
 *  - Per-subproblem arrays are row-major [S][n]: subproblem s, then the
 *    neuron index of the layer.  Convolutional neurons are flattened in
 *    (channel, y, x) order; weights of a convolution are [c_out][c_in][k][k].
 *  - Functions return asd_status; on failure no kernel has been launched and
 *    asd_last_error() describes the reason.  Calls are asynchronous on the
 *    given stream unless stated otherwise.  No call allocates device memory:
 *    all device storage comes from the caller's workspace.
 *  - One plan must not be used by two streams at once.
 */
#ifndef ASDUAL_H
#define ASDUAL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASD_ABI_VERSION 3
#define ASD_MAX_LAYERS 16
#define ASD_MAX_MASKS 8 /* compile-time cap on K_max (active masks per layer) */

typedef enum {
    ASD_OK = 0,
    ASD_EINVAL = 1,      /* invalid argument (shape, size, pointer, parameter) */
    ASD_ENOMEM = 2,      /* workspace too small */
    ASD_EDEVICE = 3,     /* a HIP runtime call failed */
    ASD_EUNSUPPORTED = 4 /* valid request outside what this build supports */
} asd_status;

typedef enum { ASD_LAYER_DENSE = 0, ASD_LAYER_CONV2D = 1 } asd_layer_kind;

/* One affine layer x_hat_k = W_k x_{k-1} + b_k (Sec. 2).  Every layer but the
 * last is followed by a ReLU.  The last layer's outputs are combined by
 * per-subproblem objective rows c (the paper's alpha_n).  It may be a
 * convolution (the sub-networks of eq:primal-intermediates end in one);
 * asd_bound_grad needs a dense one.
 * DENSE : in_c = inputs, out_c = outputs, in_h = in_w = 1, kernel/stride/pad
 *         ignored; W is [out_c][in_c] row-major.
 * CONV2D: cross-correlation with zero padding, square kernel `kernel`,
 *         same stride and padding in both directions; W is
 *         [out_c][in_c][kernel][kernel], b is [out_c]; out_h/out_w must equal
 *         (in + 2 pad - kernel) / stride + 1.
 * The input shape of layer k+1 must equal the output shape of layer k
 * (a dense layer after a convolution reads the (c, y, x) flattening). */
typedef struct {
    int32_t kind;
    int32_t in_c, in_h, in_w;
    int32_t out_c, out_h, out_w;
    int32_t kernel, stride, pad;
    const float* W; /* device, borrowed for the lifetime of the net */
    const float* b; /* device, borrowed for the lifetime of the net */
} asd_layer_desc;

typedef struct asd_net asd_net;
typedef struct asd_plan asd_plan;

/* Copies the descriptors; W and b stay borrowed until asd_net_destroy.
 * Errors: ASD_EINVAL for n_layers outside [2, ASD_MAX_LAYERS], shape
 * mismatches between consecutive layers, null pointers or non-positive
 * sizes. */
asd_status asd_net_create(const asd_layer_desc* layers /* host */, int32_t n_layers,
                          asd_net** out /* host */);
void asd_net_destroy(asd_net* net);

/* Update rules for the dual step H of Algorithm 1 (Sec. 7.1 uses Adam). */
typedef enum { ASD_RULE_ADAM = 0, ASD_RULE_SUPERGRADIENT = 1 } asd_rule;

/* Precision of a plan's state and arithmetic.  ASD_PREC_FP32 is the
 * production form (FP32 duals, moments and sums; the final bound is
 * re-evaluated in FP64).  ASD_PREC_FP64 keeps everything in FP64 (twice the
 * memory and traffic); it exists to compare whole runs with an FP64
 * reference.  ASD_PREC_MIXED is ASD_PREC_FP32 with the two Adam moments of
 * each multiplier stored together in one 32-bit word as BF16 between
 * iterations (round to nearest even; each update is computed in FP32 from
 * the stored values and steps with the unrounded result): one load and one
 * store of 4 bytes instead of two of 8, a third less state traffic per
 * multiplier.  The duals, the products and the
 * FP64 final bound are those of ASD_PREC_FP32, so the bound stays valid;
 * only the trajectory of the ascent changes.  The state calls exchange the
 * moments as float in every FP32-duals mode.  ASD_PREC_BF16 is
 * ASD_PREC_MIXED with BF16 operands in the matrix-core products of the
 * forward pass (W x* and |W| (sigma . x*), whose results form the
 * supergradient, eq:as-supergradient: weights and operands rounded to BF16,
 * nearest even, FP32 accumulation).  ASD_PREC_BF16_ALL also takes BF16
 * operands in the transposed products of the backward pass, whose results
 * f choose the minimiser (eq:as-primalk-min): near converged duals many f
 * lie within BF16 rounding of zero, and the wrong corners cost bound
 * accuracy, so the transposed products stay FP32 in ASD_PREC_BF16.  In both
 * the duals stay FP32 and the final bound is the FP64 evaluation from the
 * FP32 weights, so it stays valid; products the iteration runs on the
 * vector units (narrow convolutions, the last layer's backward pass) stay
 * FP32.  Network weights and batch inputs are FP32 in all modes. */
typedef enum {
    ASD_PREC_FP32 = 0,
    ASD_PREC_FP64 = 1,
    ASD_PREC_MIXED = 2,
    ASD_PREC_BF16 = 3,
    ASD_PREC_BF16_ALL = 4
} asd_precision;

/* Solver schedule (Sec. 7.1; readings: additions at Active Set iterations t
 * with t mod add_every < add_count while fewer than max_masks masks are
 * active; learning rates decrease linearly from lr0 at t = 0 to lr1 at
 * t = T - 1; Adam moments and step counters of alpha/beta_0/beta_1 are reset
 * when the Active Set phase starts; each added multiplier has its own). */
typedef struct {
    int32_t bigm_iters;   /* T_M, Algorithm 3 iterations (>= 0) */
    int32_t as_iters;     /* T, Algorithm 1 iterations (>= 0) */
    int32_t add_every;    /* omega (>= 1) */
    int32_t add_count;    /* V (>= 0) */
    int32_t max_masks;    /* K_max in [0, ASD_MAX_MASKS] */
    int32_t rule;         /* asd_rule */
    double bigm_lr0, bigm_lr1;
    double as_lr0, as_lr1;
    double adam_beta1, adam_beta2, adam_eps;
    int32_t precision;    /* asd_precision */
} asd_params;

/* Fills the defaults of Sec. 7.1 for CIFAR-10 branch and bound:
 * T_M = 180, T = 500, omega = 450, V = 2, K_max = 7, Adam (0.9, 0.999, 1e-8),
 * Big-M lr 1e-2 -> 1e-4, Active Set lr 1e-3 -> 1e-6, FP32. (host pointer) */
void asd_params_default(asd_params* p);

/* The problem batch: S independent subproblems on one net.  Every pointer is
 * device memory in the row-major [S][n] layout.
 *   l0, u0   [S][n_0]   input box, l0 <= u0
 *   lhat[k], uhat[k]    (k = 0 .. n_layers-2) [S][n_{k+1}] pre-activation
 *            bounds of ReLU layer k+1 (App. E), lhat <= uhat
 *   c        [S][n_last] objective rows: the bound is on c_s^T x_hat_n
 * `lhat` and `uhat` are HOST arrays of device pointers. */
typedef struct {
    int32_t S;
    const float* l0;
    const float* u0;
    const float* const* lhat; /* host array [n_layers-1] of device pointers */
    const float* const* uhat; /* host array [n_layers-1] of device pointers */
    const float* c;
} asd_batch;

/* Device workspace needed by a plan for S subproblems (host output).
 * Errors: ASD_EINVAL for S < 1 or invalid params. */
asd_status asd_plan_workspace_size(const asd_net* net, int32_t S, const asd_params* params,
                                   size_t* bytes /* host */);

/* Binds a caller-owned device workspace (>= asd_plan_workspace_size bytes,
 * 256-byte aligned) to a plan for S subproblems.  The plan keeps the
 * workspace until asd_plan_destroy.  Runs set-up kernels on `stream`
 * (sign-split weights).  Errors: ASD_EINVAL, ASD_ENOMEM if too small. */
asd_status asd_plan_create(const asd_net* net, int32_t S, const asd_params* params,
                           void* workspace, size_t bytes, hipStream_t stream,
                           asd_plan** out /* host */);
void asd_plan_destroy(asd_plan* plan);

/* Loads a batch into the plan (copies bounds into the plan's layout) and sets
 * every dual to zero with no active masks: the interval-propagation start of
 * Algorithm 3 (App. B).  The values are checked on the device (empty
 * intervals, non-finite entries) and reported per subproblem by
 * asd_check_finite.  Errors: ASD_EINVAL on S mismatch or null pointers. */
asd_status asd_init(asd_plan* plan, const asd_batch* batch, hipStream_t stream);

/* Phases of the solve. */
typedef enum { ASD_PHASE_BIGM = 0, ASD_PHASE_AS = 1 } asd_phase;

/* Runs iterations [t_begin, t_begin + n_iters) of one phase with the plan's
 * schedule (Algorithm 3 for ASD_PHASE_BIGM, Algorithm 1's inner loop with
 * active-set extension for ASD_PHASE_AS).  Starting the AS phase at
 * t_begin = 0 resets the Adam state of alpha/beta_0/beta_1.  Errors:
 * ASD_EINVAL if the range leaves [0, T) of the phase. */
asd_status asd_run(asd_plan* plan, int32_t phase /* asd_phase */, int32_t t_begin, int32_t n_iters,
                   hipStream_t stream);

/* Dual objective at the current duals (eq:dual-active-set), evaluated in FP64
 * from the FP32 duals and the FP32 weights, written to out_lb [S] (device,
 * double).  If x0 is not NULL, writes the input-layer minimiser x*_0 [S][n_0]
 * (device, float) at which the network can be evaluated for an upper bound
 * (Sec. 6.2 footnote). */
asd_status asd_bound(asd_plan* plan, double* out_lb, float* x0, hipStream_t stream);

/* Per-subproblem Active Set budgets (ragged batches of branch-and-bound
 * subdomains, each with its own iteration budget): budgets [S] (host),
 * each >= 1 and non-increasing in s (order the batch by budget).  Subproblem
 * s then runs Active Set iterations 0 .. budgets[s]-1 with its own linear
 * learning-rate schedule over budgets[s] (as a plan with T = budgets[s]
 * would), and its duals stay fixed afterwards; mask additions follow the
 * shared iteration count.  Iterations only touch the subproblems still
 * within budget (a prefix of the batch), so the work shrinks as budgets
 * run out.  The Active Set phase then has T = budgets[0] iterations.  NULL
 * clears the budgets.  Synchronises `stream` (the budgets are copied to the
 * plan's workspace).  Errors: ASD_EINVAL for a NULL plan or budgets that
 * are < 1 or increasing. */
asd_status asd_set_budgets(asd_plan* plan, const int32_t* budgets /* host */, hipStream_t stream);

/* Whole solve: asd_init, T_M Big-M iterations, T Active Set iterations
 * (T = budgets[0] with per-subproblem budgets), asd_bound.  out_lb [S]
 * device doubles. */
asd_status asd_solve(asd_plan* plan, const asd_batch* batch, double* out_lb, float* x0,
                     hipStream_t stream);

/* asd_solve with the iterations replayed from a HIP graph: the first call
 * (and the first after asd_set_budgets, asd_plan_set_tuning or
 * asd_plan_autotune) captures the Big-M and Active Set iterations of the
 * plan's schedule from `stream` into a graph and instantiates it; every call
 * runs asd_init (eager), launches the graph, then asd_bound (eager).  The
 * graph reads only the plan's workspace, so it serves any batch of the
 * plan's size.  Results equal asd_solve's.  Errors: those of asd_solve;
 * ASD_EINVAL while kernel profiling is on; ASD_EDEVICE if capture or
 * instantiation fails. */
asd_status asd_solve_graph(asd_plan* plan, const asd_batch* batch, double* out_lb, hipStream_t stream);

/* asd_solve without a plan or workspace of the caller's, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the plan is built for
 * this call over a static workspace the library holds on each GPU (64 MiB
 * per GPU, kept until the process ends), with the default kernel choices,
 * and runs asd_init, T_M Big-M and T Active Set iterations and asd_bound as
 * asd_solve does (same results).  out_lb [S] device doubles; x0 as for
 * asd_bound (may be NULL).  The call allocates nothing and calls no
 * allocating routine; all its work is stream-ordered on `stream`.  Every
 * call on one GPU uses the same workspace: calls that overlap on one GPU
 * (on different streams or threads) race, and must be serialised by the
 * caller.  Errors: ASD_EINVAL for NULL arguments, invalid params or a batch
 * whose plan would need more than the static workspace
 * (asd_plan_workspace_size > 64 MiB); ASD_EDEVICE if the workspace's device
 * address cannot be obtained. */
asd_status asd_solve_static(const asd_net* net, const asd_params* params, const asd_batch* batch,
                            double* out_lb, float* x0, hipStream_t stream);

/* Per-subproblem health of a solve: flags [S] (device, int32) receives, for
 * each subproblem s, bit 0 set if lb[s] (device [S], as written by asd_bound)
 * is not finite, bit 1 set if any multiplier of s (alpha, beta_0, beta_1,
 * the active masks' beta) is not finite, and bit 2 set if the inputs of s
 * that asd_init loaded are invalid: a non-finite value in l0, u0, lhat, uhat
 * or c, or an empty interval l0 > u0 or lhat > uhat (an infeasible subdomain,
 * Sec. 2: its bound is meaningless, not a bound); 0 for a healthy
 * subproblem.  The solve runs on such subproblems like on any other (no
 * fault, no effect on the rest of the batch).  Callers should treat flagged
 * subproblems as unverified.  Errors: ASD_EINVAL for NULL arguments or
 * before asd_init. */
asd_status asd_check_finite(asd_plan* plan, const double* lb, int32_t* flags, hipStream_t stream);

/* Solves several plans (for instance one per network of a mixed batch of
 * branch-and-bound subdomains, each plan with its own budgets) together:
 * asd_init of batches[i] into plans[i], then the Big-M and Active Set
 * iterations of all plans interleaved one iteration at a time, plan i's
 * kernels on streams[i] (host array of n_plans streams; distinct streams let
 * the plans' kernels overlap), then asd_bound into out_lb[i] (device [S_i]).
 * Each plan's result is the result of asd_solve on it alone.  Returns once
 * every launch is queued.  Errors: ASD_EINVAL for NULL entries, a repeated
 * plan, or any error of the calls above (launches already queued stay
 * queued). */
asd_status asd_solve_group(asd_plan* const* plans /* host */, const asd_batch* const* batches /* host */,
                           double* const* out_lb /* host */, int32_t n_plans, const hipStream_t* streams /* host */);

/* ---- Inspection and warm start (duals are the whole solver state) ---- */

/* State fields, per ReLU layer k = 1..n-1 and mask slot q (for ASD_F_MASK_*). */
typedef enum {
    ASD_F_ALPHA = 0, ASD_F_BETA0 = 1, ASD_F_BETA1 = 2,
    ASD_F_ALPHA_M = 3, ASD_F_ALPHA_V = 4,
    ASD_F_BETA0_M = 5, ASD_F_BETA0_V = 6,
    ASD_F_BETA1_M = 7, ASD_F_BETA1_V = 8,
    ASD_F_MASK_BETA = 9, ASD_F_MASK_M = 10, ASD_F_MASK_V = 11,
    ASD_F_MASK_LI = 12, ASD_F_MASK_UI = 13,
    /* the integral primal point the oracle was called at for slot q: z*_k of
     * layer k (0/1 per neuron) and x*_{k-1} of layer k-1 (values) */
    ASD_F_MASK_Z = 14, ASD_F_MASK_XPREV = 15
} asd_field;

/* Copies one field between the plan and a caller array [S][n] (device; float
 * for an FP32 plan, double for an FP64 plan; n = n_k, or n_{k-1} for
 * ASD_F_MASK_XPREV).  asd_state_set of ASD_F_MASK_Z /
 * ASD_F_MASK_XPREV re-derives the slot's compact mask; ASD_F_MASK_LI/UI are
 * recomputed by asd_state_set_counts (below) when `recompute` is set.
 * Errors: ASD_EINVAL for k outside [1, n-1] or q outside [0, max_masks). */
asd_status asd_state_get(asd_plan* plan, int32_t field, int32_t k, int32_t q, void* dst,
                         hipStream_t stream);
asd_status asd_state_set(asd_plan* plan, int32_t field, int32_t k, int32_t q, const void* src,
                         hipStream_t stream);

/* Scalar state: number of active masks per layer, the shared Adam step of
 * alpha/beta and each slot's Adam step (host values). */
typedef struct {
    int32_t n_masks;
    int32_t step;
    int32_t mask_step[ASD_MAX_MASKS];
} asd_counts;
asd_status asd_state_get_counts(const asd_plan* plan, asd_counts* out /* host */);
/* Sets the counts; with recompute != 0 also recomputes LI/UI of every active
 * slot from its stored primal point (runs kernels on `stream`). */
asd_status asd_state_set_counts(asd_plan* plan, const asd_counts* in /* host */, int32_t recompute,
                                hipStream_t stream);

/* ---- Fixed-dual evaluation and the separation oracle ---- */

/* Kernels asd_eval runs.  ASD_EVAL_GENERAL: the general term-wise kernels
 * (the arithmetic of FP64 plans and of the FP64 final bound).
 * ASD_EVAL_ITERATION: the kernels, kernel choices (asd_plan_autotune,
 * asd_plan_set_tuning) and shared launches an iteration of the plan runs,
 * with the dual step replaced by writing the supergradient; for an FP64 plan
 * those are the general kernels, so both paths are the same there. */
typedef enum { ASD_EVAL_GENERAL = 0, ASD_EVAL_ITERATION = 1 } asd_eval_path;

/* At the current duals and masks, computes with the plan's arithmetic:
 *   obj [S] (device, double): d_B (sum accumulated in FP64); general path
 *            only (the iteration kernels never form the objective: an FP32
 *            plan's bound is the FP64 evaluation of asd_bound),
 *   xstar[k] (k = 0..n-1) [S][n_k]: the minimiser x*_k (eq:as-primalk-min,
 *            eq:as-primal0-min), zstar[k] (k = 1..n-1) [S][n_k] 0/1 values,
 *   f[k] (k = 0..n-1), g[k] (k = 1..n-1) [S][n_k]: the coefficients of the
 *            Lagrangian in x_k and z_k (eq:dual-anderson-functions restricted
 *            to the active set, eq:dual-active-set) whose signs choose x*, z*;
 *            the iteration kernels do not form f exactly where the box of
 *            the neuron is a point (its x* is the box value whatever f is),
 *   grad_*[k] and grad_mask[k][q]: the supergradient (eq:as-supergradient)
 *            as [S][n_k] arrays.
 * Arrays are float for an FP32 or mixed plan and double for an FP64 plan.
 * Host arrays of device pointers; any entry may be NULL to skip it.  The
 * duals, moments and masks are not changed.  Errors: ASD_EINVAL for an
 * unknown path, or obj with ASD_EVAL_ITERATION in an FP32-duals plan. */
typedef struct {
    double* obj;
    void* xstar[ASD_MAX_LAYERS];
    void* zstar[ASD_MAX_LAYERS];
    void* grad_alpha[ASD_MAX_LAYERS];
    void* grad_beta0[ASD_MAX_LAYERS];
    void* grad_beta1[ASD_MAX_LAYERS];
    void* grad_mask[ASD_MAX_LAYERS][ASD_MAX_MASKS];
    void* f[ASD_MAX_LAYERS];
    void* g[ASD_MAX_LAYERS];
    int32_t path; /* asd_eval_path */
} asd_eval_out;
asd_status asd_eval(asd_plan* plan, const asd_eval_out* out /* host */, hipStream_t stream);

/* Separation oracle (Sec. 2.2, eq:oracle) for layer k at an arbitrary primal
 * point: x_prev [S][n_{k-1}] in the box of layer k-1, z [S][n_k] in [0,1]
 * (x_prev, z, LI, UI are float for an FP32 plan, double for an FP64 plan).
 * Writes the mask bits over each neuron's receptive field (fan-in F_k
 * entries per neuron in the order of the weights: dense j = 0..n_{k-1}-1;
 * conv (c_in, ky, kx), padding taps reported as 0) packed 32 per word,
 * mask_bits [S][n_k][ceil(F_k/32)] (uint32, bit t of word w is entry
 * 32 w + t), and LI, UI [S][n_k] (the row sums of W.I.Lcheck and
 * W.(1-I).Ucheck).  Uses the batch loaded by asd_init (bounds of layer k-1). */
asd_status asd_oracle(asd_plan* plan, int32_t k, const void* x_prev, const void* z,
                      uint32_t* mask_bits, void* LI, void* UI, hipStream_t stream);

/* ---- Gradient of the bound (adjoint) ---- */

/* Gradient of sum_s g[s] d_B(s) with respect to the network's weights and
 * biases and each subproblem's input box, at the plan's current duals and
 * active sets (the values asd_bound evaluates; the pre-activation bounds of
 * layers 1..n-1 are held fixed).  d_B is the minimum over the primal box of a
 * Lagrangian linear in (x, z) (constraint form of the relaxation, App. D), so
 * by Danskin's theorem its gradient is the Lagrangian's partial derivative at
 * the minimiser (x*, z*) wherever that is unique; at ties it is one
 * supergradient, with the tie rules of the minimiser (x* = u where f = 0,
 * z* = 1 where g = 0).  All sums run in FP64 (for an FP32 plan from the FP32
 * duals) in a fixed order: results are reproducible bit for bit.
 *   g      [S] (device, double): per-subproblem factors (the upstream
 *          gradient of a loss of the bounds); required.
 *   dW, db host arrays [n_layers] of device pointers (double), or NULL;
 *          any entry may be NULL to skip it.  dW[k] has the element count and
 *          order of layer k+1's W ([out_c][in_c] or [out_c][in_c][k][k]),
 *          db[k] has out_c entries; both are summed over the subproblems.
 *   dl0, du0 [S][n_0] (device, double, may be NULL): g[s] times the
 *          gradient of d_B(s) with respect to l0 and u0.
 *   reuse  nonzero: if asd_bound (or asd_bound_grad) ran last on this plan
 *          and no call has changed its state since, take the minimiser it
 *          left (the same values a recomputation gives); the caller
 *          guarantees that the network weights and the batch were not
 *          changed in place in between.  0: always recompute.
 * Overwrites the plan's minimiser buffers (as asd_bound does); the duals are
 * unchanged.  Errors: ASD_EINVAL for a NULL plan or g, before asd_init, a
 * convolutional output layer, or an l2-ball input domain. */
asd_status asd_bound_grad(asd_plan* plan, const double* g, double* const* dW /* host */,
                          double* const* db /* host */, double* dl0, double* du0, int32_t reuse,
                          hipStream_t stream);

/* ---- Input domain (Sec. 2: x_0 in a convex set C) ---- */

typedef enum { ASD_DOMAIN_BOX = 0, ASD_DOMAIN_L2 = 1 } asd_domain;

/* Input domain of the plan's subproblems, in force until the next call (a
 * plan starts with ASD_DOMAIN_BOX: the box [l0, u0] of the batch).
 * ASD_DOMAIN_L2: subproblem s ranges over the l2 ball ||x_0 - centre_s|| <=
 * radius_s (centre [S][n_0], radius [S], device floats, copied into the
 * workspace on `stream`); the batches given to asd_init must then hold the
 * ball's box hull (centre -/+ radius) as l0, u0, which bounds x_0 in the
 * check matrices of layer 1.  The minimiser x*_0 maximises f_0^T x_0 over
 * the ball (eq:as-primal0-min: centre + radius f_0 / ||f_0||, the centre
 * where f_0 = 0), in the iterations and in the final bound.  Masks added at
 * layer 1 keep multipliers 0: x*_0 lies inside the box hull, where
 * eq:oracle's rows only repeat the Big-M constraints.  asd_bound_grad
 * refuses an l2 plan.  Errors: ASD_EINVAL for a NULL plan, an unknown
 * domain, or NULL centre or radius with ASD_DOMAIN_L2. */
asd_status asd_set_input_domain(asd_plan* plan, int32_t domain, const float* centre, const float* radius,
                                hipStream_t stream);

/* ---- Intermediate bounds (App. E; interval propagation) ---- */

/* Pre-activation bounds of layers 1..n (FP64 arithmetic on the FP32 weights,
 * rounded outward to FP32): lhat[k], uhat[k] (k = 0..n_layers-1) [S][n_{k+1}] device
 * floats, host array of device pointers.  l0, u0 [S][n_0]. */
asd_status asd_interval_bounds(const asd_net* net, int32_t S, const float* l0, const float* u0,
                               float* const* lhat, float* const* uhat, hipStream_t stream);

/* ---- Intermediate bounds by the solver (App. E, eq:primal-intermediates) ---- */

/* Pre-activation bounds of the ReLU layers 1..n_layers-1 for D input boxes,
 * each from problem eq:primal-intermediates: layer 1 by interval
 * propagation (there the problem is a box-constrained LP); every neuron j of
 * a layer k >= 2 by the solver with `params` (Big-M, then Active Set, in
 * the plan precision `params->precision`) on the sub-network of layers
 * 1..k with the bounds already found for layers 1..k-1: objective row e_j
 * gives a lower bound of x_hat_k[j] and -e_j an upper bound (weak duality:
 * every dual point bounds the problem), each combined with interval
 * propagation from layer k-1 (lhat = max, uhat = min; the FP64 dual bounds
 * rounded outward to FP32).  Every bound is valid whatever the number of
 * iterations.  Layer k solves 2 n_k D subproblems on one plan in the
 * workspace; the sub-network of a convolutional layer k ends in that
 * convolution.
 *   l0, u0      [D][n_0] device floats (input boxes)
 *   lhat, uhat  host arrays [n_layers-1] of device pointers, [D][n_k]
 *               floats (outputs, k = 1..n_layers-1)
 *   workspace   device memory of at least
 *               asd_intermediate_workspace_size(net, D, params) bytes, owned
 *               by the caller (not needed, may be NULL, for 2 layers)
 * Asynchronous on `stream`.  Errors: ASD_EINVAL for NULL arguments, D < 1,
 * invalid params or a workspace that is too small. */
asd_status asd_intermediate_workspace_size(const asd_net* net, int32_t D, const asd_params* params,
                                           size_t* bytes /* host */);
asd_status asd_intermediate_bounds(const asd_net* net, int32_t D, const asd_params* params, const float* l0,
                                   const float* u0, float* const* lhat /* host */, float* const* uhat /* host */,
                                   void* workspace, size_t bytes, hipStream_t stream);

/* ---- Saddle Point (Sec. 5, Algorithm 2) and AS-SP ---- */

/* Saddle Point continues from the plan's current duals: after Big-M only
 * (asd_run of ASD_PHASE_BIGM) it is the paper's Saddle Point, after Active
 * Set iterations with masks it is AS-SP.  Its state lives in a second,
 * caller-owned workspace; the plan's own duals are read, never written.
 *   iters        T, SP-FW iterations (>= 0)
 *   gamma0       step sizes gamma_t = 1 / (t + gamma0), gamma0 >= 1 (Sec. 7.1
 *                uses 10; Sec. 5.2's 1 / (1 + t) is gamma0 = 1)
 *   init_steps   projected subgradient steps of the primal initialisation on
 *                the Big-M primal view (App. C.2), >= 0
 *   init_lr0/1   their step sizes, linear from lr0 to lr1
 *   cap_alpha    price caps (eq:price-caps): a multiplier set that is zero at
 *   cap_beta     initialisation gets this cap, > 0
 *   lds_staging  1: kernels that stage one subproblem's layer in LDS where it
 *                fits (the default); 0: every product from global memory
 *                (the same arithmetic, another summation order) */
typedef struct {
    int32_t iters;
    double gamma0;
    int32_t init_steps;
    double init_lr0, init_lr1;
    double cap_alpha, cap_beta;
    int32_t lds_staging;
} asd_sp_params;

/* Sec. 7.1 / App. C: T = 100, gamma0 = 10, 100 primal steps from 1e-2 to
 * 1e-5, caps 1e-3 for the multipliers that start at zero, LDS staging on.
 * (host pointer) */
void asd_sp_params_default(asd_sp_params* p);

/* Bytes of the Saddle Point workspace of a plan: per ReLU layer the duals
 * alpha, the four sufficient statistics of eq:suff-stats, the two price caps,
 * the primal iterate and conditional gradient, and FP64 objective terms; the
 * arrays hold the plan's precision (FP64 plans: double, otherwise float). */
asd_status asd_sp_workspace_size(const asd_plan* plan, size_t* bytes /* host */);

/* Algorithm 2's set-up on `stream`: converts the plan's duals (alpha,
 * beta_0, beta_1 and the active masks) into sufficient statistics
 * (eq:suff-stats), sets the price caps (eq:price-caps), starts the primal
 * iterate at the minimiser of the Lagrangian and runs the primal
 * initialisation.  `workspace` (256-byte aligned, >= asd_sp_workspace_size
 * bytes) stays bound to the plan until the next asd_sp_init or asd_init.
 * Errors: ASD_EINVAL before asd_init, for an l2-ball input domain, invalid
 * params, NULL or a workspace that is too small. */
asd_status asd_sp_init(asd_plan* plan, const asd_sp_params* params, void* workspace, size_t bytes,
                       hipStream_t stream);
/* SP-FW iterations t_begin .. t_begin + n_iters - 1 on `stream`: the primal
 * conditional gradient (the Lagrangian's minimiser at the current duals),
 * the dual one at the current primal iterate (eq:alphak-condg and the most
 * violated constraint per neuron, eq:betak-condg, found by the oracle
 * eq:oracle at the fractional iterate), then the convex combination with
 * gamma_t.  Errors: ASD_EINVAL without asd_sp_init, t_begin < 0. */
asd_status asd_sp_run(asd_plan* plan, int32_t t_begin, int32_t n_iters, hipStream_t stream);
/* The bound d(alpha, zeta) at the current Saddle Point duals (Algorithm 2's
 * return), evaluated in FP64 (an FP32 plan's statistics are read as stored),
 * into out_lb [S] (device doubles). */
asd_status asd_sp_bound(asd_plan* plan, double* out_lb, hipStream_t stream);
/* asd_sp_init, T iterations and asd_sp_bound. */
asd_status asd_sp_solve(asd_plan* plan, const asd_sp_params* params, void* workspace, size_t bytes,
                        double* out_lb, hipStream_t stream);

/* Arrays of the Saddle Point state, for asd_sp_read.  Layer k is a ReLU
 * layer (1..n_layers-1) except for ASD_SP_X and ASD_SP_XBAR (0..n_layers-1);
 * ASD_SP_ZETA2 of layer k has the size of layer k-1 (the coefficient of
 * x_{k-1} contributed by layer k's multipliers). */
typedef enum {
    ASD_SP_X = 0,      /* primal iterate x_k */
    ASD_SP_XBAR = 1,   /* primal conditional gradient of x_k at the current duals
                          (the Lagrangian's minimiser, used by the next iteration) */
    ASD_SP_ALPHA = 2,
    ASD_SP_ZETA1 = 3,  /* sum over masks of beta_{k,I} */
    ASD_SP_ZETA3 = 4,  /* beta_{k,1} (lhat - b) + sum_I (W . I . Lcheck) row sums beta_{k,I} */
    ASD_SP_ZETA4 = 5,  /* beta_{k,0} (uhat - b) + sum_I (W . (1-I) . Ucheck) row sums beta_{k,I} */
    ASD_SP_MU_ALPHA = 6,
    ASD_SP_MU_BETA = 7,
    ASD_SP_Z = 8,      /* primal iterate z_k */
    ASD_SP_ZETA2 = 9   /* sum_I (W_k . I)^T beta_{k,I} */
} asd_sp_field;
/* Copies one array into dst, the caller layout [S][n] in the plan's
 * precision (device), on `stream`.  Errors: ASD_EINVAL without asd_sp_init,
 * for an unknown field or a layer out of range. */
asd_status asd_sp_read(asd_plan* plan, int32_t field /* asd_sp_field */, int32_t k, void* dst,
                       hipStream_t stream);

/* ---- Autotuning of the iteration kernels ---- */

/* Kernel choices of an FP32-duals plan, per layer (index L-1 for layer L;
 * the backward entries are indexed by the neuron layer k they write):
 *   ksplit[L-1]   dense ReLU layer L: partial sums over the fan-in (1..8),
 *   fwd_mfma[L-1] convolutional ReLU layer L: forward on the matrix cores
 *                 (1; default from 32 channels) or the VALU column kernel (0),
 *   bwd_cb[k]     transposed convolution into layer k on the column kernel:
 *                 channels per thread (4 or 8; 0 = default); into a layer of
 *                 at most 4 channels (stride 2, rows of 8k positions): the
 *                 matrix-core kernel (0, default) or the VALU one (4),
 *   bwd_pos[k]    dense backward into layer k: the matrix cores (2, the
 *                 default; FP32, 64-position runs), positions on lanes (1)
 *                 or the column kernel (0),
 *   bwd_nt[k]     transposed convolution into layer k on the matrix cores:
 *                 16-position column tiles per wave (2 or 4; 0 = 2 where a
 *                 block's waves still cover every parity class at once),
 *   fwd_kw[L-1]   forward on the matrix cores: waves splitting the taps of
 *                 one 32 x 32 tile (convolution) or of one split (dense), 4 or 8,
 *   bwd_kw[k]     dense backward into layer k with positions on lanes: waves
 *                 splitting the outputs of layer k+1 (4 or 8; FP32 only). */
typedef struct {
    int32_t ksplit[ASD_MAX_LAYERS];
    int32_t fwd_mfma[ASD_MAX_LAYERS];
    int32_t bwd_cb[ASD_MAX_LAYERS];
    int32_t bwd_pos[ASD_MAX_LAYERS];
    int32_t bwd_nt[ASD_MAX_LAYERS];
    int32_t fwd_kw[ASD_MAX_LAYERS];
    int32_t bwd_kw[ASD_MAX_LAYERS];
} asd_tuning;

/* Times every alternative of the choices above on the loaded batch (each
 * kernel alone, `reps` launches after one warm-up, HIP events on `stream`)
 * with `ktune` mask slots active, and keeps the fastest.  The plan's state is
 * unchanged: the kernels run with the plain rule at step size 0 and the
 * slots beyond the active ones hold zero multipliers.  Call after asd_init
 * (before masks are added).  FP64 plans run the general kernels only: no-op.
 * Synchronises `stream`.  Errors: ASD_EINVAL before asd_init, for ktune
 * outside [0, max_masks] or below the active mask count, reps < 1. */
asd_status asd_plan_autotune(asd_plan* plan, int32_t ktune, int32_t reps, hipStream_t stream);
asd_status asd_plan_get_tuning(const asd_plan* plan, asd_tuning* out /* host */);
/* Sets the choices (entries of layers beyond the net are ignored).  Every
 * choice is valid for every shape: one a shape cannot take falls back to the
 * kernel it would use anyway.  Errors: ASD_EINVAL for values outside the
 * ranges above. */
asd_status asd_plan_set_tuning(asd_plan* plan, const asd_tuning* in /* host */);

/* ---- Kernel timing (for the benchmark's roofline figures) ---- */

/* Kernels the library launches in the iteration, by role. */
typedef enum {
    ASD_K_BACKWARD = 0,   /* f_k, inner minimisation (FP32) */
    ASD_K_FORWARD = 1,    /* products, supergradient, update */
    ASD_K_MASK = 2,       /* active-set extension */
    ASD_K_FINAL = 3,      /* FP64 final bound (all its kernels) */
    ASD_K_OTHER = 4,
    ASD_K_GRAD_WEIGHT = 5, /* asd_bound_grad: weight gradients */
    ASD_K_GRAD_BIAS = 6,   /* asd_bound_grad: bias gradients */
    ASD_K_GRAD_BOX = 7,    /* asd_bound_grad: input-box gradients */
    ASD_K_FORWARD_PASS = 8,  /* one launch holding the forward kernels of several
                                layers (layer = the lowest of them) */
    ASD_K_BACKWARD_PAIR = 9, /* one launch holding the backward kernels into the
                                last two neuron layers (layer = the lower one) */
    ASD_K_COUNT = 10
} asd_kernel_role;

typedef struct {
    int32_t role;       /* asd_kernel_role */
    int32_t layer;      /* layer index the launch works on (neuron layer for backward) */
    int32_t launches;
    double total_ms;    /* sum of HIP-event durations on the launch stream */
} asd_kernel_time;

/* Timing modes of asd_profile_enable. */
typedef enum {
    ASD_PROFILE_OFF = 0,
    ASD_PROFILE_LAUNCHES = 1, /* the launches as a solve runs them: kernels that
                                 share a launch are timed together
                                 (ASD_K_FORWARD_PASS, ASD_K_BACKWARD_PAIR) */
    ASD_PROFILE_KERNELS = 2   /* every kernel launched and timed alone */
} asd_profile_mode;

/* Starts (mode 1 or 2) or stops (0) recording a HIP event pair around every
 * iteration, mask, final-bound and gradient launch of this plan, on the
 * launch stream.  Enabling clears earlier records.  Recording adds host work
 * per launch; time runs without it.  Errors: ASD_EINVAL for another mode. */
asd_status asd_profile_enable(asd_plan* plan, int32_t mode);
/* Waits for the recorded events and writes per (role, layer) sums (host
 * array of `cap` entries); *count receives the number of entries. */
asd_status asd_profile_read(asd_plan* plan, asd_kernel_time* out /* host */, int32_t cap,
                            int32_t* count /* host */);

/* Thread-local description of the last error (never NULL). */
const char* asd_last_error(void);
int32_t asd_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ASDUAL_H */
