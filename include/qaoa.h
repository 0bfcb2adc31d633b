/*
 * qaoa.h -- C ABI of the MI355X (gfx950) QAOA statevector library.
 *
 * The library simulates depth-p QAOA for a diagonal cost C on n qubits
 * (Eq. (1)):  psi(gamma, beta) = U_M(beta_p) U_C(gamma_p) ... U_M(beta_1) U_C(gamma_1) |+>^n
 * with U_C(g) = exp(-i g C) and U_M(b) = prod_j exp(-i b X_j).
 *
 * Conventions shared by every call
 *   - Qubit / binary variable i is bit i of the basis index z (Eq. (2) uses 2^i).
 *   - Mixer sign: exp(-i b X) per qubit (the Farhi form).  The paper writes
 *     H_M = -sum X, i.e. exp(+i b X); its angles map to ours by b -> -b.
 *   - The objective is E = <psi|C|psi> with C the cut weight (MaxCut) or the
 *     0-1 polynomial value (QUBO); gradients are of E itself.
 *   - Host arrays passed in are copied during the call; the caller keeps them.
 *   - Every call validates its arguments before touching the GPU; on any error
 *     the outputs and the handle are left unchanged, except QAOA_ERR_DEVICE,
 *     which marks the handle unusable (qaoa_destroy stays valid).  Nothing
 *     throws or aborts across this boundary.
 *   - Work is ordered on the handle's HIP stream.  Calls that return values in
 *     host memory synchronise that stream before returning; device outputs are
 *     stream-ordered.  One thread may use a handle at a time; distinct handles
 *     are independent.
 *   - Complex amplitudes are interleaved (re, im): complex128 = 2 x fp64,
 *     complex64 = 2 x fp32, matching numpy/torch complex dtypes.
 */
#ifndef QAOA_MI355X_QAOA_H
#define QAOA_MI355X_QAOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qaoa_handle_s *qaoa_handle;

typedef enum {
    QAOA_OK = 0,
    QAOA_ERR_INVALID_ARGUMENT = 1, /* bad size, index, NULL pointer, non-finite value */
    QAOA_ERR_OUT_OF_MEMORY = 2,    /* device buffers do not fit (checked before allocating) */
    QAOA_ERR_DEVICE = 3,           /* a HIP call failed; the handle is now unusable */
    QAOA_ERR_NO_STATE = 4,         /* the call needs a current state (qaoa_statevector first) */
    QAOA_ERR_UNSUPPORTED = 5
} qaoa_status;

typedef enum {
    QAOA_C128 = 0, /* complex128 state, fp64 cost diagonal */
    QAOA_C64 = 1   /* complex64 state, fp32 cost diagonal; phases reduced in fp64, sums in fp64
                      (a thread's 16 pair products for one qubit are summed in fp32 first) */
} qaoa_precision;

/* Largest supported qubit count (further bounded by free device memory). */
#define QAOA_MAX_QUBITS 40

/*
 * Create a handle for weighted MaxCut (Sec. V: MaxCut benchmark; Sec. IV-A: cost
 * function representation).  C(z) = sum of w[k] over edges k = (i, j) with
 * bit i of z != bit j of z, added in edge order (so integer weights give exact
 * values).
 *   n       1 <= n <= QAOA_MAX_QUBITS
 *   m       number of edges, m >= 0
 *   edges   host int32 [m][2]; 0 <= i, j < n, i != j; repeated edges add
 *   w       host fp64 [m], finite; NULL means unit weights
 *   precision  a qaoa_precision value
 *   stream  hipStream_t to order all work on; NULL creates a private stream
 *   out     receives the handle
 * The handle allocates the state and cost diagonal on the current HIP device
 * (Sec. IV-B: state and cost arrays at initialisation, other buffers lazily when
 * first needed).  The cost diagonal is built here.
 * Errors: INVALID_ARGUMENT, OUT_OF_MEMORY (2^n buffers exceed free memory), DEVICE.
 */
qaoa_status qaoa_create_maxcut(int32_t n, int64_t m, const int32_t *edges, const double *w,
                               int32_t precision, void *stream, qaoa_handle *out);

/*
 * Create a handle for a 0-1 QUBO, the degree-2 case of Eq. (2):
 * C(z) = offset + sum_k J[k] x_i x_j + sum_i h[i] x_i,  x_i = bit i of z,
 * accumulated as offset, then pair terms in the given order, then linear
 * terms in variable order.
 *   pairs   host int32 [m][2], 0 <= i, j < n, i != j
 *   J       host fp64 [m] (may be NULL when m == 0)
 *   h       host fp64 [n] or NULL (no linear terms)
 *   offset  finite constant
 * Other arguments and errors as qaoa_create_maxcut.
 */
qaoa_status qaoa_create_qubo(int32_t n, int64_t m, const int32_t *pairs, const double *J,
                             const double *h, double offset, int32_t precision, void *stream,
                             qaoa_handle *out);

/*
 * Create a handle for a general 0-1 polynomial (Eq. (2)): term k has the
 * one-hot mask masks[k] = sum_{i in t_k} 2^i and weight w[k], and is active in
 * z iff (z AND masks[k]) == masks[k].  C(z) = offset + sum of the active
 * weights, added in term order.  A zero mask is a constant term.
 *   L       number of terms, L >= 0
 *   masks   host uint64 [L], every mask < 2^n
 *   w       host fp64 [L], finite
 * Other arguments and errors as qaoa_create_maxcut.
 */
qaoa_status qaoa_create_poly(int32_t n, int64_t L, const uint64_t *masks, const double *w,
                             double offset, int32_t precision, void *stream, qaoa_handle *out);

/*
 * Release the handle (Sec. IV-B: the handle owns the state, the cost array, a
 * stream and every buffer allocated later): waits for the handle's stream,
 * frees every device buffer through the allocator the handle was created with
 * and destroys the private stream (a caller's stream is left alone).  Valid
 * after QAOA_ERR_DEVICE.  NULL is a no-op.
 */
qaoa_status qaoa_destroy(qaoa_handle h);

/* Report n and the precision of a handle (either output pointer may be NULL). */
qaoa_status qaoa_get_info(qaoa_handle h, int32_t *n, int32_t *precision);

/*
 * Copy the cost diagonal C[0 .. 2^n) (Sec. IV-A, Eq. (2)) as fp64 into `out`.
 * For QAOA_C64 handles the stored fp32 values are widened exactly.
 *   out            fp64 [2^n], host or device memory
 *   out_is_device  nonzero if `out` is device memory (copy is stream-ordered)
 */
qaoa_status qaoa_cost_diagonal(qaoa_handle h, double *out, int32_t out_is_device);

/*
 * Minimum and maximum of the cost diagonal of Eq. (2) (Sec. IV-A), reduced on
 * the device over all 2^n entries (for approximation ratios E / C_max).  The
 * values are cached in the handle after the first call.  Synchronises the
 * stream.  Errors: INVALID_ARGUMENT (NULL outputs), DEVICE.
 */
qaoa_status qaoa_cost_extrema(qaoa_handle h, double *cmin, double *cmax);

/*
 * Prepare the QAOA state for angles gamma[p], beta[p] (Eq. (1); phase layer by
 * Euler's formula, Sec. IV-B) and make it the handle's current state.
 *   p             p >= 0 (p = 0 gives |+>^n)
 *   gamma, beta   host fp64 [p], finite (may be NULL when p == 0)
 *   out           NULL, or 2^n complex amplitudes (complex128 or complex64 per
 *                 the handle's precision) receiving a copy of the state
 *                 (Sec. IV-D: statevector export)
 *   out_is_device nonzero if `out` is device memory
 */
qaoa_status qaoa_statevector(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                             void *out, int32_t out_is_device);

/* E = sum_z C[z] |psi_z|^2 of the current state (Sec. IV-D).  NO_STATE without one. */
qaoa_status qaoa_expectation(qaoa_handle h, double *E);

/*
 * E(gamma, beta) in one fused sweep: the expectation is accumulated inside the
 * last mixer pass instead of a separate reduction.  Leaves the state current.
 */
qaoa_status qaoa_evaluate(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                          double *E);

/*
 * Expectation and its gradient with respect to all 2p angles by adjoint
 * differentiation (Sec. II-B, Sec. IV-C): dE/dtheta_k = 2 Im <lam_k|H_k|phi_k>,
 * where the layer states phi_k are recomputed by applying inverse layers to the
 * final state (none are stored) and H_k is C or sum_j X_j.
 *   E       host fp64 scalar (may be NULL)
 *   dgamma  host fp64 [p]
 *   dbeta   host fp64 [p]
 * Allocates the adjoint vector on first use.  Consumes the state: afterwards
 * the handle has no current state.
 */
qaoa_status qaoa_gradient(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                          double *E, double *dgamma, double *dbeta);

/*
 * The gradient at the angles of the handle's current state, by the adjoint
 * reverse sweep alone (Sec. II-B, IV-C): for a caller that has already run the
 * forward evolution with qaoa_evaluate or qaoa_statevector at the same
 * (gamma, beta) (an autograd forward that may or may not be followed by a
 * backward).  The first backward pass forms lam = C phi from the stored final
 * state; the layer states are recomputed by inverse layers as in
 * qaoa_gradient, whose results it matches to rounding.
 *   gamma, beta    host fp64 [p], equal (bit for bit) to the angles of the
 *                  current state
 *   dgamma, dbeta  host fp64 [p]
 * Errors: NO_STATE without a current state or with a state computed at other
 * angles.  Allocates the adjoint vector on first use.  Consumes the state.
 */
qaoa_status qaoa_gradient_from_state(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                                     double *dgamma, double *dbeta);

/*
 * qaoa_gradient without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same results as qaoa_gradient (the same kernels in the
 * same order).  The adjoint vector, the partial sums and the summed slots are
 * taken from a fixed scratch array of 16 MiB + 256 KiB that the library holds
 * on each device it runs on until the process ends; the handle's state and
 * cost diagonal (allocated at creation) are used as by qaoa_gradient.
 *   p                    0 <= p <= 32
 *   E, dgamma, dbeta     as qaoa_gradient (E may be NULL); host memory, or
 *                        device memory when out_is_device is nonzero (then
 *                        nothing is synchronised and the call can be captured
 *                        into a HIP graph)
 * Limits: the adjoint vector must fit the scratch: complex128 n <= 20,
 * complex64 n <= 21; larger n or p gives INVALID_ARGUMENT with the sizes in
 * the message.  Every call on one device shares that device's scratch, so
 * calls that overlap on one GPU (other threads, other streams) race; calls
 * ordered on one stream are safe.  Nothing in the scratch needs clearing:
 * every slot is written before it is read.  Consumes the state like
 * qaoa_gradient.  Errors: INVALID_ARGUMENT, DEVICE, UNSUPPORTED (device index
 * >= 64).
 */
qaoa_status qaoa_gradient_noalloc(qaoa_handle h, int32_t p, const double *gamma, const double *beta,
                                  double *E, double *dgamma, double *dbeta, int32_t out_is_device);

/*
 * Draw `shots` basis states from |psi_z|^2 of the current state and return
 * each with its objective value (Sec. IV-D).  Shot s uses the uniform
 * u_s = top 53 bits of Philox-4x32-10(counter = (s, 0), key = seed) * 2^-53 and
 * returns the smallest z whose cumulative probability exceeds u_s * sum|psi|^2;
 * a zero-probability state is never returned.  Results are in shot order and
 * are deterministic for a given (state, seed).
 *   z     uint64 [shots] receiving basis indices
 *   cost  fp64 [shots] receiving C[z], or NULL
 *   out_is_device  nonzero if z / cost are device memory
 * Errors: NO_STATE; INVALID_ARGUMENT for shots outside [0, 2^40] or a zero-norm
 * state; OUT_OF_MEMORY when host outputs need more device staging than is free.
 */
qaoa_status qaoa_sample(qaoa_handle h, int64_t shots, uint64_t seed, uint64_t *z, double *cost,
                        int32_t out_is_device);

/*
 * Limited-memory BFGS (Sec. V-B offers L-BFGS natively; Liu & Nocedal 1989):
 * two-loop recursion with m stored correction pairs and a strong-Wolfe line
 * search (c1 = 1e-4, c2 = 0.9).  Every trial point costs one evaluation.
 */
typedef int (*qaoa_objective_fn)(const double *x, double *f, double *g, void *user);
/* f(x) and its gradient g(x); return 0 on success, nonzero to stop the optimiser. */

typedef struct {
    int32_t max_iter;  /* accepted steps, >= 0 */
    int32_t history;   /* stored correction pairs m, >= 1 */
    double gtol;       /* stop when max_i |g_i| <= gtol */
    double ftol;       /* stop when |f_k - f_k+1| <= ftol * max(1, |f_k+1|); 0 disables */
    int32_t max_evals; /* cap on evaluations, >= 1 */
} qaoa_lbfgs_options;

/*
 * Minimise fn over R^dim starting from x (host, in-out).  opt NULL means
 * {100, 10, 1e-8, 0, 1000}.  Outputs (each may be NULL): fx = f at the returned
 * x, iters = accepted steps, evals = evaluations used, trace_x [(max_iter+1) x
 * dim] and trace_f [max_iter+1] receive the iterates x_0 .. x_iters and their f.
 * The search stops early (returning the best accepted point) when the line
 * search fails or max_evals is reached.
 * Errors: INVALID_ARGUMENT (dim < 1, NULL x/fn, bad options, non-finite x);
 * DEVICE if the first evaluation fails.
 */
qaoa_status qaoa_lbfgs_minimize(int32_t dim, double *x, qaoa_objective_fn fn, void *user,
                                const qaoa_lbfgs_options *opt, double *fx, int32_t *iters,
                                int32_t *evals, double *trace_x, double *trace_f);

/*
 * Maximise E(gamma, beta) with qaoa_lbfgs_minimize on -E, each evaluation being
 * one qaoa_gradient call.  gamma, beta (host [p], in-out) hold the start and
 * receive the optimum; E receives E at the optimum.  trace_x rows are
 * (gamma, beta) of each iterate and trace_f holds E (not -E).  The handle has
 * no current state afterwards.  Errors as qaoa_gradient and qaoa_lbfgs_minimize.
 */
qaoa_status qaoa_optimize(qaoa_handle h, int32_t p, double *gamma, double *beta,
                          const qaoa_lbfgs_options *opt, double *E, int32_t *iters, int32_t *evals,
                          double *trace_x, double *trace_f);

/*
 * Kernel timing for measurement.  While enabled, every streaming pass launch
 * (forward, turn and backward passes of qaoa_statevector / qaoa_evaluate /
 * qaoa_gradient) is bracketed by a pair of HIP events on the handle's stream.
 * qaoa_profile_enable (re)starts the counters (on != 0) or stops timing
 * (on == 0).  qaoa_profile_read synchronises the stream and reports, for one
 * pass kind (0 forward, 1 turn, 2 backward, 3 layer-boundary forward, 4
 * layer-boundary backward), the number of launches, their
 * summed GPU time in milliseconds and their summed algorithmic bytes (each
 * amplitude vector read or written once, plus one cost-diagonal read where the
 * pass applies or measures C).  Any output pointer may be NULL.
 */
qaoa_status qaoa_profile_enable(qaoa_handle h, int32_t on);
qaoa_status qaoa_profile_read(qaoa_handle h, int32_t kind, int64_t *launches, double *ms,
                              double *bytes);

/*
 * Pass plan of one mixer layer (host-side introspection; no GPU is touched).
 * The n rotations exp(-i b X_j) of a layer commute (Eq. (1)), so the library
 * applies them in a few sweeps over the state.  In sweep i one workgroup owns
 * the 2^min(n,TB) amplitudes whose indices differ only in the bits of
 * tile_bits[i] (TB = 12 for QAOA_C128, 13 for QAOA_C64: 64 KiB of state) and
 * rotates the qubits in target_bits[i]; the remaining tile bits are low
 * spectator bits kept for contiguous memory access (runs of >= 64 bytes).
 *   cap       capacity of the two output arrays
 *   npasses   receives the number of sweeps per layer
 * Errors: INVALID_ARGUMENT for n outside [1, QAOA_MAX_QUBITS], an unknown
 * precision, NULL outputs, or cap smaller than the number of sweeps.
 */
qaoa_status qaoa_pass_plan(int32_t n, int32_t precision, int32_t cap, int32_t *npasses,
                           uint64_t *tile_bits, uint64_t *target_bits);

/*
 * Batched engine: many small weighted MaxCut instances, each optimised with
 * Adam on its 2p angles, in one persistent launch (Sec. V-B: parameter
 * optimisation driven by the simulator's gradients; here every instance's loop
 * runs on the device).
 *
 * A fixed grid of workgroups takes instances from an on-device queue, largest
 * n first.  A workgroup runs one instance start to end in its own scratch slot
 * (state, adjoint vector and cost diagonal, 2^nmax amplitudes each, complex128):
 * cost diagonal (as qaoa_create_maxcut), then `steps` Adam ascent steps on
 * E(gamma, beta) / sum_k |w_k|, each step one expectation + adjoint gradient
 * with the same tiled passes as qaoa_gradient, then E at the final angles.
 * Adam (Kingma & Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * theta += lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), t = 1, 2, ...
 * The queue-reset kernel and the engine are captured once in a hipGraph and
 * replayed by every qaoa_batch_run.
 *
 * Instances of at most 12 qubits are a single 4096-amplitude tile.  With
 * resident_max_n set, those up to that size run in a second persistent launch
 * after the first, whose workgroups (one per compute unit) keep the instance's
 * state and adjoint vector in LDS through all of its Adam steps instead of
 * streaming them through the slot between passes; results are the same.  Each
 * such workgroup is faster, but the streamed launch fits two per compute unit,
 * so which mode wins depends on the batch (the autotuner measures both).
 */
typedef struct qaoa_batch_s *qaoa_batch;

/* Largest qubit count of a batched instance. */
#define QAOA_BATCH_MAX_QUBITS 24

typedef struct {
    int32_t steps;      /* Adam steps per instance, >= 0 */
    double lr;          /* step size, > 0 */
    double beta1;       /* first-moment decay, [0, 1) */
    double beta2;       /* second-moment decay, [0, 1) */
    double eps;         /* > 0 */
    int32_t workgroups; /* persistent workgroups (scratch slots); 0 = 2 per compute unit */
    int32_t max_group;  /* most qubits rotated per mixer pass after the first, 1..10 */
    int32_t use_graph;  /* nonzero: replay a captured hipGraph; 0: launch eagerly */
    int32_t waves_per_simd; /* register budget of the engine kernel: 1 or 2 waves per SIMD (0 = 1) */
    int32_t group_by_n[QAOA_BATCH_MAX_QUBITS + 1]; /* per-n override of max_group; 0 = none */
    int32_t resident_max_n; /* instances with n <= this (0..12) keep state and adjoint vector in
                               LDS; 0 = none */
} qaoa_batch_options;

/*
 * Create a batch of `count` MaxCut instances of depth p (1 <= p <= 16).
 *   n             host int32 [count], each in [2, QAOA_BATCH_MAX_QUBITS]
 *   edge_offsets  host int64 [count + 1], edge_offsets[0] = 0, non-decreasing;
 *                 instance i owns edges [edge_offsets[i], edge_offsets[i+1])
 *   edges         host int32 [E][2] with vertex indices local to the instance
 *                 (0 <= u, v < n[i], u != v); E = edge_offsets[count]
 *   w             host fp64 [E], finite; NULL means unit weights
 *   opt           NULL means {100, 0.05, 0.9, 0.999, 1e-8, 0, 10, 1, 0, {0}, 0}
 * Allocates all device memory (instances, angles, scratch slots) on the current
 * device and its own non-blocking stream; nothing is allocated by qaoa_batch_run.
 * Errors: INVALID_ARGUMENT, OUT_OF_MEMORY (slots exceed free memory), DEVICE.
 */
qaoa_status qaoa_batch_create(int32_t count, const int32_t *n, const int64_t *edge_offsets,
                              const int32_t *edges, const double *w, int32_t p,
                              const qaoa_batch_options *opt, qaoa_batch *out);

/*
 * Optimise every instance from the start angles gamma0, beta0 (host fp64
 * [count][p], finite).  Outputs (host, each may be NULL): gamma, beta
 * [count][p] the final angles; e_first [count] E at the start angles;
 * e_last [count] E at the final angles.  Synchronous.  Results depend only on
 * the inputs (each instance is processed by one workgroup in a fixed order).
 * Errors: INVALID_ARGUMENT; DEVICE (the batch is then unusable).
 */
qaoa_status qaoa_batch_run(qaoa_batch b, const double *gamma0, const double *beta0, double *gamma,
                           double *beta, double *e_first, double *e_last);

/*
 * Timeline of the last qaoa_batch_run: for every instance (host fp64 [count]
 * each, may be NULL) the time its workgroup took it from the queue and the
 * time it wrote its results, in seconds from the earliest start, read from the
 * device's constant-rate wall clock; which_launch (host int32 [count], may be
 * NULL) is 0 for the streamed launch and 1 for the LDS-resident one.  For
 * measuring how evenly the persistent workgroups are loaded.
 * Errors: INVALID_ARGUMENT (no run yet); DEVICE.
 */
qaoa_status qaoa_batch_timeline(qaoa_batch b, double *start_s, double *end_s, int32_t *which_launch);

/* Release the batch's device memory, graph and stream.  NULL is accepted. */
qaoa_status qaoa_batch_destroy(qaoa_batch b);

/*
 * Warm-start network: a message-passing network that predicts depth-p QAOA
 * angles from a weighted graph, so that an optimiser (qaoa_optimize, or the
 * batched engine) can start near good angles instead of at the linear ramp of
 * Sec. II (QAOA background: the constant-speed schedule).
 *
 *   node input   x_v = (deg_v / 8, wdeg_v / 8, 1, sqdeg_v / 8, 0 ... 0), 32
 *                features: deg_v the number of incident edges, wdeg_v the sum
 *                of their weights, sqdeg_v the sum of their squared weights
 *   layer l      H' = ReLU([H | A H] W_l^T + b_l), l = 0, 1, 2, width 128,
 *                A the symmetric weighted adjacency
 *   readout      g = mean of H over the graph's nodes
 *   head         Y = ReLU(g W_h1^T + b_h1) W_h2^T + b_h2, 2p outputs
 *   angles       gamma_i = i/p + Y_i, beta_i = 1 - i/p + Y_{p+i}, i = 1..p
 *   loss         mean over graphs and angles of (angle - target)^2
 *
 * Flat fp32 parameter vector, in this order: for l = 0, 1, 2: W_l [128][2 d_l]
 * row-major (d_0 = 32, d_1 = d_2 = 128) then b_l [128]; W_h1 [128][128],
 * b_h1 [128], W_h2 [2p][128], b_h2 [2p].
 *
 * Products run on bf16 matrix cores with fp32 accumulation; their operands
 * (activations, messages, a bf16 copy of the fp32 master weights, and the
 * gradients entering weight-gradient products) are rounded to bf16 (nearest
 * even).  Everything else is fp32.  Reductions have a fixed order.
 *
 * Graph batches use the layout of qaoa_batch_create: n [count] (1..4096 nodes
 * each, at most 2^24 in total), edge_offsets [count+1], edges [E][2] with local
 * vertex indices (no self-loops), w [E] finite or NULL for unit weights.
 */
typedef struct qaoa_mpnn_s *qaoa_mpnn;

typedef struct {
    double lr;    /* > 0 */
    double beta1; /* [0, 1) */
    double beta2; /* [0, 1) */
    double eps;   /* > 0 */
} qaoa_mpnn_adam;

/* Number of parameters of the depth-p network (1 <= p <= 16). */
qaoa_status qaoa_mpnn_num_params(int32_t p, int64_t *count);

/* Create a network with all parameters zero on the current device. */
qaoa_status qaoa_mpnn_create(int32_t p, qaoa_mpnn *out);

/* Release the network's device memory and stream.  NULL is accepted. */
qaoa_status qaoa_mpnn_destroy(qaoa_mpnn m);

/* Set the parameters from host fp32 [num_params] (finite); resets Adam's state. */
qaoa_status qaoa_mpnn_set_params(qaoa_mpnn m, const float *theta);

/* Copy the fp32 master parameters to host memory [num_params]. */
qaoa_status qaoa_mpnn_get_params(qaoa_mpnn m, float *theta);

/* Predicted angles for a batch of graphs: gamma, beta host fp64 [count][p]. */
qaoa_status qaoa_mpnn_predict(qaoa_mpnn m, int32_t count, const int32_t *n, const int64_t *edge_offsets,
                              const int32_t *edges, const double *w, double *gamma, double *beta);

/*
 * Loss against target angles (host fp64 [count][p] each, finite) and its
 * gradient with respect to the parameters (host fp32 [num_params], may be
 * NULL).  The parameters are not changed.
 */
qaoa_status qaoa_mpnn_loss_grad(qaoa_mpnn m, int32_t count, const int32_t *n, const int64_t *edge_offsets,
                                const int32_t *edges, const double *w, const double *gamma_t,
                                const double *beta_t, double *loss, float *grad);

/*
 * One training step: loss and gradient as qaoa_mpnn_loss_grad, then one Adam
 * descent step (Kingma & Ba 2015) on the fp32 master parameters, whose bf16
 * copy is refreshed.  opt NULL means {1e-3, 0.9, 0.999, 1e-8}.  loss (may be
 * NULL) receives the loss before the update.
 */
qaoa_status qaoa_mpnn_train_step(qaoa_mpnn m, int32_t count, const int32_t *n, const int64_t *edge_offsets,
                                 const int32_t *edges, const double *w, const double *gamma_t,
                                 const double *beta_t, const qaoa_mpnn_adam *opt, double *loss);

/*
 * Device-memory provider for handles (e.g. a framework's caching allocator, so
 * that the simulator's buffers share its pool).  alloc returns `bytes` of
 * device memory on the current device, usable on `stream` (the handle's
 * stream), or NULL on failure (reported as QAOA_ERR_OUT_OF_MEMORY); free
 * releases it (called after the handle's stream has been synchronised).
 */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, size_t bytes, void *stream, void *user);
    void *user;
} qaoa_allocator;

/*
 * Allocator for the state, cost diagonal, adjoint vector and scratch buffers
 * of handles created afterwards on the calling thread; each handle keeps the
 * allocator it was created with until qaoa_destroy.  NULL restores
 * hipMalloc/hipFree.  With an allocator set, the free-memory pre-checks are
 * left to it.  Errors: INVALID_ARGUMENT if alloc or free is NULL.
 */
qaoa_status qaoa_set_allocator(const qaoa_allocator *a);

/*
 * Static English description of a status code.  Together with
 * qaoa_last_error_message this is how the boundary reports errors: no call
 * throws or aborts, each returns a status (the handle of Sec. IV-B is the
 * only state a call keeps).
 */
const char *qaoa_status_string(qaoa_status s);

/* Message of the last failing call on this thread ("" if none); valid until
 * the next failing call on the same thread. */
const char *qaoa_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* QAOA_MI355X_QAOA_H */
