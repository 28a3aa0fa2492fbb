/*
 * kfac_pinn.h -- C ABI of the MI355X (gfx950) KFAC-PINN library.
 *
 * One KFAC step for a physics-informed neural network loss, as defined in
 * Dangel, Mueller & Zeinhofer, "Kronecker-Factored Approximate Curvature for
 * Physics-Informed Neural Networks" (NeurIPS 2024):
 *   forward Laplacian of a tanh MLP (Section 3.1, Eq. forward-laplacian-main),
 *   PDE residual and loss (Section 2.1, Eq. pinn-loss), output gradients by a
 *   backward pass (Algorithm 1), Kronecker factors (Section 3.2, Eq. KFAC-PINN;
 *   Eq. kfac-linear for the boundary term), EMA + damping and the inverse of
 *   the Kronecker sum (Section 3.4), momentum and grid line search (Section 3.4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Network: L = n_layers linear layers with widths[0] = d inputs, widths[L] = 1
 *   output, tanh between layers.  Parameters theta follow Section 2: layer l's
 *   augmented matrix [W | b] (h_out x (h_in+1)) is stacked column by column
 *   (bias is the last column), layers are concatenated; D = sum h_out (h_in+1).
 * Element type "real": double for KP_F64, float for KP_F32, KP_MIXED_BF16 and
 *   KP_MIXED_F16 (FP32 master parameters).  Points are row-major n x d reals, targets are n
 *   reals.  Factors, gradients and preconditioners are always double.
 * Residuals: interior r = c_t du/dx_t + c_lap sum_{i in mask} d2u/dx_i^2 - y
 *   (or c_lap sum_ij C_ij d2u/dx_i dx_j with a coefficient matrix, kp_problem),
 *   plus sum_{i in mask} (c_x x_i du/dx_i + c_g (du/dx_i)^2) + c_0 for PDEs whose
 *   residual depends on the first derivatives non-linearly (Section 3.3; the
 *   logarithmic Fokker-Planck equation of Section 4: c_t = 1, c_lap = -1,
 *   c_x = -1/2, c_g = -1, c_0 = -d_x/2, t outside the mask).  The output gradients
 *   g then use the point-dependent seed dr/dU.
 *   (Poisson -Lap u = f: c_t = 0, c_lap = -1, y = f; heat u_t = kappa Lap_x u:
 *   c_t = 1, c_lap = -kappa, t excluded from the mask); boundary r = u - y.
 *   Loss L = sum r^2/(2N) + sum r_b^2/(2M).
 * Pointers: every array argument is DEVICE memory owned by the caller unless
 *   the comment says "host".  It must stay valid until the work enqueued on the
 *   context's stream has finished.  The context owns all workspaces (allocated
 *   in kfac_pinn_create); no other entry point allocates device memory except
 *   kfac_pinn_set_line_search_lanes (which frees or re-makes the second
 *   line-search lane's buffers).  The context's internal streams (default
 *   priority) are created by its first inversion; work an entry point forks
 *   onto them (the inversion's Jacobi groups, the second line-search lane) is
 *   joined back into the context's stream before the entry point returns, so
 *   the order that the caller sees on that stream is unchanged.
 * Errors: invalid arguments return KP_ERR_ARG synchronously and enqueue
 *   nothing.  HIP launch failures return KP_ERR_HIP.  Failures found on the
 *   device set the context's device status word: a damped interior factor that
 *   is not positive definite (KP_ERR_NOT_PD), a non-finite loss at theta_t or at
 *   every line-search candidate (KP_ERR_NONFINITE; it takes precedence, being the
 *   cause of the others), an eigensolver that reached its sweep cap unconverged
 *   (KP_ERR_NOT_CONVERGED, only when nothing failed before it).  The parameter
 *   update is then skipped (theta, the momentum and the step counter stay
 *   untouched) and kfac_pinn_sync returns the code.  The Kronecker factors
 *   already hold the failed step's EMA; kfac_pinn_reset_state or
 *   kfac_pinn_set_factor restores them.
 * Threads: a context is not thread-safe; distinct contexts are independent.
 */
#ifndef KFAC_PINN_H
#define KFAC_PINN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kfac_pinn_ctx kfac_pinn_ctx;

typedef enum {
  KP_OK = 0,
  KP_ERR_ARG = 1,
  KP_ERR_OOM = 2,
  KP_ERR_HIP = 3,
  KP_ERR_NOT_PD = 4,
  KP_ERR_NONFINITE = 5,
  KP_ERR_STATE = 6,
  KP_ERR_NOT_CONVERGED = 7  /* the Jacobi eigensolver of the Kronecker-sum inverse
                               reached its sweep cap with rotations left        */
} kp_status;

typedef enum {
  KP_F64 = 0,        /* everything in FP64 (the paper's precision)                 */
  KP_F32 = 1,        /* FP32 slabs and matrix products, FP64 factors and inversion */
  KP_MIXED_BF16 = 2, /* BF16 MFMA with FP32 accumulation.  Curvature pass (forward
                        Laplacian, adjoint, factors, gradient): FP32 slabs whose
                        products run as BF16x3 (hi*hi + lo*hi + hi*lo of the BF16
                        split of each operand).  Line-search forwards: BF16 slabs
                        and BF16 weights, one MFMA per product.  FP32 elementwise
                        work, FP32 master parameters, FP64 factors and inversion */
  KP_MIXED_F16 = 3   /* as KP_MIXED_BF16, but the curvature pass runs FP16 MFMAs with
                        FP32 accumulation: FP32 slab entries are rounded once to
                        FP16 on their way into the products; the weights are split
                        into FP16 hi + lo (layer products: two MFMAs, the factor
                        and gradient products: one)                              */
} kp_precision;

typedef struct {
  int32_t n_layers;             /* L >= 1                                          */
  const int32_t* widths;        /* host, L+1 entries; widths[L] must be 1           */
  int32_t time_coord;           /* input index of t for c_t, or -1                  */
  double coef_time;             /* c_t                                              */
  double coef_lap;              /* c_lap                                            */
  const uint8_t* lap_mask;      /* host, d entries (1 = in the Laplacian row); NULL = all */
  int32_t precision;            /* kp_precision                                     */
  int32_t max_interior;         /* capacity in interior points per call             */
  int32_t max_boundary;         /* capacity in boundary points per call             */
  size_t workspace_limit_bytes; /* 0 = unlimited.  When the stored slabs of
                                   kfac_pinn_forward_laplacian would exceed it, the
                                   forward keeps no intermediates and the VJP
                                   recomputes each layer's input from x.            */
  const double* op_coef;        /* host, d x d row-major symmetric C, or NULL.  When
                                   given (lap_mask must be NULL) the second-order
                                   part is sum_ij C_ij d2u/dx_i dx_j (Section 3.1,
                                   closing paragraph; Appendix C.3), propagated
                                   along the eigenvectors of C; with a time term,
                                   C's row and column time_coord must be zero.   */
  double coef_xgrad;            /* c_x  } first-order terms of the interior residual */
  double coef_gradsq;           /* c_g  } (Section 3.3), see Residuals above; 0 for  */
  double coef_const;            /* c_0  } a linear PDE.  c_x, c_g need lap_mask form */
} kp_problem;

typedef struct {
  double lambda;        /* damping added to all four factors (Section 3.4)          */
  double beta;          /* EMA factor in [0, 1)                                     */
  double momentum;      /* mu (modes 0 and 1)                                       */
  int32_t lr_mode;      /* 0: fixed alpha = lr; 1: grid line search; 2: KFAC*, alpha
                           and mu from the quadratic model with the exact damped
                           Gramian (Section 3.4)                                     */
  double lr;            /* fixed step (lr_mode 0)                                   */
  int32_t grid_min_exp; /* grid alpha = 2^k, k = grid_max_exp .. grid_min_exp       */
  int32_t grid_max_exp; /* (the paper: -30 .. 0)                                    */
} kp_hparams;

/* Written on the device by kfac_pinn_step (when the pointer is non-NULL). */
typedef struct {
  double loss_interior;  /* L_Omega at theta_t                                     */
  double loss_boundary;  /* L_dOmega at theta_t                                    */
  double lr_chosen;      /* alpha* (0 when no step was taken)                      */
  double loss_after;     /* L(theta_t + delta_t) (grid mode; NaN in fixed mode)     */
  int32_t status;        /* kp_status of this step                                  */
  int32_t step;          /* step counter after this step                            */
  double momentum_chosen;  /* coefficient of delta_{t-1} in the applied update:
                              alpha * mu in modes 0 and 1 (0 at the first step),
                              mu* in mode 2                                        */
} kp_step_info;

/* Seeded sampler (kfac_pinn_sample).  Values come from SplitMix64 (Steele, Lea &
   Flood 2014) used as a counter-based generator, u = (z >> 11) * 2^-53. */
typedef struct {
  uint64_t seed_interior, seed_boundary, seed_initial;
  int32_t n_interior, n_boundary, n_initial;
  int32_t face_lo;      /* faces x_k in {0,1} for k >= face_lo (1 for heat: t is free) */
  int32_t target_kind;  /* 0: f = c pi^2 sum sin(pi x_i), g = c sum sin(pi x_i)
                           1: f = 2 pi^2 sin(pi x0) sin(pi x1), g = 0
                           2: heat, f = 0, g = exp(-kappa pi^2 x0) sum_{i>=1} sin(pi x_i) */
  double scale;         /* c                                                        */
  double kappa;
} kp_sampler;

/* ---- lifetime --------------------------------------------------------------
 * kfac_pinn_create: validates `problem`, allocates every workspace for the
 * stated capacities on the current HIP device, and binds `stream` (a
 * hipStream_t; NULL = the default stream).  *out receives the handle.
 * Factors start at the identity, the momentum at zero.  KP_ERR_OOM if the
 * workspaces do not fit. */
kp_status kfac_pinn_create(const kp_problem* problem, void* stream, kfac_pinn_ctx** out);
kp_status kfac_pinn_destroy(kfac_pinn_ctx* ctx);

/* Algorithm 1, step 0: every Kronecker factor to I (init_identity != 0) or 0;
   momentum and step counter to zero. */
kp_status kfac_pinn_reset_state(kfac_pinn_ctx* ctx, int32_t init_identity);

/* Number of parameters D for the given widths (host, n_layers+1 entries). */
int64_t kfac_pinn_num_params(const int32_t* widths, int32_t n_layers);

/* ---- sampling ---------------------------------------------------------------
 * Draws one batch for training step `step` (counter offset step * count *
 * draws-per-point) into x_int (n_interior x d), y_int, x_bnd and y_bnd
 * ((n_initial + n_boundary) x d; initial points first), all "real".
 * Interior points are uniform in [0,1)^d.  A boundary point picks a face with
 * one draw (f = floor(u * 2(d - face_lo)); coordinate face_lo + f/2 is set to
 * f mod 2) and its coordinates with d more.  Initial points have x_0 = 0.
 * Targets follow the manufactured solutions of Section 4 / Appendix A. */
kp_status kfac_pinn_sample(kfac_pinn_ctx* ctx, const kp_sampler* sampler, int64_t step,
                           void* x_int, void* y_int, void* x_bnd, void* y_bnd);

/* ---- forward Laplacian (Section 3.1, Eq. forward-laplacian-main) -----------
 * For n points x (n x d) computes the network value u (n), the gradient
 * du/dx (n x d, row-major; may be NULL) and the operator's second-order row
 * sum_{i in mask} d2u/dx_i^2 (n; may be NULL).  Keeps the layer slabs for a
 * following kfac_pinn_forward_laplacian_vjp unless the workspace limit forbids
 * it.  n <= max_interior. */
kp_status kfac_pinn_forward_laplacian(kfac_pinn_ctx* ctx, const void* theta, const void* x,
                                      int32_t n, void* u_out, void* grad_out, void* lap_out);

/* Vector-Jacobian product of kfac_pinn_forward_laplacian at (theta, x): given
 * cotangents u_bar (n), grad_bar (n x d) and lap_bar (n) (any may be NULL =
 * zero) writes theta_bar (D, double) and x_bar (n x d real; may be NULL).
 * It is the backward pass of Algorithm 1 with a general seed; layer inputs come
 * from the slabs of the preceding forward call on the same (theta, x, n), or
 * are recomputed from x under a workspace limit. */
kp_status kfac_pinn_forward_laplacian_vjp(kfac_pinn_ctx* ctx, const void* theta, const void* x,
                                          int32_t n, const void* u_bar, const void* grad_bar,
                                          const void* lap_bar, double* theta_bar, void* x_bar);

/* ---- curvature (Algorithm 1, steps 1-2 and 4) --------------------------------
 * Forward Laplacian over the interior points, plain forward over the boundary
 * points, residuals, one backward pass per term for the output gradients g,
 * the Kronecker factors of Eq. KFAC-PINN (interior: A = sum Z~Z~^T/(N S),
 * B = sum g g^T/N) and Eq. kfac-linear (boundary: A = sum z~z~^T/M,
 * B = sum g g^T/M), folded into the context's factors by the EMA
 * A <- beta A + (1 - beta) A_new.  Optionally writes the loss gradient
 * (grad_out, D doubles, Algorithm 1 step 4) and {L_Omega, L_dOmega}
 * (loss_out, 2 doubles). */
kp_status kfac_pinn_factors(kfac_pinn_ctx* ctx, const void* theta,
                            const void* x_int, const void* y_int, int32_t n_int,
                            const void* x_bnd, const void* y_bnd, int32_t n_bnd,
                            double beta, double* grad_out, double* loss_out);

/* ---- exact per-layer Gramian (Section 3.2, Eq. laplace_gramian_block_exact) ----
 * The block of Eq. (gramian) that KFAC approximates, for layer `layer` and one
 * term (0 interior, 1 boundary with S = 1), from the slabs of the last
 * kfac_pinn_factors / kfac_pinn_step call on this context:
 *   G = (1/n) sum_p J_p J_p^T,   J_p = sum_s z~_{p,s} (x) g_{p,s},
 * with p the parameter count h_out (h_in + 1) of the layer in the theta layout
 * (column-stacked [W | b]) and n that call's point count of the term.
 * out: p x p doubles (row-major, symmetric); work: n x p doubles of scratch;
 * both device memory owned by the caller.  For small layers: p <= 16384.
 * Errors: KP_ERR_ARG for indices, a layer above the limit, a context without
 * stored slabs (workspace limit) or without a curvature pass of that term. */
kp_status kfac_pinn_layer_gramian(kfac_pinn_ctx* ctx, int32_t layer, int32_t term, double* out,
                                  double* work);

/* ---- damped Kronecker-sum factorisation (Section 3.4) ------------------------
 * For every layer and side, damps the EMA factors (+ lambda I) and computes,
 * in FP64, P and e with P^T F1 P = I and P^T F2 P = diag(e) for the pair
 * (F1, F2) = (interior, boundary) factor: a Cholesky factor of F1, then a
 * Jacobi eigendecomposition of the whitened F2.  The inverse of the Kronecker
 * sum is then (P_A (x) P_B) (I + e_A (x) e_B)^-1 (P_A (x) P_B)^T.  The Jacobi
 * iteration starts from the eigenvectors found by the previous call on this
 * context (the identity after create/reset_state and on every 1000th call) and
 * runs until a sweep performs no rotation above its threshold, at most
 * max_sweeps sweeps (default 20), so the result does not depend on the start
 * beyond rounding.  When the context's stream is not being captured into a graph,
 * the call reads each sweep's convergence flags back to the host one sweep later
 * (so it waits on the host for all but its last sweep) and enqueues no further
 * sweeps for problems that have all converged; under capture it enqueues all
 * max_sweeps sweeps.  Both give the same result: a converged problem's launches
 * return at once.  Sets KP_ERR_NOT_PD in the device status when a damped
 * interior factor is not positive definite, and KP_ERR_NOT_CONVERGED when a
 * problem still rotated in its last allowed sweep. */
kp_status kfac_pinn_invert(kfac_pinn_ctx* ctx, double lambda);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the apply of
 * kfac_pinn_precondition for ONE layer, Delta = -(A_i (x) B_i + A_b (x) B_b)^-1 g,
 * with that layer's factorisation passed in (as kfac_pinn_get_preconditioner
 * returns it) and no context.  nA = h_in + 1, nB = h_out; PA (nA x nA, row-major),
 * a (nA), PB (nB x nB), b (nB); grad and delta_out: the layer's block of the theta
 * layout (column-major nB x nA); all device doubles owned by the caller; `stream`
 * a hipStream_t (NULL = default stream).  Nothing is allocated: the two
 * intermediate nB x nA products live in a static device array of the library,
 * 2 x 1048576 doubles (16 MiB) per GPU, held until the process ends, and the
 * product descriptors are kernel arguments.  Every call on a GPU shares that
 * array, so calls that overlap on one GPU (other streams, other threads) race;
 * nothing in it needs to start at zero.  Results equal kfac_pinn_precondition's
 * for that layer (same kernels).  Errors: KP_ERR_ARG for null pointers,
 * non-positive sizes or nA * nB > 1048576; KP_ERR_HIP. */
kp_status kfac_pinn_precondition_layer_noalloc(int32_t nA, int32_t nB, const double* PA,
                                               const double* a, const double* PB,
                                               const double* b, const double* grad,
                                               double* delta_out, void* stream);

/* Sweep cap of the Jacobi eigensolver (1 .. 64; default 20): the most sweeps a
 * call runs (and, under graph capture, the sweeps it enqueues).  Errors:
 * KP_ERR_ARG outside the range. */
kp_status kfac_pinn_set_max_sweeps(kfac_pinn_ctx* ctx, int32_t max_sweeps);

/* Early stop of the Jacobi sweeps (kfac_pinn_invert): 1 (default) lets the call
 * wait on the host for each sweep's convergence flags and stop enqueueing sweeps
 * once every problem has converged; 0 makes every call enqueue max_sweeps sweeps
 * without any host wait (as under graph capture).  The results are the same.
 * Errors: KP_ERR_ARG unless enabled is 0 or 1. */
kp_status kfac_pinn_set_sweep_wait(kfac_pinn_ctx* ctx, int32_t enabled);

/* Delta = -(A_i (x) B_i + A_b (x) B_b)^-1 g per layer with the preconditioner of
 * the last kfac_pinn_invert (grad_in, delta_out: D doubles each). */
kp_status kfac_pinn_precondition(kfac_pinn_ctx* ctx, const double* grad_in, double* delta_out);

/* ---- one full KFAC step (Algorithm 1, one iteration) -------------------------
 * Factors and gradient at theta_inout, EMA (beta), damping and inversion
 * (lambda), Delta = -C g, momentum delta^ = mu delta_{t-1} + Delta (delta_{-1} =
 * 0), the learning rate (fixed, or argmin of L(theta + 2^k delta^) over the grid
 * with ties to the larger step and non-finite losses skipped), then
 * theta_inout += alpha delta^ and delta_t = alpha delta^.
 * KFAC* (lr_mode 2, Section 3.4): delta_t = alpha* Delta + mu* delta_{t-1} with
 * (alpha*, mu*) = -Q^-1 (Delta^T g, delta_{t-1}^T g), Q_ij = d_i^T (G + lambda I) d_j
 * for d = (Delta, delta_{t-1}) and G the exact Gramian of the loss; G enters
 * through one Jacobian-vector product per direction, contracted from the slabs of
 * this step's curvature pass (so a workspace limit that drops them is an
 * argument error).  At the first step mu* = 0 and alpha* = -Delta^T g / Q_11.
 * Nothing is read back to the host; `info` (device, may be NULL) receives the
 * step's summary. */
kp_status kfac_pinn_step(kfac_pinn_ctx* ctx, void* theta_inout,
                         const void* x_int, const void* y_int, int32_t n_int,
                         const void* x_bnd, const void* y_bnd, int32_t n_bnd,
                         const kp_hparams* hp, kp_step_info* info);

/* ---- state access (tests, checkpoints) -------------------------------------
 * term: 0 interior, 1 boundary; side: 0 A ((h_in+1)^2), 1 B (h_out^2);
 * row-major dense doubles. */
kp_status kfac_pinn_get_factor(kfac_pinn_ctx* ctx, int32_t layer, int32_t term, int32_t side,
                               double* dev_out);
kp_status kfac_pinn_set_factor(kfac_pinn_ctx* ctx, int32_t layer, int32_t term, int32_t side,
                               const double* dev_in);
/* P (n x n row-major) and e (n) of the last kfac_pinn_invert for layer/side. */
kp_status kfac_pinn_get_preconditioner(kfac_pinn_ctx* ctx, int32_t layer, int32_t side,
                                       double* p_out, double* e_out);
/* The 1 + grid_max_exp - grid_min_exp candidate losses of the last grid step. */
kp_status kfac_pinn_get_line_search(kfac_pinn_ctx* ctx, double* dev_out);
/* Momentum buffer delta_{t} (D reals) and step counter. */
kp_status kfac_pinn_get_momentum(kfac_pinn_ctx* ctx, void* dev_out);
kp_status kfac_pinn_set_momentum(kfac_pinn_ctx* ctx, const void* dev_in, int64_t step);

/* ---- measurement ---------------------------------------------------------
 * While enabled, every launch of one kernel class is bracketed by HIP events on
 * the context's stream: 0 layer products of the curvature pass (forward and
 * backward), 1 factor/gradient products, 2 the whole Kronecker-sum
 * factorisation, 3 the tanh rows and their adjoint, 4 the layer products of
 * the line-search forwards; -1 disables.
 * kfac_pinn_timing_read waits for the stream and writes (host, 4 doubles):
 * launches, total milliseconds, algorithmic FLOPs and algorithmic bytes of the
 * timed launches, then resets the counters. */
kp_status kfac_pinn_timing_enable(kfac_pinn_ctx* ctx, int32_t kernel_class);
kp_status kfac_pinn_timing_read(kfac_pinn_ctx* ctx, double* out4);

/* Line-search lanes (1 or 2; default 2).  The candidates of the grid line search
 * (Section 3.4) are independent: with 2 lanes the odd candidates are enqueued on an
 * internal stream of default priority with their own slab, weight and table
 * buffers (about the size of the line-search slabs, made by kfac_pinn_create),
 * forked from and joined back to the context's stream, so that two candidates'
 * launches overlap.  Setting 1 frees those buffers (after a device-wide wait);
 * setting 2 again re-makes them (and waits for the device).  A step uses the
 * second lane once the context's internal streams exist (from its first
 * inversion on).  The results do not depend on the lane count.  Instances of a
 * batch use 1 lane.  Errors: KP_ERR_ARG for other counts, KP_ERR_HIP. */
kp_status kfac_pinn_set_line_search_lanes(kfac_pinn_ctx* ctx, int32_t lanes);

/* Jacobi sweeps used by each of the 2L eigenproblems (layer l: 2l side A, 2l+1
   side B) in the last inversion; waits for the stream.  out: host, 2L ints. */
kp_status kfac_pinn_get_sweeps(kfac_pinn_ctx* ctx, int32_t* out);

/* Whether the interior (out[0]) and boundary (out[1]) terms recompute layer inputs
   per layer instead of storing them (1) because their slabs exceed
   workspace_limit_bytes.  out: host, 2 ints. */
kp_status kfac_pinn_get_workspace(kfac_pinn_ctx* ctx, int32_t* out);

/* ---- batches of independent instances --------------------------------------
 * Not in the paper (which trains one network at a time): many small problems
 * stepped together.  kfac_pinn_batch_create creates `count` contexts from
 * problems[0..count) (host array) on internal streams of default priority;
 * instance k runs on lane k % 8, so the instances' launches overlap.
 * kfac_pinn_batch_step performs one kfac_pinn_step per instance with the same
 * hyper-parameters: thetas, x_int, y_int, x_bnd, y_bnd are host arrays of
 * `count` device pointers, n_int and n_bnd host arrays of sizes, infos a device
 * array of `count` summaries (or NULL).  Its phases:
 *   1. the curvature passes of every instance, on the lanes;
 *   2. on lane 0: the factor and gradient products of every instance, then ONE
 *      inversion launch sequence over the damped factors of all instances (each
 *      eigensolver launch covers every instance's problems);
 *   3. the directions and momenta, on the lanes;
 *   4. the line searches;
 *   5. the step sizes and updates, on the lanes.
 * Grouped launches (see kfac_pinn_batch_set_grouped): with mixed curvature
 * products (KP_MIXED_BF16, KP_MIXED_F16), stored slabs and both point sets
 * non-empty, phase 2's products are one launch per (term, layer, product) over
 * every instance plus one for its split-K reduction; with the grid line search
 * (lr_mode 1), BF16 line-search slabs and every instance on the paired
 * line-search launches (linear residuals, unit input directions), each of a
 * candidate's kernels in phase 4 is ONE launch over every instance, even
 * candidates on lane 0 and odd ones on lane 1 (each instance's second set of
 * line-search buffers).  Otherwise those launches run per instance on its lane.
 * The grouped launches read job tables in device memory, made at creation for
 * the largest point counts and rewritten when the step's buffers, point counts
 * or beta change.  The results equal those of kfac_pinn_step on each instance.
 * The Jacobi warm start and its
 * periodic cold start are counted per batch step, and the sweeps used are read
 * with kfac_pinn_batch_get_sweeps (kfac_pinn_get_sweeps on an instance's
 * context reports only its own kfac_pinn_step/invert calls).  The work is
 * ordered after the work already on `stream` and before anything enqueued
 * there later.  The first call captures each phase into HIP graphs (per lane,
 * and for the grouped line search); later calls with the same arguments replay
 * them (different arguments recapture).  The inversion (with the grouped factor
 * products) is enqueued directly, so that its sweeps stop once the host reads
 * every problem as converged (each sweep replays a graph of its own); only when
 * the convergence flags have no host buffer is it captured too, running every
 * sweep up to the cap.  With the graphs disabled
 * (kfac_pinn_batch_set_graph) every call enqueues the launches directly.
 * Errors as for kfac_pinn_step; per-instance device status is read with
 * kfac_pinn_sync on kfac_pinn_batch_context(batch, k). */
typedef struct kfac_pinn_batch kfac_pinn_batch;
kp_status kfac_pinn_batch_create(const kp_problem* problems, int32_t count, void* stream,
                                 kfac_pinn_batch** out);
kp_status kfac_pinn_batch_destroy(kfac_pinn_batch* batch);
kp_status kfac_pinn_batch_context(kfac_pinn_batch* batch, int32_t k, kfac_pinn_ctx** out);
kp_status kfac_pinn_batch_set_graph(kfac_pinn_batch* batch, int32_t enabled);
/* The grouped launches (default 1) on or off (0: every instance's factor
 * products and line-search candidates launch per instance on its lane, as
 * kfac_pinn_step does); KP_ERR_ARG for other values.  kfac_pinn_batch_is_grouped
 * writes (host) which grouped launches the last batch step took: bit 0 the line
 * search, bit 1 the factor and gradient products, bit 2 the line search on two
 * lanes (odd candidates on lane 1 with each instance's second line-search
 * buffers, made at creation). */
kp_status kfac_pinn_batch_set_grouped(kfac_pinn_batch* batch, int32_t enabled);
kp_status kfac_pinn_batch_is_grouped(kfac_pinn_batch* batch, int32_t* out);
/* Autotuning of the grouped line search (not in the paper).  Chooses, per class
 * (K = h_in + 1 rounded up to 8, h_out, rows per point S, value rows only) of the
 * grouped layer products, the tile geometry (points x neurons per workgroup:
 * 64 x 256, 128 x 128 or 256 x 64; untuned: the narrowest neuron tile covering
 * the layer) and, past the input layer, the number of derivative-row chunks (the
 * single-instance choice, 1, 2, 4 or 8), by timing the grouped launches over
 * every instance: first one policy for all classes (geometry by width or
 * 64 x 256; chunk counts as for a single instance or capped at 1, 2, 4 or 8),
 * then each class's alternatives within the launches of its layers (kept when
 * faster by more than 2 us and 0.5 %).  The arguments are those of
 * kfac_pinn_batch_step (both point sets non-empty); the instances' parameters are
 * not changed, their line-search buffers are overwritten.  cache_path (or NULL):
 * a JSON file of earlier choices per device and class, read first (cached classes
 * are not timed) and rewritten with the merged choices; an unwritable path gives
 * KP_ERR_ARG after the choices are applied.  timed (or NULL): the number of
 * classes timed.  Waits for the device.  The geometry does not change results;
 * chunk counts other than the single-instance choice make the candidates' losses
 * differ from kfac_pinn_step's in rounding (another grouping of the sums over
 * derivative rows).  KP_ERR_STATE when the instances do not take the grouped
 * line search. */
kp_status kfac_pinn_batch_tune(kfac_pinn_batch* batch, void* const* thetas,
                               const void* const* x_int, const void* const* y_int,
                               const int32_t* n_int, const void* const* x_bnd,
                               const void* const* y_bnd, const int32_t* n_bnd,
                               const char* cache_path, int32_t* timed);
/* Jacobi sweeps of instance k's eigenproblems in the last batch step (waits for
 * it): sweeps[2*layer + side] for side 0 (input factors) and 1 (output factors);
 * `sweeps` is a host array of 2 * n_layers ints. */
kp_status kfac_pinn_batch_get_sweeps(kfac_pinn_batch* batch, int32_t k, int32_t* sweeps);
kp_status kfac_pinn_batch_step(kfac_pinn_batch* batch, void* const* thetas,
                               const void* const* x_int, const void* const* y_int,
                               const int32_t* n_int, const void* const* x_bnd,
                               const void* const* y_bnd, const int32_t* n_bnd,
                               const kp_hparams* hp, kp_step_info* infos);

/* Guard check (diagnostics).  When the environment variable KFAC_PINN_GUARD_KB is
 * a positive number at kfac_pinn_create, every device buffer of the context is
 * allocated with that many KiB of guard bytes before and after it, filled with a
 * fixed pattern.  kfac_pinn_check_guards waits for the device and writes (host)
 * the number of guard bytes that no longer hold the pattern (0: no kernel wrote
 * outside a buffer by up to the guard size) and the number of guarded buffers.
 * Without guards both counts are 0. */
kp_status kfac_pinn_check_guards(kfac_pinn_ctx* ctx, int64_t* bad_bytes, int64_t* buffers);

/* Waits for the context's stream; returns the device status word (and clears it). */
kp_status kfac_pinn_sync(kfac_pinn_ctx* ctx);
const char* kfac_pinn_status_string(kp_status status);
/* Text of the last host-side error (thread-local). */
const char* kfac_pinn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KFAC_PINN_H */
