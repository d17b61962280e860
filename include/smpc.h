/*
 * smpc.h -- C ABI of the MI355X (gfx950) solver for scenario-tree stochastic
 * MPC by the accelerated dual proximal gradient method of Sampathirao,
 * Sopasakis, Bemporad and Patrinos, "GPU-accelerated stochastic predictive
 * control of drinking water networks" (arXiv 1604.01074).
 *
 * Problem solved (eq. Sc-MPC with the splitting of Sec. IV-A):
 *
 *   min  sum_n pi_n [ W_alpha (alpha1 + alpha2_{s(n)})' u_n
 *                     + (u_n - u_{a(n)})' Wu (u_n - u_{a(n)}) ]
 *      + sum_n [ cS_n dist(x_n | x >= xs) + gamma_d dist(x_n | [xmin, xmax]) ]
 *   s.t. x_n = A x_{a(n)} + B u_n + Gd d_n,  E u_n + Ed d_n = 0,
 *        umin <= u_n <= umax,  x_{a(root)} = p,  u_{a(root)} = q,
 *
 * over the decision nodes n of a scenario tree (Sec. III-C): node n sits at
 * stage s(n) in 0..N-1, has parent a(n) and probability pi_n, and carries the
 * demand d_n, the input u_n and the state x_n that follows it.  cS_n is
 * W_x * pi_n (or W_x, see weight_safety_by_prob).
 *
 * Conventions for every call:
 *  - Return value: 0 = SMPC_OK, > 0 = warning (outputs valid), < 0 = error.
 *    No C++ exception crosses the ABI.  smpc_last_error() gives the message
 *    of the last failing call on the calling thread.
 *  - Matrices are dense, row-major, float64, host memory.  Inputs are copied
 *    during the call; the caller keeps ownership of everything it passes.
 *  - Outputs go to caller-allocated host buffers of the documented size.
 *  - Node arrays use the caller's node order: stage-sorted, parent[n] < n.
 *  - A dual vector has one block (sigma~_n [nx] | zeta~_n [nx] | psi~_n [nu])
 *    per node (Sec. IV-A, dual of Hz = t), i.e. M x (2 nx + nu) row-major.
 *  - All device work of a context runs on its one HIP stream, in order.
 *    Handles are not thread-safe: use one context per host thread.
 */
#ifndef SMPC_H
#define SMPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMPC_ABI_VERSION 1

enum {
  SMPC_OK = 0,
  SMPC_MAX_ITER = 1,        /* warning: max_iter reached before tol; outputs valid */
  SMPC_PENDING = 2,         /* smpc_server_poll: the request has not finished yet  */
  SMPC_STALLED = 3,         /* warning: with stall_checks > 0, r_p made no progress
                               for stall_checks checks (e.g. an infeasible coupling
                               E u + Ed d = 0 in the u box, whose dual grows
                               without bound); outputs valid                       */
  SMPC_EINVAL = -1,         /* bad argument (NULL, negative size, bad flag)        */
  SMPC_EDIM = -2,           /* dimension outside the supported range               */
  SMPC_ENOTSPD = -3,        /* Wu not symmetric positive definite                  */
  SMPC_ERANK = -4,          /* E does not have full row rank                       */
  SMPC_EPROB = -5,          /* tree structure or probabilities inconsistent        */
  SMPC_ENOMEM = -6,         /* device allocation failed or HBM budget exceeded     */
  SMPC_EDEVICE = -7,        /* HIP runtime error                                   */
  SMPC_ENOTFACTORED = -8,   /* smpc_factor / smpc_tree_set_data not called yet     */
  SMPC_EDIVERGED = -9,      /* residual became non-finite or exploded              */
  SMPC_ENAN = -10,          /* NaN or Inf in an input                              */
  SMPC_ECANCELED = -11      /* smpc_server_cancel: the request was withdrawn        */
};

typedef struct smpc_ctx smpc_ctx;
typedef struct smpc_sys smpc_sys;
typedef struct smpc_tree smpc_tree;

/* ------------------------------------------------------------------ context
 * smpc_ctx_create: bind to HIP device `device` and to the stream `hip_stream`
 * (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream); NULL makes
 * the library create and own a stream.  `hbm_budget` caps the device bytes
 * the context may allocate (0 = no cap); exceeding it gives SMPC_ENOMEM.
 * Errors: SMPC_EINVAL (out == NULL), SMPC_EDEVICE (no such device).        */
int smpc_ctx_create(int device, void* hip_stream, size_t hbm_budget, smpc_ctx** out);
/* Frees the context.  All systems and trees of the context must be destroyed
 * first (SMPC_EINVAL otherwise).                                             */
int smpc_ctx_destroy(smpc_ctx* ctx);
/* Copies the calling thread's last error message (NUL-terminated, truncated
 * to len) into buf.  Returns the message length.                            */
int smpc_last_error(char* buf, size_t len);
/* Device bytes currently allocated by the context.                          */
int smpc_ctx_mem_used(smpc_ctx* ctx, size_t* bytes);

/* ------------------------------------------------------------------ system
 * Flow model of Sec. II (eq. model, eq. demand-control), boxes and costs of
 * Sec. III-A / III-D.  Sizes: A nx*nx, B nx*nu, Gd nx*nd, E ne*nu, Ed ne*nd
 * (E, Ed may be NULL when ne == 0), umin/umax/alpha1 nu, xmin/xmax/xs nx,
 * Wu nu*nu symmetric positive definite.
 * weight_safety_by_prob: 1 -> safety weight of node n is W_x * pi_n (the
 * expectation of the stage cost), 0 -> W_x.                                 */
typedef struct {
  int nx, nu, nd, ne;
  const double *A, *B, *Gd, *E, *Ed;
  const double *umin, *umax, *xmin, *xmax, *xs;
  double W_alpha, W_x, gamma_d;
  const double *alpha1, *Wu;
  int weight_safety_by_prob;
} smpc_sys_desc;

/* Copies the system, checks it (SMPC_ENAN, SMPC_EDIM, SMPC_EINVAL for
 * umin > umax or xmin > xmax, SMPC_ENOTSPD for Wu, SMPC_ERANK for E) and runs
 * the tree-independent part of the factor step (App. A / App. B) in float64
 * on the host.  Supported: 1 <= nx <= 128, 1 <= nu <= 128, 0 <= nd <= 4096,
 * 0 <= ne < nu.                                                             */
int smpc_sys_create(smpc_ctx* ctx, const smpc_sys_desc* desc, smpc_sys** out);
int smpc_sys_destroy(smpc_sys* sys);   /* SMPC_EINVAL while trees still use it */

/* ------------------------------------------------------------------ tree
 * Scenario tree (Sec. III-C) with N stages and M decision nodes, stage-sorted:
 * stage[0] = 0, parent[0] = -1, parent[n] < n, stage[parent[n]] = stage[n]-1,
 * every node at stage < N-1 has a child, prob > 0, prob[0] = 1 and the
 * children of each node sum to its probability (relative 1e-9).
 * Violations give SMPC_EPROB; M (2 nx + nu) >= 2^31 gives SMPC_EDIM.
 * Allocates the tree's device buffers.                                      */
int smpc_tree_create(smpc_sys* sys, int N, int M, const int32_t* stage,
                     const int32_t* parent, const double* prob, smpc_tree** out);
int smpc_tree_destroy(smpc_tree* tree);

/* Cost update of App. A (Alg. 2, step 2) for new node demands d (M*nd,
 * caller's node order; NULL = zero when nd = 0) and pumping costs alpha2
 * (N*nu; NULL = zero).  d and alpha2 are copied to the device, where float64
 * kernels compute per node the particular input uhat_n (minimum-norm
 * solution of E u + Ed d_n = 0), e_n = B uhat_n + Gd d_n and the linear cost
 * of the input
 *   beta_n = pi_n W_alpha (alpha1 + alpha2_{s(n)})
 *            + 2 Wu (pibar_n uhat_n - pi_n uhat_{a(n)} - sum_c pi_c uhat_c),
 *   pibar_n = pi_n + sum over the children c of pi_c
 * (App. A writes its v-space form L' beta_n); the root's term in the previous
 * input q is added by each solve.  Errors: SMPC_ENAN, SMPC_EDEVICE.         */
int smpc_tree_set_data(smpc_tree* tree, const double* d, const double* alpha2);
/* The node data the device holds, in the caller's node order (any pointer
 * may be NULL): uhat (M*nu), e (M*nx), beta (M*nu; the root row includes the
 * q term of the last solve, or none before the first).                      */
int smpc_tree_get_data(smpc_tree* tree, double* uhat, double* e, double* beta);

/* Step size and dual scaling (Sec. IV-D).
 * precond: 0 -> no scaling; 1 -> one scalar per (node, dual block), the
 *   inverse square root of the dual Hessian's diagonal averaged over the
 *   block, taken from a single branch of the tree and divided by pi_n;
 *   2 -> the same diagonal to the power -1/4 (the square root of 1's
 *   scaling), which needed about half the iterations of 1 on the
 *   Barcelona-shaped trees.
 * scale: optional M*3 caller-given scaling (overrides precond when non-NULL).
 * power_iters: the least number of power-iteration steps on the device for
 *   the largest eigenvalue L of the (scaled) dual Hessian (default 200 when
 *   <= 0); the iteration then goes on, 10 steps at a time, until its
 *   Rayleigh quotient (which approaches L from below) changes by less than
 *   1e-5 relative over 10 steps, for at most 10 x power_iters steps in all.
 * lambda_override > 0 skips the power iteration and uses that step size.
 * The step used is lambda = 1 / (L * (1 + margin)), margin = 0.02 when L
 * comes from the power iteration.                                            */
typedef struct {
  int precond;
  int power_iters;
  double lambda_override;
  const double* scale;
} smpc_factor_opts;
int smpc_factor(smpc_tree* tree, const smpc_factor_opts* opts);
/* Step size lambda and, when scale != NULL, the M*3 dual scaling in use.    */
int smpc_tree_get_factor(smpc_tree* tree, double* lambda, double* scale);
/* Number of decision nodes, horizon, number of chains (maximal single-child
 * paths) and chain levels of the tree.                                      */
int smpc_tree_info(smpc_tree* tree, int* M, int* N, int* n_chains, int* n_levels);

/* ------------------------------------------------------------------ solve
 * APG iteration (eq. apg-iteration) from y^0 = y^{-1} and theta_0 = theta_{-1}
 * = 1.  Every check_every iterations (and at the last one) the primal
 * residual r_p = ||Hz - t||_inf is reduced in float64 and the solve stops when
 * r_p <= tol * (1 + max(||Hz||_inf, ||t||_inf)); tol = 0 runs max_iter.
 * precision 64: every step in float64.  precision 32: the solve step, prox and
 * extrapolation run in float32 until the stop test passes (or max_iter -
 * polish_iters is reached), then polish_iters more iterations run in float64
 * from the float32 dual iterates.  A float32 phase whose r_p has not fallen
 * below 0.99 of its best value for stall_checks consecutive checks has met
 * the accuracy floor of float32: that tree continues in float64 until the
 * stop test passes or max_iter is reached (stall_checks 0 -> 100, < 0 ->
 * never; not applied when tol = 0).  With stall_checks > 0 the same rule
 * also ends a precision-64 solve with SMPC_STALLED: in float64 a stall means
 * the iteration makes no progress, as when E u + Ed d = 0 has no solution in
 * the u box (the dual then grows without bound while r_p levels off); the
 * window must be longer than the plateaus of the accelerated iteration on
 * the problems at hand.  Reductions are float64 in both modes.
 * warm_start: 0 -> y0 = 0; 1 -> y^0 = y^{-1} = the tree's resident dual of
 * its previous solve, shifted by smpc_shift_warm_start (no host copy);
 * 2 -> y^0 = y0 and y^{-1} = y_prev0 (or y0 when y_prev0 is NULL), both
 * M*(2nx+nu) in the caller's node order.
 * Chunk lengths (nodes a kernel stages between barriers; a launch-shape
 * choice that never changes the result, which is bit-identical for every
 * length): chunk32 / chunk64 = {backward, forward} lengths for the float32 /
 * float64 iterations, each 0 or a length smpc_chunk_lengths lists.  A
 * precision with a nonzero entry uses exactly those lengths (0 -> the
 * default).  Otherwise tune 0 uses the defaults, and tune 1 uses the lengths
 * an earlier tuned solve of the same launch plan (the tree, or the same set
 * of trees in smpc_solve_batch) chose, or, if none has, times every listed
 * pair on the first iteration blocks of this solve (two timed blocks each,
 * after one that warms the pair up; these are ordinary iterations of the
 * solve) and keeps the fastest for the plan and as the system's choice for
 * servers.  A solve whose trees all stop before every pair is timed leaves
 * the plan untuned.
 * unfused: 0 -> each APG iteration after the first is one launch (the
 * forward rollout of iteration nu and the backward sweep of iteration nu + 1
 * in the same workgroups); 1 -> two launches per iteration (backward, then
 * forward).  Results are identical.
 * dual64 (precision 32 only): 1 -> the float32 phase keeps the dual iterates
 * y^nu, y^{nu-1}, y^{nu+1} in float64 and runs the extrapolation, the prox
 * and the dual update in float64; the solve step (its matrix-vector
 * products, the recursions over the tree and the node data) stays float32.
 * Rounding the stored dual to float32 limits how far the float32 iteration
 * gets (r_p stalls on some trees), while float32 errors in the solve step
 * only perturb each dual gradient, so with dual64 the float32 phase follows
 * the float64 iteration to the tolerance.  The stall rule then applies only
 * when stall_checks > 0.  0 -> the dual is stored in float32 too.          */
typedef struct {
  double tol;
  int max_iter;
  int check_every;
  int precision;
  int polish_iters;
  int warm_start;
  const double* y0;
  const double* y_prev0;
  int stall_checks;
  int tune;
  int chunk32[2];
  int chunk64[2];
  int unfused;
  int gap;  /* 1: fill smpc_result.cost and .gap (smpc_tree_objective)   */
  int dual64;
} smpc_solve_opts;

/* Chunk lengths built into the library for `precision` (32 or 64) and
 * kernel `which` (0 backward, 1 forward), default first: up to cap entries
 * are written to out and their number to *n.                               */
int smpc_chunk_lengths(int precision, int which, int* out, int cap, int* n);

/* Caller-allocated outputs; any pointer may be NULL.  u0: nu, x: M*nx,
 * u: M*nu (last primal iterate z^nu), y: M*(2nx+nu) (y^{nu+1}).
 * iterations counts all iterations, fp32_iterations the float32 ones.
 * status: SMPC_OK (stop test passed), SMPC_MAX_ITER, SMPC_STALLED or
 * SMPC_EDIVERGED.
 * cost and gap: with opts.gap = 1, the primal cost of z^nu and the duality
 * gap of smpc_tree_objective; 0 otherwise.                                  */
typedef struct {
  double* u0;
  double* x;
  double* u;
  double* y;
  int iterations;
  int fp32_iterations;
  double r_primal;
  double hz_t_max;
  int status;
  double queue_ms;  /* server requests: submit -> admission; 0 otherwise */
  double run_ms;    /* server requests: admission -> result; 0 otherwise  */
  int chunk32[2];   /* {backward, forward} chunk lengths the float32 / float64 */
  int chunk64[2];   /* iterations ended with; {0, 0} for a precision not run  */
  double cost;
  double gap;
} smpc_result;

/* Solve one tree from initial state p (nx) and previous input q (nu).
 * Returns the result status (or an error).                                  */
int smpc_solve(smpc_tree* tree, const double* p, const double* q,
               const smpc_solve_opts* opts, smpc_result* res);

/* Solve n distinct trees of one system together: every kernel launch covers
 * the chains of all trees; a tree that has met its stop test stops iterating
 * while the others go on.  Each tree's result equals its smpc_solve result
 * bit for bit.  p[i], q[i] as in smpc_solve; res has n entries.  With
 * warm_start 2, y0 (and y_prev0) hold the trees' dual vectors one after the
 * other in batch order.  Returns the worst status over the trees.            */
int smpc_solve_batch(smpc_tree* const* trees, int n, const double* const* p,
                     const double* const* q, const smpc_solve_opts* opts,
                     smpc_result* res);

/* Receding-horizon warm start (closed loop of Alg. 2; the paper restarts from
 * y0 = 0, any dual point is a valid start).  Prepares the next solve of the
 * same tree with warm_start 1 from the dual the last solve left on the
 * device.  The next tree's root takes the place of child `realized` of the
 * root (in the caller's order of the root's children); a deeper node takes
 * the place of the child of its parent's image with the same child index
 * (the last child when there are fewer); below the last stage the image
 * stays (the last stage is repeated).  The safety block (when weighted by
 * probability) and the input-box block are rescaled by pi_new / pi_old, the
 * state-box block is kept.  realized = -1 resumes from the dual unshifted.
 * SMPC_EINVAL without a previous solve (smpc_factor and smpc_solve_step
 * discard the resident dual) or for a realized index out of range.         */
int smpc_shift_warm_start(smpc_tree* tree, int realized);

/* ------------------------------------------------------------------ objective
 * Objectives of eq. optim:prob and the a-posteriori duality gap of
 * Sec. IV-E at the iterates the tree's last solve left on the device: the
 * last primal iterate z^nu, the prox output t^nu (recovered from the dual
 * update) and the dual y^{nu+1} (unscaled).  In float64:
 *   cost   = V(z^nu): the objective of eq. Sc-MPC at z^nu (soft terms at the
 *            states x_n themselves, i.e. t = Hz)
 *   primal = f(z^nu) + g(t^nu)
 *   dual   = D(y) = f*(-H'y) + g*(y), f*(-H'y) = -(f(z_y) + <y, H z_y>) with
 *            z_y the solve step at y (one extra solve step), g* the support
 *            functions of the sets of g
 *   gap    = primal + dual (>= 0 for y in dom g* by weak duality, -> 0 at
 *            the optimum by strong duality, Sec. IV-A)
 *   dual_violation = the largest violation of dom g* (y_sigma <= 0 and the
 *            norm balls of radius cS_n and cd); <= 0 means y lies in it.
 * The extra solve step overwrites the tree's primal iterate and the dual slot
 * of y^{nu-1} (the resident dual for warm starts is kept); the values are
 * cached, so later calls return the same numbers until the next solve.
 * Errors: SMPC_EINVAL when the tree has no finished solve (or smpc_factor /
 * smpc_solve_step ran since).  Device scratch: allocated by the library on
 * first use (see smpc_tree_objective_noalloc).                              */
typedef struct {
  double cost;
  double primal;
  double dual;
  double gap;
  double dual_violation;
} smpc_objective;
int smpc_tree_objective(smpc_tree* tree, smpc_objective* out);
/* smpc_tree_objective for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the partial sums in a
 * fixed device array of the library (8 * 1025 doubles, 65.6 KB per GPU,
 * held until the process ends; the kernels stride over the nodes, so every
 * tree size fits).  Calls no hipMalloc / hipFree and records no profiling
 * events.  Needs the tree's single-tree launch plan, which smpc_solve of
 * that tree and smpc_factor's power iteration create (SMPC_EINVAL otherwise:
 * a tree factored with lambda_override and solved only in batches has
 * none).  Every call on one GPU shares the array: calls that overlap on
 * a GPU (other host threads, other contexts) race and must be serialised by
 * the caller.                                                              */
int smpc_tree_objective_noalloc(smpc_tree* tree, smpc_objective* out);

/* ------------------------------------------------------------------ closed loop
 * The loop of Alg. 2 around the solver: apply u0, move the plant, solve
 * again.  smpc_plant_step is the flow model of Sec. II (eq. model),
 *   x_next = A x + B u + Gd d      (x: nx, u: nu, d: nd; float64, host)
 * with the realised demand d.  smpc_closed_loop_kpi evaluates the key
 * performance indicators of Sec. V-B over a run of Hs steps: u (Hs*nu) the
 * applied inputs u_1..u_Hs, x (Hs*nx) the states they lead to, alpha2
 * (Hs*nu, NULL = zero) the pumping cost of each step, u_prev (nu) the input
 * before the first step:
 *   E  = (1/Hs) sum_k (alpha1 + alpha2_k)' |u_k|        average economic cost
 *   dU = (1/Hs) sum_k ||u_k - u_{k-1}||_2^2              smoothness
 *   S  = sum_k ||[xs - x_k]_+||_1                        water taken from the
 *                                                        safety storage
 *   R  = ||xs||_1 / ((1/Hs) sum_k ||x_k||_1) * 100       safety volume in % of
 *                                                        the mean volume
 * Errors: SMPC_EINVAL (NULL, Hs < 1), SMPC_ENAN.                            */
int smpc_plant_step(smpc_sys* sys, const double* x, const double* u, const double* d, double* x_next);
typedef struct {
  double E, dU, S, R;
} smpc_kpi;
int smpc_closed_loop_kpi(smpc_sys* sys, int Hs, const double* u, const double* x, const double* alpha2,
                         const double* u_prev, smpc_kpi* out);

/* ------------------------------------------------------------------ serving
 * Continuous batching of closed-loop MPC steps (the loop of Alg. 2 for many
 * controllers).  A server owns a worker thread that drives the context's
 * stream.  Queued requests are admitted between iteration blocks; an
 * admitted request loads its data into its tree, starts its dual (cold, or
 * from the tree's resident dual shifted as by smpc_shift_warm_start) and
 * iterates in the launch group of its current precision; each tree leaves as
 * soon as it stops, so short requests do not wait for long ones.  A result
 * equals that of smpc_solve on the same tree and inputs bit for bit.
 * Admission: at most max_active trees iterate at once (0: no limit); a tree
 * runs one request at a time, in submission order.  A request whose tree
 * needs float32 buffers is admitted only when they fit both the context's
 * HBM budget and the device's free memory (hipMemGetInfo, less a 1/16
 * reserve); otherwise the server first releases the float32 buffers of idle
 * trees (least recently finished first; a tree whose resident dual is
 * float32 keeps them), and if that is not enough the request waits, ahead
 * of later requests and in submission order, until a running request
 * finishes.  With nothing running it fails with SMPC_ENOMEM.  While a server
 * exists, its system and trees are used only through the server calls.     */
typedef struct smpc_server smpc_server;
typedef struct {
  smpc_solve_opts solve;  /* tol, max_iter, check_every, precision, polish_iters,
                             stall_checks, chunk32, chunk64 (tune 1: the
                             system's tuned lengths where it has them; the
                             server itself does not time); warm_start must be
                             0 (per request)                                  */
  int max_active;
} smpc_server_opts;
int smpc_server_create(smpc_sys* sys, const smpc_server_opts* opts, smpc_server** out);
/* One MPC step for `tree`: d (M*nd) and alpha2 (N*nu) replace the tree's
 * data as smpc_tree_set_data does (d NULL: keep the data), p and q as in
 * smpc_solve; warm 0: cold start, 1: resident dual shifted along root child
 * `realized` (-1: unshifted).  Inputs are copied.  *ticket identifies it.  */
int smpc_server_submit(smpc_server* srv, smpc_tree* tree, const double* d, const double* alpha2,
                       const double* p, const double* q, int warm, int realized, uint64_t* ticket);
/* Wait up to wait_ms (< 0: without limit) for the request; SMPC_PENDING if
 * it is not done, else its status with res filled (u0 copied when res->u0 is
 * set; x, u, y must be NULL) and the ticket released.                      */
int smpc_server_poll(smpc_server* srv, uint64_t ticket, smpc_result* res, int wait_ms);
/* Withdraws a request: a queued one never starts, a running one stops at
 * the end of its current iteration block.  Its poll then returns
 * SMPC_ECANCELED (no outputs).  A request that has already finished keeps
 * its result.  SMPC_EINVAL for an unknown ticket.                          */
int smpc_server_cancel(smpc_server* srv, uint64_t ticket);
/* Finishes the queued and running requests, then stops the worker.         */
int smpc_server_destroy(smpc_server* srv);

/* Solve step alone (Alg. 1): the primal point z(w) = argmin <z, H'w> + f(z)
 * for a dual point w (M*(2nx+nu), caller's order), i.e. the dual gradient of
 * Sec. IV-B.  precision 64 or 32.  Outputs x (M*nx) and u (M*nu).           */
int smpc_solve_step(smpc_tree* tree, const double* p, const double* q,
                    const double* w, int precision, double* x, double* u);

/* ------------------------------------------------------------------ profiling
 * With profiling on, every kernel launch is bracketed by HIP events on the
 * context stream.  smpc_ctx_kernel_stats synchronises the stream and returns
 * per-kernel totals since the last reset (up to cap entries, *n set to the
 * number of distinct kernels).                                               */
typedef struct {
  char name[48];
  int launches;
  double total_ms;
} smpc_kernel_stat;
int smpc_ctx_set_profiling(smpc_ctx* ctx, int enable);
int smpc_ctx_kernel_stats(smpc_ctx* ctx, smpc_kernel_stat* out, int cap, int* n);
int smpc_ctx_reset_stats(smpc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SMPC_H */
