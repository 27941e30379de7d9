/*
 * rd.h - resistance distance by Lanczos iteration on AMD Instinct MI355X (gfx950).
 *
 * The library computes r(s,t) = (e_s - e_t)^T L^+ (e_s - e_t) (paper Section 2.1,
 * definition of resistance distance) for an undirected, connected, optionally
 * weighted graph, with the Lanczos iteration of the paper's Algorithm 3
 * (Section 3): a three-term Krylov recurrence on the normalised adjacency
 * D^{-1/2} W D^{-1/2} started from (e_s/sqrt(d_s) - e_t/sqrt(d_t)), whose
 * tridiagonal coefficients give r_hat = (1/d_s + 1/d_t) e_1^T (I - T)^{-1} e_1
 * (Eq. approx_formula). Potentials phi = L^+ (e_s - e_t) and flows follow the
 * electric-flow definition of Section 6.3 and the potential estimate of
 * Algorithm 5.
 *
 * Entry points: graphs (rd_init_graph, rd_set_weights, rd_graph_info,
 * rd_free_graph); Algorithm 3 for one pair (rd_query, and rd_query_trace for
 * its coefficients) or many (rd_query_batch, with rd_tune_width and
 * rd_batch_schedule for its launch shape); the edge-weight gradient
 * (rd_grad_edges); potentials (rd_potentials); the Power Method of Algorithm 1
 * (rd_power_method); Lanczos Push of Algorithm 4 (rd_lanczos_push); extreme
 * Ritz values and the condition-number estimate (rd_ritz_bounds);
 * diagnostics (rd_kernel_stats, rd_status_string, rd_last_error).
 *
 * Conventions shared by every entry point:
 *  - Every call returns rd_status; nothing throws across the ABI. A handle is
 *    not thread-safe: calls on one handle must not overlap.
 *  - Node ids are int32 in [0, n). Edges are undirected, given once each as
 *    (u[e], v[e]); edge ids are positions in that list.
 *  - Inputs are copied; the caller may free them when the call returns.
 *  - Unless RD_DEVICE_PTRS is passed, every pointer argument is host memory.
 *    With RD_DEVICE_PTRS, array arguments (edge lists, weights, pair lists,
 *    result arrays, gradients) are device pointers on the handle's device
 *    (for instance torch CUDA tensors' data_ptr()).
 *  - Work is enqueued on rd_options.stream (a hipStream_t; NULL means the
 *    handle's own stream). Every call returns only after its outputs are
 *    written (it synchronises that stream).
 *  - Errors: RD_E_ARG for invalid arguments (ids out of range, self-loops,
 *    duplicate edges, non-finite or non-positive weights, bad sizes),
 *    RD_E_NOT_CONNECTED for a disconnected graph, RD_E_OOM when device memory
 *    runs out, RD_E_DEVICE for a HIP runtime failure. rd_last_error(g) then
 *    holds a message. Per-query outcomes are reported in rd_result.status.
 */
#ifndef RD_H_
#define RD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rd_graph_s *rd_graph; /* opaque handle, owned by the library */

typedef enum {
  RD_OK = 0,
  RD_E_ARG = 1,
  RD_E_NOT_CONNECTED = 2,
  RD_E_OOM = 3,
  RD_E_DEVICE = 4,
  RD_E_NOT_CONVERGED = 5, /* per query: iteration cap reached; r holds the last estimate */
  RD_E_BREAKDOWN = 6      /* per query: non-positive pivot or non-finite value; r holds the last good estimate */
} rd_status;

/* flags */
#define RD_DEVICE_PTRS 0x1u
#define RD_PROFILE 0x2u /* rd_options.flags: time the sparse-product and edge-pass launches (see rd_kernel_stats) */
#define RD_GENERAL_PATH 0x4u /* rd_options.flags: never use the single-workgroup path that
                                rd_query, rd_query_trace and rd_query_batch (without refine)
                                take when both n-vectors of a run fit in one workgroup's LDS */

#define RD_REORDER 0x8u /* rd_init_graph flags: number the nodes internally by decreasing
                           degree (ties by id) so that the vector entries that the sparse
                           products gather most often share cache lines. Every argument and
                           result stays in the caller's node ids and edge order. */

#define RD_NO_COMPACT 0x10u /* rd_options.flags: rd_query_batch keeps its block width to the end.
                               By default, once every pair has started and at most half of the
                               columns still run, the running columns move to a block of half
                               the width (repeatedly, down to 16), so a tail of slow pairs does
                               not pay for idle columns. Results differ only by rounding. */

#define RD_NO_SPARSE2 0x20u /* rd_options.flags: run the second Lanczos iteration of every
                               pair as a dense product. By default (precision either,
                               reorth 0), a pair whose second product touches few adjacency
                               entries computes it from the support of q_2 alone,
                               N(s) u N(t) u {s, t}: each entry (u, v), u in that support,
                               adds w_uv w_1[u] / d_v to v's sum in 64-bit fixed point
                               (integer sums do not depend on the order, so results stay the
                               same from run to run), and the pair joins the dense iterations
                               at the third. rd_query_batch, rd_grad_edges and refine (which
                               also write the potentials' second terms on that support) take
                               the step when the scatter costs less than a dense column of the
                               autotuned product; rd_query when it has at most nnz/64
                               entries; rd_query_trace never. Results differ only by
                               rounding. */

/* weight / vector dtypes */
#define RD_F64 0
#define RD_F32 1

typedef struct {
  int32_t precision;   /* RD_F64: vectors and sparse products in FP64.
                          RD_F32: vectors and sparse products in FP32 with FP32
                          accumulation; inner products summed in FP64; the
                          Lanczos scalars and the tridiagonal solve in FP64. */
  int32_t max_iters;   /* iteration cap; 0 = max(fixed_k, min(n, 100000)) */
  int32_t fixed_k;     /* > 0: run exactly k iterations, as Algorithm 3 states
                          it (eps is ignored; an exact breakdown still stops) */
  int32_t delay;       /* window d of the stopping estimator; 0 = 8 */
  int32_t block_width; /* rd_query_batch: columns per sweep, 0 = autotuned */
  int32_t err_mode;    /* 0: eps is relative to r_hat; 1: eps is absolute
                          (the paper's error notion, Definition of
                          epsilon-absolute error) */
  uint32_t flags;      /* RD_DEVICE_PTRS: the array arguments of rd_query_batch
                          and rd_grad_edges are device pointers */
  int32_t refine;      /* rd_query_batch only. 1: report the FP64 energy
                          J = 2 b^T phi - phi^T L phi (b = e_s - e_t) of the
                          potential phi accumulated by the run (the estimate
                          of Algorithm 5) instead of r_hat. J <= r, and r - J equals
                          the squared energy-norm error of phi, so rounding in
                          FP32 vectors enters only to second order. Pairs run
                          with refill; finished potentials are harvested into
                          blocks of block_width whose energies are taken per
                          block. */
  int32_t reorth;      /* re-orthogonalisation of w after w -= alpha_i v_i
                          (not in Algorithm 3, which relies on v_1 being
                          exactly orthogonal to u_1 = D^{1/2} 1 / sqrt(vol),
                          the eigenvector of calA for eigenvalue 1), with FP64
                          coefficients all taken from that w:
                          0: none (the paper's loop);
                          1: w -= (u_1^T w) u_1;
                          2: also w -= (v_i^T w) v_i + (v_{i-1}^T w) v_{i-1}.
                          From the second iteration on (v_1 is orthogonal to
                          u_1 by construction). Costs one more vector pass
                          per iteration; graphs small enough for the
                          single-workgroup path take the general path. */
  void *stream;        /* hipStream_t, NULL = the handle's stream */
} rd_options;

typedef struct {
  double r;       /* r_hat(s,t) */
  double err_est; /* stopping estimate of r - r_hat (absolute) */
  int32_t iters;  /* Lanczos iterations performed */
  int32_t status; /* RD_OK, RD_E_NOT_CONVERGED or RD_E_BREAKDOWN */
} rd_result;

/* Fill *o with the defaults (FP64, eps relative, delay 8, autotuned width). */
void rd_default_options(rd_options *o);

/*
 * Build a graph handle on the current HIP device.
 *  n        number of nodes (>= 2)
 *  m        number of undirected edges (>= 1)
 *  u, v     int32[m] endpoints of edge e (u[e] != v[e]; each pair at most once)
 *  w        weights[m] of dtype w_dtype (RD_F64 or RD_F32), finite and > 0;
 *           NULL means unit weights (the unweighted graphs the paper focuses on,
 *           Section 2.1; weighted graphs by the direct generalisation stated there)
 *  flags    RD_DEVICE_PTRS if u, v, w are device pointers; RD_REORDER to
 *           relabel the nodes internally by decreasing degree
 *  out      receives the handle (NULL on failure)
 * Builds the symmetric CSR, weighted degrees d_u = sum_v w_uv in FP64 and the
 * launch schedule on the device; checks connectivity (RD_E_NOT_CONNECTED).
 */
rd_status rd_init_graph(int32_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w,
                        int32_t w_dtype, uint32_t flags, rd_graph *out);

/* Replace the edge weights: w[m] in the edge-list order of rd_init_graph,
 * finite and > 0 (checked first: RD_E_ARG, and the handle keeps its old
 * weights). Degrees, their inverses and vol are recomputed;
 * the structure, and so connectivity, is unchanged. flags: RD_DEVICE_PTRS if w
 * is a device pointer. */
rd_status rd_set_weights(rd_graph g, const void *w, int32_t w_dtype, uint32_t flags);

/* n, m and the number of stored adjacency entries (2m). Any pointer may be NULL. */
rd_status rd_graph_info(rd_graph g, int32_t *n, int64_t *m, int64_t *nnz);

/*
 * One pair, the plain single-pair loop: Algorithm 3 (Section 3) with
 * r_hat = (1/d_s + 1/d_t) e_1^T (I - T)^{-1} e_1 (Eq. approx_formula).
 * s == t gives r = 0 with iters = 0. eps > 0 is the stopping tolerance
 * (relative unless o->err_mode = 1) unless o->fixed_k > 0. o may be NULL
 * (defaults). out is host memory (RD_DEVICE_PTRS is not accepted here).
 * Returns RD_E_ARG for s or t outside [0, n) or eps <= 0 without fixed_k;
 * otherwise RD_OK, with the query's own outcome in out->status (RD_OK,
 * RD_E_NOT_CONVERGED when max_iters ran out, RD_E_BREAKDOWN) and out->r the
 * last estimate.
 */
rd_status rd_query(rd_graph g, int32_t s, int32_t t, double eps, const rd_options *o,
                   rd_result *out);

/*
 * Diagnostic form of rd_query: runs exactly k iterations (stopping early only
 * at an exact breakdown) and writes, for i = 1..iters, alpha_i, beta_{i+1} and
 * r_hat_i to alpha[i-1], beta[i-1], rhat[i-1] (host arrays of length k).
 * *iters receives the number of iterations performed.
 */
rd_status rd_query_trace(rd_graph g, int32_t s, int32_t t, int32_t k, const rd_options *o,
                         double *alpha, double *beta, double *rhat, int32_t *iters);

/*
 * Extreme Ritz values of a k-step Lanczos run from the pair's start vector
 * (Section 3): the smallest and largest eigenvalues theta_min, theta_max of
 * the tridiagonal T_k of alpha_1..alpha_k and beta_2..beta_k (*iters = the
 * steps done, fewer at an exact breakdown). v_1 is orthogonal to D^{1/2} 1,
 * so both lie in [lambda_min(calA), lambda_2(calA)] (the Ritz-containment
 * check of Assumption 1), theta_max rises towards lambda_2 as k grows, and
 * kappa_hat = 2 / (1 - theta_max) is a lower bound of the condition number
 * kappa = 2 / mu_2 (Section 2.1) that converges to it. The run always deflates
 * u_1 = D^{1/2} 1 / sqrt(vol) (reorth >= 1): without it, rounding brings the
 * eigenvalue-1 direction back in long runs and theta_max drifts to 1. The
 * eigenvalues of T_k are found on the host by bisection on the Sturm count.
 * Options as for rd_query_trace (precision, reorth 2 adds the local
 * Gram-Schmidt pass). s == t, ids outside [0, n) or k < 1 return RD_E_ARG.
 */
rd_status rd_ritz_bounds(rd_graph g, int32_t s, int32_t t, int32_t k, const rd_options *o,
                         double *theta_min, double *theta_max, int32_t *iters);

/*
 * Lanczos Push (Algorithm 4, Section 4.1) for npairs pairs, k iterations of
 * the subset Lanczos recurrence with threshold eps >= 0: a nonzero entry
 * v_i(u) is pushed along edge (u, v) only when |v_i(u)| > eps sqrt(d_u d_v)
 * (Definition of AMV), and the alpha and beta terms are subtracted only on
 * S_i = {u : |v_i(u)| > eps d_u}. out[p].r = r' = (1/d_s + 1/d_t) v_1^T V
 * (I - T)^{-1} e_1, out[p].iters = the iterations done (fewer than k at an
 * exact breakdown), out[p].err_est = 0, status RD_OK; s == t gives 0. With
 * eps = 0 this is Algorithm 3 at k iterations. One workgroup per pair keeps
 * the nonzero entries as lists over per-slot node arrays, so the work follows
 * the pushed edges. Each node's AMV sum runs in adjacency order and alpha,
 * beta^2 are summed in fixed point, so results are the same bit for bit from
 * call to call (and agree with the sequential algorithm to rounding). FP64
 * throughout; options: the
 * RD_DEVICE_PTRS flag (s, t, out device memory) and stream. Device memory:
 * 40 bytes per node per concurrent pair (at most 512 pairs and 48 GB),
 * allocated per call. npairs < 0, k < 1, eps < 0 or ids outside [0, n) return
 * RD_E_ARG.
 */
rd_status rd_lanczos_push(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t, int32_t k,
                          double eps, const rd_options *o, rd_result *out);

/*
 * Many pairs: npairs independent runs of Algorithm 3 advanced together as the
 * block columns of one sparse product per iteration; a column whose run stops
 * is retired and its slot refilled with the next pending pair (pairs with
 * s == t get r = 0 without a slot). s, t are int32[npairs] and out
 * rd_result[npairs]; all three are device pointers when o->flags has
 * RD_DEVICE_PTRS. Options: precision, block_width (0: autotuned), reorth,
 * refine, and the flags RD_NO_COMPACT, RD_NO_SPARSE2, RD_GENERAL_PATH,
 * RD_PROFILE. Each result is that of the same run done alone, up to rounding,
 * and the same from call to call bit for bit. Returns RD_E_ARG for an id
 * outside [0, n) (checked on the device), an unsupported block_width or
 * eps <= 0 without fixed_k; per-pair outcomes are in out[p].status as for
 * rd_query. Device memory kept on the handle for later calls: three n x width
 * vector blocks (RD_E_OOM when they do not fit), and for the sparse second
 * iteration 8 bytes per node and column plus lists of 2 * max_degree + 2
 * entries per column (when these would pass 24 GB or do not fit, the call
 * takes dense second iterations instead).
 */
rd_status rd_query_batch(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t,
                         double eps, const rd_options *o, rd_result *out);

/*
 * The block width rd_query_batch uses when rd_options.block_width is 0, and
 * the row-bin schedule of its sparse product. First the width among 32, 64,
 * 128, 256 (not wider than needed for npairs) whose sparse product takes the
 * least time per column on this graph (the fastest of five products each; a
 * wider width only when it is at least 2% faster per column than the narrower
 * best); then, at that width, the schedule
 * (entries per wavefront work item: 128, 256 or 512; rows longer than 512,
 * 1024 or 2048 entries get a workgroup of their own) with the least time.
 * Measured on first use with HIP events on `stream` (NULL: the handle's
 * stream) and kept on the handle per precision; with the environment variable
 * RD_AUTOTUNE_CACHE naming a file, choices are also read from and appended to
 * that file (one line per graph and precision: key, width, entries per work
 * item, long-row threshold, product time per column in ms). The chosen
 * schedule stays in effect for later calls, also with an explicit
 * block_width. The measured time per column also sets which pairs take the
 * sparse second iteration (see RD_NO_SPARSE2) when a run uses the tuned width.
 */
rd_status rd_tune_width(rd_graph g, int32_t precision, int32_t npairs, void *stream, int32_t *width);

/* The row-bin schedule currently in effect for rd_query_batch on g: entries
 * per wavefront work item and the row length above which a row gets a
 * workgroup of its own (defaults 256 and 1024 until the autotuner runs).
 * Either pointer may be NULL. */
rd_status rd_batch_schedule(rd_graph g, int32_t *wave_nnz, int32_t *long_deg);

/*
 * Edge-weight gradient of L = sum_p grad_r[p] r(s_p, t_p):
 *   grad_w[e] = -sum_p grad_r[p] (phi_p(u_e) - phi_p(v_e))^2,
 * the derivative of r = b^T L^+ b (b = e_s - e_t, Section 2.1) through
 * L = sum_e w_e b_e b_e^T, evaluated at the potential phi_p = L^+ b of the
 * electric-flow definition (Section 6.3), estimated as in Algorithm 5 from
 * the same Lanczos run that gives r_hat (it is the gradient
 * of the exact r at phi_hat, not of the truncated r_hat_k). grad_r may be
 * NULL (all ones). fwd, when not NULL, receives the forward results
 * (rd_result[npairs]). grad_w is float[m] in edge-list order, accumulated in
 * FP64. When o->flags has RD_DEVICE_PTRS, s, t, grad_r, fwd and grad_w are
 * device pointers. block_width 0 is autotuned; refine is ignored. Errors as
 * for rd_query_batch; grad_w == NULL is RD_E_ARG. Device memory kept on the
 * handle besides rd_query_batch's: three more n x width blocks in the vector
 * precision (search directions, potentials, finished potentials) and an FP64
 * accumulator of 8 bytes per adjacency entry (16 bytes per edge).
 */
rd_status rd_grad_edges(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t,
                        const double *grad_r, double eps, const rd_options *o, rd_result *fwd,
                        float *grad_w);

/*
 * Power Method (Algorithm 1, Section 2.2) for npairs pairs (s[p], t[p]):
 *   r_bar = sum_{i=0}^{l} r_i(s) / (2 d_s) - r_i(t) / (2 d_t),
 *   r_0 = e_s - e_t,  r_{i+1} = (I/2 + P/2) r_i,  P = A D^{-1},
 * the series of Eq. er_laylor_expansion cut after l + 1 terms; the Power
 * Method theorem gives |r_bar - r| <= eps for l = 2 kappa log(kappa / eps).
 * out[p].r = r_bar, out[p].err_est = the last term added, out[p].iters = l
 * (the number of products), out[p].status = RD_OK. Vectors in o->precision
 * (FP32 or FP64), the sum in FP64. When both n-vectors fit in one
 * workgroup's LDS (and RD_GENERAL_PATH is not set), one workgroup runs all l
 * steps of a pair; otherwise B pairs at a time run on the batched product
 * kernels. Options: precision, block_width (batched runs; 0: the width
 * rd_tune_width picks), RD_DEVICE_PTRS (s, t, out are device memory),
 * RD_GENERAL_PATH, RD_PROFILE (batched runs: the first 64 products of each
 * group are timed for rd_kernel_stats which = 0).
 * l < 0, ids outside [0, n) (checked on the device) or an unsupported
 * block_width return RD_E_ARG; s == t gives 0. Device memory: the vector
 * blocks of rd_query_batch (kept on the handle).
 */
rd_status rd_power_method(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t, int32_t l,
                          const rd_options *o, rd_result *out);

/*
 * Electric potentials (Section 6.3, the potential estimate of Algorithm 5):
 * for each pair p, phi_p = Pi sqrt(c) D^{-1/2} V (I - T)^{-1} e_1 from the
 * same Lanczos run that estimates r(s_p, t_p) (c = 1/d_s + 1/d_t, V the Lanczos
 * vectors, T the tridiagonal matrix), which tends to L^+ (e_s - e_t); Pi
 * removes the mean, so phi_p sums to zero as L^+ b does. The flow of edge
 * e = (u, v) is f(e) = w_e (phi_p(u) - phi_p(v)). phi is double[npairs * n],
 * row p holding phi_p in the caller's node order. out (may be NULL) receives
 * the r_hat of each run as rd_query_batch gives it. The pairs run with refill
 * on block_width columns (0: the width rd_tune_width picks) and the stopping
 * rule of rd_query_batch; each finished potential moves to a slot of a block
 * of the same width, which is copied out when full (and once at the end).
 * The error of phi is of the order of the square root of r's (r's error is
 * second order in phi's). Options as for rd_query_batch (refine is ignored).
 * When o->flags has RD_DEVICE_PTRS, s, t, out and phi are device pointers.
 * Errors as for rd_query_batch; phi == NULL is RD_E_ARG. Device memory: three
 * more n x width blocks than rd_query_batch (search directions, potentials,
 * finished potentials), plus npairs * n doubles for phi when it is host
 * memory.
 */
rd_status rd_potentials(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t, double eps,
                        const rd_options *o, rd_result *out, double *phi);

/*
 * Diagnostic: timing of the sparse-product launches recorded by calls made
 * with RD_PROFILE in rd_options.flags, since the previous rd_kernel_stats call
 * (which resets the counters). which = 0: the batched product over the rows
 * up to the long-row threshold (k_spmm_short); which = 1: the single-pair
 * product (k_spmv); which = 2: the edge pass of rd_grad_edges (k_grad_edges;
 * the pass over the last block of finished potentials of each call is timed).
 * Durations come from HIP events recorded around
 * each launch on the stream it runs on. alg_bytes receives the mean
 * algorithmic bytes per counted launch (a batched run that narrows its block
 * counts each launch at its own width). Products: adjacency
 * indices (and values, if weighted) of the rows covered, row offsets, the
 * gathered vector block read once, the previous block read and the result
 * block written, and the degree arrays. Edge pass: its work items, the column
 * and edge id of every edge, the FP64 accumulator read and written, and the
 * potential block (stored in the run's vector precision) read once.
 */
rd_status rd_kernel_stats(rd_graph g, int32_t which, double *total_ms, int64_t *launches,
                          double *alg_bytes);

/* Release the handle and its device memory. NULL is ignored. */
void rd_free_graph(rd_graph g);

/* Static description of a status code. */
const char *rd_status_string(rd_status s);

/* Message of the last failing call on g (empty if none); valid until the next
 * call on g. With g == NULL: the message of this thread's last failed
 * rd_init_graph. */
const char *rd_last_error(rd_graph g);

#ifdef __cplusplus
}
#endif

#endif /* RD_H_ */
