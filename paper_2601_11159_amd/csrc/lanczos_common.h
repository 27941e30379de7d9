// Device helpers shared by the single-pair and batched Lanczos paths:
// fixed-order reductions and the per-run scalar logic (tridiagonal solve and
// stopping test), all in FP64.
#pragma once

#include <hip/hip_runtime.h>

#include "rd_internal.h"

// Sum over a full 64-lane wavefront in a fixed butterfly order.
template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Block-wide sum (blockDim.x a multiple of 64, at most 1024), fixed order.
// The result is valid in every thread. `sm` needs blockDim.x/64 slots.
template <typename T>
__device__ __forceinline__ T block_sum(T x, T *sm) {
  x = wave_sum(x);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sm[wid] = x;
  __syncthreads();
  T r = (lane < nw) ? sm[lane] : T(0);
  r = wave_sum(r);
  return r;
}

// Stopping estimate of the remaining error of r_hat_k from the recent values
// (reading of the paper, which fixes k): with window d = min(delay, k-2),
// inc_now = r_k - r_{k-1}, inc_prev = r_{k-1} - r_{k-2},
// inc_then = r_{k-d} - r_{k-d-1} and mean per-step contraction
// q = (inc_now/inc_then)^(1/d): eight times the geometric tail of the latest
// increment, max(8 inc_now q/(1-q), inc_now), with q capped at 0.9999;
// infinite when q >= 1; |inc_now| + |inc_prev| once an increment is not
// positive (rounding floor).
__device__ __forceinline__ double stop_estimate(const LzState &S) {
  const int k = S.k;
  if (k < 3) return INFINITY;
  const int d = min(S.delay, k - 2);
  auto h = [&](int j) { return S.hist[(j - 1) % RD_HIST]; };  // r_hat_j, 1-based
  const double inow = h(k) - h(k - 1);
  const double iprev = h(k - 1) - h(k - 2);
  const double ithen = h(k - d) - h(k - d - 1);
  if (inow <= 0.0 || ithen <= 0.0) return fabs(inow) + fabs(iprev);
  double q = pow(inow / ithen, 1.0 / (double)d);
  if (q >= 1.0) return INFINITY;
  q = fmin(q, 0.9999);
  return fmax(8.0 * inow * q / (1.0 - q), inow);
}

// Iteration i = S.k + 1 has produced alpha_i. Extend the LDL^T factorisation
// of I - T_i (pivots delta, e_1 component omega) and the value
// g_i = e_1^T (I - T_i)^{-1} e_1 = sum_j omega_j^2 / delta_j, so that
// r_hat_i = c g_i (the output formula of Algorithm 3), then apply the
// stopping test. Returns false on a non-positive pivot or non-finite value.
__device__ __forceinline__ void scalar_after_alpha(LzState &S, double alpha, double *tr_alpha,
                                                   double *tr_rhat) {
  const int i = S.k + 1;
  double delta, omega, g;
  if (i == 1) {
    delta = 1.0 - alpha;
    omega = 1.0;
    g = 1.0 / delta;
  } else {
    omega = S.omega * S.beta / S.delta;
    delta = (1.0 - alpha) - S.beta * S.beta / S.delta;
    g = S.g + omega * omega / delta;
  }
  if (!(delta > 0.0) || !isfinite(g) || !isfinite(alpha)) {
    S.status = LZ_BREAKDOWN;  // keep the last good r_hat
    return;
  }
  S.alpha = alpha;
  S.delta = delta;
  S.omega = omega;
  S.g = g;
  S.rhat = S.c * g;
  S.k = i;
  S.hist[(i - 1) % RD_HIST] = S.rhat;
  if (tr_alpha) tr_alpha[i - 1] = alpha;
  if (tr_rhat) tr_rhat[i - 1] = S.rhat;
  if (S.fixed_k == 0) {
    const double est = stop_estimate(S);
    S.err_est = est;
    const double thr = S.err_mode == 0 ? S.tol * S.rhat : S.tol;
    if (est <= thr) S.status = LZ_DONE;
  }
}

// beta_{i+1} = sqrt(bb) is known: exact breakdown, caps, and the scale-on-read
// coefficients of the next iteration.
__device__ __forceinline__ void scalar_after_beta(LzState &S, double bb, double *tr_beta) {
  const int i = S.k;
  const double beta_next = sqrt(bb);
  if (tr_beta) tr_beta[i - 1] = beta_next;
  if (!isfinite(beta_next)) {
    S.status = LZ_BREAKDOWN;
    return;
  }
  if (beta_next <= 1e-13 * (fabs(S.alpha) + S.beta)) {
    S.status = LZ_DONE;  // invariant Krylov space: r_hat_i is exact
    S.err_est = 0.0;
    return;
  }
  S.prev_coef = beta_next * S.sig_cur;
  S.sig_prev = S.sig_cur;
  S.sig_cur = 1.0 / beta_next;
  S.beta = beta_next;
  if (S.fixed_k > 0 && i >= S.fixed_k) S.status = LZ_DONE;
  else if (i >= S.max_iters) S.status = LZ_NOT_CONVERGED;
}

__device__ __forceinline__ void state_start(LzState &S, int32_t s, int32_t t, double c, double tol,
                                            int32_t max_iters, int32_t fixed_k, int32_t delay,
                                            int32_t err_mode, int32_t pair) {
  S.c = c;
  S.sig_cur = 1.0;
  S.sig_prev = 0.0;
  S.ro_mu = S.ro_c = S.ro_p = 0.0;
  S.prev_coef = 0.0;
  S.beta = 0.0;
  S.alpha = 0.0;
  S.delta = 1.0;
  S.omega = 1.0;
  S.g = 0.0;
  S.rhat = 0.0;
  S.err_est = INFINITY;
  S.tol = tol;
  for (int j = 0; j < RD_HIST; ++j) S.hist[j] = 0.0;
  S.k = 0;
  S.status = LZ_RUNNING;
  S.max_iters = max_iters;
  S.fixed_k = fixed_k;
  S.delay = delay;
  S.err_mode = err_mode;
  S.s = s;
  S.t = t;
  S.pair = pair;
}

// Position of `target` in the ascending adjacency row r, or -1.
__device__ __forceinline__ int32_t row_find(const int32_t *__restrict__ row_ptr,
                                            const int32_t *__restrict__ col, int32_t r,
                                            int32_t target) {
  int32_t lo = row_ptr[r], hi = row_ptr[r + 1];
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    const int32_t c = col[mid];
    if (c == target) return mid;
    if (c < target) lo = mid + 1; else hi = mid;
  }
  return -1;
}

// The first iteration of Algorithm 3 computed from the adjacency rows of s and
// t only: q_1 = (e_s/d_s - e_t/d_t)/sqrt(c) has two non-zeros, so
// y_1 = D^{-1} W q_1 lives on N(s) u N(t), alpha_1 = <y_1, q_1>_D involves
// rows s and t alone, and w_1 = y_1 - alpha_1 q_1 lives on N(s) u N(t) u {s, t}.
// Every entry of w_1 is passed once to store(u, value, pos) (which returns the
// value as stored, e.g. rounded to FP32). pos is the entry's slot in a list
// of deg_s + deg_t + 2 slots (deg_x = row length): entries of row s take their
// adjacency position, entries of row t not in row s take deg_s + theirs, and
// s and t, when they are not neighbours, the last two. The slots of row-t
// entries that are also in row s (and the last two when s ~ t) stay unused.
// The block returns alpha_1 and ||w_1||_D^2 (summed in a fixed order) in every
// thread. All threads of the block must call it. `sm` needs blockDim.x/64 + 2 doubles.
template <typename Store>
__device__ void first_iteration(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                const double *__restrict__ w64, const double *__restrict__ deg,
                                int32_t s, int32_t t, double c, Store store, double *sm,
                                double &alpha1, double &bb) {
  const double rc = 1.0 / sqrt(c);
  const double ds = deg[s], dt = deg[t];
  const double q1s = rc / ds, q1t = -rc / dt;
  const int nw = blockDim.x >> 6;
  if (threadIdx.x == 0) {
    const int32_t p = row_find(row_ptr, col, s, t);
    const double wst = p < 0 ? 0.0 : (w64 ? w64[p] : 1.0);
    const double y1s = wst * q1t / ds, y1t = wst * q1s / dt;
    sm[nw] = ds * y1s * q1s + dt * y1t * q1t;
    sm[nw + 1] = p < 0 ? 0.0 : 1.0;
  }
  __syncthreads();
  const double a1 = sm[nw];
  const bool adjacent = sm[nw + 1] != 0.0;
  double acc = 0.0;
  // u in N(s): y_1[u] = (w_us q1s + w_ut q1t)/d_u, the second term if u ~ t
  for (int32_t p = row_ptr[s] + threadIdx.x; p < row_ptr[s + 1]; p += blockDim.x) {
    const int32_t u = col[p];
    double val = (w64 ? w64[p] : 1.0) * q1s;
    const int32_t pt = row_find(row_ptr, col, t, u);
    if (pt >= 0) val += (w64 ? w64[pt] : 1.0) * q1t;
    val /= deg[u];
    if (u == t) val -= a1 * q1t;
    const double stored = store(u, val, p - row_ptr[s]);
    acc += deg[u] * stored * stored;
  }
  // u in N(t) \ N(s)
  for (int32_t p = row_ptr[t] + threadIdx.x; p < row_ptr[t + 1]; p += blockDim.x) {
    const int32_t u = col[p];
    if (row_find(row_ptr, col, s, u) >= 0) continue;
    double val = (w64 ? w64[p] : 1.0) * q1t / deg[u];
    if (u == s) val -= a1 * q1s;
    const double stored = store(u, val, (row_ptr[s + 1] - row_ptr[s]) + (p - row_ptr[t]));
    acc += deg[u] * stored * stored;
  }
  // s and t themselves when they are not neighbours (then y_1[s] = y_1[t] = 0)
  if (threadIdx.x == 0 && !adjacent) {
    const int32_t base = (row_ptr[s + 1] - row_ptr[s]) + (row_ptr[t + 1] - row_ptr[t]);
    const double vs = store(s, -a1 * q1s, base);
    const double vt = store(t, -a1 * q1t, base + 1);
    acc += ds * vs * vs + dt * vt * vt;
  }
  bb = block_sum(acc, sm);
  alpha1 = a1;
}

__host__ __device__ inline rd_status status_of(int32_t st) {
  switch (st) {
    case LZ_DONE: return RD_OK;
    case LZ_NOT_CONVERGED: return RD_E_NOT_CONVERGED;
    case LZ_BREAKDOWN: return RD_E_BREAKDOWN;
    default: return RD_E_NOT_CONVERGED;
  }
}
