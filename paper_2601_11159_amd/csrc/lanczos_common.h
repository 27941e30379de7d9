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
// inc_now = r_k - r_{k-1}, inc_then = r_{k-d} - r_{k-d-1}, span = r_k - r_{k-d}
// and per-step contraction q = (inc_now/inc_then)^(1/d): the geometric tail
// max(span q/(1-q), inc_now) with q capped at 0.9999; infinite when q >= 1;
// |span| + |inc_now| once an increment is not positive (rounding floor).
__device__ __forceinline__ double stop_estimate(const LzState &S) {
  const int k = S.k;
  if (k < 3) return INFINITY;
  const int d = min(S.delay, k - 2);
  auto h = [&](int j) { return S.hist[(j - 1) % RD_HIST]; };  // r_hat_j, 1-based
  const double inow = h(k) - h(k - 1);
  const double ithen = h(k - d) - h(k - d - 1);
  const double span = h(k) - h(k - d);
  if (inow <= 0.0 || ithen <= 0.0) return fabs(span) + fabs(inow);
  double q = pow(inow / ithen, 1.0 / (double)d);
  if (q >= 1.0) return INFINITY;
  q = fmin(q, 0.9999);
  return fmax(span * q / (1.0 - q), inow);
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

__host__ __device__ inline rd_status status_of(int32_t st) {
  switch (st) {
    case LZ_DONE: return RD_OK;
    case LZ_NOT_CONVERGED: return RD_E_NOT_CONVERGED;
    case LZ_BREAKDOWN: return RD_E_BREAKDOWN;
    default: return RD_E_NOT_CONVERGED;
  }
}
