// Small graphs: one workgroup runs the whole Lanczos iteration of one pair.
//
// When both n-vectors fit in LDS, the per-iteration cost of the general path
// (four launches, device-wide reductions, host polling) dominates. Here a
// workgroup keeps U_cur and U_prev in LDS, reads the CSR from L2, and
// synchronises with block barriers; the host launches once per batch (one
// workgroup per pair). The arithmetic is that of the general path: the same
// degree-scaled recurrence, scale-on-read normalisation, FP64 sums and the
// same scalar update and stopping test (lanczos_common.h).

#include <algorithm>

#include "lanczos_common.h"

namespace {

constexpr int SMALL_THREADS = 512;

template <typename VT, bool WEIGHTED>
__global__ __launch_bounds__(SMALL_THREADS) void k_small(
    int32_t n, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const VT *__restrict__ w, const VT *__restrict__ invdeg, const double *__restrict__ deg,
    int32_t npairs, const int32_t *__restrict__ ps, const int32_t *__restrict__ pt, int32_t s0,
    int32_t t0, double tol,
    int32_t max_iters, int32_t fixed_k, int32_t delay, int32_t err_mode, rd_result *__restrict__ out,
    double *tr_alpha, double *tr_beta, double *tr_rhat) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  VT *bufA = reinterpret_cast<VT *>(lds_raw);
  VT *bufB = bufA + n;
  __shared__ double red[SMALL_THREADS / 64];
  __shared__ LzState S;
  const int32_t pair = blockIdx.x;
  if (pair >= npairs) return;
  const int32_t s = ps ? ps[pair] : s0, t = pt ? pt[pair] : t0;
  if (s == t) {
    if (threadIdx.x == 0) out[pair] = rd_result{0.0, 0.0, 0, RD_OK};
    return;
  }
  const double c = 1.0 / deg[s] + 1.0 / deg[t];
  const double rc = 1.0 / sqrt(c);
  for (int32_t r = threadIdx.x; r < n; r += SMALL_THREADS) {
    double x = 0.0;
    if (r == s) x = rc / deg[s];
    if (r == t) x = -rc / deg[t];
    bufA[r] = (VT)x;  // q_1
  }
  if (threadIdx.x == 0) state_start(S, s, t, c, tol, max_iters, fixed_k, delay, err_mode, pair);
  __syncthreads();
  VT *Ucur = bufA, *Uprev = bufB;
  for (;;) {
    const VT sig = (VT)S.sig_cur, pc = (VT)S.prev_coef;
    const bool has_prev = S.prev_coef != 0.0;
    // y = sig D^{-1} W U_cur - pc U_prev, over U_prev; <y, q>_D
    double apart = 0.0;
    for (int32_t r = threadIdx.x; r < n; r += SMALL_THREADS) {
      VT acc = 0;
      for (int32_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p) {
        const VT x = Ucur[col[p]];
        acc += WEIGHTED ? w[p] * x : x;
      }
      VT y = sig * acc * invdeg[r];
      if (has_prev) y -= pc * Uprev[r];
      Uprev[r] = y;
      apart += deg[r] * (double)y * ((double)sig * (double)Ucur[r]);
    }
    const double alpha = block_sum(apart, red);
    if (threadIdx.x == 0) scalar_after_alpha(S, alpha, tr_alpha, tr_rhat);
    __syncthreads();
    if (S.status != LZ_RUNNING) break;
    // w = y - alpha q_i; ||w||_D^2
    const VT coef = (VT)(S.alpha * S.sig_cur);
    double bacc = 0.0;
    for (int32_t r = threadIdx.x; r < n; r += SMALL_THREADS) {
      const VT x = Uprev[r] - coef * Ucur[r];
      Uprev[r] = x;
      bacc += deg[r] * ((double)x * (double)x);
    }
    const double bb = block_sum(bacc, red);
    if (threadIdx.x == 0) scalar_after_beta(S, bb, tr_beta);
    __syncthreads();
    if (S.status != LZ_RUNNING) break;
    VT *tmp = Ucur;
    Ucur = Uprev;
    Uprev = tmp;
  }
  if (threadIdx.x == 0) {
    rd_result res;
    res.r = S.rhat;
    res.err_est = S.err_est;
    res.iters = S.k;
    res.status = (int32_t)status_of(S.status);
    out[pair] = res;
  }
}

}  // namespace

// Largest dynamic LDS per workgroup the small path may use.
static size_t small_lds_limit(rd_graph g) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, g->device) != hipSuccess) return 64 * 1024;
  return std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024) - 1024;
}

bool small_eligible(rd_graph g, const rd_options &o) {
  if ((o.flags & RD_GENERAL_PATH) || o.reorth > 0) return false;
  const size_t vt = o.precision == RD_F64 ? sizeof(double) : sizeof(float);
  return 2 * (size_t)g->n * vt <= small_lds_limit(g);
}

// npairs pairs (device arrays), one workgroup each; results to device `out`.
// ps == nullptr: a single pair (s0, t0).
void small_run(rd_graph g, int32_t npairs, const int32_t *ps, const int32_t *pt, int32_t s0,
               int32_t t0, double eps, const rd_options &o, hipStream_t st, rd_result *out,
               double *tr_alpha, double *tr_beta, double *tr_rhat) {
  if (npairs <= 0) return;
  const size_t vt = o.precision == RD_F64 ? sizeof(double) : sizeof(float);
  const size_t lds = 2 * (size_t)g->n * vt;
  const dim3 grid(npairs), block(SMALL_THREADS);
  if (o.precision == RD_F64) {
    if (g->unit)
      hipLaunchKernelGGL((k_small<double, false>), grid, block, lds, st, g->n, g->row_ptr, g->col,
                         (const double *)nullptr, (const double *)g->invdeg, g->deg, npairs, ps, pt,
                         s0, t0, eps, o.max_iters, o.fixed_k, o.delay, o.err_mode, out, tr_alpha, tr_beta,
                         tr_rhat);
    else
      hipLaunchKernelGGL((k_small<double, true>), grid, block, lds, st, g->n, g->row_ptr, g->col,
                         (const double *)g->w64, (const double *)g->invdeg, g->deg, npairs, ps, pt,
                         s0, t0, eps, o.max_iters, o.fixed_k, o.delay, o.err_mode, out, tr_alpha, tr_beta,
                         tr_rhat);
  } else {
    if (g->unit)
      hipLaunchKernelGGL((k_small<float, false>), grid, block, lds, st, g->n, g->row_ptr, g->col,
                         (const float *)nullptr, (const float *)g->invdeg32, g->deg, npairs, ps, pt,
                         s0, t0, eps, o.max_iters, o.fixed_k, o.delay, o.err_mode, out, tr_alpha, tr_beta,
                         tr_rhat);
    else
      hipLaunchKernelGGL((k_small<float, true>), grid, block, lds, st, g->n, g->row_ptr, g->col,
                         (const float *)g->w32, (const float *)g->invdeg32, g->deg, npairs, ps, pt,
                         s0, t0, eps, o.max_iters, o.fixed_k, o.delay, o.err_mode, out, tr_alpha, tr_beta,
                         tr_rhat);
  }
  RD_HIP(hipGetLastError());
}
