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
constexpr int HOIST_ROWS = 8;  // rows per thread whose degrees stay in registers (n <= 4096)

// CSR_LDS: the row offsets, column ids (and weights) are copied to LDS once,
// after the two vectors, so an iteration touches no global memory.
// HOIST: each thread's (at most HOIST_ROWS) rows keep d_u and 1/d_u in registers.
template <typename VT, bool WEIGHTED, bool CSR_LDS, bool HOIST>
__global__ __launch_bounds__(SMALL_THREADS) void k_small(
    int32_t n, int32_t nnz, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
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
  const int32_t *RP = row_ptr;
  const int32_t *CL = col;
  const VT *WL = w;
  if constexpr (CSR_LDS) {
    int32_t *rp_l = reinterpret_cast<int32_t *>(bufB + n);
    int32_t *col_l = rp_l + (n + 1);
    for (int32_t i = threadIdx.x; i <= n; i += SMALL_THREADS) rp_l[i] = row_ptr[i];
    for (int32_t i = threadIdx.x; i < nnz; i += SMALL_THREADS) col_l[i] = col[i];
    if constexpr (WEIGHTED) {
      // weights after the column ids, aligned to their size
      const size_t off = ((size_t)(n + 1 + nnz) * 4 + sizeof(VT) - 1) / sizeof(VT) * sizeof(VT);
      VT *w_l = reinterpret_cast<VT *>(reinterpret_cast<unsigned char *>(rp_l) + off);
      for (int32_t i = threadIdx.x; i < nnz; i += SMALL_THREADS) w_l[i] = w[i];
      WL = w_l;
    }
    RP = rp_l;
    CL = col_l;
  }
  double dg[HOIST ? HOIST_ROWS : 1];
  VT idg[HOIST ? HOIST_ROWS : 1];
  int32_t rb[HOIST ? HOIST_ROWS : 1], re[HOIST ? HOIST_ROWS : 1];
  if constexpr (HOIST) {
    if constexpr (CSR_LDS) __syncthreads();  // the row offsets in LDS are complete
#pragma unroll
    for (int k = 0; k < HOIST_ROWS; ++k) {
      const int32_t r = threadIdx.x + k * SMALL_THREADS;
      dg[k] = r < n ? deg[r] : 0.0;
      idg[k] = r < n ? invdeg[r] : VT(0);
      rb[k] = r < n ? RP[r] : 0;
      re[k] = r < n ? RP[r + 1] : 0;
    }
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
  // one row of y = sig D^{-1} W U_cur - pc U_prev (over U_prev); returns its
  // contribution to <y, q>_D
  auto spmv_row = [&](int32_t r, VT sig, VT pc, bool has_prev, double d, VT id) {
    VT acc = 0;
    const int32_t pe = RP[r + 1];
    for (int32_t p = RP[r]; p < pe; ++p) {
      const VT x = Ucur[CL[p]];
      acc += WEIGHTED ? WL[p] * x : x;
    }
    VT y = sig * acc * id;
    if (has_prev) y -= pc * Uprev[r];
    Uprev[r] = y;
    return d * (double)y * ((double)sig * (double)Ucur[r]);
  };
  for (;;) {
    const VT sig = (VT)S.sig_cur, pc = (VT)S.prev_coef;
    const bool has_prev = S.prev_coef != 0.0;
    double apart = 0.0;
    if constexpr (HOIST) {
      // the first FRONT entries of all of this thread's rows in flight
      // together: every column id, then every gather
      constexpr int FRONT = 4;
      int32_t ci[HOIST_ROWS][FRONT];
#pragma unroll
      for (int k = 0; k < HOIST_ROWS; ++k)
#pragma unroll
        for (int e = 0; e < FRONT; ++e) ci[k][e] = rb[k] + e < re[k] ? CL[rb[k] + e] : -1;
      VT acc[HOIST_ROWS];
#pragma unroll
      for (int k = 0; k < HOIST_ROWS; ++k) {
        VT x[FRONT];
#pragma unroll
        for (int e = 0; e < FRONT; ++e) x[e] = ci[k][e] >= 0 ? Ucur[ci[k][e]] : VT(0);
        VT a = 0;
#pragma unroll
        for (int e = 0; e < FRONT; ++e) a += WEIGHTED && ci[k][e] >= 0 ? WL[rb[k] + e] * x[e] : x[e];
        acc[k] = a;
      }
#pragma unroll
      for (int k = 0; k < HOIST_ROWS; ++k) {
        const int32_t r = threadIdx.x + k * SMALL_THREADS;
        if (r >= n) continue;
        for (int32_t p = rb[k] + FRONT; p < re[k]; ++p) {
          const VT x = Ucur[CL[p]];
          acc[k] += WEIGHTED ? WL[p] * x : x;
        }
        VT y = sig * acc[k] * idg[k];
        if (has_prev) y -= pc * Uprev[r];
        Uprev[r] = y;
        apart += dg[k] * (double)y * ((double)sig * (double)Ucur[r]);
      }
    } else {
      for (int32_t r = threadIdx.x; r < n; r += SMALL_THREADS)
        apart += spmv_row(r, sig, pc, has_prev, deg[r], invdeg[r]);
    }
    const double alpha = block_sum(apart, red);
    if (threadIdx.x == 0) scalar_after_alpha(S, alpha, tr_alpha, tr_rhat);
    __syncthreads();
    if (S.status != LZ_RUNNING) break;
    // w = y - alpha q_i; ||w||_D^2
    const VT coef = (VT)(S.alpha * S.sig_cur);
    double bacc = 0.0;
    if constexpr (HOIST) {
#pragma unroll
      for (int k = 0; k < HOIST_ROWS; ++k) {
        const int32_t r = threadIdx.x + k * SMALL_THREADS;
        if (r < n) {
          const VT x = Uprev[r] - coef * Ucur[r];
          Uprev[r] = x;
          bacc += dg[k] * ((double)x * (double)x);
        }
      }
    } else {
      for (int32_t r = threadIdx.x; r < n; r += SMALL_THREADS) {
        const VT x = Uprev[r] - coef * Ucur[r];
        Uprev[r] = x;
        bacc += deg[r] * ((double)x * (double)x);
      }
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

// Power Method (Algorithm 1) for one pair per workgroup. With x = D^{-1} r
// in LDS, each step is x <- x/2 + D^{-1} A x / 2 (P = A D^{-1}); before each
// step thread 0 adds r(s)/(2 d_s) - r(t)/(2 d_t) = (x(s) - x(t)) / 2 to the
// FP64 sum. A block barrier separates the steps; the two buffers alternate.
template <typename VT, bool WEIGHTED, bool CSR_LDS>
__global__ __launch_bounds__(SMALL_THREADS) void k_pm_small(
    int32_t n, int32_t nnz, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const VT *__restrict__ w, const VT *__restrict__ invdeg, const double *__restrict__ deg,
    int32_t npairs, const int32_t *__restrict__ ps, const int32_t *__restrict__ pt, int32_t l,
    rd_result *__restrict__ out) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  VT *xa = reinterpret_cast<VT *>(lds_raw);
  VT *xb = xa + n;
  const int32_t pair = blockIdx.x;
  if (pair >= npairs) return;
  const int32_t s = ps[pair], t = pt[pair];
  if (s == t) {
    if (threadIdx.x == 0) out[pair] = rd_result{0.0, 0.0, l, RD_OK};
    return;
  }
  const int32_t *RP = row_ptr;
  const int32_t *CL = col;
  const VT *WL = w;
  if constexpr (CSR_LDS) {
    int32_t *rp_l = reinterpret_cast<int32_t *>(xb + n);
    int32_t *col_l = rp_l + (n + 1);
    for (int32_t i = threadIdx.x; i <= n; i += SMALL_THREADS) rp_l[i] = row_ptr[i];
    for (int32_t i = threadIdx.x; i < nnz; i += SMALL_THREADS) col_l[i] = col[i];
    if constexpr (WEIGHTED) {
      const size_t off = ((size_t)(n + 1 + nnz) * 4 + sizeof(VT) - 1) / sizeof(VT) * sizeof(VT);
      VT *w_l = reinterpret_cast<VT *>(reinterpret_cast<unsigned char *>(rp_l) + off);
      for (int32_t i = threadIdx.x; i < nnz; i += SMALL_THREADS) w_l[i] = w[i];
      WL = w_l;
    }
    RP = rp_l;
    CL = col_l;
  }
  const VT xs = (VT)(1.0 / deg[s]), xt = (VT)(-1.0 / deg[t]);
  for (int32_t r = threadIdx.x; r < n; r += SMALL_THREADS) xa[r] = r == s ? xs : (r == t ? xt : VT(0));
  __syncthreads();
  double sum = 0.0, last = 0.0;
  VT *cur = xa, *nxt = xb;
  for (int32_t i = 0;; ++i) {
    if (threadIdx.x == 0) {
      last = 0.5 * ((double)cur[s] - (double)cur[t]);
      sum += last;
    }
    if (i == l) break;
    for (int32_t r = threadIdx.x; r < n; r += SMALL_THREADS) {
      VT acc = 0;
      const int32_t pe = RP[r + 1];
      for (int32_t p = RP[r]; p < pe; ++p) acc += WEIGHTED ? WL[p] * cur[CL[p]] : cur[CL[p]];
      nxt[r] = VT(0.5) * acc * invdeg[r] + VT(0.5) * cur[r];
    }
    __syncthreads();
    VT *tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (threadIdx.x == 0) out[pair] = rd_result{sum, last, l, RD_OK};
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

// LDS bytes of the two vectors and, when csr, of the row offsets, column ids
// and weights after them.
static size_t small_lds_bytes(rd_graph g, size_t vt, bool csr) {
  size_t b = 2 * (size_t)g->n * vt;
  if (csr) {
    b += ((size_t)(g->n + 1) + (size_t)g->nnz) * 4;
    if (!g->unit) b = (b + vt - 1) / vt * vt + (size_t)g->nnz * vt;
  }
  return b;
}

template <typename VT, bool WEIGHTED>
static void small_launch(rd_graph g, int32_t npairs, const int32_t *ps, const int32_t *pt, int32_t s0,
                         int32_t t0, double eps, const rd_options &o, hipStream_t st, rd_result *out,
                         double *tr_alpha, double *tr_beta, double *tr_rhat) {
  const bool csr = small_lds_bytes(g, sizeof(VT), true) <= small_lds_limit(g);
  const bool hoist = g->n <= SMALL_THREADS * HOIST_ROWS;
  const size_t lds = small_lds_bytes(g, sizeof(VT), csr);
  const VT *w = (const VT *)(sizeof(VT) == 8 ? (const void *)g->w64 : (const void *)g->w32);
  const VT *id = (const VT *)(sizeof(VT) == 8 ? (const void *)g->invdeg : (const void *)g->invdeg32);
  const dim3 grid(npairs), block(SMALL_THREADS);
#define RD_SMALL_LAUNCH(CSR, HOIST)                                                                  \
  hipLaunchKernelGGL((k_small<VT, WEIGHTED, CSR, HOIST>), grid, block, lds, st, g->n, (int32_t)g->nnz, \
                     g->row_ptr, g->col, WEIGHTED ? w : (const VT *)nullptr, id, g->deg, npairs, ps,  \
                     pt, s0, t0, eps, o.max_iters, o.fixed_k, o.delay, o.err_mode, out, tr_alpha,     \
                     tr_beta, tr_rhat)
  if (csr && hoist) RD_SMALL_LAUNCH(true, true);
  else if (csr) RD_SMALL_LAUNCH(true, false);
  else if (hoist) RD_SMALL_LAUNCH(false, true);
  else RD_SMALL_LAUNCH(false, false);
#undef RD_SMALL_LAUNCH
}

// npairs pairs (device arrays), one workgroup each; results to device `out`.
// ps == nullptr: a single pair (s0, t0).
void small_run(rd_graph g, int32_t npairs, const int32_t *ps, const int32_t *pt, int32_t s0,
               int32_t t0, double eps, const rd_options &o, hipStream_t st, rd_result *out,
               double *tr_alpha, double *tr_beta, double *tr_rhat) {
  if (npairs <= 0) return;
  if (o.precision == RD_F64) {
    if (g->unit)
      small_launch<double, false>(g, npairs, ps, pt, s0, t0, eps, o, st, out, tr_alpha, tr_beta, tr_rhat);
    else
      small_launch<double, true>(g, npairs, ps, pt, s0, t0, eps, o, st, out, tr_alpha, tr_beta, tr_rhat);
  } else {
    if (g->unit)
      small_launch<float, false>(g, npairs, ps, pt, s0, t0, eps, o, st, out, tr_alpha, tr_beta, tr_rhat);
    else
      small_launch<float, true>(g, npairs, ps, pt, s0, t0, eps, o, st, out, tr_alpha, tr_beta, tr_rhat);
  }
  RD_HIP(hipGetLastError());
}

template <typename VT, bool WEIGHTED>
static void pm_small_launch(rd_graph g, int32_t npairs, const int32_t *ps, const int32_t *pt, int32_t l,
                            hipStream_t st, rd_result *out) {
  const bool csr = small_lds_bytes(g, sizeof(VT), true) <= small_lds_limit(g);
  const size_t lds = small_lds_bytes(g, sizeof(VT), csr);
  const VT *w = (const VT *)(sizeof(VT) == 8 ? (const void *)g->w64 : (const void *)g->w32);
  const VT *id = (const VT *)(sizeof(VT) == 8 ? (const void *)g->invdeg : (const void *)g->invdeg32);
  if (csr)
    hipLaunchKernelGGL((k_pm_small<VT, WEIGHTED, true>), dim3(npairs), dim3(SMALL_THREADS), lds, st, g->n,
                       (int32_t)g->nnz, g->row_ptr, g->col, WEIGHTED ? w : (const VT *)nullptr, id, g->deg,
                       npairs, ps, pt, l, out);
  else
    hipLaunchKernelGGL((k_pm_small<VT, WEIGHTED, false>), dim3(npairs), dim3(SMALL_THREADS), lds, st, g->n,
                       (int32_t)g->nnz, g->row_ptr, g->col, WEIGHTED ? w : (const VT *)nullptr, id, g->deg,
                       npairs, ps, pt, l, out);
}

// Power Method for graphs whose two vectors fit in LDS: one workgroup per pair.
void pm_small_run(rd_graph g, int32_t npairs, const int32_t *ps, const int32_t *pt, int32_t l,
                  const rd_options &o, hipStream_t st, rd_result *out) {
  if (npairs <= 0) return;
  if (o.precision == RD_F64) {
    if (g->unit) pm_small_launch<double, false>(g, npairs, ps, pt, l, st, out);
    else pm_small_launch<double, true>(g, npairs, ps, pt, l, st, out);
  } else {
    if (g->unit) pm_small_launch<float, false>(g, npairs, ps, pt, l, st, out);
    else pm_small_launch<float, true>(g, npairs, ps, pt, l, st, out);
  }
  RD_HIP(hipGetLastError());
}
