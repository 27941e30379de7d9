// Single-pair Lanczos iteration (Algorithm 3) on the device.
//
// Vectors are kept in the degree-scaled basis q_i = D^{-1/2} v_i. The
// recurrence of Eq. lz_recurrence, beta_{i+1} v_{i+1} = (calA - alpha_i) v_i -
// beta_i v_{i-1} with calA = D^{-1/2} W D^{-1/2}, becomes
//     beta_{i+1} q_{i+1} = (D^{-1} W - alpha_i) q_i - beta_i q_{i-1},
// and the inner products <x, y> of v-vectors become sum_u d_u x_u y_u. The
// alpha_i, beta_i, T and r_hat are identical; for unit weights the product
// needs no stored matrix values and no per-entry scale factors.
//
// Each vector is stored unnormalised together with a scale (q_i = sig * U_i),
// so the division by beta_{i+1} is applied when the vector is next read.
//
// Three vector buffers rotate (q_{i-1}, q_i and the new vector). One iteration
// = four launches on one stream:
//   k_spmv          y = sig_i D^{-1} W U_i - beta_i q_{i-1}   (+ per-block <y, q_i>_D)
//   k_reduce_alpha  alpha_i, LDL^T update of I - T_i, r_hat_i, stopping test
//   k_update        w = y - alpha_i q_i                       (+ per-block ||w||_D^2)
//   k_reduce_beta   beta_{i+1}, breakdown test, next scales
// With re-orthogonalisation, k_update also sums the coefficients and
// k_reorth_coef + k_reorth_apply remove the components before k_reduce_beta.
// (The partial sums are combined by separate one-block launches: a last-block
// reduction inside the producing kernel needs a device-scope release per block,
// which writes back the whole L2 of its XCD and made the product 6x slower.)
// Every kernel returns at once when the run has stopped, so the host may
// enqueue iterations ahead of the stopping decision.

#include <algorithm>
#include <cmath>
#include <vector>

#include "lanczos_common.h"

namespace {

constexpr int SPMV_THREADS = 256;
constexpr int BLOCK_NNZ = SPMV_BLOCK_NNZ;    // adjacency entries staged per multi-row block
constexpr int BLOCK_ROWS = SPMV_BLOCK_ROWS;  // rows per multi-row block (the schedule guarantees it)
static_assert(BLOCK_ROWS == SPMV_THREADS, "one epilogue row per thread");
static_assert(BLOCK_NNZ % SPMV_THREADS == 0, "whole gather rounds");
constexpr int UPD_THREADS = 256;
constexpr int RED_THREADS = 1024;

template <typename VT>
struct VecTraits;
template <>
struct VecTraits<double> {
  static const double *w(rd_graph g) { return g->w64; }
  static const double *invdeg(rd_graph g) { return g->invdeg; }
};
template <>
struct VecTraits<float> {
  static const float *w(rd_graph g) { return g->w32; }
  static const float *invdeg(rd_graph g) { return g->invdeg32; }
};

// Fixed-order sum of nb partials by one block.
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int nb, double *sm) {
  double a = 0.0;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) a += part[j];
  return block_sum(a, sm);
}

// y_u = sig (1/d_u) sum_v w_uv U_cur[v] - prev_coef U_prev[u] into Y (the third
// vector buffer); per-block partial of sum_u d_u y_u (sig U_cur[u]).
//
// Multi-row blocks run in three phases so no global load sits on a serial
// chain: (1) stage the block's row offsets and the gathered products
// w_uv U_cur[v] in LDS with coalesced index loads; (2) groups of 2^lanes
// threads reduce rows from LDS in a fixed order; (3) one thread per row applies
// the recurrence with coalesced per-row loads and stores.
template <typename VT, bool WEIGHTED>
__global__ __launch_bounds__(SPMV_THREADS) void k_spmv(
    const int32_t *__restrict__ blk_row, const int8_t *__restrict__ blk_lanes,
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const VT *__restrict__ w, const VT *__restrict__ invdeg, const double *__restrict__ deg,
    const VT *__restrict__ Ucur, const VT *__restrict__ Uprev, VT *__restrict__ Y,
    double *__restrict__ part, const LzState *__restrict__ st) {
  if (st->status != LZ_RUNNING) return;
  __shared__ VT vals[BLOCK_NNZ];
  __shared__ VT rsum[BLOCK_ROWS];
  __shared__ int32_t rp[BLOCK_ROWS + 1];
  __shared__ double red[SPMV_THREADS / 64];
  __shared__ VT vred[SPMV_THREADS / 64];
  const double sigd = st->sig_cur, pcd = st->prev_coef;
  const VT sig = (VT)sigd, pc = (VT)pcd;
  const bool has_prev = pcd != 0.0;
  const int b = blockIdx.x, tid = threadIdx.x;
  const int32_t r0 = blk_row[b], r1 = blk_row[b + 1];
  const int lg = blk_lanes[b];
  double apart = 0.0;
  if (lg < 0) {
    const int32_t p0 = row_ptr[r0], p1 = row_ptr[r0 + 1];
    VT acc[4] = {0, 0, 0, 0};
    int32_t p = p0 + tid;
    for (; p + 3 * SPMV_THREADS < p1; p += 4 * SPMV_THREADS) {
      int32_t c[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] = col[p + k * SPMV_THREADS];
      VT x[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = Ucur[c[k]];
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] += WEIGHTED ? w[p + k * SPMV_THREADS] * x[k] : x[k];
    }
    for (; p < p1; p += SPMV_THREADS) {
      const VT x = Ucur[col[p]];
      acc[0] += WEIGHTED ? w[p] * x : x;
    }
    VT a = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    a = block_sum(a, vred);
    if (tid == 0) {
      VT y = sig * a * invdeg[r0];
      if (has_prev) y -= pc * Uprev[r0];
      Y[r0] = y;
      apart = deg[r0] * (double)y * ((double)sig * (double)Ucur[r0]);
    }
  } else {
    const int32_t nrows = r1 - r0;
    const int32_t p0 = row_ptr[r0], p1 = row_ptr[r1];
    for (int32_t j = tid; j <= nrows; j += SPMV_THREADS) rp[j] = row_ptr[r0 + j];
    // operands of this thread's epilogue row, loaded while the products are gathered
    const bool mine = tid < nrows;
    const int32_t r = r0 + tid;
    VT e_id = 0, e_u = 0, e_y = 0;
    double e_d = 0.0;
    if (mine) {
      e_id = invdeg[r];
      e_u = Ucur[r];
      e_d = deg[r];
      if (has_prev) e_y = Uprev[r];
    }
    // at most BLOCK_NNZ entries: every index load, then every gather, in flight at once
    constexpr int PER = BLOCK_NNZ / SPMV_THREADS;
    int32_t c[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int32_t p = p0 + tid + k * SPMV_THREADS;
      c[k] = p < p1 ? col[p] : -1;
    }
    VT x[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) x[k] = c[k] >= 0 ? Ucur[c[k]] : VT(0);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int32_t p = p0 + tid + k * SPMV_THREADS;
      if (p < p1) vals[p - p0] = WEIGHTED ? w[p] * x[k] : x[k];
    }
    __syncthreads();
    const int gsz = 1 << lg, lane = tid & (gsz - 1);
    const int ngrp = SPMV_THREADS >> lg;
    for (int32_t j = tid >> lg; j < nrows; j += ngrp) {
      const int32_t qb = rp[j] - p0, qe = rp[j + 1] - p0;
      VT acc = 0;
      for (int32_t q = qb + lane; q < qe; q += gsz) acc += vals[q];
      for (int off = gsz >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, gsz);
      if (lane == 0) rsum[j] = acc;
    }
    __syncthreads();
    if (mine) {
      VT y = sig * rsum[tid] * e_id;
      if (has_prev) y -= pc * e_y;
      Y[r] = y;
      apart = e_d * (double)y * ((double)sig * (double)e_u);
    }
  }
  apart = block_sum(apart, red);
  if (tid == 0) part[b] = apart;
}

// alpha_i from the product's partials (fixed order), the LDL^T update of
// I - T_i, r_hat_i and the stopping test.
__global__ __launch_bounds__(RED_THREADS) void k_reduce_alpha(const double *__restrict__ part, int nb,
                                                              LzState *__restrict__ st,
                                                              double *tr_alpha, double *tr_rhat) {
  if (st->status != LZ_RUNNING) return;
  __shared__ double sm[RED_THREADS / 64];
  const double a = sum_partials(part, nb, sm);
  if (threadIdx.x == 0) {
    LzState S = *st;
    scalar_after_alpha(S, a, tr_alpha, tr_rhat);
    *st = S;
  }
}


// w = y - alpha_i sig_i U_cur, in place over y; per-block partials (slab j at
// part + j * nb): sum d w^2; RO >= 1: sum d w; RO == 2: sum d w U_cur and
// sum d w U_prev (the coefficients of the re-orthogonalisation).
template <typename VT, int RO>
__global__ __launch_bounds__(UPD_THREADS) void k_update(int32_t n, const double *__restrict__ deg,
                                                        const VT *__restrict__ Ucur,
                                                        const VT *__restrict__ Uprev,
                                                        VT *__restrict__ Y, double *__restrict__ part,
                                                        const LzState *__restrict__ st) {
  if (st->status != LZ_RUNNING) return;
  __shared__ double red[UPD_THREADS / 64];
  const VT a = (VT)(st->alpha * st->sig_cur);
  double acc = 0.0, a1 = 0.0, ac = 0.0, ap = 0.0;
  for (int32_t i = blockIdx.x * UPD_THREADS + threadIdx.x; i < n; i += gridDim.x * UPD_THREADS) {
    const VT u = Ucur[i];
    VT x = Y[i] - a * u;
    Y[i] = x;
    const double d = deg[i], dx = d * (double)x;
    acc += dx * (double)x;
    if constexpr (RO >= 1) a1 += dx;
    if constexpr (RO == 2) {
      ac += dx * (double)u;
      ap += dx * (double)Uprev[i];
    }
  }
  const int nb = gridDim.x;
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
  if constexpr (RO >= 1) {
    a1 = block_sum(a1, red);
    if (threadIdx.x == 0) part[nb + blockIdx.x] = a1;
  }
  if constexpr (RO == 2) {
    ac = block_sum(ac, red);
    ap = block_sum(ap, red);
    if (threadIdx.x == 0) {
      part[2 * nb + blockIdx.x] = ac;
      part[3 * nb + blockIdx.x] = ap;
    }
  }
}

// Coefficients of the re-orthogonalisation from the partials of k_update (fixed
// order), in terms of the stored vectors: with S1 = sum d w, Sc = sum d w U_cur,
// Sp = sum d w U_prev, the components of w along u_1 (in the scaled basis the
// constant vector), q_i = sig_cur U_cur and q_{i-1} = sig_prev U_prev are
// removed by w -= (S1/vol) 1 + sig_cur^2 Sc U_cur + sig_prev^2 Sp U_prev.
template <int RO>
__global__ __launch_bounds__(RED_THREADS) void k_reorth_coef(const double *__restrict__ part, int nb,
                                                             double vol, LzState *__restrict__ st) {
  if (st->status != LZ_RUNNING) return;
  __shared__ double sm[RED_THREADS / 64];
  const double s1 = sum_partials(part + nb, nb, sm);
  double sc = 0.0, sp = 0.0;
  if constexpr (RO == 2) {
    sc = sum_partials(part + 2 * nb, nb, sm);
    sp = sum_partials(part + 3 * nb, nb, sm);
  }
  if (threadIdx.x == 0) {
    LzState S = *st;
    S.ro_mu = s1 / vol;
    S.ro_c = S.sig_cur * S.sig_cur * sc;
    S.ro_p = S.sig_prev * S.sig_prev * sp;
    *st = S;
  }
}

// w -= ro_mu 1 + ro_c U_cur + ro_p U_prev, per-block partial of sum d w^2.
template <typename VT, int RO>
__global__ __launch_bounds__(UPD_THREADS) void k_reorth_apply(int32_t n, const double *__restrict__ deg,
                                                              const VT *__restrict__ Ucur,
                                                              const VT *__restrict__ Uprev,
                                                              VT *__restrict__ Y,
                                                              double *__restrict__ part,
                                                              const LzState *__restrict__ st) {
  if (st->status != LZ_RUNNING) return;
  __shared__ double red[UPD_THREADS / 64];
  const VT mu = (VT)st->ro_mu, cc = (VT)st->ro_c, cp = (VT)st->ro_p;
  double acc = 0.0;
  for (int32_t i = blockIdx.x * UPD_THREADS + threadIdx.x; i < n; i += gridDim.x * UPD_THREADS) {
    VT x = Y[i] - mu;
    if constexpr (RO == 2) x -= cc * Ucur[i] + cp * Uprev[i];
    Y[i] = x;
    acc += deg[i] * ((double)x * (double)x);
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// beta_{i+1} (fixed order), breakdown test, next scales.
__global__ __launch_bounds__(RED_THREADS) void k_reduce_beta(const double *__restrict__ part, int nb,
                                                             LzState *__restrict__ st,
                                                             double *tr_beta) {
  if (st->status != LZ_RUNNING) return;
  __shared__ double sm[RED_THREADS / 64];
  const double bb = sum_partials(part, nb, sm);
  if (threadIdx.x == 0) {
    LzState S = *st;
    scalar_after_beta(S, bb, tr_beta);
    *st = S;
  }
}

// q_1 = (e_s/d_s - e_t/d_t)/sqrt(c), c = 1/d_s + 1/d_t (v_1 of Algorithm 3 in the scaled basis).
template <typename VT>
__global__ void k_init(int32_t n, VT *__restrict__ U, VT *__restrict__ U1, VT *__restrict__ U2,
                       const double *__restrict__ deg, int32_t s, int32_t t, double tol,
                       int32_t max_iters, int32_t fixed_k, int32_t delay, int32_t err_mode,
                       LzState *__restrict__ st) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double c = 1.0 / deg[s] + 1.0 / deg[t];
    const double rc = 1.0 / sqrt(c);
    double x = 0.0;
    if (i == s) x = rc / deg[s];
    if (i == t) x = -rc / deg[t];
    U[i] = (VT)x;
    U1[i] = VT(0);
    U2[i] = VT(0);  // the sparse second iteration writes w_2 into a zero vector
    if (i == 0) {
      LzState S;
      state_start(S, s, t, c, tol, max_iters, fixed_k, delay, err_mode, 0);
      *st = S;
    }
  }
}

// Iteration 1 from the adjacency rows of s and t (q_1 has two non-zeros):
// w_1 is scattered into U1 (zeroed by k_init), then alpha_1 and beta_2 go
// through the same scalar update as every later iteration.
template <typename VT>
__global__ __launch_bounds__(256) void k_first(const int32_t *__restrict__ row_ptr,
                                               const int32_t *__restrict__ col,
                                               const double *__restrict__ w64,
                                               const double *__restrict__ deg, VT *__restrict__ U1,
                                               LzState *__restrict__ st, double *tr_alpha,
                                               double *tr_beta, double *tr_rhat) {
  __shared__ double sm[256 / 64 + 2];
  __shared__ int32_t s, t;
  __shared__ double c;
  if (threadIdx.x == 0) {
    s = st->s;
    t = st->t;
    c = st->c;
  }
  __syncthreads();
  double a1, bb;
  first_iteration(
      row_ptr, col, w64, deg, s, t, c,
      [&](int32_t u, double val, int32_t) {
        const VT x = (VT)val;
        U1[u] = x;
        return (double)x;
      },
      sm, a1, bb);
  if (threadIdx.x == 0) {
    LzState S = *st;
    scalar_after_alpha(S, a1, tr_alpha, tr_rhat);
    if (S.status == LZ_RUNNING) scalar_after_beta(S, bb, tr_beta);
    *st = S;
  }
}

}  // namespace

struct PlainWork {
  int32_t n = 0;
  void *U[3] = {nullptr, nullptr, nullptr};  // n doubles each (room for either precision)
  double *part = nullptr;
  int32_t npart = 0;
  LzState *st = nullptr;
  LzState *st_host = nullptr;  // pinned
  int upd_blocks = 0;
  int last_k = 8;  // iterations of the previous query: first chunk size
};

void plain_free(rd_graph g) {
  PlainWork *pw = g->plain;
  if (!pw) return;
  for (void *u : pw->U) dev_free(u);
  dev_free(pw->part);
  dev_free(pw->st);
  if (pw->st_host) (void)hipHostFree(pw->st_host);
  delete pw;
  g->plain = nullptr;
}

static PlainWork *plain_get(rd_graph g) {
  if (g->plain) return g->plain;
  PlainWork *pw = new PlainWork();
  try {
    pw->n = g->n;
    pw->U[0] = dev_alloc((size_t)g->n * sizeof(double));
    pw->U[1] = dev_alloc((size_t)g->n * sizeof(double));
    pw->U[2] = dev_alloc((size_t)g->n * sizeof(double));
    int dev_cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) dev_cus = prop.multiProcessorCount;
    pw->upd_blocks = std::max(1, std::min<int>((g->n + UPD_THREADS * 4 - 1) / (UPD_THREADS * 4),
                                               dev_cus * 8));
    pw->npart = std::max(g->nblk, 4 * pw->upd_blocks);  // four slabs for the re-orthogonalisation
    pw->part = (double *)dev_alloc((size_t)pw->npart * sizeof(double));
    pw->st = (LzState *)dev_alloc(sizeof(LzState));
    RD_HIP(hipHostMalloc((void **)&pw->st_host, sizeof(LzState), hipHostMallocDefault));
  } catch (...) {
    g->plain = pw;
    plain_free(g);
    throw;
  }
  g->plain = pw;
  return pw;
}

template <typename VT, int RO>
static void enqueue_update(rd_graph g, PlainWork *pw, const VT *Ucur, const VT *Uprev, VT *Y,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_update<VT, RO>), dim3(pw->upd_blocks), dim3(UPD_THREADS), 0, st, g->n, g->deg,
                     Ucur, Uprev, Y, pw->part, pw->st);
  if constexpr (RO > 0) {
    hipLaunchKernelGGL(k_reorth_coef<RO>, dim3(1), dim3(RED_THREADS), 0, st, pw->part, pw->upd_blocks,
                       g->vol, pw->st);
    hipLaunchKernelGGL((k_reorth_apply<VT, RO>), dim3(pw->upd_blocks), dim3(UPD_THREADS), 0, st, g->n,
                       g->deg, Ucur, Uprev, Y, pw->part, pw->st);
  }
}

// One dense iteration: product of U[cur] (q_i) with U[prv] (q_{i-1}) into U[nxt].
template <typename VT>
static void enqueue_iteration(rd_graph g, PlainWork *pw, int cur, int prv, int nxt, int reorth,
                              hipStream_t st, double *tr_alpha, double *tr_beta, double *tr_rhat,
                              bool prof) {
  const VT *Ucur = (const VT *)pw->U[cur];
  const VT *Uprev = (const VT *)pw->U[prv];
  VT *Y = (VT *)pw->U[nxt];
  std::pair<hipEvent_t, hipEvent_t> ev{};
  if (prof) {
    const double sv = sizeof(VT);
    ev = g->timer[1].next((double)g->nnz * (4.0 + (g->unit ? 0.0 : sv)) + 4.0 * (g->n + 1) +
                          3.0 * sv * g->n + (sv + 8.0) * g->n);
    RD_HIP(hipEventRecord(ev.first, st));
  }
  if (g->unit)
    hipLaunchKernelGGL((k_spmv<VT, false>), dim3(g->nblk), dim3(SPMV_THREADS), 0, st, g->blk_row,
                       g->blk_lanes, g->row_ptr, g->col, (const VT *)nullptr,
                       VecTraits<VT>::invdeg(g), g->deg, Ucur, Uprev, Y, pw->part, pw->st);
  else
    hipLaunchKernelGGL((k_spmv<VT, true>), dim3(g->nblk), dim3(SPMV_THREADS), 0, st, g->blk_row,
                       g->blk_lanes, g->row_ptr, g->col, VecTraits<VT>::w(g),
                       VecTraits<VT>::invdeg(g), g->deg, Ucur, Uprev, Y, pw->part, pw->st);
  if (prof) RD_HIP(hipEventRecord(ev.second, st));
  hipLaunchKernelGGL(k_reduce_alpha, dim3(1), dim3(RED_THREADS), 0, st, pw->part, g->nblk, pw->st,
                     tr_alpha, tr_rhat);
  if (reorth == 0) enqueue_update<VT, 0>(g, pw, Ucur, Uprev, Y, st);
  else if (reorth == 1) enqueue_update<VT, 1>(g, pw, Ucur, Uprev, Y, st);
  else enqueue_update<VT, 2>(g, pw, Ucur, Uprev, Y, st);
  hipLaunchKernelGGL(k_reduce_beta, dim3(1), dim3(RED_THREADS), 0, st, pw->part, pw->upd_blocks,
                     pw->st, tr_beta);
}

template <typename VT>
static void plain_run_t(rd_graph g, int32_t s, int32_t t, double eps, const rd_options &o,
                        hipStream_t st, rd_result *out, double *tr_alpha, double *tr_beta,
                        double *tr_rhat) {
  PlainWork *pw = plain_get(g);
  hipLaunchKernelGGL(k_init<VT>, dim3((g->n + 255) / 256), dim3(256), 0, st, g->n, (VT *)pw->U[0],
                     (VT *)pw->U[1], (VT *)pw->U[2], g->deg, s, t, eps, o.max_iters, o.fixed_k, o.delay,
                     o.err_mode, pw->st);
  hipLaunchKernelGGL(k_first<VT>, dim3(1), dim3(256), 0, st, g->row_ptr, g->col,
                     (const double *)g->w64, g->deg, (VT *)pw->U[1], pw->st, tr_alpha, tr_beta, tr_rhat);
  RD_HIP(hipGetLastError());
  const int cap = o.fixed_k > 0 ? o.fixed_k : o.max_iters;
  // iteration 1 is done; the dense iterations start from U[1] (w_1) and U[0] (q_1)
  int done_iters = 1, prv = 0, cur = 1, nxt = 2;
  // the second iteration from the support of q_2 (not with re-orthogonalisation
  // or a trace, which records every iteration's scalars): then the dense
  // iterations start from U[2] (w_2) and U[1] (w_1)
  if (o.reorth == 0 && !tr_alpha && !(o.flags & RD_NO_SPARSE2) && cap >= 2 &&
      sparse_second_single(g, sizeof(VT) == 8 ? RD_F64 : RD_F32, pw->U[1], pw->U[2], pw->st, st)) {
    RD_HIP(hipMemcpyAsync(pw->st_host, pw->st, sizeof(LzState), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    if (pw->st_host->k == 2) {
      done_iters = 2;
      prv = 1;
      cur = 2;
      nxt = 0;
    }
  }
  const int sparse_iters = done_iters;
  // iterations enqueued between two looks at the state: first what the
  // previous query needed (a launch after the stop still dispatches every
  // workgroup of the product before returning, about 0.3 ms on a 4M-node
  // graph), then 2, then doubling for long runs
  int chunk = o.fixed_k > 0 ? o.fixed_k - done_iters : std::max(1, std::min(pw->last_k, 64) - done_iters);
  bool first_chunk = true;
  for (;;) {
    const int todo = std::min(chunk, cap - done_iters);
    for (int j = 0; j < todo; ++j) {
      enqueue_iteration<VT>(g, pw, cur, prv, nxt, o.reorth, st, tr_alpha, tr_beta, tr_rhat,
                            o.flags & RD_PROFILE);
      const int old_prv = prv;
      prv = cur;
      cur = nxt;
      nxt = old_prv;
    }
    RD_HIP(hipGetLastError());
    done_iters += todo;
    RD_HIP(hipMemcpyAsync(pw->st_host, pw->st, sizeof(LzState), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    if (pw->st_host->status != LZ_RUNNING || done_iters >= cap) break;
    chunk = first_chunk ? 2 : std::min(2 * chunk, 256);
    first_chunk = false;
  }
  const LzState &S = *pw->st_host;
  // launches after the stopping iteration returned at once: the dense
  // products of iterations sparse_iters + 1 .. k did work
  if (o.flags & RD_PROFILE) g->timer[1].resolve((size_t)std::max(0, S.k - sparse_iters));
  int32_t status = S.status;
  if (status == LZ_RUNNING) status = LZ_NOT_CONVERGED;  // cap reached while still running
  out->r = S.rhat;
  out->err_est = S.err_est;
  out->iters = S.k;
  out->status = status_of(status);
  pw->last_k = std::max(2, S.k);
}

void plain_run(rd_graph g, int32_t s, int32_t t, double eps, const rd_options &o, hipStream_t st,
               rd_result *out, double *tr_alpha, double *tr_beta, double *tr_rhat, int32_t) {
  if (small_eligible(g, o)) {
    // both vectors fit in LDS: one workgroup runs the whole iteration
    PlainWork *pw = plain_get(g);
    rd_result *dres = reinterpret_cast<rd_result *>(pw->st);
    small_run(g, 1, nullptr, nullptr, s, t, eps, o, st, dres, tr_alpha, tr_beta, tr_rhat);
    rd_result *hres = reinterpret_cast<rd_result *>(pw->st_host);
    RD_HIP(hipMemcpyAsync(hres, dres, sizeof(rd_result), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    *out = *hres;
    return;
  }
  if (o.precision == RD_F64)
    plain_run_t<double>(g, s, t, eps, o, st, out, tr_alpha, tr_beta, tr_rhat);
  else
    plain_run_t<float>(g, s, t, eps, o, st, out, tr_alpha, tr_beta, tr_rhat);
}

extern "C" {

rd_status rd_query(rd_graph g, int32_t s, int32_t t, double eps, const rd_options *o,
                   rd_result *out) {
  if (!g || !out) return RD_E_ARG;
  try {
    g->err.clear();
    rd_options opt = resolve_options(g, o);
    RD_REQUIRE(s >= 0 && s < g->n && t >= 0 && t < g->n, "s and t must be in [0, n)");
    RD_REQUIRE(opt.fixed_k > 0 || eps > 0.0, "eps must be > 0 unless fixed_k is set");
    if (s == t) {
      *out = rd_result{0.0, 0.0, 0, RD_OK};
      return RD_OK;
    }
    RD_HIP(hipSetDevice(g->device));
    if (g->perm) {
      s = g->perm_host[s];
      t = g->perm_host[t];
    }
    plain_run(g, s, t, eps, opt, pick_stream(g, o), out, nullptr, nullptr, nullptr, 0);
    return RD_OK;
  } catch (const RdError &e) {
    g->err = e.msg;
    return e.code;
  }
}

rd_status rd_query_trace(rd_graph g, int32_t s, int32_t t, int32_t k, const rd_options *o,
                         double *alpha, double *beta, double *rhat, int32_t *iters) {
  if (!g || !alpha || !beta || !rhat || !iters || k < 1) return RD_E_ARG;
  double *dtr = nullptr;
  try {
    g->err.clear();
    rd_options opt = resolve_options(g, o);
    RD_REQUIRE(s >= 0 && s < g->n && t >= 0 && t < g->n && s != t, "need s != t in [0, n)");
    opt.fixed_k = k;
    RD_HIP(hipSetDevice(g->device));
    if (g->perm) {
      s = g->perm_host[s];
      t = g->perm_host[t];
    }
    hipStream_t st = pick_stream(g, o);
    dtr = (double *)dev_alloc(3 * (size_t)k * sizeof(double));
    RD_HIP(hipMemsetAsync(dtr, 0, 3 * (size_t)k * sizeof(double), st));
    rd_result res;
    plain_run(g, s, t, 1.0, opt, st, &res, dtr, dtr + k, dtr + 2 * k, k);
    std::vector<double> h(3 * (size_t)k);
    RD_HIP(hipMemcpyAsync(h.data(), dtr, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    std::copy(h.begin(), h.begin() + k, alpha);
    std::copy(h.begin() + k, h.begin() + 2 * k, beta);
    std::copy(h.begin() + 2 * k, h.end(), rhat);
    *iters = res.iters;
    dev_free(dtr);
    return RD_OK;
  } catch (const RdError &e) {
    dev_free(dtr);
    g->err = e.msg;
    return e.code;
  }
}

}  // extern "C"

// The smallest and largest eigenvalues of the symmetric tridiagonal matrix
// with diagonal a[0..k) and off-diagonal b[0..k-1) (b[j] couples rows j and
// j+1): bisection on the Sturm count, the number of negative pivots of the
// LDL^T factorisation of T - x I, which equals the number of eigenvalues
// below x.
static int32_t sturm_below(const double *a, const double *b, int32_t k, double x) {
  int32_t neg = 0;
  double d = 1.0;
  for (int32_t j = 0; j < k; ++j) {
    d = a[j] - x - (j ? b[j - 1] * b[j - 1] / d : 0.0);
    if (d == 0.0) d = -1e-300;  // a zero pivot counts as an eigenvalue at x
    if (d < 0.0) ++neg;
  }
  return neg;
}

static double tridiag_eig(const double *a, const double *b, int32_t k, int32_t idx, double lo, double hi) {
  // the idx-th smallest eigenvalue (0-based) in [lo, hi]
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(lo) + std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b, k, mid) > idx) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

extern "C" rd_status rd_ritz_bounds(rd_graph g, int32_t s, int32_t t, int32_t k, const rd_options *o,
                                    double *theta_min, double *theta_max, int32_t *iters) {
  if (!g || !theta_min || !theta_max || !iters || k < 1) return RD_E_ARG;
  rd_options o2;
  try {
    o2 = resolve_options(g, o);
  } catch (const RdError &e) {
    g->err = e.msg;
    return e.code;
  }
  // without deflation, rounding brings back the direction D^{1/2} 1 of
  // eigenvalue 1 in long runs and the top Ritz value drifts to 1
  o2.reorth = std::max(o2.reorth, 1);
  o2.max_iters = 0;
  o2.fixed_k = 0;
  std::vector<double> a(k), b(k), r(k);
  const rd_status rc = rd_query_trace(g, s, t, k, &o2, a.data(), b.data(), r.data(), iters);
  if (rc != RD_OK) return rc;
  const int32_t kk = *iters;
  // Gershgorin interval of T_k
  double lo = 1e300, hi = -1e300;
  for (int32_t j = 0; j < kk; ++j) {
    const double rad = (j ? std::fabs(b[j - 1]) : 0.0) + (j + 1 < kk ? std::fabs(b[j]) : 0.0);
    lo = std::min(lo, a[j] - rad);
    hi = std::max(hi, a[j] + rad);
  }
  *theta_min = tridiag_eig(a.data(), b.data(), kk, 0, lo, hi);
  *theta_max = tridiag_eig(a.data(), b.data(), kk, kk - 1, lo, hi);
  return RD_OK;
}
