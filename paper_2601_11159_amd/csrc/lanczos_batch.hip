// Batched Lanczos iteration: many (s,t) pairs advanced together.
//
// B independent runs of Algorithm 3 share one pass over the graph per
// iteration. The vectors of all runs form n x B row-major blocks (column j =
// slot j), so the sparse product reads each neighbour row X[v, 0:B] as one
// contiguous segment (B FP32 values = B*4 bytes) instead of B scattered words.
// The runs are independent (no coupling between columns); each column keeps its
// own FP64 scalars, tridiagonal solve and stopping test. A column whose run
// stops is retired and refilled with the next pending pair in the same
// iteration, so slots stay busy while pairs of uneven length stream through.
//
// Vectors use the degree-scaled basis q = D^{-1/2} v and scale-on-read
// normalisation as in the single-pair path (see lanczos_plain.hip).
//
// One iteration:
//   k_spmm_short / k_spmm_long   Y = sig D^{-1} W U_cur - pc U_prev (+ per-block <Y, q>_D per column)
//   k_col_sum                    alpha_j for every column
//   k_control                    scalar update, stopping test, retire + refill (one block, fixed order)
//   k_update                     W = Y - alpha sig U_cur, or the start vector of a refilled column
//   k_col_sum + k_beta           beta_{j, i+1} and next scales

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "lanczos_common.h"

namespace {

constexpr int SHORT_THREADS = 256;
constexpr int LONG_THREADS = 1024;
// default row-bin schedule (the autotuner may choose another per graph)
constexpr int LONG_DEG = 1024;   // rows longer than this go to the split-row kernel
constexpr int WAVE_NNZ = 256;    // adjacency entries per wave work item (short rows)
constexpr int COL_THREADS = 256;

// COL_FINAL: the run stopped at this iteration; only the potential is updated
// (gradient mode), then the column is idle.
// Gradient mode with refill ("harvest"): a finished column's potential is
// copied into slot hslot of the block of finished potentials (COL_FINAL with
// hslot >= 0, or COL_HARVEST for a potential already complete); COL_PENDING
// waits for a free slot. The slot is refilled after its potential is copied.
// COL_FINAL_REFILL / COL_HARVEST_REFILL: the same, and in the same update the
// column starts the next pair (its potential columns are zeroed after the copy).
enum : int32_t {
  COL_RUN = 0,
  COL_REFILL = 1,
  COL_IDLE = 2,
  COL_FINAL = 3,
  COL_HARVEST = 4,
  COL_PENDING = 5,
  COL_FINAL_REFILL = 6,
  COL_HARVEST_REFILL = 7
};

__device__ __forceinline__ bool starts_pair(int32_t mode) {
  return mode == COL_REFILL || mode == COL_FINAL_REFILL || mode == COL_HARVEST_REFILL;
}

// gradient handling of a batched run
enum : int32_t { GRAD_NONE = 0, GRAD_HARVEST = 2 };

struct ColCtrl {
  double sig;   // q = sig * U_cur[:, j]
  double pc;    // coefficient of U_prev[:, j] (0: the previous vector is not used)
  double coef;  // alpha * sig for the update
  double vs;    // start vector entries of a refilled column at rows s and t
  double vt;
  double pa;    // gradient mode: p_i = q_i + pa p_{i-1}
  double xb;    //                x_i = x_{i-1} + xb p_i
  double ro_mu;  // re-orthogonalisation: W -= ro_mu + ro_c U_cur + ro_p U_prev
  double ro_c;
  double ro_p;
  int32_t mode;  // COL_*
  int32_t s, t;
  int32_t prev_sparse;  // the previous vector is q_1 (vs at s, vt at t, zero elsewhere)
  int32_t upd_sparse;   // the same, for the update of the current iteration
  int32_t hslot;        // harvest slot of the finished potential (-1: none)
  int32_t plist;        // 1 + list id: the previous vector is q_2 of a sparse second
                        // iteration, held in that list (the product reads zeros for it)
};

template <typename VT, int N>
struct alignas(sizeof(VT) * N) VecN {
  VT v[N];
};

template <typename VT, int N>
__device__ __forceinline__ VecN<VT, N> vload(const VT *p) {
  return *reinterpret_cast<const VecN<VT, N> *>(p);
}
template <typename VT, int N>
__device__ __forceinline__ void vstore(VT *p, const VecN<VT, N> &x) {
  *reinterpret_cast<VecN<VT, N> *>(p) = x;
}
// the same with the non-temporal hint (streams read or written once)
template <typename VT, int N>
__device__ __forceinline__ VecN<VT, N> vload_nt(const VT *p) {
  VecN<VT, N> r;
  if constexpr (N == 1) {
    r.v[0] = __builtin_nontemporal_load(p);
  } else {
    typedef VT E __attribute__((ext_vector_type(N)));
    const E e = __builtin_nontemporal_load(reinterpret_cast<const E *>(p));
#pragma unroll
    for (int i = 0; i < N; ++i) r.v[i] = e[i];
  }
  return r;
}
template <typename VT, int N>
__device__ __forceinline__ void vstore_nt(VT *p, const VecN<VT, N> &x) {
  if constexpr (N == 1) {
    __builtin_nontemporal_store(x.v[0], p);
  } else {
    typedef VT E __attribute__((ext_vector_type(N)));
    E e;
#pragma unroll
    for (int i = 0; i < N; ++i) e[i] = x.v[i];
    __builtin_nontemporal_store(e, reinterpret_cast<E *>(p));
  }
}
// loads of stored values widened to FP64, stores of FP64 values rounded once
template <typename T, int N>
__device__ __forceinline__ VecN<double, N> vload_f64(const T *p) {
  const VecN<T, N> x = vload<T, N>(p);
  VecN<double, N> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.v[i] = (double)x.v[i];
  return r;
}
template <typename T, int N>
__device__ __forceinline__ void vstore_from_f64(T *p, const VecN<double, N> &x) {
  VecN<T, N> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.v[i] = (T)x.v[i];
  vstore<T, N>(p, r);
}

template <int B>
struct Shape {
  static constexpr int VEC = B >= 64 ? B / 64 : 1;  // columns per lane
  static constexpr int LPR = B / VEC;               // lanes per row
  static constexpr int RPW = 64 / LPR;              // rows per wavefront
};

// Fold the per-lane column partials of all rows handled by a block into
// part[j * ldp + slot] (fixed order: sub-rows of a wave, then waves). Ends with
// a barrier, so `sm` may be reused by a following call.
template <int B, int VEC>
__device__ __forceinline__ void block_column_partials(double (&apart)[VEC], double *sm, double *part,
                                                      int32_t ldp, int32_t slot) {
  using S = Shape<B>;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int v = 0; v < VEC; ++v)
    for (int off = S::LPR; off < 64; off <<= 1) apart[v] += __shfl_xor(apart[v], off, 64);
  if (lane < S::LPR) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) sm[wid * B + lane * VEC + v] = apart[v];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < B; j += blockDim.x) {
    double a = 0.0;
    for (int w = 0; w < nw; ++w) a += sm[w * B + j];
    part[(size_t)j * ldp + slot] = a;
  }
  __syncthreads();
}

// Rows of length <= long_deg. Wave work items are contiguous row ranges of
// bounded adjacency length; items are dealt to wavefronts round-robin (a fixed
// assignment, so the partial sums do not depend on timing).
template <typename VT, int B, bool WEIGHTED>
__global__ __launch_bounds__(SHORT_THREADS) void k_spmm_short(
    int32_t nwi, const int32_t *__restrict__ witem_row, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col, const VT *__restrict__ w, const VT *__restrict__ invdeg,
    const double *__restrict__ deg, const VT *__restrict__ Ucur, const VT *__restrict__ Uprev,
    VT *__restrict__ Y, const ColCtrl *__restrict__ ctrl, double *__restrict__ part, int32_t ldp,
    const int32_t *__restrict__ active, int32_t long_deg) {
  if (*active == 0) return;
  using S = Shape<B>;
  constexpr int VEC = S::VEC;
  using V = VecN<VT, VEC>;
  // lanes holding at most 4 bytes of a row: registers to spare for a wider
  // gather front (measured: -12% per launch at FP32 width 64, +3% in FP64)
  constexpr bool NARROW = sizeof(VT) * VEC <= 4;
  // gathers in flight per lane: 8, or 4 for 32-byte lanes (FP64 at width 256),
  // where 8 needs 138 VGPRs (3 waves per SIMD) and 4 fits in 106 (4 waves);
  // measured 8% faster per launch on a road-like graph
  constexpr int UNR = sizeof(VT) * VEC >= 32 ? 4 : 8;
  __shared__ double sm[(SHORT_THREADS / 64) * B];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int sub = lane / S::LPR, c0 = (lane % S::LPR) * VEC;
  VT sig[VEC], pc[VEC], pvs[VEC], pvt[VEC];
  int32_t pss[VEC], pst[VEC];
  bool hp[VEC], psp[VEC];
  double apart[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const ColCtrl &cc = ctrl[c0 + v];
    sig[v] = (VT)cc.sig;
    pc[v] = (VT)cc.pc;
    hp[v] = cc.pc != 0.0;
    psp[v] = cc.prev_sparse != 0;
    pss[v] = cc.s;
    pst[v] = cc.t;
    pvs[v] = (VT)cc.vs;
    pvt[v] = (VT)cc.vt;
    apart[v] = 0.0;
  }
  const int gw = blockIdx.x * (SHORT_THREADS / 64) + wid;
  const int nwv = gridDim.x * (SHORT_THREADS / 64);
  for (int32_t it = gw; it < nwi; it += nwv) {
    const int32_t rb = witem_row[2 * it], re = witem_row[2 * it + 1];
    for (int32_t r = rb + sub; r < re; r += S::RPW) {
      const int32_t pb = row_ptr[r], pe = row_ptr[r + 1];
      if (pe - pb > long_deg) continue;
      // the row's own operands, loaded ahead of the gathers (narrow lanes only:
      // wider ones lose more to occupancy than they gain)
      V up, uc;
      if constexpr (NARROW) {
        up = vload<VT, VEC>(Uprev + (size_t)r * B + c0);
        uc = vload<VT, VEC>(Ucur + (size_t)r * B + c0);
      }
      VT acc[VEC];
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] = 0;
      int32_t p = pb;
      for (; p + UNR <= pe; p += UNR) {
        int32_t ci[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) ci[k] = col[p + k];
        V x[UNR];
#pragma unroll
        for (int k = 0; k < UNR; ++k) x[k] = vload<VT, VEC>(Ucur + (size_t)ci[k] * B + c0);
#pragma unroll
        for (int k = 0; k < UNR; ++k) {
          const VT wk = WEIGHTED ? w[p + k] : VT(1);
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[v] += WEIGHTED ? wk * x[k].v[v] : x[k].v[v];
        }
      }
      // the last (fewer than UNR) entries - all of a row on low-degree graphs:
      // every index load, then every gather, in flight together
      const int rem = pe - p;
      if (!NARROW) {
        for (; p < pe; ++p) {
          const V x = vload<VT, VEC>(Ucur + (size_t)col[p] * B + c0);
          const VT wk = WEIGHTED ? w[p] : VT(1);
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[v] += WEIGHTED ? wk * x.v[v] : x.v[v];
        }
      } else if (rem > 0) {
        int32_t ci[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) ci[k] = k < rem ? col[p + k] : 0;
        V x[7];
#pragma unroll
        for (int k = 0; k < 7; ++k)
          if (k < rem) x[k] = vload<VT, VEC>(Ucur + (size_t)ci[k] * B + c0);
#pragma unroll
        for (int k = 0; k < 7; ++k) {
          if (k < rem) {
            const VT wk = WEIGHTED ? w[p + k] : VT(1);
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[v] += WEIGHTED ? wk * x[k].v[v] : x[k].v[v];
          }
        }
      }
      const VT id = invdeg[r];
      const double dr = deg[r];
      if constexpr (!NARROW) {
        up = vload<VT, VEC>(Uprev + (size_t)r * B + c0);
        uc = vload<VT, VEC>(Ucur + (size_t)r * B + c0);
      }
      V y;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        VT yy = sig[v] * acc[v] * id;
        if (hp[v]) {
          const VT prev = psp[v] ? (r == pss[v] ? pvs[v] : (r == pst[v] ? pvt[v] : VT(0))) : up.v[v];
          yy -= pc[v] * prev;
        }
        y.v[v] = yy;
        apart[v] += dr * (double)yy * ((double)sig[v] * (double)uc.v[v]);
      }
      vstore<VT, VEC>(Y + (size_t)r * B + c0, y);
    }
  }
  block_column_partials<B, VEC>(apart, sm, part, ldp, blockIdx.x);
}

// Rows longer than long_deg: one block per row, entries split over all
// sub-rows of the block and combined in LDS in a fixed order.
template <typename VT, int B, bool WEIGHTED>
__global__ __launch_bounds__(LONG_THREADS) void k_spmm_long(
    const int32_t *__restrict__ long_rows, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col, const VT *__restrict__ w, const VT *__restrict__ invdeg,
    const double *__restrict__ deg, const VT *__restrict__ Ucur, const VT *__restrict__ Uprev,
    VT *__restrict__ Y, const ColCtrl *__restrict__ ctrl, double *__restrict__ part, int32_t ldp,
    int32_t poff, const int32_t *__restrict__ active) {
  if (*active == 0) return;
  using S = Shape<B>;
  constexpr int VEC = S::VEC;
  constexpr int NG = (LONG_THREADS / 64) * S::RPW;  // sub-rows per block
  using V = VecN<VT, VEC>;
  __shared__ VT acc_sm[NG * B];
  __shared__ double sm[(LONG_THREADS / 64) * B];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int sub = lane / S::LPR, c0 = (lane % S::LPR) * VEC;
  const int g = wid * S::RPW + sub;
  const int32_t r = long_rows[blockIdx.x];
  const int32_t pb = row_ptr[r], pe = row_ptr[r + 1];
  VT acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0;
  // UNR gathers in flight per lane (as in k_spmm_short), and the column ids of
  // the next UNR entries loaded while those gathers run: a hub row's sub-row
  // walks hundreds of entries, so its dependent loads set the launch's length
  constexpr int UNR = sizeof(VT) * VEC >= 32 ? 4 : 8;
  int32_t p = pb + g;
  int32_t ci[UNR];
  if (p + (UNR - 1) * NG < pe) {
#pragma unroll
    for (int k = 0; k < UNR; ++k) ci[k] = col[p + k * NG];
  }
  for (; p + (UNR - 1) * NG < pe; p += UNR * NG) {
    V x[UNR];
#pragma unroll
    for (int k = 0; k < UNR; ++k) x[k] = vload<VT, VEC>(Ucur + (size_t)ci[k] * B + c0);
    const int32_t pn = p + UNR * NG;
    if (pn + (UNR - 1) * NG < pe) {
#pragma unroll
      for (int k = 0; k < UNR; ++k) ci[k] = col[pn + k * NG];
    }
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      const VT wk = WEIGHTED ? w[p + k * NG] : VT(1);
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[v] += WEIGHTED ? wk * x[k].v[v] : x[k].v[v];
    }
  }
  for (; p < pe; p += NG) {
    const V x = vload<VT, VEC>(Ucur + (size_t)col[p] * B + c0);
    const VT wk = WEIGHTED ? w[p] : VT(1);
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += WEIGHTED ? wk * x.v[v] : x.v[v];
  }
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc_sm[g * B + c0 + v] = acc[v];
  __syncthreads();
  double apart[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) apart[v] = 0.0;
  if (g == 0) {
    VT tot[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      tot[v] = 0;
      for (int h = 0; h < NG; ++h) tot[v] += acc_sm[h * B + c0 + v];
    }
    const VT id = invdeg[r];
    const double dr = deg[r];
    const V up = vload<VT, VEC>(Uprev + (size_t)r * B + c0);
    const V uc = vload<VT, VEC>(Ucur + (size_t)r * B + c0);
    V y;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const ColCtrl &cc = ctrl[c0 + v];
      const VT sg = (VT)cc.sig;
      const double pcd = cc.pc;
      VT yy = sg * tot[v] * id;
      if (pcd != 0.0) {
        const VT prev =
            cc.prev_sparse ? (r == cc.s ? (VT)cc.vs : (r == cc.t ? (VT)cc.vt : VT(0))) : up.v[v];
        yy -= (VT)pcd * prev;
      }
      y.v[v] = yy;
      apart[v] = dr * (double)yy * ((double)sg * (double)uc.v[v]);
    }
    vstore<VT, VEC>(Y + (size_t)r * B + c0, y);
  }
  block_column_partials<B, VEC>(apart, sm, part, ldp, poff + blockIdx.x);
}

// out[j] = sum_k part[j * ldp + k], k < np (block j, fixed order).
__global__ __launch_bounds__(COL_THREADS) void k_col_sum(const double *__restrict__ part, int32_t ldp,
                                                         int32_t np, double *__restrict__ out,
                                                         const int32_t *__restrict__ active) {
  if (*active == 0) return;
  __shared__ double sm[COL_THREADS / 64];
  const double *p = part + (size_t)blockIdx.x * ldp;
  double a = 0.0;
  for (int k = threadIdx.x; k < np; k += COL_THREADS) a += p[k];
  a = block_sum(a, sm);
  if (threadIdx.x == 0) out[blockIdx.x] = a;
}

struct RunParams {
  double tol;
  int32_t max_iters, fixed_k, delay, err_mode;
  int32_t npairs;
  int32_t reorth;
  int32_t gmode;          // GRAD_NONE or GRAD_HARVEST
  const double *grad_r;   // harvest mode: weight of each pair (nullptr: ones)
  int32_t s2;             // sparse second iterations on
  int64_t s2_ecap;        // at most this many scatter entries per column
  int32_t *slot_pair = nullptr;  // harvest mode for potentials and energies: pair of each slot
  double *phi = nullptr;         // the potentials' destination [npairs][n], or nullptr
  int32_t refine = 0;            // 1: r of each pair as the FP64 energy of its potential
};

__device__ __forceinline__ void write_result(rd_result *out, const LzState &S) {
  rd_result r;
  r.r = S.rhat;
  r.err_est = S.err_est;
  r.iters = S.k;
  r.status = (int32_t)status_of(S.status);
  out[S.pair] = r;
}

// Scalar step for every column after alpha, then retirement and refill in
// column order (one block; thread 0 pops the pair queue and hands out harvest
// slots serially, so the assignment of pairs and slots is deterministic).
// grad: GRAD_NONE or GRAD_HARVEST (a stopped run adds its last
// term and its potential is copied to a harvest slot, with weight
// cw[slot] = grad_r[pair] * c, before the column is refilled).
__global__ __launch_bounds__(256) void k_control(int32_t B, LzState *__restrict__ st,
                                                 ColCtrl *__restrict__ ctrl,
                                                 const double *__restrict__ alpha, RunParams prm,
                                                 const int32_t *__restrict__ ps,
                                                 const int32_t *__restrict__ pt,
                                                 const double *__restrict__ deg,
                                                 rd_result *__restrict__ out,
                                                 int32_t *__restrict__ qstate, int32_t grad,
                                                 const double *__restrict__ grad_r, double *__restrict__ cw) {
  // qstate: [0] next pair, [1] active columns, [2] iterations with work, [3] constant 1,
  // [4] harvest slots in use.
  // Every call but the first (which fills the slots) returns once no column is active.
  if (qstate[1] == 0 && qstate[2] > 0) return;
  __shared__ int32_t need[256];
  __shared__ int32_t wants[256];
  __shared__ int32_t newpair[256];
  __shared__ int32_t slot[256];
  const int j = threadIdx.x;
  const bool harvest = grad == GRAD_HARVEST;
  LzState S;
  double pa = 0.0, xb = 0.0;
  bool advanced = false, fin = false, pending = false;
  if (j < B) {
    S = st[j];
    const ColCtrl &pc = ctrl[j];
    // harvest mode: a finished potential still waiting for a slot
    pending = harvest && (pc.mode == COL_PENDING || (pc.mode == COL_FINAL && pc.hslot < 0));
    const bool was_running = S.status == LZ_RUNNING;
    const double delta_prev = S.delta, beta_i = S.beta;
    const int32_t k_prev = S.k;
    if (was_running) scalar_after_alpha(S, alpha[j], nullptr, nullptr);
    // coefficients of the potential recurrence for iteration i = S.k: with
    // I - T_i = L D L^T (unit lower bidiagonal L, subdiagonal -beta_i/delta_{i-1}),
    // x_i = Q_i (I - T_i)^{-1} e_1 = x_{i-1} + (omega_i/delta_i) p_i and
    // p_i = q_i + (beta_i/delta_{i-1}) p_{i-1}
    advanced = was_running && S.k == k_prev + 1;
    if (advanced) {
      pa = S.k > 1 ? beta_i / delta_prev : 0.0;
      xb = S.omega / S.delta;
    }
    fin = S.status == LZ_DONE || S.status == LZ_NOT_CONVERGED || S.status == LZ_BREAKDOWN;
    if (fin) write_result(out, S);
    if (harvest) {
      wants[j] = (fin || pending) ? 1 : 0;
      need[j] = (!fin && !pending && S.status == LZ_IDLE) ? 1 : 0;
    } else {
      wants[j] = 0;
      need[j] = (fin || S.status == LZ_IDLE) ? 1 : 0;
    }
  }
  __syncthreads();
  if (j == 0) {
    int32_t head = qstate[0];
    int32_t used = qstate[4];
    for (int c = 0; c < B; ++c) {
      slot[c] = -1;
      if (wants[c] && used < B) slot[c] = used++;
      newpair[c] = -2;
      // a finished column whose potential gets a slot now starts the next pair at once
      if (!need[c] && !(wants[c] && slot[c] >= 0)) continue;
      int32_t idx = -1;
      while (head < prm.npairs) {
        const int32_t cand = head++;
        if (ps[cand] == pt[cand]) {
          out[cand] = rd_result{0.0, 0.0, 0, RD_OK};
          continue;
        }
        idx = cand;
        break;
      }
      newpair[c] = idx;
    }
    qstate[0] = head;
    qstate[4] = used;
  }
  __syncthreads();
  int32_t active = 0;
  if (j < B) {
    ColCtrl cc = ctrl[j];
    const int32_t np = newpair[j];
    if (harvest && (fin || pending)) {
      // finished: last potential term (if this iteration added one), then the
      // copy to a harvest slot, or wait for one; with a slot and a pair left,
      // the next pair starts in the same update (cc.sig keeps the finished
      // run's scale for its last term; k_first_batch sets the new one)
      const bool final_term = fin && advanced && S.status != LZ_BREAKDOWN;
      const int32_t sl = slot[j];
      if (sl >= 0) {
        cw[sl] = (grad_r ? grad_r[S.pair] : 1.0) * S.c;
        if (prm.slot_pair) prm.slot_pair[sl] = S.pair;
      }
      cc.hslot = sl;
      cc.pa = pa;
      cc.xb = xb;
      cc.pc = 0.0;
      cc.coef = 0.0;
      cc.upd_sparse = 0;
      if (sl >= 0 && np >= 0) {
        const int32_t s = ps[np], t = pt[np];
        const double c = 1.0 / deg[s] + 1.0 / deg[t];
        state_start(S, s, t, c, prm.tol, prm.max_iters, prm.fixed_k, prm.delay, prm.err_mode, np);
        const double rc = 1.0 / sqrt(c);
        cc.mode = final_term ? COL_FINAL_REFILL : COL_HARVEST_REFILL;
        cc.vs = rc / deg[s];
        cc.vt = -rc / deg[t];
        cc.prev_sparse = 0;
        cc.s = s;
        cc.t = t;
      } else {
        S.status = LZ_IDLE;
        cc.mode = final_term ? COL_FINAL : (sl >= 0 ? COL_HARVEST : COL_PENDING);
      }
      active = 1;
    } else if (np >= 0) {
      const int32_t s = ps[np], t = pt[np];
      const double c = 1.0 / deg[s] + 1.0 / deg[t];
      state_start(S, s, t, c, prm.tol, prm.max_iters, prm.fixed_k, prm.delay, prm.err_mode, np);
      const double rc = 1.0 / sqrt(c);
      cc.mode = COL_REFILL;
      cc.sig = 1.0;
      cc.pc = 0.0;
      cc.coef = 0.0;
      cc.vs = rc / deg[s];
      cc.vt = -rc / deg[t];
      cc.prev_sparse = 0;
      cc.upd_sparse = 0;
      cc.hslot = -1;
      cc.s = s;
      cc.t = t;
      active = 1;
    } else if (np == -1) {
      // no pair left (without harvest: the finished potential is not kept);
      // the column is idle afterwards
      S.status = LZ_IDLE;
      cc.mode = COL_IDLE;
      cc.hslot = -1;
      cc.pa = pa;
      cc.xb = xb;
      cc.pc = 0.0;
      cc.coef = 0.0;
      cc.upd_sparse = 0;
      cc.sig = 0.0;
    } else {
      cc.mode = COL_RUN;
      cc.coef = S.alpha * S.sig_cur;
      cc.upd_sparse = cc.prev_sparse;  // the update still needs to know
      cc.prev_sparse = 0;  // the sparse q_1 was consumed by this iteration's product
      cc.pa = pa;
      cc.xb = xb;
      active = 1;
    }
    st[j] = S;
    ctrl[j] = cc;
  }
  // count active columns
  __shared__ int32_t cnt[4];
  int32_t a = active;
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if ((j & 63) == 0) cnt[j >> 6] = a;
  __syncthreads();
  if (j == 0) {
    const int32_t total = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    qstate[1] = total;
    if (total > 0) qstate[2] += 1;  // the next sparse product does work
  }
}

// W = Y - alpha sig U_cur for running columns (in place over Y), the start
// vector for refilled columns, zero for idle ones; per-block sum d W^2.
// RO (re-orthogonalisation runs only, so the default keeps no registers for
// it): ro >= 1 also sums d W per block (slab 0 of rpart); ro == 2 also sums
// d W U_cur and d W U_prev (slabs 1 and 2), the coefficients of the
// re-orthogonalisation.
// GRAD: also advance the potential of running (and just-stopped) columns,
// p = sig U_cur + pa p, x = x + xb p (arrays P, X of the same shape).
template <typename VT, int B, bool GRAD, bool RO>
__global__ __launch_bounds__(SHORT_THREADS) void k_update(int32_t n, const double *__restrict__ deg,
                                                          const VT *__restrict__ Ucur,
                                                          const VT *__restrict__ Uprev,
                                                          VT *__restrict__ Y,
                                                          const ColCtrl *__restrict__ ctrl,
                                                          double *__restrict__ part, int32_t ldp,
                                                          const int32_t *__restrict__ active,
                                                          VT *__restrict__ P, VT *__restrict__ X,
                                                          int32_t ro, double *__restrict__ rpart,
                                                          VT *__restrict__ Xf) {
  if (*active == 0) return;
  using S = Shape<B>;
  constexpr int VEC = S::VEC;
  using V = VecN<VT, VEC>;
  __shared__ double sm[(SHORT_THREADS / 64) * B];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int sub = lane / S::LPR, c0 = (lane % S::LPR) * VEC;
  VT coef[VEC], vs[VEC], vt[VEC], sig[VEC];
  double pa[VEC], xb[VEC];
  int32_t mode[VEC], cs[VEC], ct[VEC], hs[VEC];
  bool psp[VEC];
  bool pot = false;
  double acc[VEC], a1[VEC], ac[VEC], ap[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const ColCtrl &cc = ctrl[c0 + v];
    coef[v] = (VT)cc.coef;
    vs[v] = (VT)cc.vs;
    vt[v] = (VT)cc.vt;
    sig[v] = (VT)cc.sig;
    pa[v] = cc.pa;
    xb[v] = cc.xb;
    mode[v] = cc.mode;
    cs[v] = cc.s;
    ct[v] = cc.t;
    psp[v] = cc.upd_sparse != 0;
    hs[v] = cc.hslot;
    acc[v] = a1[v] = ac[v] = ap[v] = 0.0;
    pot = pot || (mode[v] != COL_IDLE && mode[v] != COL_PENDING);
  }
  // lanes of at most 4 bytes (FP32 up to width 64) stream Y and U_cur with the
  // non-temporal hint: -12% per launch on a 4M-node power-law graph at FP32
  // width 64, +2% on FP64 width 256 (a road-like graph), so wider lanes do not
  constexpr bool NT = !GRAD && !RO && sizeof(VT) * VEC <= 4;
  const int gw = blockIdx.x * (SHORT_THREADS / 64) + wid;
  const int nwv = gridDim.x * (SHORT_THREADS / 64);
  for (int32_t r = gw * S::RPW + sub; r < n; r += nwv * S::RPW) {
    const V y = NT ? vload_nt<VT, VEC>(Y + (size_t)r * B + c0) : vload<VT, VEC>(Y + (size_t)r * B + c0);
    const V uc = NT ? vload_nt<VT, VEC>(Ucur + (size_t)r * B + c0) : vload<VT, VEC>(Ucur + (size_t)r * B + c0);
    const double dr = deg[r];
    V up;
    if (RO && ro == 2) up = vload<VT, VEC>(Uprev + (size_t)r * B + c0);
    V o;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      VT x;
      if (mode[v] == COL_RUN) {
        x = y.v[v] - coef[v] * uc.v[v];
        const double dx = dr * (double)x;
        acc[v] += dx * (double)x;
        if (RO && ro >= 1) a1[v] += dx;
        if (RO && ro == 2) {
          const VT pv = psp[v] ? (r == cs[v] ? vs[v] : (r == ct[v] ? vt[v] : VT(0))) : up.v[v];
          ac[v] += dx * (double)uc.v[v];
          ap[v] += dx * (double)pv;
        }
      } else {
        // refilled columns: the first iteration's vector is scattered by
        // k_first_batch; idle and finished columns hold zeros
        x = VT(0);
      }
      o.v[v] = x;
    }
    if constexpr (NT) vstore_nt<VT, VEC>(Y + (size_t)r * B + c0, o);
    else vstore<VT, VEC>(Y + (size_t)r * B + c0, o);
    if constexpr (GRAD) {
      if (pot) {
        VecN<double, VEC> pv = vload_f64<VT, VEC>(P + (size_t)r * B + c0);
        VecN<double, VEC> xv = vload_f64<VT, VEC>(X + (size_t)r * B + c0);
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int32_t m = mode[v];
          if (m == COL_RUN || m == COL_FINAL || m == COL_FINAL_REFILL) {
            const double p = (double)sig[v] * (double)uc.v[v] + pa[v] * pv.v[v];
            pv.v[v] = p;
            xv.v[v] += xb[v] * p;
          }
          // a finished potential goes to its harvest slot
          if ((m == COL_FINAL || m == COL_HARVEST || m == COL_FINAL_REFILL || m == COL_HARVEST_REFILL) &&
              hs[v] >= 0)
            Xf[(size_t)r * B + hs[v]] = (VT)xv.v[v];
          if (starts_pair(m)) {
            pv.v[v] = 0.0;  // a new run's potential starts from zero
            xv.v[v] = 0.0;
          }
        }
        vstore_from_f64<VT, VEC>(P + (size_t)r * B + c0, pv);
        vstore_from_f64<VT, VEC>(X + (size_t)r * B + c0, xv);
      }
    }
  }
  block_column_partials<B, VEC>(acc, sm, part, ldp, blockIdx.x);
  if (RO && ro >= 1) block_column_partials<B, VEC>(a1, sm, rpart, ldp, blockIdx.x);
  if (RO && ro == 2) {
    block_column_partials<B, VEC>(ac, sm, rpart + (size_t)B * ldp, ldp, blockIdx.x);
    block_column_partials<B, VEC>(ap, sm, rpart + 2 * (size_t)B * ldp, ldp, blockIdx.x);
  }
}

// Coefficients of the re-orthogonalisation of every running column from the
// column sums of k_update (sums[k * B + j], slab k), in terms of the stored
// vectors: the components of W along u_1 (the constant vector in the scaled
// basis), q_i = sig_cur U_cur and q_{i-1} = sig_prev U_prev are
// (sum d W)/vol, sig_cur^2 sum d W U_cur and sig_prev^2 sum d W U_prev.
__global__ void k_reorth_coef(int32_t B, int32_t ro, double vol, const double *__restrict__ sums,
                              const LzState *__restrict__ st, ColCtrl *__restrict__ ctrl,
                              const int32_t *__restrict__ active) {
  if (*active == 0) return;
  const int j = threadIdx.x;
  if (j >= B) return;
  ColCtrl cc = ctrl[j];
  const LzState &S = st[j];
  const bool run = cc.mode == COL_RUN;
  cc.ro_mu = run ? sums[j] / vol : 0.0;
  cc.ro_c = run && ro == 2 ? S.sig_cur * S.sig_cur * sums[B + j] : 0.0;
  cc.ro_p = run && ro == 2 ? S.sig_prev * S.sig_prev * sums[2 * B + j] : 0.0;
  ctrl[j] = cc;
}

// W -= ro_mu + ro_c U_cur + ro_p U_prev for running columns; per-block sum d W^2.
template <typename VT, int B>
__global__ __launch_bounds__(SHORT_THREADS) void k_reorth_apply(int32_t n, const double *__restrict__ deg,
                                                                const VT *__restrict__ Ucur,
                                                                const VT *__restrict__ Uprev,
                                                                VT *__restrict__ Y,
                                                                const ColCtrl *__restrict__ ctrl,
                                                                double *__restrict__ part, int32_t ldp,
                                                                const int32_t *__restrict__ active,
                                                                int32_t ro) {
  if (*active == 0) return;
  using S = Shape<B>;
  constexpr int VEC = S::VEC;
  using V = VecN<VT, VEC>;
  __shared__ double sm[(SHORT_THREADS / 64) * B];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int sub = lane / S::LPR, c0 = (lane % S::LPR) * VEC;
  VT mu[VEC], kc[VEC], kp[VEC], vs[VEC], vt[VEC];
  int32_t cs[VEC], ct[VEC];
  bool run[VEC], psp[VEC];
  double acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) {
    const ColCtrl &cc = ctrl[c0 + v];
    run[v] = cc.mode == COL_RUN;
    mu[v] = (VT)cc.ro_mu;
    kc[v] = (VT)cc.ro_c;
    kp[v] = (VT)cc.ro_p;
    vs[v] = (VT)cc.vs;
    vt[v] = (VT)cc.vt;
    cs[v] = cc.s;
    ct[v] = cc.t;
    psp[v] = cc.upd_sparse != 0;
    acc[v] = 0.0;
  }
  const int gw = blockIdx.x * (SHORT_THREADS / 64) + wid;
  const int nwv = gridDim.x * (SHORT_THREADS / 64);
  for (int32_t r = gw * S::RPW + sub; r < n; r += nwv * S::RPW) {
    V w = vload<VT, VEC>(Y + (size_t)r * B + c0);
    V uc, up;
    if (ro == 2) {
      uc = vload<VT, VEC>(Ucur + (size_t)r * B + c0);
      up = vload<VT, VEC>(Uprev + (size_t)r * B + c0);
    }
    const double dr = deg[r];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      if (!run[v]) continue;
      VT x = w.v[v] - mu[v];
      if (ro == 2) {
        const VT pv = psp[v] ? (r == cs[v] ? vs[v] : (r == ct[v] ? vt[v] : VT(0))) : up.v[v];
        x -= kc[v] * uc.v[v] + kp[v] * pv;
      }
      w.v[v] = x;
      acc[v] += dr * ((double)x * (double)x);
    }
    vstore<VT, VEC>(Y + (size_t)r * B + c0, w);
  }
  block_column_partials<B, VEC>(acc, sm, part, ldp, blockIdx.x);
}

// Sum over the LPR lanes of a row segment (result in every lane of it).
template <int LPR>
__device__ __forceinline__ double segment_sum(double x) {
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Eight segment sums at once (LPR >= 8 lanes): the first three butterfly
// stages each hand half of the values to the partner lane, so every stage
// moves half as many values as the one before; the rest sum one value. The
// total of value k ends in the lanes whose bits LPR/2, LPR/4, LPR/8 spell k;
// the lane cl = k * LPR / 8 holds it.
template <int LPR>
__device__ __forceinline__ double segment_sums8(const double (&a)[8], int cl) {
  double v4[4], v2[2];
  {
    constexpr int o = LPR / 2;
    const bool up = cl & o;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double keep = up ? a[i + 4] : a[i];
      const double give = up ? a[i] : a[i + 4];
      v4[i] = keep + __shfl_xor(give, o, 64);
    }
  }
  {
    constexpr int o = LPR / 4;
    const bool up = cl & o;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const double keep = up ? v4[i + 2] : v4[i];
      const double give = up ? v4[i] : v4[i + 2];
      v2[i] = keep + __shfl_xor(give, o, 64);
    }
  }
  double x;
  {
    constexpr int o = LPR / 8;
    const bool up = cl & o;
    const double keep = up ? v2[1] : v2[0];
    const double give = up ? v2[0] : v2[1];
    x = keep + __shfl_xor(give, o, 64);
  }
#pragma unroll
  for (int off = LPR / 16; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Edge gradient for the pairs held in the columns of X (the accumulated
// potentials in the scaled basis: phi_p = sqrt(c_p) X[:, p]), for the
// adjacency entry a = (u, v > u) of every edge:
//   gacc[a] += -sum_p cw[p] (X[u, p] - X[v, p])^2,  cw[p] = grad_r[pair] * c_pair.
// The accumulator is in adjacency order, so a chunk's words are contiguous;
// k_gacc_out applies the edge ids once per call. One row segment (LPR lanes
// over the columns) per edge chunk; EU edges in flight per segment; FP64 sums
// in a fixed order.
// gate != nullptr: run only when *gate == B (a full block of harvested potentials).
template <typename PT, int B>
__global__ __launch_bounds__(SHORT_THREADS) void k_grad_edges(
    int32_t nch, const int4 *__restrict__ chunk, const int32_t *__restrict__ col,
    const PT *__restrict__ X, const double *__restrict__ cw, double *__restrict__ gacc,
    const int32_t *__restrict__ gate) {
  if (gate && *gate != B) return;
  using S = Shape<B>;
  constexpr int VEC = S::VEC;
  constexpr int EU = 8;  // one lane per edge writes its sum (a segment has >= 16 lanes)
  using XV = VecN<double, VEC>;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int sub = lane / S::LPR, cl = lane % S::LPR, c0 = cl * VEC;
  double w[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) w[v] = cw[c0 + v];
  const int gw = blockIdx.x * (SHORT_THREADS / 64) + wid;
  const int nwv = gridDim.x * (SHORT_THREADS / 64);
  const int32_t stride = nwv * S::RPW;
  int32_t ic = gw * S::RPW + sub;
  int4 nx = ic < nch ? chunk[ic] : make_int4(0, 0, 0, 0);
  for (; ic < nch; ic += stride) {
    // the next chunk's bounds load while this one is processed
    const int4 ch = nx;
    if (ic + stride < nch) nx = chunk[ic + stride];
    const int32_t u = ch.x, pe = ch.z;
    const XV xu = vload_f64<PT, VEC>(X + (size_t)u * B + c0);
    int32_t p = ch.y;
    for (; p + EU <= pe; p += EU) {
      XV xv[EU];
#pragma unroll
      for (int k = 0; k < EU; ++k) xv[k] = vload_f64<PT, VEC>(X + (size_t)col[p + k] * B + c0);
      // lane cl = k * LPR / 8 writes edge k's sum
      constexpr int WS = S::LPR / EU;
      const bool writer = cl % WS == 0;
      const int32_t kw = cl / WS;
      const double g0 = writer ? gacc[p + kw] : 0.0;  // loaded with the gathers
      double a[EU];
#pragma unroll
      for (int k = 0; k < EU; ++k) {
        a[k] = 0.0;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const double d = xu.v[v] - xv[k].v[v];
          a[k] += w[v] * d * d;
        }
      }
      const double mine = segment_sums8<S::LPR>(a, cl);
      if (writer) gacc[p + kw] = g0 - mine;
    }
    for (; p < pe; ++p) {
      const XV xv = vload_f64<PT, VEC>(X + (size_t)col[p] * B + c0);
      double a = 0.0;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const double d = xu.v[v] - xv.v[v];
        a += w[v] * d * d;
      }
      a = segment_sum<S::LPR>(a);
      if (cl == 0) gacc[p] -= a;
    }
  }
}

// After the edge pass of a full harvest block: the slots are free again and
// their weights zero (so a final pass over a partly filled block counts only
// the slots in use).
__global__ void k_harvest_reset(int32_t B, int32_t *__restrict__ qstate, double *__restrict__ cw,
                                int32_t *__restrict__ slot_pair) {
  if (qstate[4] != B) return;
  __syncthreads();
  for (int j = threadIdx.x; j < B; j += blockDim.x) {
    cw[j] = 0.0;
    if (slot_pair) slot_pair[j] = -1;
  }
  __syncthreads();
  if (threadIdx.x == 0) qstate[4] = 0;
}

// Per-column energy of the accumulated potentials, sum_e w_e (X[u,p] - X[v,p])^2
// in FP64, as per-block column partials (edge chunks as in k_grad_edges).
template <typename PT, int B, bool WEIGHTED>
__global__ __launch_bounds__(SHORT_THREADS) void k_energy(
    int32_t nch, const int4 *__restrict__ chunk, const int32_t *__restrict__ col,
    const double *__restrict__ w64, const PT *__restrict__ X, double *__restrict__ part,
    int32_t ldp, const int32_t *__restrict__ active) {
  if (*active == 0) return;
  using S = Shape<B>;
  constexpr int VEC = S::VEC;
  using XV = VecN<double, VEC>;
  __shared__ double sm[(SHORT_THREADS / 64) * B];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int sub = lane / S::LPR, c0 = (lane % S::LPR) * VEC;
  double acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0.0;
  const int gw = blockIdx.x * (SHORT_THREADS / 64) + wid;
  const int nwv = gridDim.x * (SHORT_THREADS / 64);
  for (int32_t ic = gw * S::RPW + sub; ic < nch; ic += nwv * S::RPW) {
    const int4 ch = chunk[ic];
    const int32_t u = ch.x, pe = ch.z;
    const XV xu = vload_f64<PT, VEC>(X + (size_t)u * B + c0);
    int32_t p = ch.y;
    for (; p + 4 <= pe; p += 4) {
      XV xv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) xv[k] = vload_f64<PT, VEC>(X + (size_t)col[p + k] * B + c0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double we = WEIGHTED ? w64[p + k] : 1.0;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const double d = xu.v[v] - xv[k].v[v];
          acc[v] += we * d * d;
        }
      }
    }
    for (; p < pe; ++p) {
      const XV xv = vload_f64<PT, VEC>(X + (size_t)col[p] * B + c0);
      const double we = WEIGHTED ? w64[p] : 1.0;
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const double d = xu.v[v] - xv.v[v];
        acc[v] += we * d * d;
      }
    }
  }
  block_column_partials<B, VEC>(acc, sm, part, ldp, blockIdx.x);
}

// r = J(phi) = 2 (phi_s - phi_t) - phi^T L phi with phi = sqrt(c) Xf[:, j] (FP64)
// for the pair p held by harvest slot j (cw[j] = c_p; energy[j] = the column's
// sum_e w_e (Xf[u, j] - Xf[v, j])^2).
template <typename VT, int B>
__global__ void k_refine_out(const int32_t *__restrict__ slot_pair, const int32_t *__restrict__ ps,
                             const int32_t *__restrict__ pt, const double *__restrict__ cw,
                             const VT *__restrict__ X, const double *__restrict__ energy,
                             rd_result *__restrict__ out, const int32_t *__restrict__ active) {
  if (*active == 0) return;
  const int j = threadIdx.x;
  if (j >= B) return;
  const int32_t pair = slot_pair[j];
  if (pair < 0) return;
  const double c = cw[j];
  const double xs = (double)X[(size_t)ps[pair] * B + j], xt = (double)X[(size_t)pt[pair] * B + j];
  out[pair].r = 2.0 * sqrt(c) * (xs - xt) - c * energy[j];
}

// Per-column partial sums of X over the rows (fixed order, as the products).
template <typename VT, int B>
__global__ __launch_bounds__(SHORT_THREADS) void k_col_reduce(int32_t n, const VT *__restrict__ X,
                                                            double *__restrict__ part, int32_t ldp,
                                                            const int32_t *__restrict__ active) {
  if (*active == 0) return;
  using S = Shape<B>;
  constexpr int VEC = S::VEC;
  __shared__ double sm[(SHORT_THREADS / 64) * B];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int sub = lane / S::LPR, c0 = (lane % S::LPR) * VEC;
  double acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0.0;
  const int gw = blockIdx.x * (SHORT_THREADS / 64) + wid;
  const int nwv = gridDim.x * (SHORT_THREADS / 64);
  for (int32_t r = gw * S::RPW + sub; r < n; r += nwv * S::RPW) {
    const VecN<VT, VEC> x = vload<VT, VEC>(X + (size_t)r * B + c0);
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += (double)x.v[v];
  }
  block_column_partials<B, VEC>(acc, sm, part, ldp, blockIdx.x);
}

// 1 when the block of harvested potentials is full (qstate[4] == B), else 0.
__global__ void k_full_flag(int32_t B, const int32_t *__restrict__ qstate, int32_t *__restrict__ flag) {
  if (threadIdx.x == 0) *flag = qstate[4] == B ? 1 : 0;
}

// phi_p = Pi sqrt(c_p) Xf[:, j] for the pair p held by harvest slot j, in the
// caller's node order (perm: caller id -> row; nullptr: the identity), one row
// of n values per pair; colsum[j] is the column's sum, so the mean is removed
// (phi sums to zero, as L^+ b does); cw[j] = c_p (the pairs' weights are ones).
template <typename VT, int B>
__global__ __launch_bounds__(256) void k_pot_out(int32_t n, const int32_t *__restrict__ perm,
                                                 const int32_t *__restrict__ slot_pair,
                                                 const double *__restrict__ cw, const VT *__restrict__ X,
                                                 const double *__restrict__ colsum, double *__restrict__ phi,
                                                 const int32_t *__restrict__ active) {
  if (*active == 0) return;
  // tiles of 64 nodes x TJ slots through LDS: the block is read a row segment
  // per node and phi written 64 consecutive nodes per slot (both coalesced);
  // grid-stride over the tiles, so a gated-off launch is cheap
  constexpr int TJ = B < 64 ? B : 64;
  constexpr int JT = B / TJ;
  __shared__ double tile[TJ][65];
  const int32_t ntile = (int32_t)((n + 63) / 64) * JT;
  for (int32_t t = blockIdx.x; t < ntile; t += gridDim.x) {
    const int32_t u0 = (t / JT) * 64;
    const int j0 = (t % JT) * TJ;
    for (int e = threadIdx.x; e < 64 * TJ; e += 256) {
      const int jj = e % TJ, uu = e / TJ;
      const int32_t u = u0 + uu;
      double x = 0.0;
      if (u < n) x = (double)X[(size_t)(perm ? perm[u] : u) * B + j0 + jj];
      tile[jj][uu] = x;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * TJ; e += 256) {
      const int uu = e % 64, jj = e / 64;
      const int32_t u = u0 + uu;
      const int j = j0 + jj;
      const int32_t pair = slot_pair[j];
      if (u < n && pair >= 0) phi[(size_t)pair * n + u] = sqrt(cw[j]) * (tile[jj][uu] - colsum[j] / n);
    }
    __syncthreads();
  }
}

// grad_w in caller edge order from the adjacency-order accumulator (one
// thread per edge chunk).
__global__ void k_gacc_out(int32_t nch, const int4 *__restrict__ chunk, const int32_t *__restrict__ eid,
                           const double *__restrict__ gacc, float *__restrict__ grad_w) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nch) return;
  const int4 ch = chunk[i];
  for (int32_t p = ch.y; p < ch.z; ++p) grad_w[eid[p]] = (float)gacc[p];
}

// beta_{i+1} of every running column and the next scales.
__global__ __launch_bounds__(COL_THREADS) void k_beta(const double *__restrict__ part, int32_t ldp,
                                                      int32_t np, LzState *__restrict__ st,
                                                      ColCtrl *__restrict__ ctrl,
                                                      const int32_t *__restrict__ active) {
  if (*active == 0) return;
  __shared__ double sm[COL_THREADS / 64];
  const int j = blockIdx.x;
  const double *p = part + (size_t)j * ldp;
  double a = 0.0;
  for (int k = threadIdx.x; k < np; k += COL_THREADS) a += p[k];
  a = block_sum(a, sm);
  if (threadIdx.x == 0) {
    ColCtrl cc = ctrl[j];
    if (cc.mode != COL_RUN) return;
    LzState S = st[j];
    if (S.status != LZ_RUNNING) return;
    scalar_after_beta(S, a, nullptr);
    cc.sig = S.sig_cur;
    cc.pc = S.prev_coef;
    st[j] = S;
    ctrl[j] = cc;
  }
}

// ---------------------------------------------------------------------------
// Sparse second iteration. After the sparse first iteration a refilled column
// holds w_1 on S = N(s) u N(t) u {s, t}, so q_2 = w_1 / beta_2 has that support
// and y_2 = D^{-1} W q_2 - beta_2 q_1 lives on N(S), which contains S. Each
// adjacency entry (u in S, v in N(u)) adds w_uv w_1[u] / d_v to the sum of v
// and 1 to its count, packed in one 64-bit fixed-point word (sum << 16 | count):
// integer addition does not depend on the order, so the sums, and the run,
// are the same every time. The entry whose add found a zero count owns the
// node (an ownership bit per entry). alpha_2 comes from the sums on S. Each
// owner writes y_2[v] into the column, adds d_v y_2[v]^2 to ||w_2||_D^2 (in
// fixed point, so the order of the adds does not matter) and clears the word;
// a pass over S subtracts alpha_2 q_2 there and corrects the norm.
// The column joins the dense iterations at i = 3; that product reads zeros for
// q_2, and k_s2_prev adds its term from the list of S afterwards.
// ---------------------------------------------------------------------------
constexpr int S2_PIECE = 256;           // scatter entries of one row per wavefront step
constexpr int32_t S2_LCAP_MAX = 65535;  // list slots per column at most (deg_s + deg_t + 2),
                                        // so a count (at most |S|) fits 16 bits
constexpr int S2_CNT_BITS = 16;
constexpr double S2_ENTRY_NS = 0.125;  // measured cost of the sparse step per scatter entry (MI355X)
constexpr double S2_BETA_UNIT = 0x1p58;  // fixed-point units of the ||w_2||^2 terms (<= 1)
constexpr double S2_BETA_SUB = 0x1p32;   // second word: 2^-90

struct S2Col {
  int64_t E;       // scatter entries of the current step (0: none)
  int32_t L;       // list slots of the column's current list (deg_s + deg_t + 2)
  int32_t nch;     // pieces: rows of the list cut into S2_PIECE entries
  int32_t sexp;    // the sums are kept in units of 2^-sexp
  int32_t adv;     // alpha_2 advanced the run (the potentials take their second term)
  double alpha;    // alpha_2
  double pa, xb;   // potentials: p_2 = q_2 + pa p_1, x_2 = x_1 + xb p_2
  unsigned long long bhi, blo;  // ||w_2||_D^2 in units of 2^-58 (two's complement) and 2^-90
};

// The rest of a column's list once its slots hold (node, stored w_1) or a
// hole (node -1), for all 256 threads of a block: exclusive prefix sums of the
// rows' piece counts into lp, the number of scatter entries, the fixed-point
// unit from max |w_1| (mx: each thread's part), and, when the scatter has at
// most s2_ecap entries, the column's record *sc and the slot of every piece.
__device__ void s2_finish_list(const int32_t *__restrict__ row_ptr, int32_t L, const int32_t *__restrict__ lu,
                               int64_t *__restrict__ lp, double mx, int64_t s2_ecap, S2Col *__restrict__ sc,
                               int32_t *__restrict__ ps) {
  __shared__ int64_t wsum[256 / 64];
  __shared__ double wmax[256 / 64];
  __shared__ int32_t go;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t carry = 0, ent = 0;
  for (int32_t base = 0; base < L; base += 256) {
    const int32_t k = base + threadIdx.x;
    int64_t d = 0;
    if (k < L) {
      const int32_t u = lu[k];
      if (u >= 0) {
        const int32_t len = row_ptr[u + 1] - row_ptr[u];
        d = (len + S2_PIECE - 1) / S2_PIECE;
        ent += len;
      }
    }
    int64_t x = d;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    int64_t before = carry, tot = 0;
    for (int w = 0; w < 256 / 64; ++w) {
      if (w < wid) before += wsum[w];
      tot += wsum[w];
    }
    if (k < L) lp[k] = before + x - d;
    __syncthreads();
    carry += tot;
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  ent = wave_sum(ent);
  if (lane == 0) {
    wmax[wid] = mx;
    wsum[wid] = ent;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    lp[L] = carry;
    ent = 0;
    for (int w = 0; w < 256 / 64; ++w) {
      mx = fmax(mx, wmax[w]);
      ent += wsum[w];
    }
    S2Col c = *sc;
    c.L = L;
    c.E = 0;
    // (at most 2^22 pieces per column keeps the piece offsets of 256 columns in int32)
    if (ent > 0 && ent <= s2_ecap && carry <= (1 << 22) && mx > 0.0) {
      // |sum_u w_uv w_1[u] / d_v| <= max |w_1| < 2^e: units of 2^(e - 46) keep
      // every sum below 2^46, which leaves 16 bits of the word for the count
      int e;
      (void)frexp(mx, &e);
      c.E = ent;
      c.nch = (int32_t)carry;
      c.sexp = 46 - e;
      c.bhi = c.blo = 0;
    }
    *sc = c;
    go = c.E > 0;
  }
  __syncthreads();
  if (!go) return;
  for (int32_t k = threadIdx.x; k < L; k += blockDim.x)
    for (int64_t r = lp[k]; r < lp[k + 1]; ++r) ps[r] = k;
}

// First iteration of every refilled column from the adjacency rows of s and t
// (block j: column j). Writes w_1 into column j of W (zeroed by k_update),
// completes iteration 1 of the column's scalars, and arms the next product to
// read the previous vector q_1 analytically. GRAD: p_1 = q_1, x_1 = q_1/delta_1.
// s2: also the list of S (slot, node, stored w_1) with the exclusive prefix
// sums of the rows' piece counts, and the sparse second step when its scatter
// has at most s2_ecap entries.
template <typename VT, int B, bool GRAD>
__global__ __launch_bounds__(256) void k_first_batch(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const double *__restrict__ w64, const double *__restrict__ deg, VT *__restrict__ W,
    LzState *__restrict__ st, ColCtrl *__restrict__ ctrl, VT *__restrict__ P, VT *__restrict__ X,
    const int32_t *__restrict__ active, int32_t s2, int64_t s2_ecap, int32_t lcap,
    int32_t *__restrict__ Lu, double *__restrict__ Lw, int64_t *__restrict__ Lp,
    S2Col *__restrict__ s2c, int32_t *__restrict__ pslot, int64_t pcap) {
  if (*active == 0) return;
  const int j = blockIdx.x;
  if (!starts_pair(ctrl[j].mode)) return;
  __shared__ double sm[256 / 64 + 2];
  __shared__ LzState S0;
  __shared__ int32_t take;
  if (threadIdx.x == 0) S0 = st[j];
  __syncthreads();
  const int32_t s = S0.s, t = S0.t;
  const int32_t L = (row_ptr[s + 1] - row_ptr[s]) + (row_ptr[t + 1] - row_ptr[t]) + 2;
  const bool lst = s2 && L <= lcap;
  int32_t *lu = Lu + (size_t)j * lcap;
  double *lw = Lw + (size_t)j * lcap;
  int64_t *lp = Lp + (size_t)j * (lcap + 1);
  if (lst) {
    for (int32_t k = threadIdx.x; k < L; k += blockDim.x) lu[k] = -1;
    __syncthreads();
  }
  double mx = 0.0;
  double a1, bb;
  first_iteration(
      row_ptr, col, w64, deg, s, t, S0.c,
      [&](int32_t u, double val, int32_t pos) {
        const VT x = (VT)val;
        W[(size_t)u * B + j] = x;
        if (lst) {
          lu[pos] = u;
          lw[pos] = (double)x;
          mx = fmax(mx, fabs((double)x));
        }
        return (double)x;
      },
      sm, a1, bb);
  if (threadIdx.x == 0) {
    LzState S = S0;
    ColCtrl cc = ctrl[j];
    scalar_after_alpha(S, a1, nullptr, nullptr);
    const bool advanced = S.k == 1;
    if (S.status == LZ_RUNNING) scalar_after_beta(S, bb, nullptr);
    if (GRAD && advanced) {
      const double rc = 1.0 / sqrt(S.c);
      const double q1s = rc / deg[s], q1t = -rc / deg[t];
      P[(size_t)s * B + j] = (VT)q1s;
      P[(size_t)t * B + j] = (VT)q1t;
      X[(size_t)s * B + j] = (VT)(q1s / S.delta);
      X[(size_t)t * B + j] = (VT)(q1t / S.delta);
    }
    cc.mode = COL_RUN;
    cc.coef = 0.0;
    cc.plist = 0;
    if (S.status == LZ_RUNNING) {
      cc.sig = S.sig_cur;     // 1 / beta_2
      cc.pc = S.prev_coef;    // beta_2 (q_1 is stored with scale 1)
      cc.prev_sparse = 1;     // cc.vs, cc.vt hold q_1 at s and t
    } else {
      cc.sig = 0.0;  // finished after one iteration: retired by the next control step
      cc.pc = 0.0;
      cc.prev_sparse = 0;
    }
    st[j] = S;
    ctrl[j] = cc;
    take = lst && S.status == LZ_RUNNING;
  }
  __syncthreads();
  if (!take) return;
  s2_finish_list(row_ptr, L, lu, lp, mx, s2_ecap, s2c + j, pslot + (size_t)j * pcap);
}

// Piece offsets of the columns taking the sparse step, computed by every
// workgroup into LDS: cp[j] = sum of nch over the columns before j, cp[B] the
// total (B <= 256, a block of 256 threads).
__device__ __forceinline__ void s2_offsets(int32_t B, const S2Col *__restrict__ s2c, int32_t *cp) {
  __shared__ int32_t wtot[256 / 64];
  const int j = threadIdx.x, lane = j & 63, wid = j >> 6;
  const int32_t d = (j < B && s2c[j].E > 0) ? s2c[j].nch : 0;
  int32_t x = d;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wtot[wid] = x;
  __syncthreads();
  int32_t before = 0, tot = 0;
  for (int w = 0; w < 256 / 64; ++w) {
    if (w < wid) before += wtot[w];
    tot += wtot[w];
  }
  if (j < B) cp[j] = before + x - d;
  if (j == 0) cp[B] = tot;
  __syncthreads();
}

// Column of piece c (the last j with cpre[j] <= c; cpre[0] = 0 <= c < cpre[B]).
__device__ __forceinline__ int32_t s2_column(const int32_t *cpre, int32_t B, int32_t c) {
  int32_t lo = 0, hi = B;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (cpre[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

// A global piece c: its column j, list slot k (holding u) and the row
// entries [pb, pe) it covers. cp: the piece offsets (in LDS).
struct S2Piece {
  int32_t j, k, u, pb, pe;
};
__device__ __forceinline__ S2Piece s2_piece(const int32_t *cp, int32_t B, int32_t c, int32_t lcap,
                                            int64_t pcap, const int32_t *__restrict__ pslot,
                                            const int32_t *__restrict__ Lu, const int64_t *__restrict__ Lp,
                                            const int32_t *__restrict__ row_ptr) {
  S2Piece q;
  q.j = s2_column(cp, B, c);
  const int32_t r = c - cp[q.j];
  q.k = pslot[(size_t)q.j * pcap + r];
  q.u = Lu[(size_t)q.j * lcap + q.k];
  const int64_t first = Lp[(size_t)q.j * (lcap + 1) + q.k];
  q.pb = row_ptr[q.u] + (int32_t)(r - first) * S2_PIECE;
  q.pe = min(q.pb + S2_PIECE, row_ptr[q.u + 1]);
  return q;
}

// the sum and the count of a packed word
__device__ __forceinline__ double s2_sum(unsigned long long a, double inv_unit) {
  return (double)((long long)a >> S2_CNT_BITS) * inv_unit;
}
__device__ __forceinline__ bool s2_count_is_zero(unsigned long long a) {
  return (a & ((1ull << S2_CNT_BITS) - 1)) == 0;
}

// The scatter, one row piece per wavefront: piece r of column j covers
// entries q*S2_PIECE .. of the row of the list slot k holding u (q = r - lp[k]);
// each entry (u, v) adds w_uv w_1[u] / d_v, in units of 2^-sexp, and a count
// of 1 to the word acc[j][v] (two's complement in unsigned 64-bit words). Bit
// `lane` of own[c][i] marks the entry pb + lane + 64 i of global piece c whose
// add found the count at zero: one entry per node.
template <bool WEIGHTED>
__global__ __launch_bounds__(256) void k_s2_scatter(
    int32_t B, int32_t n, const S2Col *__restrict__ s2c, int32_t lcap,
    int64_t pcap, const int32_t *__restrict__ pslot, const int32_t *__restrict__ Lu,
    const double *__restrict__ Lw, const int64_t *__restrict__ Lp, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col, const double *__restrict__ w64, const double *__restrict__ deg,
    unsigned long long *__restrict__ acc, unsigned long long *__restrict__ own,
    const int32_t *__restrict__ active) {
  if (*active == 0) return;
  constexpr int NI = S2_PIECE / 64;
  __shared__ int32_t cp[257];
  s2_offsets(B, s2c, cp);
  const int32_t total = cp[B];
  const int lane = threadIdx.x & 63;
  const int32_t nwv = gridDim.x * (256 / 64);
  for (int32_t c = blockIdx.x * (256 / 64) + (threadIdx.x >> 6); c < total; c += nwv) {
    const S2Piece q = s2_piece(cp, B, c, lcap, pcap, pslot, Lu, Lp, row_ptr);
    const double wu = Lw[(size_t)q.j * lcap + q.k];
    const double unit = ldexp(1.0, s2c[q.j].sexp);
    unsigned long long *aj = acc + (size_t)q.j * n;
    // the piece's entries: every load first, then every add
    int32_t v[NI];
    double f[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int32_t p = q.pb + lane + 64 * i;
      v[i] = p < q.pe ? col[p] : -1;
      f[i] = (WEIGHTED && p < q.pe) ? w64[p] : 1.0;
    }
#pragma unroll
    for (int i = 0; i < NI; ++i)
      if (v[i] >= 0) f[i] *= wu / deg[v[i]];
    unsigned long long old[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      old[i] = 1ull;  // not an owner
      if (v[i] >= 0) {
        const long long fx = llrint(f[i] * unit);
        old[i] = atomicAdd(aj + v[i], ((unsigned long long)fx << S2_CNT_BITS) + 1ull);
      }
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const unsigned long long m = __ballot(s2_count_is_zero(old[i]));
      if (lane == 0) own[(size_t)c * NI + i] = m;
    }
  }
}

// alpha_2 = <y_2, q_2>_D over S (block j: column j, fixed order), then the
// column's scalar step.
__global__ __launch_bounds__(256) void k_s2_alpha(int32_t n, S2Col *__restrict__ s2c, int32_t lcap,
                                                  const int32_t *__restrict__ Lu, const double *__restrict__ Lw,
                                                  const double *__restrict__ deg,
                                                  const unsigned long long *__restrict__ acc,
                                                  LzState *__restrict__ st, const int32_t *__restrict__ active) {
  if (*active == 0) return;
  const int j = blockIdx.x;
  if (s2c[j].E == 0) return;
  __shared__ double sm[256 / 64];
  const LzState S0 = st[j];
  const int32_t L = s2c[j].L;
  const double inv = ldexp(1.0, -s2c[j].sexp);
  const double sig = S0.sig_cur, beta = S0.beta;  // 1/beta_2, beta_2
  const double rc = 1.0 / sqrt(S0.c);
  const double q1s = rc / deg[S0.s], q1t = -rc / deg[S0.t];
  const int32_t *lu = Lu + (size_t)j * lcap;
  const double *lw = Lw + (size_t)j * lcap;
  const unsigned long long *aj = acc + (size_t)j * n;
  double a = 0.0;
  for (int32_t k = threadIdx.x; k < L; k += blockDim.x) {
    const int32_t u = lu[k];
    if (u < 0) continue;
    const double q1 = u == S0.s ? q1s : (u == S0.t ? q1t : 0.0);
    const double y = sig * s2_sum(aj[u], inv) - beta * q1;
    a += deg[u] * y * (sig * lw[k]);
  }
  a = block_sum(a, sm);
  if (threadIdx.x == 0) {
    LzState S = S0;
    const double delta_prev = S.delta, beta_i = S.beta;
    scalar_after_alpha(S, a, nullptr, nullptr);
    s2c[j].alpha = a;
    // coefficients of the potential recurrence for i = 2 (as in k_control)
    const bool adv = S.k == 2;
    s2c[j].adv = adv ? 1 : 0;
    s2c[j].pa = adv ? beta_i / delta_prev : 0.0;
    s2c[j].xb = adv ? S.omega / S.delta : 0.0;
    st[j] = S;
  }
}

// The owner of each node v of N(S) writes y_2[v] into column j of W, adds
// d_v y_2[v]^2 to the fixed-point norm and clears the node's word (a column
// that stopped at alpha_2 only clears).
template <typename VT, int B>
__global__ __launch_bounds__(256) void k_s2_write(
    int32_t n, S2Col *__restrict__ s2c, int32_t lcap, int64_t pcap,
    const int32_t *__restrict__ pslot, const int32_t *__restrict__ Lu, const int64_t *__restrict__ Lp,
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ deg,
    unsigned long long *__restrict__ acc, const unsigned long long *__restrict__ own,
    const LzState *__restrict__ st, VT *__restrict__ W, const int32_t *__restrict__ active) {
  if (*active == 0) return;
  constexpr int NI = S2_PIECE / 64;
  __shared__ int32_t cp[257];
  s2_offsets(B, s2c, cp);
  const int32_t total = cp[B];
  const int lane = threadIdx.x & 63;
  const int32_t nwv = gridDim.x * (256 / 64);
  // one row piece per wavefront, as in k_s2_scatter
  for (int32_t c = blockIdx.x * (256 / 64) + (threadIdx.x >> 6); c < total; c += nwv) {
    const S2Piece q = s2_piece(cp, B, c, lcap, pcap, pslot, Lu, Lp, row_ptr);
    const int32_t j = q.j;
    const LzState &S = st[j];
    const bool running = S.status == LZ_RUNNING;
    const double inv = ldexp(1.0, -s2c[j].sexp);
    const double sig = S.sig_cur, beta = S.beta;
    const int32_t s = S.s, t = S.t;
    const double rc = 1.0 / sqrt(S.c);
    const double q1s = rc / deg[s], q1t = -rc / deg[t];
    unsigned long long *aj = acc + (size_t)j * n;
    // the owned entries: every load first
    int32_t v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int32_t p = q.pb + lane + 64 * i;
      const bool mine = p < q.pe && ((own[(size_t)c * NI + i] >> lane) & 1ull);
      v[i] = mine ? col[p] : -1;
    }
    unsigned long long a[NI];
    double dv[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      a[i] = 0ull;
      dv[i] = 0.0;
      if (v[i] >= 0) {
        a[i] = aj[v[i]];
        dv[i] = deg[v[i]];
      }
    }
#pragma unroll
    for (int i = 0; i < NI; ++i)
      if (v[i] >= 0) aj[v[i]] = 0ull;
    // each node's term of the norm in fixed point on its own, so the total
    // does not depend on which entry owned the node
    unsigned long long hi = 0, lo = 0;
    if (running) {
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        if (v[i] < 0) continue;
        const double q1 = v[i] == s ? q1s : (v[i] == t ? q1t : 0.0);
        const VT x = (VT)(sig * s2_sum(a[i], inv) - beta * q1);
        W[(size_t)v[i] * B + j] = x;
        const double th = dv[i] * (double)x * (double)x * S2_BETA_UNIT;
        const double fh = floor(th);
        hi += (unsigned long long)fh;
        lo += (unsigned long long)((th - fh) * S2_BETA_SUB);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      hi += __shfl_xor(hi, off, 64);
      lo += __shfl_xor(lo, off, 64);
    }
    if (lane == 0 && running && (hi | lo)) {
      atomicAdd(&s2c[j].bhi, hi);
      atomicAdd(&s2c[j].blo, lo);
    }
  }
}

// On S (block j: column j, fixed order): w_2 = y_2 - alpha_2 q_2 in place of the
// y_2 that k_s2_write stored (S is inside N(S)), and the norm corrected by the
// difference. GRAD: the potentials' second terms, which live on S too:
// p_2 = q_2 + pa p_1 and x_2 = x_1 + xb p_2 (also when the run stopped at
// alpha_2, as the dense update adds a stopped run's last term).
template <typename VT, int B, bool GRAD>
__global__ __launch_bounds__(256) void k_s2_fix(S2Col *__restrict__ s2c, int32_t lcap,
                                                const int32_t *__restrict__ Lu, const double *__restrict__ Lw,
                                                const double *__restrict__ deg, const LzState *__restrict__ st,
                                                VT *__restrict__ W, VT *__restrict__ P, VT *__restrict__ X,
                                                const int32_t *__restrict__ active) {
  if (*active == 0) return;
  const int j = blockIdx.x;
  if (s2c[j].E == 0) return;
  const bool running = st[j].status == LZ_RUNNING;
  const bool pot = GRAD && s2c[j].adv;
  if (!running && !pot) return;
  __shared__ double sm[256 / 64];
  const LzState &S = st[j];
  const int32_t L = s2c[j].L;
  const double alpha = s2c[j].alpha;
  const double pa = s2c[j].pa, xb = s2c[j].xb;
  const double sig = S.sig_cur;
  const int32_t *lu = Lu + (size_t)j * lcap;
  const double *lw = Lw + (size_t)j * lcap;
  double d = 0.0;
  for (int32_t k = threadIdx.x; k < L; k += blockDim.x) {
    const int32_t u = lu[k];
    if (u < 0) continue;
    const size_t ix = (size_t)u * B + j;
    const double q2 = sig * lw[k];
    if (running) {
      const double x0 = (double)W[ix];  // y_2[u] as k_s2_write stored it
      const VT x = (VT)(x0 - alpha * q2);
      W[ix] = x;
      d += deg[u] * ((double)x * (double)x - x0 * x0);
    }
    if (pot) {
      const double p = q2 + pa * (double)P[ix];
      P[ix] = (VT)p;
      X[ix] = (VT)((double)X[ix] + xb * p);
    }
  }
  d = block_sum(d, sm);
  if (threadIdx.x == 0 && running) {
    // the norm's two words take the signed correction: hi floor, lo >= 0
    const double th = d * S2_BETA_UNIT;
    const double fh = floor(th);
    s2c[j].bhi += (unsigned long long)(long long)fh;
    s2c[j].blo += (unsigned long long)((th - fh) * S2_BETA_SUB);
  }
}

// beta_3 of every column that took the sparse step, its scales for the dense
// iterations, and the previous-vector list (one thread per column).
__global__ void k_s2_beta(int32_t B, S2Col *__restrict__ s2c, LzState *__restrict__ st,
                          ColCtrl *__restrict__ ctrl, const int32_t *__restrict__ active) {
  if (*active == 0) return;
  const int j = threadIdx.x;
  if (j >= B || s2c[j].E == 0) return;
  S2Col c = s2c[j];
  const double bb = ldexp((double)(long long)c.bhi, -58) + ldexp((double)c.blo, -90);
  c.bhi = c.blo = 0;
  c.E = 0;
  s2c[j] = c;
  LzState S = st[j];
  ColCtrl cc = ctrl[j];
  if (S.status == LZ_RUNNING) scalar_after_beta(S, bb, nullptr);
  if (S.status == LZ_RUNNING) {
    cc.sig = S.sig_cur;   // 1 / beta_3 (W holds w_2)
    cc.pc = S.prev_coef;  // beta_3 / beta_2: the list holds w_1 = beta_2 q_2
    cc.prev_sparse = 1;   // the product reads zeros for q_2 ...
    cc.vs = cc.vt = 0.0;
    cc.plist = j + 1;     // ... and k_s2_prev adds its term
  } else {
    cc.sig = 0.0;  // stopped at the second iteration: retired by the next control step
    cc.pc = 0.0;
    cc.prev_sparse = 0;
    cc.plist = 0;
  }
  st[j] = S;
  ctrl[j] = cc;
}

// After the product of a column whose previous vector is a listed q_2:
// Y -= pc w_1 on S, and the change of <Y, q_i>_D into partial slot `slot`
// (zero for the other columns). Block j: column j.
template <typename VT, int B>
__global__ __launch_bounds__(256) void k_s2_prev(const S2Col *__restrict__ s2c, int32_t lcap,
                                                 const int32_t *__restrict__ Lu, const double *__restrict__ Lw,
                                                 const double *__restrict__ deg, const VT *__restrict__ Ucur,
                                                 VT *__restrict__ Y, ColCtrl *__restrict__ ctrl,
                                                 double *__restrict__ part, int32_t ldp, int32_t slot,
                                                 const int32_t *__restrict__ active) {
  if (*active == 0) return;
  __shared__ double sm[256 / 64];
  const int j = blockIdx.x;
  const int32_t pl = ctrl[j].plist;
  double a = 0.0;
  if (pl > 0) {
    const int32_t id = pl - 1;
    const int32_t L = s2c[id].L;
    const VT pc = (VT)ctrl[j].pc;
    const double sg = (double)(VT)ctrl[j].sig;
    const int32_t *lu = Lu + (size_t)id * lcap;
    const double *lw = Lw + (size_t)id * lcap;
    for (int32_t k = threadIdx.x; k < L; k += blockDim.x) {
      const int32_t u = lu[k];
      if (u < 0) continue;
      const size_t ix = (size_t)u * B + j;
      const VT old = Y[ix];
      const VT nv = old - pc * (VT)lw[k];
      Y[ix] = nv;
      a += deg[u] * ((double)nv - (double)old) * (sg * (double)Ucur[ix]);
    }
  }
  a = block_sum(a, sm);
  if (threadIdx.x == 0) {
    part[(size_t)j * ldp + slot] = a;
    if (pl > 0) ctrl[j].plist = 0;
  }
}

// The list of S for a single-pair run, built from w_1 as its first iteration
// stored it (U1, zero off S) with the slots k_first_batch uses, then finished
// as there (slot 0 of the column arrays). No list when the run stopped or
// the list would not fit.
template <typename VT>
__global__ __launch_bounds__(256) void k_s2_list_single(const int32_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col, const VT *__restrict__ U1,
                                                        const LzState *__restrict__ st, int64_t s2_ecap,
                                                        int32_t lcap, int32_t *__restrict__ Lu,
                                                        double *__restrict__ Lw, int64_t *__restrict__ Lp,
                                                        S2Col *__restrict__ s2c, int32_t *__restrict__ pslot) {
  const int32_t s = st->s, t = st->t;
  const int32_t rs = row_ptr[s], ds = row_ptr[s + 1] - rs;
  const int32_t rt = row_ptr[t], dt = row_ptr[t + 1] - rt;
  const int32_t L = ds + dt + 2;
  if (st->status != LZ_RUNNING || L > lcap) {
    if (threadIdx.x == 0) s2c->E = 0;
    return;
  }
  for (int32_t k = threadIdx.x; k < L; k += blockDim.x) Lu[k] = -1;
  __syncthreads();
  double mx = 0.0;
  auto put = [&](int32_t pos, int32_t u) {
    const double x = (double)U1[u];
    Lu[pos] = u;
    Lw[pos] = x;
    mx = fmax(mx, fabs(x));
  };
  for (int32_t p = threadIdx.x; p < ds; p += blockDim.x) put(p, col[rs + p]);
  for (int32_t p = threadIdx.x; p < dt; p += blockDim.x) {
    const int32_t u = col[rt + p];
    if (row_find(row_ptr, col, s, u) < 0) put(ds + p, u);
  }
  if (threadIdx.x == 0 && row_find(row_ptr, col, s, t) < 0) {
    put(L - 2, s);
    put(L - 1, t);
  }
  __syncthreads();
  s2_finish_list(row_ptr, L, Lu, Lp, mx, s2_ecap, s2c, pslot);
}

__global__ void k_batch_reset(int32_t B, LzState *__restrict__ st, ColCtrl *__restrict__ ctrl,
                              int32_t *__restrict__ qstate, S2Col *__restrict__ s2c) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (s2c && j < B) {
    s2c[j].E = 0;
    s2c[j].bhi = s2c[j].blo = 0;
  }
  if (j < B) {
    LzState S;
    state_start(S, 0, 0, 0.0, 0.0, 0, 0, 4, 0, -1);
    S.status = LZ_IDLE;
    st[j] = S;
    ColCtrl cc{};
    cc.mode = COL_IDLE;
    cc.s = -1;
    cc.t = -1;
    cc.hslot = -1;
    ctrl[j] = cc;
  }
  if (j == 0) {
    qstate[0] = 0;
    qstate[1] = 0;
    qstate[2] = 0;
    qstate[3] = 1;
    qstate[4] = 0;
  }
}

__global__ void k_check_pairs(int32_t npairs, int32_t n, const int32_t *__restrict__ s,
                              const int32_t *__restrict__ t, int32_t *__restrict__ flag) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < npairs && (s[i] < 0 || s[i] >= n || t[i] < 0 || t[i] >= n)) atomicOr(flag, 1);
}

// caller ids -> internal ids of a reordered graph
__global__ void k_map_pairs(int32_t npairs, const int32_t *__restrict__ perm,
                            const int32_t *__restrict__ s, const int32_t *__restrict__ t,
                            int32_t *__restrict__ ms, int32_t *__restrict__ mt) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  ms[i] = perm[s[i]];
  mt[i] = perm[t[i]];
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct BatchWork {
  // row-bin schedule (independent of B and precision): wave work items of at
  // most wave_nnz entries over rows of at most long_deg entries, longer rows
  // listed separately
  int32_t wave_nnz = 0, long_deg = 0;
  std::vector<int32_t> rp_host;  // row offsets, kept to rebuild the schedule
  int32_t nwi = 0, nlong = 0;
  int64_t nnz_short = 0;  // adjacency entries of rows handled by k_spmm_short
  int32_t n_short = 0;    // rows handled by k_spmm_short
  int32_t *witem_row = nullptr;  // [2*nwi]: [begin, end) row range of each work item
  int32_t *long_rows = nullptr;  // [nlong]
  int32_t grid_short = 0, grid_upd = 0;
  // buffers sized for the widest run so far
  size_t vec_bytes = 0;
  void *X[3] = {nullptr, nullptr, nullptr};  // q_{i-1}, q_i and the new vector rotate
  int32_t Bcap = 0;
  double *part = nullptr;  // [Bcap][ldp_cap]
  int32_t ldp = 0;      // partial slots per column of the current schedule
  int32_t ldp_cap = 0;  // slots the partial buffers were sized for
  double *colsum = nullptr;  // [Bcap]
  double *rpart = nullptr;   // re-orthogonalisation partials [3][Bcap][ldp]
  double *rsum = nullptr;    // [3 * 256]
  // gradient mode: search directions and potentials (n x B each), edge accumulator
  void *P = nullptr, *Xp = nullptr;
  void *Xf = nullptr;  // gradient harvest mode: n x B finished potentials
  size_t pot_bytes = 0;
  double *gacc = nullptr;  // [nnz]: edge gradient by adjacency entry (upper entries used)
  double *cw = nullptr;    // [256]
  // potentials harvest mode: column partials and sums of the block, the pair
  // of each slot, the full-block flag
  double *ppart = nullptr;  // [256][grid_upd]
  double *psum = nullptr;   // [256]
  int32_t *spair = nullptr; // [256]
  int32_t *pflag = nullptr;
  int32_t ppart_ld = 0;
  LzState *st = nullptr;
  ColCtrl *ctrl = nullptr;
  int32_t *qstate = nullptr;       // [8]: queue head, active columns, working iterations, 1,
                                   // harvest slots in use
  int32_t *qstate_host = nullptr;  // pinned
  int32_t *flag = nullptr;
  int32_t *cmap = nullptr;  // [128] source columns of a compaction
  // sparse second iterations: per column, a fixed-point word per node and the
  // list of S with the prefix sums of its rows' piece counts
  int32_t s2_slots = 0, s2_lcap = 0;
  unsigned long long *s2_acc = nullptr;  // [s2_slots][n]
  int32_t *s2_lu = nullptr;              // [s2_slots][s2_lcap]
  double *s2_lw = nullptr;               // [s2_slots][s2_lcap]
  int64_t *s2_lp = nullptr;              // [s2_slots][s2_lcap + 1]
  unsigned long long *s2_own = nullptr;  // ownership bits: [s2_slots * s2_pcap][S2_PIECE / 64]
  int32_t *s2_pslot = nullptr;           // list slot of every piece: [s2_slots][s2_pcap]
  int64_t s2_pcap = 0;                   // row pieces per column at most
  S2Col *s2c = nullptr;                  // [256]
  // autotune cache: chosen width and schedule per precision
  int32_t tuned[2] = {0, 0};
  int32_t tuned_wave[2] = {0, 0}, tuned_long[2] = {0, 0};
  double tuned_col_ms[2] = {0.0, 0.0};  // product time per column at that width and schedule
};

void batch_free(rd_graph g) {
  BatchWork *bw = g->batch;
  if (!bw) return;
  dev_free(bw->witem_row);
  dev_free(bw->long_rows);
  for (void *x : bw->X) dev_free(x);
  dev_free(bw->part);
  dev_free(bw->colsum);
  dev_free(bw->rpart);
  dev_free(bw->rsum);
  dev_free(bw->P);
  dev_free(bw->Xp);
  dev_free(bw->Xf);
  dev_free(bw->gacc);
  dev_free(bw->cw);
  dev_free(bw->ppart);
  dev_free(bw->psum);
  dev_free(bw->spair);
  dev_free(bw->pflag);
  dev_free(bw->st);
  dev_free(bw->ctrl);
  dev_free(bw->qstate);
  dev_free(bw->flag);
  dev_free(bw->cmap);
  dev_free(bw->s2_acc);
  dev_free(bw->s2_own);
  dev_free(bw->s2_pslot);
  dev_free(bw->s2_lu);
  dev_free(bw->s2_lw);
  dev_free(bw->s2_lp);
  dev_free(bw->s2c);
  if (bw->qstate_host) (void)hipHostFree(bw->qstate_host);
  delete bw;
  g->batch = nullptr;
}

// (Re)build the row-bin schedule: [begin, end) ranges of consecutive rows of at
// most long_deg entries holding at most wave_nnz entries (or one row), and the
// list of longer rows.
static void build_schedule(rd_graph g, BatchWork *bw, int32_t wave_nnz, int32_t long_deg) {
  if (bw->witem_row && wave_nnz == bw->wave_nnz && long_deg == bw->long_deg) return;
  const std::vector<int32_t> &rp = bw->rp_host;
  std::vector<int32_t> items, longs;
  items.reserve(g->nnz / wave_nnz + 16);
  int32_t r = 0;
  while (r < g->n) {
    if (rp[r + 1] - rp[r] > long_deg) {
      longs.push_back(r);
      ++r;
      continue;
    }
    const int32_t begin = r;
    int64_t acc = 0;
    while (r < g->n) {
      const int32_t len = rp[r + 1] - rp[r];
      if (len > long_deg || (acc > 0 && acc + len > wave_nnz)) break;
      acc += len;
      ++r;
    }
    items.push_back(begin);
    items.push_back(r);
  }
  dev_free(bw->witem_row);
  dev_free(bw->long_rows);
  bw->witem_row = bw->long_rows = nullptr;
  bw->nwi = (int32_t)items.size() / 2;
  bw->n_short = g->n - (int32_t)longs.size();
  bw->nnz_short = g->nnz;
  for (int32_t lr : longs) bw->nnz_short -= rp[lr + 1] - rp[lr];
  bw->nlong = (int32_t)longs.size();
  bw->witem_row = (int32_t *)dev_alloc(std::max<size_t>(2, items.size()) * sizeof(int32_t));
  if (!items.empty())
    RD_HIP(hipMemcpy(bw->witem_row, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  bw->long_rows = (int32_t *)dev_alloc(std::max<size_t>(1, longs.size()) * sizeof(int32_t));
  if (!longs.empty())
    RD_HIP(hipMemcpy(bw->long_rows, longs.data(), longs.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) cus = prop.multiProcessorCount;
  // persistent-style grids: enough waves to fill the chip, a fixed count so
  // the number of partial sums per column is fixed
  bw->grid_short = std::max(1, std::min<int32_t>(cus * 8, (bw->nwi + 3) / 4));
  bw->grid_upd = std::max(1, std::min<int32_t>(cus * 8, cdiv(g->n, 64)));
  // one slot more than the products write: the sparse-step correction
  bw->ldp = std::max(bw->grid_short + bw->nlong + 1, bw->grid_upd);
  bw->wave_nnz = wave_nnz;
  bw->long_deg = long_deg;
}

static BatchWork *batch_get(rd_graph g) {
  if (g->batch) return g->batch;
  BatchWork *bw = new BatchWork();
  g->batch = bw;
  bw->rp_host.resize((size_t)g->n + 1);
  RD_HIP(hipMemcpy(bw->rp_host.data(), g->row_ptr, (g->n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
  build_schedule(g, bw, WAVE_NNZ, LONG_DEG);
  bw->st = (LzState *)dev_alloc(256 * sizeof(LzState));
  bw->ctrl = (ColCtrl *)dev_alloc(256 * sizeof(ColCtrl));
  bw->colsum = (double *)dev_alloc(256 * sizeof(double));
  bw->qstate = (int32_t *)dev_alloc(8 * sizeof(int32_t));
  {
    // [3] is the constant 1 that gates launches outside a batched run
    const int32_t q0[8] = {0, 0, 0, 1, 0, 0, 0, 0};
    RD_HIP(hipMemcpy(bw->qstate, q0, sizeof(q0), hipMemcpyHostToDevice));
  }
  bw->flag = (int32_t *)dev_alloc(sizeof(int32_t));
  bw->cmap = (int32_t *)dev_alloc(128 * sizeof(int32_t));
  bw->s2c = (S2Col *)dev_alloc(256 * sizeof(S2Col));
  RD_HIP(hipMemset(bw->s2c, 0, 256 * sizeof(S2Col)));
  RD_HIP(hipHostMalloc((void **)&bw->qstate_host, 4 * sizeof(int32_t), hipHostMallocDefault));
  return bw;
}

// Buffers of the sparse second iterations for B columns. Returns false (the
// run then uses dense second iterations) when the per-node arrays would take
// more than S2_MAX_BYTES or device memory runs out.
constexpr size_t S2_MAX_BYTES = (size_t)24 << 30;
static bool s2_reserve(rd_graph g, BatchWork *bw, int32_t B, hipStream_t st) {
  if (B <= bw->s2_slots) return true;
  const size_t per = (size_t)g->n * sizeof(unsigned long long);
  if (per * B > S2_MAX_BYTES) return false;
  dev_free(bw->s2_acc);
  dev_free(bw->s2_own);
  dev_free(bw->s2_pslot);
  dev_free(bw->s2_lu);
  dev_free(bw->s2_lw);
  dev_free(bw->s2_lp);
  bw->s2_acc = nullptr;
  bw->s2_own = nullptr;
  bw->s2_pslot = nullptr;
  bw->s2_lu = nullptr;
  bw->s2_lw = nullptr;
  bw->s2_lp = nullptr;
  bw->s2_slots = 0;
  const int32_t lcap = (int32_t)std::min<int64_t>(2 * (int64_t)g->max_deg + 2, S2_LCAP_MAX);
  // a column's pieces: at most one per list slot plus entries / S2_PIECE, and
  // at most s2_ecap <= nnz * 8 / 128 entries
  const int64_t pcap = lcap + g->nnz * 8 / 128 / S2_PIECE + 1;
  try {
    bw->s2_acc = (unsigned long long *)dev_alloc((size_t)B * g->n * sizeof(unsigned long long));
    bw->s2_lu = (int32_t *)dev_alloc((size_t)B * lcap * sizeof(int32_t));
    bw->s2_lw = (double *)dev_alloc((size_t)B * lcap * sizeof(double));
    bw->s2_lp = (int64_t *)dev_alloc((size_t)B * (lcap + 1) * sizeof(int64_t));
    bw->s2_own = (unsigned long long *)dev_alloc((size_t)B * pcap * (S2_PIECE / 64) * sizeof(unsigned long long));
    bw->s2_pslot = (int32_t *)dev_alloc((size_t)B * pcap * sizeof(int32_t));
  } catch (const RdError &e) {
    if (e.code != RD_E_OOM) throw;
    // not enough device memory: this run takes dense second iterations
    for (void **x : {(void **)&bw->s2_acc, (void **)&bw->s2_lu, (void **)&bw->s2_lw, (void **)&bw->s2_lp,
                     (void **)&bw->s2_own, (void **)&bw->s2_pslot}) {
      dev_free(*x);
      *x = nullptr;
    }
    return false;
  }
  bw->s2_pcap = pcap;
  RD_HIP(hipMemsetAsync(bw->s2_acc, 0, (size_t)B * g->n * sizeof(unsigned long long), st));
  RD_HIP(hipMemsetAsync(bw->s2c, 0, 256 * sizeof(S2Col), st));
  bw->s2_lcap = lcap;
  bw->s2_slots = B;
  return true;
}

static void batch_reserve(rd_graph g, BatchWork *bw, int32_t B, size_t elem) {
  const size_t need = (size_t)g->n * B * elem;
  if (need > bw->vec_bytes) {
    for (void *&x : bw->X) {
      dev_free(x);
      x = nullptr;
    }
    bw->vec_bytes = 0;
    for (void *&x : bw->X) x = dev_alloc(need);
    bw->vec_bytes = need;
  }
  if (B > bw->Bcap || bw->ldp > bw->ldp_cap) {
    dev_free(bw->part);
    dev_free(bw->rpart);
    bw->part = bw->rpart = nullptr;
    bw->Bcap = std::max(B, bw->Bcap);
    bw->ldp_cap = std::max(bw->ldp, bw->ldp_cap);
    bw->part = (double *)dev_alloc((size_t)bw->Bcap * bw->ldp_cap * sizeof(double));
  }
}

// Partial and column-sum buffers of the re-orthogonalisation (on first use).
static void reorth_reserve(BatchWork *bw) {
  if (!bw->rpart) bw->rpart = (double *)dev_alloc(3 * (size_t)bw->Bcap * bw->ldp_cap * sizeof(double));
  if (!bw->rsum) bw->rsum = (double *)dev_alloc(3 * 256 * sizeof(double));
}

template <typename VT, int B, bool WEIGHTED>
static void launch_spmm(rd_graph g, BatchWork *bw, const VT *Ucur, const VT *Uprev, VT *Y,
                        hipStream_t st, const int32_t *active, bool prof = false) {
  const VT *w = nullptr;
  const VT *invdeg;
  if constexpr (sizeof(VT) == 8) {
    w = (const VT *)g->w64;
    invdeg = (const VT *)g->invdeg;
  } else {
    w = (const VT *)g->w32;
    invdeg = (const VT *)g->invdeg32;
  }
  std::pair<hipEvent_t, hipEvent_t> ev{};
  if (prof) {
    const double sv = sizeof(VT);
    ev = g->timer[0].next((double)bw->nnz_short * (4.0 + (WEIGHTED ? sv : 0.0)) +
                          4.0 * ((double)bw->n_short + 2.0 * bw->nwi) +
                          sv * B * ((double)g->n + 2.0 * bw->n_short) + (sv + 8.0) * (double)bw->n_short);
    RD_HIP(hipEventRecord(ev.first, st));
  }
  hipLaunchKernelGGL((k_spmm_short<VT, B, WEIGHTED>), dim3(bw->grid_short), dim3(SHORT_THREADS), 0, st,
                     bw->nwi, bw->witem_row, g->row_ptr, g->col, w, invdeg, g->deg, Ucur, Uprev, Y,
                     bw->ctrl, bw->part, bw->ldp, active, bw->long_deg);
  if (prof) RD_HIP(hipEventRecord(ev.second, st));
  if (bw->nlong > 0)
    hipLaunchKernelGGL((k_spmm_long<VT, B, WEIGHTED>), dim3(bw->nlong), dim3(LONG_THREADS), 0, st,
                       bw->long_rows, g->row_ptr, g->col, w, invdeg, g->deg, Ucur, Uprev, Y,
                       bw->ctrl, bw->part, bw->ldp, bw->grid_short, active);
}

template <typename VT, int B, bool GRAD>
static void launch_first(rd_graph g, BatchWork *bw, VT *W, const RunParams &prm, hipStream_t st) {
  const int32_t *active = bw->qstate + 1;
  const bool s2 = prm.s2;
  hipLaunchKernelGGL((k_first_batch<VT, B, GRAD>), dim3(B), dim3(256), 0, st, g->row_ptr, g->col,
                     (const double *)g->w64, g->deg, W, bw->st, bw->ctrl, (VT *)bw->P, (VT *)bw->Xp,
                     active, s2 ? 1 : 0, prm.s2_ecap, bw->s2_lcap, bw->s2_lu, bw->s2_lw, bw->s2_lp, bw->s2c,
                     bw->s2_pslot, bw->s2_pcap);
  if (!s2) return;
  const int32_t grid = 2048;  // 8192 wavefronts over the row pieces
  if (g->unit)
    hipLaunchKernelGGL(k_s2_scatter<false>, dim3(grid), dim3(256), 0, st, B, g->n,
                       (const S2Col *)bw->s2c, bw->s2_lcap, bw->s2_pcap,
                       (const int32_t *)bw->s2_pslot, (const int32_t *)bw->s2_lu, (const double *)bw->s2_lw,
                       (const int64_t *)bw->s2_lp,
                       g->row_ptr, g->col, (const double *)nullptr, g->deg, bw->s2_acc, bw->s2_own, active);
  else
    hipLaunchKernelGGL(k_s2_scatter<true>, dim3(grid), dim3(256), 0, st, B, g->n,
                       (const S2Col *)bw->s2c, bw->s2_lcap, bw->s2_pcap,
                       (const int32_t *)bw->s2_pslot, (const int32_t *)bw->s2_lu, (const double *)bw->s2_lw,
                       (const int64_t *)bw->s2_lp,
                       g->row_ptr, g->col, (const double *)g->w64, g->deg, bw->s2_acc, bw->s2_own, active);
  hipLaunchKernelGGL(k_s2_alpha, dim3(B), dim3(256), 0, st, g->n, bw->s2c, bw->s2_lcap,
                     (const int32_t *)bw->s2_lu, (const double *)bw->s2_lw, g->deg,
                     (const unsigned long long *)bw->s2_acc, bw->st, active);
  hipLaunchKernelGGL((k_s2_write<VT, B>), dim3(grid), dim3(256), 0, st, g->n, bw->s2c, bw->s2_lcap,
                     bw->s2_pcap, (const int32_t *)bw->s2_pslot,
                     (const int32_t *)bw->s2_lu, (const int64_t *)bw->s2_lp, g->row_ptr, g->col, g->deg,
                     bw->s2_acc, (const unsigned long long *)bw->s2_own, (const LzState *)bw->st, W, active);
  hipLaunchKernelGGL((k_s2_fix<VT, B, GRAD>), dim3(B), dim3(256), 0, st, bw->s2c, bw->s2_lcap,
                     (const int32_t *)bw->s2_lu, (const double *)bw->s2_lw, g->deg, (const LzState *)bw->st,
                     W, (VT *)bw->P, (VT *)bw->Xp, active);
  hipLaunchKernelGGL(k_s2_beta, dim3(1), dim3(256), 0, st, B, bw->s2c, bw->st, bw->ctrl, active);
}

// The sparse second iteration of a single-pair run, one column of the batched
// machinery: U1 holds w_1 (zero off S), U2 (zero) receives w_2, st is the
// run's state after iteration 1. Enqueued on the stream; the step was taken
// when the state then shows k = 2.
template <typename VT>
static void single_second_t(rd_graph g, BatchWork *bw, const VT *U1, VT *U2, LzState *st, int64_t ecap,
                            hipStream_t stream) {
  const int32_t *one = bw->qstate + 3;
  const int32_t grid = 256;
  hipLaunchKernelGGL(k_s2_list_single<VT>, dim3(1), dim3(256), 0, stream, g->row_ptr, g->col, U1,
                     (const LzState *)st, ecap, bw->s2_lcap, bw->s2_lu, bw->s2_lw, bw->s2_lp, bw->s2c,
                     bw->s2_pslot);
  if (g->unit)
    hipLaunchKernelGGL(k_s2_scatter<false>, dim3(grid), dim3(256), 0, stream, 1, g->n, (const S2Col *)bw->s2c,
                       bw->s2_lcap, bw->s2_pcap, (const int32_t *)bw->s2_pslot, (const int32_t *)bw->s2_lu,
                       (const double *)bw->s2_lw, (const int64_t *)bw->s2_lp, g->row_ptr, g->col,
                       (const double *)nullptr, g->deg, bw->s2_acc, bw->s2_own, one);
  else
    hipLaunchKernelGGL(k_s2_scatter<true>, dim3(grid), dim3(256), 0, stream, 1, g->n, (const S2Col *)bw->s2c,
                       bw->s2_lcap, bw->s2_pcap, (const int32_t *)bw->s2_pslot, (const int32_t *)bw->s2_lu,
                       (const double *)bw->s2_lw, (const int64_t *)bw->s2_lp, g->row_ptr, g->col,
                       (const double *)g->w64, g->deg, bw->s2_acc, bw->s2_own, one);
  hipLaunchKernelGGL(k_s2_alpha, dim3(1), dim3(256), 0, stream, g->n, bw->s2c, bw->s2_lcap,
                     (const int32_t *)bw->s2_lu, (const double *)bw->s2_lw, g->deg,
                     (const unsigned long long *)bw->s2_acc, st, one);
  hipLaunchKernelGGL((k_s2_write<VT, 1>), dim3(grid), dim3(256), 0, stream, g->n, bw->s2c, bw->s2_lcap,
                     bw->s2_pcap, (const int32_t *)bw->s2_pslot, (const int32_t *)bw->s2_lu,
                     (const int64_t *)bw->s2_lp, g->row_ptr, g->col, g->deg, bw->s2_acc,
                     (const unsigned long long *)bw->s2_own, (const LzState *)st, U2, one);
  hipLaunchKernelGGL((k_s2_fix<VT, 1, false>), dim3(1), dim3(256), 0, stream, bw->s2c, bw->s2_lcap,
                     (const int32_t *)bw->s2_lu, (const double *)bw->s2_lw, g->deg, (const LzState *)st, U2,
                     (VT *)nullptr, (VT *)nullptr, one);
  // the column record's scales go to a spare control slot; the single-pair
  // kernels read theirs from the state
  hipLaunchKernelGGL(k_s2_beta, dim3(1), dim3(256), 0, stream, 1, bw->s2c, st, bw->ctrl, one);
}

bool sparse_second_single(rd_graph g, int32_t precision, void *U1, void *U2, LzState *st, hipStream_t stream) {
  BatchWork *bw = batch_get(g);
  if (!s2_reserve(g, bw, 1, stream)) return false;
  // one column: the step pays while its scatter costs less than one dense
  // single-pair iteration, which gathers nnz vector entries (8-byte gathers
  // pulling whole lines): taken as nnz / 64 entries
  const int64_t ecap = std::max<int64_t>(1, std::min<int64_t>(g->nnz / 64, g->nnz * 8 / 128));
  if (precision == RD_F64)
    single_second_t<double>(g, bw, (const double *)U1, (double *)U2, st, ecap, stream);
  else
    single_second_t<float>(g, bw, (const float *)U1, (float *)U2, st, ecap, stream);
  RD_HIP(hipGetLastError());
  return true;
}

// What a full block of harvested potentials gives besides the edge gradient:
// the potentials themselves (column sums, then the copy-out of the slots in
// use) and/or the FP64 energy of each one (r rewritten as J(phi)). gated: only
// when the block is full (the flag is set first); otherwise active is the
// constant 1 (the last, partly filled block).
template <typename VT, int B>
static void launch_block_out(rd_graph g, BatchWork *bw, const RunParams &prm, const int32_t *ps,
                             const int32_t *pt, rd_result *out, bool gated, hipStream_t st) {
  const int32_t *active = bw->qstate + 3;
  if (gated) {
    hipLaunchKernelGGL(k_full_flag, dim3(1), dim3(64), 0, st, B, (const int32_t *)bw->qstate, bw->pflag);
    active = bw->pflag;
  }
  if (prm.phi) {
    hipLaunchKernelGGL((k_col_reduce<VT, B>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->n,
                       (const VT *)bw->Xf, bw->ppart, bw->ppart_ld, active);
    hipLaunchKernelGGL(k_col_sum, dim3(B), dim3(COL_THREADS), 0, st, (const double *)bw->ppart,
                       bw->ppart_ld, bw->grid_upd, bw->psum, active);
    hipLaunchKernelGGL((k_pot_out<VT, B>), dim3(std::min<int64_t>(cdiv(g->n, 64) * (B < 64 ? 1 : B / 64), 4096)),
                       dim3(256), 0, st, g->n,
                       (const int32_t *)g->perm, (const int32_t *)prm.slot_pair, (const double *)bw->cw,
                       (const VT *)bw->Xf, (const double *)bw->psum, prm.phi, active);
  }
  if (prm.refine) {
    if (g->unit)
      hipLaunchKernelGGL((k_energy<VT, B, false>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->nch,
                         (const int4 *)g->echunk, g->col, (const double *)nullptr, (const VT *)bw->Xf,
                         bw->ppart, bw->ppart_ld, active);
    else
      hipLaunchKernelGGL((k_energy<VT, B, true>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->nch,
                         (const int4 *)g->echunk, g->col, (const double *)g->w64, (const VT *)bw->Xf,
                         bw->ppart, bw->ppart_ld, active);
    hipLaunchKernelGGL(k_col_sum, dim3(B), dim3(COL_THREADS), 0, st, (const double *)bw->ppart,
                       bw->ppart_ld, bw->grid_upd, bw->psum, active);
    hipLaunchKernelGGL((k_refine_out<VT, B>), dim3(1), dim3(256), 0, st, (const int32_t *)prm.slot_pair, ps, pt,
                       (const double *)bw->cw, (const VT *)bw->Xf, (const double *)bw->psum, out, active);
  }
}

// The three vector blocks of a run: q_{i-1}, q_i and the block the next
// product writes (they rotate every iteration).
struct RunBufs {
  void *prv, *cur, *nxt;
  void rotate() {
    void *old = prv;
    prv = cur;
    cur = nxt;
    nxt = old;
  }
};

template <typename VT, int B, bool GRAD>
static void enqueue_batch_iteration(rd_graph g, BatchWork *bw, const RunBufs &rb,
                                    const RunParams &prm, const int32_t *ps, const int32_t *pt,
                                    rd_result *out, hipStream_t st, bool prof) {
  const VT *Ucur = (const VT *)rb.cur;
  const VT *Uprev = (const VT *)rb.prv;
  VT *Y = (VT *)rb.nxt;
  const int32_t *active = bw->qstate + 1;
  if (g->unit)
    launch_spmm<VT, B, false>(g, bw, Ucur, Uprev, Y, st, active, prof);
  else
    launch_spmm<VT, B, true>(g, bw, Ucur, Uprev, Y, st, active, prof);
  int32_t np = bw->grid_short + bw->nlong;
  if (prm.s2) {
    hipLaunchKernelGGL((k_s2_prev<VT, B>), dim3(B), dim3(256), 0, st, (const S2Col *)bw->s2c, bw->s2_lcap,
                       (const int32_t *)bw->s2_lu, (const double *)bw->s2_lw, g->deg, Ucur, Y, bw->ctrl,
                       bw->part, bw->ldp, np, active);
    np += 1;
  }
  hipLaunchKernelGGL(k_col_sum, dim3(B), dim3(COL_THREADS), 0, st, bw->part, bw->ldp, np, bw->colsum,
                     active);
  hipLaunchKernelGGL(k_control, dim3(1), dim3(256), 0, st, B, bw->st, bw->ctrl,
                     (const double *)bw->colsum, prm, ps, pt, g->deg, out, bw->qstate, prm.gmode,
                     prm.grad_r, bw->cw);
  if (prm.reorth > 0)
    hipLaunchKernelGGL((k_update<VT, B, GRAD, true>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->n,
                       g->deg, Ucur, Uprev, Y, bw->ctrl, bw->part, bw->ldp, active, (VT *)bw->P,
                       (VT *)bw->Xp, prm.reorth, bw->rpart, (VT *)bw->Xf);
  else
    hipLaunchKernelGGL((k_update<VT, B, GRAD, false>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->n,
                       g->deg, Ucur, Uprev, Y, bw->ctrl, bw->part, bw->ldp, active, (VT *)bw->P,
                       (VT *)bw->Xp, 0, bw->rpart, (VT *)bw->Xf);
  if (prm.gmode == GRAD_HARVEST) {
    // a full block of harvested potentials: its edge pass (or, for potentials,
    // its copy-out), then the slots are free
    if (prm.slot_pair)
      launch_block_out<VT, B>(g, bw, prm, ps, pt, out, true, st);
    else
      hipLaunchKernelGGL((k_grad_edges<VT, B>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->nch,
                         (const int4 *)g->echunk, g->col, (const VT *)bw->Xf, (const double *)bw->cw, bw->gacc,
                         (const int32_t *)(bw->qstate + 4));
    hipLaunchKernelGGL(k_harvest_reset, dim3(1), dim3(256), 0, st, B, bw->qstate, bw->cw, prm.slot_pair);
  }
  if (prm.reorth > 0) {
    // column sums of the three coefficient slabs (rpart holds [3][B][ldp])
    hipLaunchKernelGGL(k_col_sum, dim3(3 * B), dim3(COL_THREADS), 0, st, bw->rpart, bw->ldp,
                       bw->grid_upd, bw->rsum, active);
    hipLaunchKernelGGL(k_reorth_coef, dim3(1), dim3(256), 0, st, B, prm.reorth, g->vol,
                       (const double *)bw->rsum, (const LzState *)bw->st, bw->ctrl, active);
    hipLaunchKernelGGL((k_reorth_apply<VT, B>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->n,
                       g->deg, Ucur, Uprev, Y, (const ColCtrl *)bw->ctrl, bw->part, bw->ldp, active,
                       prm.reorth);
  }
  hipLaunchKernelGGL(k_beta, dim3(B), dim3(COL_THREADS), 0, st, bw->part, bw->ldp, bw->grid_upd,
                     bw->st, bw->ctrl, active);
  launch_first<VT, B, GRAD>(g, bw, Y, prm, st);
}

// Tail compaction: the running columns of a B-wide run (their q_i and q_{i-1}
// and their state) move to columns 0..count-1 of a B/2-wide run, the other
// columns of which are idle. map[c] is the source column of column c (-1: none),
// increasing in c, so map[c] >= c.
template <typename VT, int B>
__global__ void k_compact_vectors(int32_t n, const int32_t *__restrict__ map,
                                  const VT *__restrict__ cur, const VT *__restrict__ prv,
                                  VT *__restrict__ cur2, VT *__restrict__ prv2) {
  constexpr int H = B / 2;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * H) return;
  const int64_t r = i / H;
  const int c = (int)(i - r * H);
  const int src = map[c];
  cur2[i] = src >= 0 ? cur[r * B + src] : VT(0);
  prv2[i] = src >= 0 ? prv[r * B + src] : VT(0);
}

// In place, by one thread in increasing column order (map[c] >= c, so no
// source is overwritten before it is read).
__global__ void k_compact_state(int32_t H, const int32_t *__restrict__ map, LzState *__restrict__ st,
                                ColCtrl *__restrict__ ctrl) {
  if (threadIdx.x != 0) return;
  for (int c = 0; c < H; ++c) {
    const int src = map[c];
    if (src >= 0) {
      if (src != c) {
        st[c] = st[src];
        ctrl[c] = ctrl[src];
      }
    } else {
      LzState S = st[c];
      S.status = LZ_IDLE;
      S.pair = -1;
      st[c] = S;
      ColCtrl cc = ctrl[c];
      cc.mode = COL_IDLE;
      cc.sig = cc.pc = cc.coef = 0.0;
      cc.prev_sparse = cc.upd_sparse = 0;
      ctrl[c] = cc;
    }
  }
}

// Iterate a B-wide run until every column has stopped. Iterations are
// enqueued in growing chunks and the host reads the queue state in between.
// Once the pair queue is empty and at most half of the columns still run, the
// run continues at half the width (compact_ok, down to 16 columns).
// Returns the number of iterations enqueued.
template <typename VT, int B, bool GRAD>
static int64_t batch_loop(rd_graph g, BatchWork *bw, RunBufs rb, int32_t npairs, const int32_t *ps,
                          const int32_t *pt, const RunParams &prm, rd_result *out, hipStream_t st,
                          bool prof, bool compact_ok, int64_t iters, int64_t cap) {
  int chunk = 4;
  for (;;) {
    for (int j = 0; j < chunk; ++j) {
      enqueue_batch_iteration<VT, B, GRAD>(g, bw, rb, prm, ps, pt, out, st, prof);
      rb.rotate();
    }
    iters += chunk;
    RD_HIP(hipGetLastError());
    RD_HIP(hipMemcpyAsync(bw->qstate_host, bw->qstate, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    if (bw->qstate_host[1] == 0) return iters;
    RD_REQUIRE(iters < cap, "batched run did not drain (internal error)");
    if constexpr (B > 16) {
      if (compact_ok && bw->qstate_host[0] >= npairs && bw->qstate_host[1] <= B / 2) {
        constexpr int H = B / 2;
        std::vector<ColCtrl> cc(B);
        RD_HIP(hipMemcpyAsync(cc.data(), bw->ctrl, B * sizeof(ColCtrl), hipMemcpyDeviceToHost, st));
        RD_HIP(hipStreamSynchronize(st));
        int32_t map[256];
        int count = 0;
        for (int c = 0; c < B; ++c)
          if (cc[c].mode == COL_RUN) map[count++] = c;
        RD_REQUIRE(count <= H, "compaction: more running columns than the narrower block holds");
        for (int c = count; c < H; ++c) map[c] = -1;
        RD_HIP(hipMemcpyAsync(bw->cmap, map, H * sizeof(int32_t), hipMemcpyHostToDevice, st));
        // q_i and q_{i-1} go to the two halves of the free block; the old q_i
        // block becomes the next product's output
        VT *cur2 = (VT *)rb.nxt;
        VT *prv2 = cur2 + (size_t)g->n * H;
        hipLaunchKernelGGL((k_compact_vectors<VT, B>), dim3(cdiv((int64_t)g->n * H, 256)), dim3(256), 0,
                           st, g->n, (const int32_t *)bw->cmap, (const VT *)rb.cur, (const VT *)rb.prv,
                           cur2, prv2);
        hipLaunchKernelGGL(k_compact_state, dim3(1), dim3(64), 0, st, H, (const int32_t *)bw->cmap,
                           bw->st, bw->ctrl);
        RD_HIP(hipGetLastError());
        RunBufs nb{prv2, cur2, rb.cur};
        return batch_loop<VT, H, GRAD>(g, bw, nb, npairs, ps, pt, prm, out, st, prof, compact_ok, iters,
                                       cap);
      }
    }
    // once every pair has started, look at the state more often so the tail
    // is caught while it can still be narrowed
    const bool tail = compact_ok && B > 16 && bw->qstate_host[0] >= npairs;
    chunk = std::min(chunk * 2, tail ? 8 : 64);
  }
}

// Run all pairs through B slots. Returns the number of iterations enqueued.
// GRAD: npairs <= B (no refill) and the potentials of the B runs are
// accumulated in bw->Xp (bw->P, bw->Xp zeroed by the caller); no compaction.
template <typename VT, int B, bool GRAD = false>
static int64_t batch_run_t(rd_graph g, BatchWork *bw, int32_t npairs, const int32_t *ps,
                           const int32_t *pt, const RunParams &prm_in, rd_result *out, hipStream_t st,
                           bool prof, bool compact_ok = false) {
  batch_reserve(g, bw, B, sizeof(VT));
  RunParams prm = prm_in;
  if (prm.reorth > 0) reorth_reserve(bw);
  // sparse second steps (not with re-orthogonalisation or potentials) for
  // columns whose scatter costs less than the dense iteration it replaces:
  // the autotuned product time per column (times 1.15 for the update and
  // reductions around it) over the cost of one scatter entry, else
  // nnz * size / 256 entries (the two measured optima were nnz * 4 / 512 for
  // a power-law graph in FP32 and nnz * 8 / 128 for another in FP64)
  prm.s2 = prm.s2 && prm.reorth == 0 && s2_reserve(g, bw, B, st);
  const int pi = sizeof(VT) == 8 ? RD_F64 : RD_F32;
  if (bw->tuned[pi] == B && bw->tuned_col_ms[pi] > 0.0)
    prm.s2_ecap = (int64_t)(bw->tuned_col_ms[pi] * 1.15 * 1e6 / S2_ENTRY_NS);
  else
    prm.s2_ecap = g->nnz * (int64_t)sizeof(VT) / 256;
  prm.s2_ecap = std::min<int64_t>(std::max<int64_t>(prm.s2_ecap, 1), g->nnz * 8 / 128);
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, st, B, bw->st, bw->ctrl, bw->qstate,
                     bw->s2c);
  // fill the slots: control with every column idle pops the first B pairs,
  // then the update writes their start vectors (and zeros elsewhere)
  hipLaunchKernelGGL(k_control, dim3(1), dim3(256), 0, st, B, bw->st, bw->ctrl,
                     (const double *)bw->colsum, prm, ps, pt, g->deg, out, bw->qstate, prm.gmode,
                     prm.grad_r, bw->cw);
  hipLaunchKernelGGL((k_update<VT, B, false, false>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->n,
                     g->deg, (const VT *)bw->X[1], (const VT *)bw->X[2], (VT *)bw->X[0], bw->ctrl,
                     bw->part, bw->ldp, bw->qstate + 1, (VT *)nullptr, (VT *)nullptr, 0,
                     (double *)nullptr, (VT *)nullptr);
  launch_first<VT, B, GRAD>(g, bw, (VT *)bw->X[0], prm, st);
  RD_HIP(hipGetLastError());
  // every column starts from the sparse q_1, so the first product reads no
  // previous vector; X[0] holds w_1
  const RunBufs rb{bw->X[1], bw->X[0], bw->X[2]};
  const int64_t cap = (int64_t)prm.max_iters * ((npairs + B - 1) / B + 1) + 16;
  const int64_t iters =
      batch_loop<VT, B, GRAD>(g, bw, rb, npairs, ps, pt, prm, out, st, prof, compact_ok && !GRAD, 0, cap);
  // sparse products enqueued after the last active iteration returned at once
  if (prof) g->timer[0].resolve((size_t)bw->qstate_host[2]);
  return iters;
}

template <typename VT>
static int64_t batch_dispatch(rd_graph g, BatchWork *bw, int32_t B, int32_t npairs, const int32_t *ps,
                              const int32_t *pt, const RunParams &prm, rd_result *out, hipStream_t st,
                              bool prof, bool compact) {
  switch (B) {
    case 16: return batch_run_t<VT, 16>(g, bw, npairs, ps, pt, prm, out, st, prof, compact);
    case 32: return batch_run_t<VT, 32>(g, bw, npairs, ps, pt, prm, out, st, prof, compact);
    case 64: return batch_run_t<VT, 64>(g, bw, npairs, ps, pt, prm, out, st, prof, compact);
    case 128: return batch_run_t<VT, 128>(g, bw, npairs, ps, pt, prm, out, st, prof, compact);
    case 256: return batch_run_t<VT, 256>(g, bw, npairs, ps, pt, prm, out, st, prof, compact);
  }
  throw RdError{RD_E_ARG, "block_width must be one of 16, 32, 64, 128, 256"};
}

// Edge gradient of sum_p grad_r[p] r(s_p, t_p) (grad_w != nullptr): one run
// over all pairs with refill. Potentials are accumulated during each pair's
// run; a finished potential is copied to a slot of the harvest block Xf and
// the column is refilled; every full block of B harvested potentials gets one
// edge pass into the FP64 accumulator, and the last, partly filled block one
// more at the end.
// grad_w == nullptr, phi != nullptr: the same run; each block's potentials are
// copied out (mean removed, caller's node order) instead of the edge pass.
// grad_w == nullptr, phi == nullptr: refinement; each block's potentials give
// their pairs r = J(phi), the FP64 energy, in place of r_hat.
template <typename VT, int B>
static void grad_run_t(rd_graph g, BatchWork *bw, int32_t npairs, const int32_t *ps,
                       const int32_t *pt, const double *grad_r, const RunParams &prm0,
                       rd_result *out, float *grad_w, hipStream_t st, bool prof, double *phi = nullptr) {
  // all three modes run with refill and harvest finished potentials into
  // blocks: the edge gradient, the potentials' copy-out, or the energies (refine)
  const bool pots = phi != nullptr;
  const bool refine = grad_w == nullptr && !pots;
  const bool grad = grad_w != nullptr;
  batch_reserve(g, bw, B, sizeof(VT));
  const size_t need = (size_t)g->n * B * sizeof(VT);  // potentials stored like the vectors
  if (need > bw->pot_bytes) {
    dev_free(bw->P);
    dev_free(bw->Xp);
    dev_free(bw->Xf);
    bw->P = bw->Xp = bw->Xf = nullptr;
    bw->pot_bytes = 0;
    bw->P = dev_alloc(need);
    bw->Xp = dev_alloc(need);
    bw->pot_bytes = need;
  }
  if (!bw->Xf) bw->Xf = dev_alloc(bw->pot_bytes);
  if (grad && !bw->gacc) bw->gacc = (double *)dev_alloc((size_t)g->nnz * sizeof(double));
  if (!grad && (!bw->ppart || bw->ppart_ld < bw->grid_upd)) {
    dev_free(bw->ppart);
    bw->ppart = nullptr;
    bw->ppart = (double *)dev_alloc((size_t)256 * bw->grid_upd * sizeof(double));
    bw->ppart_ld = bw->grid_upd;
  }
  if (!grad && !bw->psum) bw->psum = (double *)dev_alloc(256 * sizeof(double));
  if (!grad && !bw->spair) bw->spair = (int32_t *)dev_alloc(256 * sizeof(int32_t));
  if (!grad && !bw->pflag) bw->pflag = (int32_t *)dev_alloc(sizeof(int32_t));
  if (!bw->cw) bw->cw = (double *)dev_alloc(256 * sizeof(double));
  edge_chunks(g, st);
  {
    if (grad) RD_HIP(hipMemsetAsync(bw->gacc, 0, (size_t)g->nnz * sizeof(double), st));
    RD_HIP(hipMemsetAsync(bw->P, 0, need, st));
    RD_HIP(hipMemsetAsync(bw->Xp, 0, need, st));
    RD_HIP(hipMemsetAsync(bw->Xf, 0, need, st));
    RD_HIP(hipMemsetAsync(bw->cw, 0, 256 * sizeof(double), st));
    RunParams prm = prm0;
    prm.gmode = GRAD_HARVEST;
    prm.grad_r = grad_r;
    if (!grad) {
      RD_HIP(hipMemsetAsync(bw->spair, 0xff, 256 * sizeof(int32_t), st));  // -1: no pair
      prm.slot_pair = bw->spair;
      prm.phi = phi;
      prm.refine = refine ? 1 : 0;
    }
    if (npairs > 0) batch_run_t<VT, B, true>(g, bw, npairs, ps, pt, prm, out, st, prof);
    if (!grad) {
      // the last, partly filled block (unused slots hold no pair)
      launch_block_out<VT, B>(g, bw, prm, ps, pt, out, false, st);
      RD_HIP(hipGetLastError());
      return;
    }
    // the last, partly filled harvest block (unused slots have weight zero)
    std::pair<hipEvent_t, hipEvent_t> ev{};
    if (prof) {
      // chunks, column ids of the upper entries, the accumulator read and
      // written, the potential block read once
      ev = g->timer[2].next(16.0 * g->nch + 4.0 * (double)g->m + 16.0 * (double)g->m +
                            (double)sizeof(VT) * B * (double)g->n + 8.0 * B);
      RD_HIP(hipEventRecord(ev.first, st));
    }
    hipLaunchKernelGGL((k_grad_edges<VT, B>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->nch,
                       (const int4 *)g->echunk, g->col, (const VT *)bw->Xf, (const double *)bw->cw, bw->gacc,
                       (const int32_t *)nullptr);
    if (prof) RD_HIP(hipEventRecord(ev.second, st));
    hipLaunchKernelGGL(k_gacc_out, dim3(cdiv(g->nch, 256)), dim3(256), 0, st, g->nch, (const int4 *)g->echunk,
                       g->eid, (const double *)bw->gacc, grad_w);
    RD_HIP(hipGetLastError());
    if (prof) {
      RD_HIP(hipStreamSynchronize(st));
      g->timer[2].resolve(g->timer[2].used);
    }
    return;
  }
}

template <typename VT>
static void grad_dispatch(rd_graph g, BatchWork *bw, int32_t B, int32_t npairs, const int32_t *ps,
                          const int32_t *pt, const double *grad_r, const RunParams &prm,
                          rd_result *out, float *grad_w, hipStream_t st, bool prof,
                          double *phi = nullptr) {
  switch (B) {
    case 16: return grad_run_t<VT, 16>(g, bw, npairs, ps, pt, grad_r, prm, out, grad_w, st, prof, phi);
    case 32: return grad_run_t<VT, 32>(g, bw, npairs, ps, pt, grad_r, prm, out, grad_w, st, prof, phi);
    case 64: return grad_run_t<VT, 64>(g, bw, npairs, ps, pt, grad_r, prm, out, grad_w, st, prof, phi);
    case 128: return grad_run_t<VT, 128>(g, bw, npairs, ps, pt, grad_r, prm, out, grad_w, st, prof, phi);
    case 256: return grad_run_t<VT, 256>(g, bw, npairs, ps, pt, grad_r, prm, out, grad_w, st, prof, phi);
  }
  throw RdError{RD_E_ARG, "block_width must be one of 16, 32, 64, 128, 256"};
}

// Time of one sparse product at width B (vectors of arbitrary content).
template <typename VT, int B>
static float probe_spmm(rd_graph g, BatchWork *bw, hipStream_t st) {
  batch_reserve(g, bw, B, sizeof(VT));
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(256), 0, st, B, bw->st, bw->ctrl, bw->qstate,
                     bw->s2c);
  hipLaunchKernelGGL((k_update<VT, B, false, false>), dim3(bw->grid_upd), dim3(SHORT_THREADS), 0, st, g->n,
                     g->deg, (const VT *)bw->X[1], (const VT *)bw->X[2], (VT *)bw->X[0], bw->ctrl,
                     bw->part, bw->ldp, bw->qstate + 3, (VT *)nullptr, (VT *)nullptr, 0,
                     (double *)nullptr, (VT *)nullptr);
  constexpr int NT = 5;
  hipEvent_t ev[NT + 1];
  for (hipEvent_t &e : ev) RD_HIP(hipEventCreate(&e));
  auto once = [&]() {
    if (g->unit)
      launch_spmm<VT, B, false>(g, bw, (const VT *)bw->X[0], (const VT *)bw->X[2], (VT *)bw->X[1], st,
                                bw->qstate + 3);
    else
      launch_spmm<VT, B, true>(g, bw, (const VT *)bw->X[0], (const VT *)bw->X[2], (VT *)bw->X[1], st,
                               bw->qstate + 3);
  };
  once();
  RD_HIP(hipEventRecord(ev[0], st));
  for (int k = 0; k < NT; ++k) {
    once();
    RD_HIP(hipEventRecord(ev[k + 1], st));
  }
  RD_HIP(hipEventSynchronize(ev[NT]));
  // the fastest of the products: the least disturbed by other work on the chip
  float best = 1e30f;
  for (int k = 0; k < NT; ++k) {
    float ms = 0.f;
    RD_HIP(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
    best = std::min(best, ms);
  }
  for (hipEvent_t &e : ev) (void)hipEventDestroy(e);
  return best;
}

template <typename VT>
static float probe_dispatch(rd_graph g, BatchWork *bw, int32_t B, hipStream_t st) {
  switch (B) {
    case 16: return probe_spmm<VT, 16>(g, bw, st);
    case 32: return probe_spmm<VT, 32>(g, bw, st);
    case 64: return probe_spmm<VT, 64>(g, bw, st);
    case 128: return probe_spmm<VT, 128>(g, bw, st);
    case 256: return probe_spmm<VT, 256>(g, bw, st);
  }
  return 1e30f;
}

static std::string tune_key(rd_graph g, int prec) {
  std::ostringstream k;
  k << "n=" << g->n << ",nnz=" << g->nnz << ",maxdeg=" << g->max_deg << ",w=" << (g->unit ? 0 : 1)
    << ",prec=" << prec;
  return k.str();
}

// Block width and row-bin schedule with the least sparse-product time per
// column: first the width (candidates that fit the number of pairs) under the
// default schedule, then the schedule at that width (entries per wave work
// item 128/256/512, long-row threshold 512/1024/2048). Remembered per handle
// and precision and, when the environment variable RD_AUTOTUNE_CACHE names a
// file, read from and appended to that file. Leaves the chosen schedule
// built; returns the width.
static int32_t autotune_width(rd_graph g, BatchWork *bw, int prec, int32_t npairs, hipStream_t st) {
  auto valid_width = [](int32_t B) { return B == 16 || B == 32 || B == 64 || B == 128 || B == 256; };
  if (!bw->tuned[prec]) {
    const char *path = std::getenv("RD_AUTOTUNE_CACHE");
    const std::string key = tune_key(g, prec);
    if (path) {
      std::ifstream f(path);
      std::string line;
      while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string k;
        int32_t B = 0, wv = 0, ld = 0;
        double cm = 0.0;
        if ((in >> k >> B >> wv >> ld) && k == key && valid_width(B) && wv >= 32 && ld >= 64) {
          if (!(in >> cm) || !(cm > 0.0)) cm = 0.0;  // optional fifth field
          bw->tuned[prec] = B;
          bw->tuned_wave[prec] = wv;
          bw->tuned_long[prec] = ld;
          bw->tuned_col_ms[prec] = cm;
        }
      }
    }
    if (!bw->tuned[prec]) {
      auto probe = [&](int32_t B) {
        return prec == RD_F64 ? probe_dispatch<double>(g, bw, B, st) : probe_dispatch<float>(g, bw, B, st);
      };
      build_schedule(g, bw, WAVE_NNZ, LONG_DEG);
      int32_t best = 0;
      double best_t = 1e300;
      for (int32_t B : {32, 64, 128, 256}) {
        if (B > 32 && B / 2 >= npairs) break;  // wider than the work: no gain
        const double per_col = probe(B) / B;
        // a wider block must be faster per column by more than the probe's
        // noise: it also leaves a longer tail of idle columns
        if (per_col < best_t * 0.98) {
          best_t = per_col;
          best = B;
        }
      }
      int32_t best_wave = WAVE_NNZ, best_long = LONG_DEG;
      double best_s = probe(best);  // the default schedule, measured again next to the others
      for (int32_t wv : {128, 256, 512}) {
        for (int32_t ld : {512, 1024, 2048}) {
          if (wv == WAVE_NNZ && ld == LONG_DEG) continue;
          build_schedule(g, bw, wv, ld);
          const double t = probe(best);
          if (t < best_s) {
            best_s = t;
            best_wave = wv;
            best_long = ld;
          }
        }
      }
      bw->tuned[prec] = best;
      bw->tuned_wave[prec] = best_wave;
      bw->tuned_long[prec] = best_long;
      bw->tuned_col_ms[prec] = best_s / best;
      if (path) {
        std::ofstream f(path, std::ios::app);
        f << key << " " << best << " " << best_wave << " " << best_long << " " << bw->tuned_col_ms[prec]
          << "\n";
      }
    }
  }
  build_schedule(g, bw, bw->tuned_wave[prec], bw->tuned_long[prec]);
  return bw->tuned[prec];
}

// ---------------------------------------------------------------------------
// Power Method (Algorithm 1) for B pairs at a time on the batched product.
// With x = D^{-1} r, the lazy step r <- (I/2 + P/2) r with P = A D^{-1} reads
// x <- x/2 + D^{-1} A x / 2: the product kernels with column scale 1/2 and
// coefficient -1/2 on the previous-vector operand, which is x itself. Before
// each step the sum takes r(s)/(2 d_s) - r(t)/(2 d_t) = (x(s) - x(t)) / 2.

// Column controls, sums and start vectors x_0 = e_s / d_s - e_t / d_t of one
// group (X zeroed before; columns >= cnt stay zero).
template <typename VT, int B>
__global__ void k_pm_init(int32_t cnt, const int32_t *__restrict__ ps, const int32_t *__restrict__ pt,
                          const double *__restrict__ deg, ColCtrl *__restrict__ ctrl, VT *__restrict__ X,
                          double *__restrict__ sums) {
  const int j = threadIdx.x;
  if (j >= B) return;
  ColCtrl c{};
  c.sig = 0.5;
  c.pc = -0.5;
  c.hslot = -1;
  ctrl[j] = c;
  sums[j] = 0.0;
  sums[B + j] = 0.0;
  if (j < cnt) {
    const int32_t s = ps[j], t = pt[j];
    X[(size_t)s * B + j] = (VT)(1.0 / deg[s]);
    X[(size_t)t * B + j] -= (VT)(1.0 / deg[t]);  // s == t leaves zero
  }
}

// sums[j] += (x(s_j) - x(t_j)) / 2 in FP64; sums[B + j] keeps the last term.
template <typename VT, int B>
__global__ void k_pm_acc(int32_t cnt, const int32_t *__restrict__ ps, const int32_t *__restrict__ pt,
                         const VT *__restrict__ X, double *__restrict__ sums) {
  const int j = threadIdx.x;
  if (j >= cnt) return;
  const double term = 0.5 * ((double)X[(size_t)ps[j] * B + j] - (double)X[(size_t)pt[j] * B + j]);
  sums[j] += term;
  sums[B + j] = term;
}

template <int B>
__global__ void k_pm_out(int32_t cnt, int32_t l, const double *__restrict__ sums, rd_result *__restrict__ out) {
  const int j = threadIdx.x;
  if (j >= cnt) return;
  rd_result r;
  r.r = sums[j];
  r.err_est = sums[B + j];
  r.iters = l;
  r.status = RD_OK;
  out[j] = r;
}

template <typename VT, int B>
static void pm_run_t(rd_graph g, BatchWork *bw, int32_t npairs, const int32_t *ps, const int32_t *pt,
                     int32_t l, rd_result *out, double *sums, hipStream_t st, bool prof) {
  batch_reserve(g, bw, B, sizeof(VT));
  const size_t bytes = (size_t)g->n * B * sizeof(VT);
  const int32_t *gate = bw->qstate + 3;  // the constant 1
  constexpr int32_t PROF_STEPS = 64;    // products timed per group under RD_PROFILE
  for (int32_t p0 = 0; p0 < npairs; p0 += B) {
    const int32_t cnt = std::min<int32_t>(B, npairs - p0);
    VT *cur = (VT *)bw->X[0], *nxt = (VT *)bw->X[1];
    RD_HIP(hipMemsetAsync(cur, 0, bytes, st));
    hipLaunchKernelGGL((k_pm_init<VT, B>), dim3(1), dim3(256), 0, st, cnt, ps + p0, pt + p0, g->deg,
                       bw->ctrl, cur, sums);
    for (int32_t i = 0;; ++i) {
      hipLaunchKernelGGL((k_pm_acc<VT, B>), dim3(1), dim3(256), 0, st, cnt, ps + p0, pt + p0,
                         (const VT *)cur, sums);
      if (i == l) break;
      const bool tm = prof && i < PROF_STEPS;
      if (g->unit)
        launch_spmm<VT, B, false>(g, bw, cur, cur, nxt, st, gate, tm);
      else
        launch_spmm<VT, B, true>(g, bw, cur, cur, nxt, st, gate, tm);
      std::swap(cur, nxt);
    }
    hipLaunchKernelGGL((k_pm_out<B>), dim3(1), dim3(256), 0, st, cnt, l, (const double *)sums, out + p0);
    RD_HIP(hipGetLastError());
    if (prof) {
      RD_HIP(hipStreamSynchronize(st));
      g->timer[0].resolve(g->timer[0].used);
    }
  }
}

template <typename VT>
static void pm_dispatch(rd_graph g, BatchWork *bw, int32_t B, int32_t npairs, const int32_t *ps,
                        const int32_t *pt, int32_t l, rd_result *out, double *sums, hipStream_t st,
                        bool prof) {
  switch (B) {
    case 16: return pm_run_t<VT, 16>(g, bw, npairs, ps, pt, l, out, sums, st, prof);
    case 32: return pm_run_t<VT, 32>(g, bw, npairs, ps, pt, l, out, sums, st, prof);
    case 64: return pm_run_t<VT, 64>(g, bw, npairs, ps, pt, l, out, sums, st, prof);
    case 128: return pm_run_t<VT, 128>(g, bw, npairs, ps, pt, l, out, sums, st, prof);
    case 256: return pm_run_t<VT, 256>(g, bw, npairs, ps, pt, l, out, sums, st, prof);
  }
  throw RdError{RD_E_ARG, "block_width must be one of 16, 32, 64, 128, 256"};
}

extern "C" {

rd_status rd_query_batch(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t, double eps,
                         const rd_options *o, rd_result *out) {
  if (!g || npairs < 0 || (npairs > 0 && (!s || !t || !out))) return RD_E_ARG;
  std::vector<void *> owned;
  try {
    g->err.clear();
    rd_options opt = resolve_options(g, o);
    RD_REQUIRE(opt.fixed_k > 0 || eps > 0.0, "eps must be > 0 unless fixed_k is set");
    if (npairs == 0) return RD_OK;
    RD_HIP(hipSetDevice(g->device));
    hipStream_t st = pick_stream(g, o);
    BatchWork *bw = batch_get(g);
    const bool dp = opt.flags & RD_DEVICE_PTRS;
    const int32_t *ds = s, *dt = t;
    rd_result *dout = out;
    if (!dp) {
      int32_t *tmp = (int32_t *)dev_alloc(2 * (size_t)npairs * sizeof(int32_t));
      owned.push_back(tmp);
      RD_HIP(hipMemcpyAsync(tmp, s, npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
      RD_HIP(hipMemcpyAsync(tmp + npairs, t, npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
      ds = tmp;
      dt = tmp + npairs;
      dout = (rd_result *)dev_alloc((size_t)npairs * sizeof(rd_result));
      owned.push_back(dout);
    }
    RD_HIP(hipMemsetAsync(bw->flag, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_check_pairs, dim3(cdiv(npairs, 256)), dim3(256), 0, st, npairs, g->n, ds, dt,
                       bw->flag);
    int32_t bad = 0;
    RD_HIP(hipMemcpyAsync(&bad, bw->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    RD_REQUIRE(!bad, "pair node ids must be in [0, n)");
    if (g->perm) {
      int32_t *mp = (int32_t *)dev_alloc(2 * (size_t)npairs * sizeof(int32_t));
      owned.push_back(mp);
      hipLaunchKernelGGL(k_map_pairs, dim3(cdiv(npairs, 256)), dim3(256), 0, st, npairs, g->perm, ds,
                         dt, mp, mp + npairs);
      RD_HIP(hipGetLastError());
      ds = mp;
      dt = mp + npairs;
    }
    int32_t B = opt.block_width;
    RD_REQUIRE(B == 0 || B == 16 || B == 32 || B == 64 || B == 128 || B == 256,
               "block_width must be 0 or one of 16, 32, 64, 128, 256");
    if (!opt.refine && small_eligible(g, opt)) {
      // both vectors of a run fit in LDS: one workgroup per pair
      small_run(g, npairs, ds, dt, 0, 0, eps, opt, st, dout, nullptr, nullptr, nullptr);
      if (!dp)
        RD_HIP(hipMemcpyAsync(out, dout, (size_t)npairs * sizeof(rd_result), hipMemcpyDeviceToHost, st));
      RD_HIP(hipStreamSynchronize(st));
      for (void *p : owned) dev_free(p);
      return RD_OK;
    }
    if (B == 0) B = autotune_width(g, bw, opt.precision, npairs, st);
    RunParams prm{eps,       opt.max_iters, opt.fixed_k, opt.delay, opt.err_mode, npairs, opt.reorth,
                  GRAD_NONE, nullptr,       (opt.flags & RD_NO_SPARSE2) ? 0 : 1, 0};
    const bool prof = opt.flags & RD_PROFILE;
    if (opt.refine) {
      // runs with potentials (harvested per block), r reported as the FP64 energy
      if (opt.precision == RD_F64)
        grad_dispatch<double>(g, bw, B, npairs, ds, dt, nullptr, prm, dout, nullptr, st, prof);
      else
        grad_dispatch<float>(g, bw, B, npairs, ds, dt, nullptr, prm, dout, nullptr, st, prof);
    } else {
      const bool compact = !(opt.flags & RD_NO_COMPACT);
      if (opt.precision == RD_F64)
        batch_dispatch<double>(g, bw, B, npairs, ds, dt, prm, dout, st, prof, compact);
      else
        batch_dispatch<float>(g, bw, B, npairs, ds, dt, prm, dout, st, prof, compact);
    }
    if (!dp) {
      RD_HIP(hipMemcpyAsync(out, dout, (size_t)npairs * sizeof(rd_result), hipMemcpyDeviceToHost, st));
    }
    RD_HIP(hipStreamSynchronize(st));
    for (void *p : owned) dev_free(p);
    return RD_OK;
  } catch (const RdError &e) {
    (void)hipDeviceSynchronize();
    for (void *p : owned) dev_free(p);
    g->err = e.msg;
    return e.code;
  }
}

rd_status rd_power_method(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t, int32_t l,
                          const rd_options *o, rd_result *out) {
  if (!g || npairs < 0 || l < 0 || (npairs > 0 && (!s || !t || !out))) return RD_E_ARG;
  std::vector<void *> owned;
  try {
    g->err.clear();
    rd_options opt = resolve_options(g, o);
    if (npairs == 0) return RD_OK;
    RD_HIP(hipSetDevice(g->device));
    hipStream_t st = pick_stream(g, o);
    BatchWork *bw = batch_get(g);
    const bool dp = opt.flags & RD_DEVICE_PTRS;
    const int32_t *ds = s, *dt = t;
    rd_result *dout = out;
    if (!dp) {
      int32_t *tmp = (int32_t *)dev_alloc(2 * (size_t)npairs * sizeof(int32_t));
      owned.push_back(tmp);
      RD_HIP(hipMemcpyAsync(tmp, s, npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
      RD_HIP(hipMemcpyAsync(tmp + npairs, t, npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
      ds = tmp;
      dt = tmp + npairs;
      dout = (rd_result *)dev_alloc((size_t)npairs * sizeof(rd_result));
      owned.push_back(dout);
    }
    RD_HIP(hipMemsetAsync(bw->flag, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_check_pairs, dim3(cdiv(npairs, 256)), dim3(256), 0, st, npairs, g->n, ds, dt,
                       bw->flag);
    int32_t bad = 0;
    RD_HIP(hipMemcpyAsync(&bad, bw->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    RD_REQUIRE(!bad, "pair node ids must be in [0, n)");
    if (g->perm) {
      int32_t *mp = (int32_t *)dev_alloc(2 * (size_t)npairs * sizeof(int32_t));
      owned.push_back(mp);
      hipLaunchKernelGGL(k_map_pairs, dim3(cdiv(npairs, 256)), dim3(256), 0, st, npairs, g->perm, ds,
                         dt, mp, mp + npairs);
      RD_HIP(hipGetLastError());
      ds = mp;
      dt = mp + npairs;
    }
    int32_t B = opt.block_width;
    RD_REQUIRE(B == 0 || B == 16 || B == 32 || B == 64 || B == 128 || B == 256,
               "block_width must be 0 or one of 16, 32, 64, 128, 256");
    if (small_eligible(g, opt)) {
      // both vectors fit in LDS: one workgroup per pair runs all l steps
      pm_small_run(g, npairs, ds, dt, l, opt, st, dout);
    } else {
      if (B == 0) B = autotune_width(g, bw, opt.precision, npairs, st);
      double *sums = (double *)dev_alloc(2 * 256 * sizeof(double));
      owned.push_back(sums);
      const bool prof = opt.flags & RD_PROFILE;
      if (opt.precision == RD_F64)
        pm_dispatch<double>(g, bw, B, npairs, ds, dt, l, dout, sums, st, prof);
      else
        pm_dispatch<float>(g, bw, B, npairs, ds, dt, l, dout, sums, st, prof);
    }
    if (!dp)
      RD_HIP(hipMemcpyAsync(out, dout, (size_t)npairs * sizeof(rd_result), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    for (void *p : owned) dev_free(p);
    return RD_OK;
  } catch (const RdError &e) {
    (void)hipDeviceSynchronize();
    for (void *p : owned) dev_free(p);
    g->err = e.msg;
    return e.code;
  }
}

rd_status rd_potentials(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t, double eps,
                        const rd_options *o, rd_result *out, double *phi) {
  if (!g || npairs < 0 || (npairs > 0 && (!s || !t || !phi))) return RD_E_ARG;
  std::vector<void *> owned;
  try {
    g->err.clear();
    rd_options opt = resolve_options(g, o);
    RD_REQUIRE(opt.fixed_k > 0 || eps > 0.0, "eps must be > 0 unless fixed_k is set");
    if (npairs == 0) return RD_OK;
    RD_HIP(hipSetDevice(g->device));
    hipStream_t st = pick_stream(g, o);
    BatchWork *bw = batch_get(g);
    const bool dp = opt.flags & RD_DEVICE_PTRS;
    const int32_t *ds = s, *dt = t;
    rd_result *dout = out;
    double *dphi = phi;
    const size_t phi_bytes = (size_t)npairs * g->n * sizeof(double);
    if (!dp) {
      int32_t *tmp = (int32_t *)dev_alloc(2 * (size_t)npairs * sizeof(int32_t));
      owned.push_back(tmp);
      RD_HIP(hipMemcpyAsync(tmp, s, npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
      RD_HIP(hipMemcpyAsync(tmp + npairs, t, npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
      ds = tmp;
      dt = tmp + npairs;
      dphi = (double *)dev_alloc(phi_bytes);
      owned.push_back(dphi);
    }
    if (!dp || !out) {
      dout = (rd_result *)dev_alloc((size_t)npairs * sizeof(rd_result));
      owned.push_back(dout);
    }
    RD_HIP(hipMemsetAsync(bw->flag, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_check_pairs, dim3(cdiv(npairs, 256)), dim3(256), 0, st, npairs, g->n, ds, dt,
                       bw->flag);
    int32_t bad = 0;
    RD_HIP(hipMemcpyAsync(&bad, bw->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    RD_REQUIRE(!bad, "pair node ids must be in [0, n)");
    if (g->perm) {
      int32_t *mp = (int32_t *)dev_alloc(2 * (size_t)npairs * sizeof(int32_t));
      owned.push_back(mp);
      hipLaunchKernelGGL(k_map_pairs, dim3(cdiv(npairs, 256)), dim3(256), 0, st, npairs, g->perm, ds,
                         dt, mp, mp + npairs);
      RD_HIP(hipGetLastError());
      ds = mp;
      dt = mp + npairs;
    }
    int32_t B = opt.block_width;
    RD_REQUIRE(B == 0 || B == 16 || B == 32 || B == 64 || B == 128 || B == 256,
               "block_width must be 0 or one of 16, 32, 64, 128, 256");
    if (B == 0) B = autotune_width(g, bw, opt.precision, npairs, st);
    RD_HIP(hipMemsetAsync(dphi, 0, phi_bytes, st));
    // runs with potentials, harvested per block and copied out
    RunParams prm{eps,       opt.max_iters, opt.fixed_k, opt.delay, opt.err_mode, npairs, opt.reorth,
                  GRAD_NONE, nullptr,       (opt.flags & RD_NO_SPARSE2) ? 0 : 1, 0};
    const bool prof = opt.flags & RD_PROFILE;
    if (opt.precision == RD_F64)
      grad_dispatch<double>(g, bw, B, npairs, ds, dt, nullptr, prm, dout, nullptr, st, prof, dphi);
    else
      grad_dispatch<float>(g, bw, B, npairs, ds, dt, nullptr, prm, dout, nullptr, st, prof, dphi);
    if (!dp) {
      RD_HIP(hipMemcpyAsync(phi, dphi, phi_bytes, hipMemcpyDeviceToHost, st));
      if (out)
        RD_HIP(hipMemcpyAsync(out, dout, (size_t)npairs * sizeof(rd_result), hipMemcpyDeviceToHost, st));
    }
    RD_HIP(hipStreamSynchronize(st));
    for (void *p : owned) dev_free(p);
    return RD_OK;
  } catch (const RdError &e) {
    (void)hipDeviceSynchronize();
    for (void *p : owned) dev_free(p);
    g->err = e.msg;
    return e.code;
  }
}

rd_status rd_grad_edges(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t,
                        const double *grad_r, double eps, const rd_options *o, rd_result *fwd,
                        float *grad_w) {
  if (!g || npairs < 0 || !grad_w || (npairs > 0 && (!s || !t))) return RD_E_ARG;
  std::vector<void *> owned;
  try {
    g->err.clear();
    rd_options opt = resolve_options(g, o);
    RD_REQUIRE(opt.fixed_k > 0 || eps > 0.0, "eps must be > 0 unless fixed_k is set");
    RD_HIP(hipSetDevice(g->device));
    hipStream_t st = pick_stream(g, o);
    BatchWork *bw = batch_get(g);
    const bool dp = opt.flags & RD_DEVICE_PTRS;
    auto tmp = [&](size_t bytes) {
      void *p = dev_alloc(bytes);
      owned.push_back(p);
      return p;
    };
    const int32_t *ds = s, *dt = t;
    const double *dg = grad_r;
    rd_result *dout = fwd;
    float *dgw = grad_w;
    if (!dp) {
      if (npairs > 0) {
        int32_t *pp = (int32_t *)tmp(2 * (size_t)npairs * sizeof(int32_t));
        RD_HIP(hipMemcpyAsync(pp, s, npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
        RD_HIP(hipMemcpyAsync(pp + npairs, t, npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
        ds = pp;
        dt = pp + npairs;
        if (grad_r) {
          double *d = (double *)tmp((size_t)npairs * sizeof(double));
          RD_HIP(hipMemcpyAsync(d, grad_r, npairs * sizeof(double), hipMemcpyHostToDevice, st));
          dg = d;
        }
      }
      dout = nullptr;
      dgw = (float *)tmp((size_t)g->m * sizeof(float));
    }
    if (!dout) dout = (rd_result *)tmp(std::max<size_t>(1, npairs) * sizeof(rd_result));
    if (npairs > 0) {
      RD_HIP(hipMemsetAsync(bw->flag, 0, sizeof(int32_t), st));
      hipLaunchKernelGGL(k_check_pairs, dim3(cdiv(npairs, 256)), dim3(256), 0, st, npairs, g->n, ds,
                         dt, bw->flag);
      int32_t bad = 0;
      RD_HIP(hipMemcpyAsync(&bad, bw->flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      RD_HIP(hipStreamSynchronize(st));
      RD_REQUIRE(!bad, "pair node ids must be in [0, n)");
      if (g->perm) {
        int32_t *mp = (int32_t *)tmp(2 * (size_t)npairs * sizeof(int32_t));
        hipLaunchKernelGGL(k_map_pairs, dim3(cdiv(npairs, 256)), dim3(256), 0, st, npairs, g->perm,
                           ds, dt, mp, mp + npairs);
        RD_HIP(hipGetLastError());
        ds = mp;
        dt = mp + npairs;
      }
    }
    int32_t B = opt.block_width;
    if (B == 0) B = autotune_width(g, bw, opt.precision, std::max(npairs, 1), st);
    RD_REQUIRE(B == 16 || B == 32 || B == 64 || B == 128 || B == 256,
               "block_width must be 0 or one of 16, 32, 64, 128, 256");
    RunParams prm{eps,       opt.max_iters, opt.fixed_k, opt.delay, opt.err_mode, npairs, opt.reorth,
                  GRAD_NONE, nullptr,       (opt.flags & RD_NO_SPARSE2) ? 0 : 1, 0};
    if (opt.precision == RD_F64)
      grad_dispatch<double>(g, bw, B, npairs, ds, dt, dg, prm, dout, dgw, st, opt.flags & RD_PROFILE);
    else
      grad_dispatch<float>(g, bw, B, npairs, ds, dt, dg, prm, dout, dgw, st, opt.flags & RD_PROFILE);
    if (!dp) {
      if (fwd && npairs > 0)
        RD_HIP(hipMemcpyAsync(fwd, dout, (size_t)npairs * sizeof(rd_result), hipMemcpyDeviceToHost, st));
      RD_HIP(hipMemcpyAsync(grad_w, dgw, (size_t)g->m * sizeof(float), hipMemcpyDeviceToHost, st));
    }
    RD_HIP(hipStreamSynchronize(st));
    for (void *p : owned) dev_free(p);
    return RD_OK;
  } catch (const RdError &e) {
    (void)hipDeviceSynchronize();
    for (void *p : owned) dev_free(p);
    g->err = e.msg;
    return e.code;
  }
}

}  // extern "C"

extern "C" rd_status rd_batch_schedule(rd_graph g, int32_t *wave_nnz, int32_t *long_deg) {
  if (!g) return RD_E_ARG;
  try {
    g->err.clear();
    RD_HIP(hipSetDevice(g->device));
    BatchWork *bw = batch_get(g);
    if (wave_nnz) *wave_nnz = bw->wave_nnz;
    if (long_deg) *long_deg = bw->long_deg;
    return RD_OK;
  } catch (const RdError &e) {
    g->err = e.msg;
    return e.code;
  }
}

extern "C" rd_status rd_tune_width(rd_graph g, int32_t precision, int32_t npairs, void *stream,
                                   int32_t *width) {
  if (!g || !width || npairs < 1 || (precision != RD_F64 && precision != RD_F32)) return RD_E_ARG;
  try {
    g->err.clear();
    RD_HIP(hipSetDevice(g->device));
    hipStream_t st = stream ? (hipStream_t)stream : g->own_stream;
    *width = autotune_width(g, batch_get(g), precision, npairs, st);
    return RD_OK;
  } catch (const RdError &e) {
    g->err = e.msg;
    return e.code;
  }
}
