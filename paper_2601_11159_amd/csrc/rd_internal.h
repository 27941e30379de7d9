// Internal declarations of the resistance-distance library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "rd.h"

// ---------------------------------------------------------------------------
// Error plumbing
// ---------------------------------------------------------------------------

struct RdError {
  rd_status code;
  std::string msg;
};

#define RD_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw RdError{e_ == hipErrorOutOfMemory ? RD_E_OOM : RD_E_DEVICE,                   \
                    std::string(#call) + ": " + hipGetErrorString(e_)};                   \
  } while (0)

#define RD_REQUIRE(cond, msg)                                         \
  do {                                                                \
    if (!(cond)) throw RdError{RD_E_ARG, std::string(msg)};           \
  } while (0)

// ---------------------------------------------------------------------------
// Per-run Lanczos scalars (FP64), one record per query slot, device resident.
// ---------------------------------------------------------------------------

enum : int32_t { LZ_RUNNING = 0, LZ_DONE = 1, LZ_NOT_CONVERGED = 2, LZ_BREAKDOWN = 3, LZ_IDLE = 4 };

constexpr int RD_HIST = 16;  // ring of recent r_hat values for the stopping estimator (delay <= 14)

struct LzState {
  double c;          // 1/d_s + 1/d_t
  double sig_cur;    // q_i = sig_cur * U_cur (scale-on-read normalisation)
  double sig_prev;   // q_{i-1} = sig_prev * U_prev
  double prev_coef;  // beta_i * sig_prev: coefficient of U_prev in the recurrence (0 when i = 1)
  double beta;       // beta_i
  double alpha;      // alpha_i of the current iteration
  double delta;      // pivot of the LDL^T factorisation of I - T_i
  double omega;      // |(L^{-1} e_1)_i|
  double g;          // e_1^T (I - T_i)^{-1} e_1
  double rhat;       // c * g
  double err_est;    // stopping estimate (absolute)
  double tol;        // stopping tolerance (relative or absolute per err_mode)
  double ro_mu, ro_c, ro_p;  // re-orthogonalisation: w -= ro_mu 1 + ro_c U_cur + ro_p U_prev
  double hist[RD_HIST];
  int32_t k;         // iterations completed
  int32_t status;    // LZ_*
  int32_t max_iters;
  int32_t fixed_k;
  int32_t delay;
  int32_t err_mode;
  int32_t s, t;
  int32_t pair;      // index of the pair held by this slot (batched runs)
  int32_t pad;
};

// ---------------------------------------------------------------------------
// Graph handle
// ---------------------------------------------------------------------------

struct PlainWork;
struct BatchWork;

// Event-timed launches of one kernel (RD_PROFILE).
struct KernelTimer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  std::vector<double> bytes;  // algorithmic bytes of each recorded launch
  size_t used = 0;            // events recorded in the current call
  double total_ms = 0;        // resolved durations since the last read
  double total_bytes = 0;     // and their algorithmic bytes
  int64_t launches = 0;
  std::pair<hipEvent_t, hipEvent_t> next(double alg_bytes);
  void resolve(size_t valid);  // after the stream is synchronised: count the first `valid` launches
  void release();
};

struct rd_graph_s {
  int device = 0;
  hipStream_t own_stream = nullptr;
  int32_t n = 0;
  int64_t m = 0, nnz = 0;
  bool unit = true;
  int32_t max_deg = 0;
  double vol = 0.0;  // sum of the weighted degrees

  int32_t *row_ptr = nullptr;  // [n+1]
  int32_t *col = nullptr;      // [nnz] neighbour ids, ascending within a row
  int32_t *eid = nullptr;      // [nnz] edge id of each adjacency entry
  double *w64 = nullptr;       // [nnz] weights in adjacency order (weighted graphs)
  float *w32 = nullptr;        // [nnz] same, FP32
  double *deg = nullptr;       // [n] weighted degree (FP64)
  double *invdeg = nullptr;    // [n] 1/d (FP64)
  float *invdeg32 = nullptr;   // [n] 1/d (FP32)
  float *deg32 = nullptr;      // [n] d (FP32)

  // plain SpMV launch schedule: row blocks of bounded adjacency length
  int32_t nblk = 0;
  int32_t *blk_row = nullptr;  // [nblk+1] first row of each block
  int8_t *blk_lanes = nullptr; // [nblk] log2(lanes per row) for multi-row blocks, -1 for one long row

  // edge-pass work items (built on first use): the entries (u, v > u) of
  // each row cut into chunks of at most EDGE_CHUNK, as (u, begin, end, 0)
  int32_t nch = 0;
  int4 *echunk = nullptr;

  // RD_REORDER: internal id of every caller id (nullptr: identity)
  int32_t *perm = nullptr;
  std::vector<int32_t> perm_host;

  KernelTimer timer[3];  // 0: batched short-row product, 1: single-pair product, 2: edge gradient
  PlainWork *plain = nullptr;
  BatchWork *batch = nullptr;

  std::string err;
};

// ---------------------------------------------------------------------------
// Shared helpers
// ---------------------------------------------------------------------------

void *dev_alloc(size_t bytes);
void dev_free(void *p);
hipStream_t pick_stream(rd_graph g, const rd_options *o);
rd_options resolve_options(rd_graph g, const rd_options *o);

// Row blocks of the single-pair product: at most SPMV_BLOCK_NNZ adjacency
// entries and SPMV_BLOCK_ROWS rows each (a longer row is a block of its own).
constexpr int SPMV_BLOCK_NNZ = 1024;
constexpr int SPMV_BLOCK_ROWS = 256;

// Work items of the edge passes (gradient, energy): every undirected edge once,
// as the adjacency entry (u, v) with v > u. Columns ascend within a row, so
// these entries are a suffix of row u; the suffix is cut into chunks of at most
// EDGE_CHUNK entries so that the edges of a hub row spread over many wavefronts.
constexpr int EDGE_CHUNK = 32;
void edge_chunks(rd_graph g, hipStream_t st);

// plain single-pair path (lanczos_plain.hip)
void plain_free(rd_graph g);
void plain_run(rd_graph g, int32_t s, int32_t t, double eps, const rd_options &o, hipStream_t st,
               rd_result *out, double *tr_alpha, double *tr_beta, double *tr_rhat, int32_t trace_k);

// batched path (lanczos_batch.hip)
void batch_free(rd_graph g);
// the sparse second iteration of a single-pair run (see lanczos_batch.hip);
// false when its buffers are not available
bool sparse_second_single(rd_graph g, int32_t precision, void *U1, void *U2, LzState *st, hipStream_t stream);

// one workgroup per pair for graphs whose two vectors fit in LDS (lanczos_small.hip)
bool small_eligible(rd_graph g, const rd_options &o);
void small_run(rd_graph g, int32_t npairs, const int32_t *ps, const int32_t *pt, int32_t s0,
               int32_t t0, double eps, const rd_options &o, hipStream_t st, rd_result *out,
               double *tr_alpha, double *tr_beta, double *tr_rhat);
// the Power Method (Algorithm 1) on the same single-workgroup layout
void pm_small_run(rd_graph g, int32_t npairs, const int32_t *ps, const int32_t *pt, int32_t l,
                  const rd_options &o, hipStream_t st, rd_result *out);
