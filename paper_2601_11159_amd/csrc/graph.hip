// Graph preparation on the device: validation, symmetric CSR, weighted
// degrees, connectivity, and the row-block schedule of the single-pair SpMV.
//
// The operator of the Lanczos recurrence is built from the graph exactly as
// Section 2.1/2.2 define it: W (A for unit weights), d_u = sum_v w_uv and the
// normalised adjacency D^{-1/2} W D^{-1/2}. Entries are kept as CSR in
// ascending column order so every reduction over a row has a fixed order.

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "rd_internal.h"

namespace {

enum : int32_t { BAD_RANGE = 1, BAD_LOOP = 2, BAD_WEIGHT = 4, BAD_DUP = 8, BAD_ISOLATED = 16 };

template <typename WT>
__global__ void k_validate_keys(int64_t m, int32_t n, const int32_t *__restrict__ u,
                                const int32_t *__restrict__ v, const WT *__restrict__ w,
                                uint64_t *__restrict__ keys, int32_t *__restrict__ vals,
                                int32_t *__restrict__ flags) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  int32_t a = u[e], b = v[e];
  int32_t f = 0;
  if (a < 0 || a >= n || b < 0 || b >= n) f |= BAD_RANGE;
  if (a == b) f |= BAD_LOOP;
  if (w) {
    double x = (double)w[e];
    if (!(x > 0.0) || !isfinite(x)) f |= BAD_WEIGHT;
  }
  if (f) atomicOr(flags, f);
  uint32_t ua = (uint32_t)a, ub = (uint32_t)b;
  keys[2 * e] = ((uint64_t)ua << 32) | ub;
  keys[2 * e + 1] = ((uint64_t)ub << 32) | ua;
  vals[2 * e] = (int32_t)e;
  vals[2 * e + 1] = (int32_t)e;
}

__global__ void k_count_degree(int64_t m, const int32_t *__restrict__ u, const int32_t *__restrict__ v,
                               int32_t *__restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  atomicAdd(&cnt[u[e]], 1);
  atomicAdd(&cnt[v[e]], 1);
}

// ascending sort keys for descending degree
__global__ void k_degree_keys(int32_t n, const int32_t *__restrict__ cnt, uint32_t *__restrict__ key,
                              int32_t *__restrict__ ids) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = 0xffffffffu - (uint32_t)cnt[i];
  ids[i] = i;
}

// perm[old id] = rank of the old id in the sorted order
__global__ void k_rank_of(int32_t n, const int32_t *__restrict__ order, int32_t *__restrict__ perm) {
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) perm[order[r]] = r;
}

__global__ void k_relabel_keys(int64_t nnz, const int32_t *__restrict__ perm,
                               uint64_t *__restrict__ keys) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const uint64_t k = keys[p];
  const uint32_t a = (uint32_t)perm[k >> 32], b = (uint32_t)perm[k & 0xffffffffu];
  keys[p] = ((uint64_t)a << 32) | b;
}

__global__ void k_split_keys(int64_t nnz, const uint64_t *__restrict__ keys,
                             int32_t *__restrict__ col, int32_t *__restrict__ flags) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  uint64_t k = keys[p];
  col[p] = (int32_t)(k & 0xffffffffu);
  if (p + 1 < nnz && keys[p + 1] == k) atomicOr(flags, BAD_DUP);
}

// row_ptr[r] = first position whose row id is >= r (binary search over sorted keys)
__global__ void k_row_ptr(int32_t n, int64_t nnz, const uint64_t *__restrict__ keys,
                          int32_t *__restrict__ row_ptr) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > n) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((int64_t)(keys[mid] >> 32) < r) lo = mid + 1; else hi = mid;
  }
  row_ptr[r] = (int32_t)lo;
}

template <typename WT>
__global__ void k_gather_weights(int64_t nnz, const int32_t *__restrict__ eid,
                                 const WT *__restrict__ w, double *__restrict__ w64,
                                 float *__restrict__ w32) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  WT x = w[eid[p]];
  w64[p] = (double)x;
  w32[p] = (float)x;
}

// d_u = sum of the row's weights in adjacency order (FP64); unit weights: row length.
__global__ void k_degrees(int32_t n, const int32_t *__restrict__ row_ptr,
                          const double *__restrict__ w64, double *__restrict__ deg,
                          double *__restrict__ invdeg, float *__restrict__ invdeg32,
                          float *__restrict__ deg32, int32_t *__restrict__ flags,
                          int32_t *__restrict__ maxdeg) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int32_t b = row_ptr[r], e = row_ptr[r + 1];
  double d;
  if (w64) {
    d = 0.0;
    for (int32_t p = b; p < e; ++p) d += w64[p];
  } else {
    d = (double)(e - b);
  }
  if (e == b) atomicOr(flags, BAD_ISOLATED);
  atomicMax(maxdeg, e - b);
  deg[r] = d;
  invdeg[r] = 1.0 / d;
  invdeg32[r] = (float)(1.0 / d);
  deg32[r] = (float)d;
}

__global__ void k_bfs_seed(int32_t n, int32_t *__restrict__ visited, int32_t *__restrict__ frontier) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) visited[r] = (r == 0);
  if (r == 0) frontier[0] = 0;
}

// One BFS level: a wavefront per frontier node, lanes over its neighbours.
__global__ void k_bfs_level(int32_t nf, const int32_t *__restrict__ frontier,
                            const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                            int32_t *__restrict__ visited, int32_t *__restrict__ next,
                            int32_t *__restrict__ next_count) {
  int32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
  int32_t lane = threadIdx.x & 63;
  if (wave >= nf) return;
  int32_t x = frontier[wave];
  for (int32_t p = row_ptr[x] + lane; p < row_ptr[x + 1]; p += 64) {
    int32_t y = col[p];
    if (atomicExch(&visited[y], 1) == 0) next[atomicAdd(next_count, 1)] = y;
  }
}

inline unsigned grid_for(int64_t work, int threads) {
  return (unsigned)((work + threads - 1) / threads);
}

// Row blocks for the single-pair SpMV: at most `max_rows` consecutive rows
// whose adjacency entries total at most `budget`, or one row alone when it is
// longer. Each
// multi-row block records log2 of the lanes that cooperate on one row.
void build_row_blocks(rd_graph g, const std::vector<int32_t> &rp, int32_t budget, int32_t max_rows) {
  std::vector<int32_t> start;
  std::vector<int8_t> lanes;
  const int32_t n = g->n;
  int32_t r = 0;
  start.reserve(n / 8 + 16);
  while (r < n) {
    int32_t len = rp[r + 1] - rp[r];
    if (len > budget) {
      start.push_back(r);
      lanes.push_back((int8_t)-1);
      ++r;
      continue;
    }
    int32_t r1 = r + 1;
    while (r1 < n && r1 - r < max_rows && rp[r1 + 1] - rp[r] <= budget) ++r1;
    int32_t rows = r1 - r;
    int32_t avg = (rp[r1] - rp[r]) / rows;
    int lg = 0;
    while (lg < 6 && (2 << lg) <= avg) ++lg;
    start.push_back(r);
    lanes.push_back((int8_t)lg);
    r = r1;
  }
  start.push_back(n);
  g->nblk = (int32_t)lanes.size();
  g->blk_row = (int32_t *)dev_alloc(start.size() * sizeof(int32_t));
  g->blk_lanes = (int8_t *)dev_alloc(lanes.size() * sizeof(int8_t));
  RD_HIP(hipMemcpy(g->blk_row, start.data(), start.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  RD_HIP(hipMemcpy(g->blk_lanes, lanes.data(), lanes.size() * sizeof(int8_t), hipMemcpyHostToDevice));
}

bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// Copy (or alias) a caller array onto the device.
template <typename T>
const T *to_device(const T *p, int64_t count, bool device_ptrs, std::vector<void *> &owned) {
  if (!p) return nullptr;
  if (device_ptrs) {
    RD_REQUIRE(is_device_ptr(p), "RD_DEVICE_PTRS given but an array is not device memory");
    return p;
  }
  T *d = (T *)dev_alloc(count * sizeof(T));
  owned.push_back(d);
  RD_HIP(hipMemcpy(d, p, count * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

// vol = sum_u d_u in FP64, summed on the host in node order.
static void compute_volume(rd_graph g) {
  std::vector<double> d(g->n);
  RD_HIP(hipMemcpy(d.data(), g->deg, (size_t)g->n * sizeof(double), hipMemcpyDeviceToHost));
  double v = 0.0;
  for (double x : d) v += x;
  g->vol = v;
}

void set_weights_impl(rd_graph g, const void *w, int32_t w_dtype, uint32_t flags) {
  RD_REQUIRE(w_dtype == RD_F64 || w_dtype == RD_F32, "w_dtype must be RD_F64 or RD_F32");
  std::vector<void *> owned;
  try {
    bool dp = flags & RD_DEVICE_PTRS;
    int32_t *dflags = (int32_t *)dev_alloc(2 * sizeof(int32_t));
    owned.push_back(dflags);
    RD_HIP(hipMemset(dflags, 0, 2 * sizeof(int32_t)));
    if (!g->w64) {
      g->w64 = (double *)dev_alloc(g->nnz * sizeof(double));
      g->w32 = (float *)dev_alloc(g->nnz * sizeof(float));
    }
    // validate the weights with the edge-list kernel's weight test
    if (w_dtype == RD_F64) {
      const double *dw = to_device((const double *)w, g->m, dp, owned);
      hipLaunchKernelGGL(k_gather_weights<double>, dim3(grid_for(g->nnz, 256)), dim3(256), 0, 0,
                         g->nnz, g->eid, dw, g->w64, g->w32);
    } else {
      const float *dw = to_device((const float *)w, g->m, dp, owned);
      hipLaunchKernelGGL(k_gather_weights<float>, dim3(grid_for(g->nnz, 256)), dim3(256), 0, 0,
                         g->nnz, g->eid, dw, g->w64, g->w32);
    }
    RD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(g->n, 256)), dim3(256), 0, 0, g->n, g->row_ptr,
                       (const double *)g->w64, g->deg, g->invdeg, g->invdeg32, g->deg32, dflags,
                       dflags + 1);
    RD_HIP(hipGetLastError());
    RD_HIP(hipDeviceSynchronize());
    g->unit = false;
    compute_volume(g);
    for (void *p : owned) dev_free(p);
    owned.clear();
  } catch (...) {
    for (void *p : owned) dev_free(p);
    throw;
  }
}

// Weight validity check on the caller's array (range of values), done on the device.
template <typename WT>
__global__ void k_check_weights(int64_t m, const WT *__restrict__ w, int32_t *__restrict__ flags) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  double x = (double)w[e];
  if (!(x > 0.0) || !isfinite(x)) atomicOr(flags, BAD_WEIGHT);
}

}  // namespace

// ---------------------------------------------------------------------------
// Shared helpers
// ---------------------------------------------------------------------------

void *dev_alloc(size_t bytes) {
  void *p = nullptr;
  if (bytes == 0) bytes = 1;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw RdError{e == hipErrorOutOfMemory ? RD_E_OOM : RD_E_DEVICE,
                  std::string("hipMalloc failed: ") + hipGetErrorString(e)};
  }
  return p;
}

void dev_free(void *p) {
  if (p) (void)hipFree(p);
}

hipStream_t pick_stream(rd_graph g, const rd_options *o) {
  return (o && o->stream) ? (hipStream_t)o->stream : g->own_stream;
}

rd_options resolve_options(rd_graph g, const rd_options *o) {
  rd_options r;
  rd_default_options(&r);
  if (o) r = *o;
  RD_REQUIRE(r.precision == RD_F64 || r.precision == RD_F32, "precision must be RD_F64 or RD_F32");
  RD_REQUIRE(r.max_iters >= 0 && r.fixed_k >= 0, "max_iters and fixed_k must be >= 0");
  if (r.max_iters == 0) r.max_iters = std::max(r.fixed_k, std::min<int32_t>(g->n, 100000));
  if (r.delay == 0) r.delay = 8;
  RD_REQUIRE(r.delay >= 1 && r.delay <= RD_HIST - 2, "delay must be in [1, 14]");
  RD_REQUIRE(r.err_mode == 0 || r.err_mode == 1, "err_mode must be 0 or 1");
  RD_REQUIRE(r.block_width >= 0 && r.block_width <= 256, "block_width must be in [0, 256]");
  RD_REQUIRE(r.refine == 0 || r.refine == 1, "refine must be 0 or 1");
  RD_REQUIRE(r.reorth >= 0 && r.reorth <= 2, "reorth must be 0, 1 or 2");
  return r;
}

std::pair<hipEvent_t, hipEvent_t> KernelTimer::next(double alg_bytes) {
  if (used == pool.size()) {
    hipEvent_t a, b;
    RD_HIP(hipEventCreate(&a));
    RD_HIP(hipEventCreate(&b));
    pool.push_back({a, b});
    bytes.push_back(0.0);
  }
  bytes[used] = alg_bytes;
  return pool[used++];
}

void KernelTimer::resolve(size_t valid) {
  for (size_t i = 0; i < used && i < valid; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pool[i].first, pool[i].second) == hipSuccess) {
      total_ms += ms;
      total_bytes += bytes[i];
      ++launches;
    } else {
      (void)hipGetLastError();
    }
  }
  used = 0;
}

void KernelTimer::release() {
  for (auto &p : pool) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  pool.clear();
  bytes.clear();
  used = 0;
}

__global__ void k_upper_count(int32_t n, const int32_t *__restrict__ row_ptr,
                              const int32_t *__restrict__ col, int32_t *__restrict__ ub,
                              int32_t *__restrict__ cnt) {
  const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int32_t lo = row_ptr[u], hi = row_ptr[u + 1];
  const int32_t re = hi;
  while (lo < hi) {  // first entry with col > u
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (col[mid] > u) hi = mid;
    else lo = mid + 1;
  }
  ub[u] = lo;
  cnt[u] = (re - lo + EDGE_CHUNK - 1) / EDGE_CHUNK;
}

__global__ void k_upper_fill(int32_t n, const int32_t *__restrict__ row_ptr,
                             const int32_t *__restrict__ ub, const int32_t *__restrict__ cnt,
                             const int32_t *__restrict__ off, int4 *__restrict__ chunk) {
  const int32_t u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int32_t re = row_ptr[u + 1], nc = cnt[u], o = off[u];
  int32_t p = ub[u];
  for (int32_t c = 0; c < nc; ++c, p += EDGE_CHUNK) chunk[o + c] = make_int4(u, p, min(p + EDGE_CHUNK, re), 0);
}

void edge_chunks(rd_graph g, hipStream_t st) {
  if (g->echunk) return;
  const int32_t n = g->n;
  std::vector<void *> tmp;
  try {
    int32_t *buf = (int32_t *)dev_alloc(3 * (size_t)n * sizeof(int32_t));
    tmp.push_back(buf);
    int32_t *ub = buf, *cnt = buf + n, *off = buf + 2 * (size_t)n;
    hipLaunchKernelGGL(k_upper_count, dim3(grid_for(n, 256)), dim3(256), 0, st, n, g->row_ptr, g->col,
                       ub, cnt);
    size_t tb = 0;
    RD_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, off, n, st));
    void *scan_tmp = dev_alloc(tb);
    tmp.push_back(scan_tmp);
    RD_HIP(hipcub::DeviceScan::ExclusiveSum(scan_tmp, tb, cnt, off, n, st));
    int32_t last[2];
    RD_HIP(hipMemcpyAsync(&last[0], off + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RD_HIP(hipMemcpyAsync(&last[1], cnt + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    RD_HIP(hipStreamSynchronize(st));
    const int32_t nch = last[0] + last[1];
    int4 *ch = (int4 *)dev_alloc(std::max<size_t>(1, nch) * sizeof(int4));
    tmp.push_back(ch);
    hipLaunchKernelGGL(k_upper_fill, dim3(grid_for(n, 256)), dim3(256), 0, st, n, g->row_ptr,
                       (const int32_t *)ub, (const int32_t *)cnt, (const int32_t *)off, ch);
    RD_HIP(hipGetLastError());
    RD_HIP(hipStreamSynchronize(st));
    tmp.pop_back();
    g->echunk = ch;
    g->nch = nch;
  } catch (...) {
    for (void *p : tmp) dev_free(p);
    throw;
  }
  for (void *p : tmp) dev_free(p);
}

static void free_graph_memory(rd_graph g) {
  for (KernelTimer &k : g->timer) k.release();
  plain_free(g);
  batch_free(g);
  dev_free(g->row_ptr);
  dev_free(g->col);
  dev_free(g->eid);
  dev_free(g->w64);
  dev_free(g->w32);
  dev_free(g->deg);
  dev_free(g->invdeg);
  dev_free(g->invdeg32);
  dev_free(g->deg32);
  dev_free(g->blk_row);
  dev_free(g->blk_lanes);
  dev_free(g->perm);
  dev_free(g->echunk);
  if (g->own_stream) (void)hipStreamDestroy(g->own_stream);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void rd_default_options(rd_options *o) {
  if (!o) return;
  o->precision = RD_F64;
  o->max_iters = 0;
  o->fixed_k = 0;
  o->delay = 8;
  o->refine = 0;
  o->reorth = 0;
  o->block_width = 0;
  o->err_mode = 0;
  o->flags = 0;
  o->stream = nullptr;
}

const char *rd_status_string(rd_status s) {
  switch (s) {
    case RD_OK: return "ok";
    case RD_E_ARG: return "invalid argument";
    case RD_E_NOT_CONNECTED: return "graph is not connected";
    case RD_E_OOM: return "out of device memory";
    case RD_E_DEVICE: return "HIP runtime error";
    case RD_E_NOT_CONVERGED: return "iteration cap reached before the tolerance";
    case RD_E_BREAKDOWN: return "numerical breakdown (non-positive pivot or non-finite value)";
  }
  return "unknown status";
}

// Messages of failed rd_init_graph calls (no handle exists then), per thread.
static thread_local std::string g_init_error;

const char *rd_last_error(rd_graph g) { return g ? g->err.c_str() : g_init_error.c_str(); }

rd_status rd_kernel_stats(rd_graph g, int32_t which, double *total_ms, int64_t *launches,
                          double *alg_bytes) {
  if (!g || which < 0 || which > 2) return RD_E_ARG;
  KernelTimer &k = g->timer[which];
  if (total_ms) *total_ms = k.total_ms;
  if (launches) *launches = k.launches;
  if (alg_bytes) *alg_bytes = k.launches ? k.total_bytes / (double)k.launches : 0.0;
  k.total_ms = 0;
  k.total_bytes = 0;
  k.launches = 0;
  return RD_OK;
}

rd_status rd_graph_info(rd_graph g, int32_t *n, int64_t *m, int64_t *nnz) {
  if (!g) return RD_E_ARG;
  if (n) *n = g->n;
  if (m) *m = g->m;
  if (nnz) *nnz = g->nnz;
  return RD_OK;
}

rd_status rd_init_graph(int32_t n, int64_t m, const int32_t *u, const int32_t *v, const void *w,
                        int32_t w_dtype, uint32_t flags, rd_graph *out) {
  g_init_error.clear();
  if (!out) return RD_E_ARG;
  *out = nullptr;
  if (n < 2 || m < 1 || !u || !v || m > (int64_t)0x3fffffff) {
    g_init_error = "need n >= 2, 1 <= m < 2^30 and non-null edge arrays";
    return RD_E_ARG;
  }
  if (w && w_dtype != RD_F64 && w_dtype != RD_F32) {
    g_init_error = "w_dtype must be RD_F64 or RD_F32";
    return RD_E_ARG;
  }
  rd_graph g = new (std::nothrow) rd_graph_s();
  if (!g) return RD_E_OOM;
  std::vector<void *> owned;
  try {
    RD_HIP(hipGetDevice(&g->device));
    RD_HIP(hipStreamCreateWithFlags(&g->own_stream, hipStreamNonBlocking));
    g->n = n;
    g->m = m;
    g->nnz = 2 * m;
    const bool dp = flags & RD_DEVICE_PTRS;
    const int32_t *du = to_device(u, m, dp, owned);
    const int32_t *dv = to_device(v, m, dp, owned);

    int32_t *dflags = (int32_t *)dev_alloc(2 * sizeof(int32_t));
    owned.push_back(dflags);
    RD_HIP(hipMemset(dflags, 0, 2 * sizeof(int32_t)));

    uint64_t *keys = (uint64_t *)dev_alloc(g->nnz * sizeof(uint64_t));
    owned.push_back(keys);
    uint64_t *keys2 = (uint64_t *)dev_alloc(g->nnz * sizeof(uint64_t));
    owned.push_back(keys2);
    int32_t *vals = (int32_t *)dev_alloc(g->nnz * sizeof(int32_t));
    owned.push_back(vals);
    g->eid = (int32_t *)dev_alloc(g->nnz * sizeof(int32_t));

    const void *dw = nullptr;
    if (w && w_dtype == RD_F64) {
      dw = to_device((const double *)w, m, dp, owned);
      hipLaunchKernelGGL(k_validate_keys<double>, dim3(grid_for(m, 256)), dim3(256), 0, 0, m, n, du,
                         dv, (const double *)dw, keys, vals, dflags);
    } else if (w) {
      dw = to_device((const float *)w, m, dp, owned);
      hipLaunchKernelGGL(k_validate_keys<float>, dim3(grid_for(m, 256)), dim3(256), 0, 0, m, n, du,
                         dv, (const float *)dw, keys, vals, dflags);
    } else {
      hipLaunchKernelGGL(k_validate_keys<double>, dim3(grid_for(m, 256)), dim3(256), 0, 0, m, n, du,
                         dv, (const double *)nullptr, keys, vals, dflags);
    }
    RD_HIP(hipGetLastError());
    int32_t hflags = 0;
    RD_HIP(hipMemcpy(&hflags, dflags, sizeof(int32_t), hipMemcpyDeviceToHost));
    RD_REQUIRE(!(hflags & BAD_RANGE), "node id out of range [0, n)");
    RD_REQUIRE(!(hflags & BAD_LOOP), "self-loop in the edge list");
    RD_REQUIRE(!(hflags & BAD_WEIGHT), "edge weights must be finite and > 0");

    if (flags & RD_REORDER) {
      // internal ids by decreasing degree (ties by id): the most gathered
      // entries of a vector share cache lines
      int32_t *cnt = (int32_t *)dev_alloc((size_t)n * sizeof(int32_t));
      owned.push_back(cnt);
      RD_HIP(hipMemset(cnt, 0, (size_t)n * sizeof(int32_t)));
      hipLaunchKernelGGL(k_count_degree, dim3(grid_for(m, 256)), dim3(256), 0, 0, m, du, dv, cnt);
      uint32_t *dk = (uint32_t *)dev_alloc(2 * (size_t)n * sizeof(uint32_t));
      owned.push_back(dk);
      int32_t *ids = (int32_t *)dev_alloc(2 * (size_t)n * sizeof(int32_t));
      owned.push_back(ids);
      hipLaunchKernelGGL(k_degree_keys, dim3(grid_for(n, 256)), dim3(256), 0, 0, n, cnt, dk, ids);
      size_t tb = 0;
      RD_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, dk, dk + n, ids, ids + n, n, 0, 32,
                                                (hipStream_t)0));
      void *tmp0 = dev_alloc(tb);
      owned.push_back(tmp0);
      RD_HIP(hipcub::DeviceRadixSort::SortPairs(tmp0, tb, dk, dk + n, ids, ids + n, n, 0, 32,
                                                (hipStream_t)0));
      g->perm = (int32_t *)dev_alloc((size_t)n * sizeof(int32_t));
      hipLaunchKernelGGL(k_rank_of, dim3(grid_for(n, 256)), dim3(256), 0, 0, n,
                         (const int32_t *)(ids + n), g->perm);
      hipLaunchKernelGGL(k_relabel_keys, dim3(grid_for(g->nnz, 256)), dim3(256), 0, 0, g->nnz,
                         (const int32_t *)g->perm, keys);
      RD_HIP(hipGetLastError());
      g->perm_host.resize(n);
      RD_HIP(hipMemcpy(g->perm_host.data(), g->perm, (size_t)n * sizeof(int32_t),
                       hipMemcpyDeviceToHost));
    }

    // sort the 2m directed entries by (row, column); values carry the edge id
    int end_bit = 32;
    while (end_bit < 64 && ((uint64_t)(n - 1) >> (end_bit - 32)) != 0) ++end_bit;
    size_t tmp_bytes = 0;
    RD_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, keys2, vals, g->eid,
                                              (int)g->nnz, 0, end_bit, (hipStream_t)0));
    void *tmp = dev_alloc(tmp_bytes);
    owned.push_back(tmp);
    RD_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, keys2, vals, g->eid, (int)g->nnz,
                                              0, end_bit, (hipStream_t)0));

    g->col = (int32_t *)dev_alloc(g->nnz * sizeof(int32_t));
    g->row_ptr = (int32_t *)dev_alloc((size_t)(n + 1) * sizeof(int32_t));
    hipLaunchKernelGGL(k_split_keys, dim3(grid_for(g->nnz, 256)), dim3(256), 0, 0, g->nnz, keys2,
                       g->col, dflags);
    hipLaunchKernelGGL(k_row_ptr, dim3(grid_for((int64_t)n + 1, 256)), dim3(256), 0, 0, n, g->nnz,
                       keys2, g->row_ptr);
    RD_HIP(hipGetLastError());

    g->deg = (double *)dev_alloc(n * sizeof(double));
    g->invdeg = (double *)dev_alloc(n * sizeof(double));
    g->invdeg32 = (float *)dev_alloc(n * sizeof(float));
    g->deg32 = (float *)dev_alloc(n * sizeof(float));
    if (w) {
      g->w64 = (double *)dev_alloc(g->nnz * sizeof(double));
      g->w32 = (float *)dev_alloc(g->nnz * sizeof(float));
      if (w_dtype == RD_F64)
        hipLaunchKernelGGL(k_gather_weights<double>, dim3(grid_for(g->nnz, 256)), dim3(256), 0, 0,
                           g->nnz, g->eid, (const double *)dw, g->w64, g->w32);
      else
        hipLaunchKernelGGL(k_gather_weights<float>, dim3(grid_for(g->nnz, 256)), dim3(256), 0, 0,
                           g->nnz, g->eid, (const float *)dw, g->w64, g->w32);
      g->unit = false;
    }
    hipLaunchKernelGGL(k_degrees, dim3(grid_for(n, 256)), dim3(256), 0, 0, n, g->row_ptr,
                       (const double *)g->w64, g->deg, g->invdeg, g->invdeg32, g->deg32, dflags,
                       dflags + 1);
    RD_HIP(hipGetLastError());
    int32_t hf[2];
    RD_HIP(hipMemcpy(hf, dflags, 2 * sizeof(int32_t), hipMemcpyDeviceToHost));
    RD_REQUIRE(!(hf[0] & BAD_DUP), "duplicate edge in the edge list");
    if (hf[0] & BAD_ISOLATED) throw RdError{RD_E_NOT_CONNECTED, "graph has an isolated node"};
    g->max_deg = hf[1];
    compute_volume(g);

    // connectivity: level-synchronous BFS from node 0
    {
      int32_t *visited = (int32_t *)keys;  // reuse sort buffers (nnz*8 bytes >= 3n*4)
      int32_t *fa = visited + n;
      int32_t *fb = (int32_t *)keys2;
      int32_t *cnt = dflags + 1;
      hipLaunchKernelGGL(k_bfs_seed, dim3(grid_for(n, 256)), dim3(256), 0, 0, n, visited, fa);
      int32_t nf = 1;
      int64_t reached = 1;
      while (nf > 0) {
        RD_HIP(hipMemset(cnt, 0, sizeof(int32_t)));
        hipLaunchKernelGGL(k_bfs_level, dim3(grid_for((int64_t)nf * 64, 256)), dim3(256), 0, 0, nf,
                           fa, g->row_ptr, g->col, visited, fb, cnt);
        RD_HIP(hipGetLastError());
        RD_HIP(hipMemcpy(&nf, cnt, sizeof(int32_t), hipMemcpyDeviceToHost));
        reached += nf;
        std::swap(fa, fb);
      }
      if (reached != n) throw RdError{RD_E_NOT_CONNECTED, "graph is not connected"};
    }

    std::vector<int32_t> rp(n + 1);
    RD_HIP(hipMemcpy(rp.data(), g->row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    build_row_blocks(g, rp, SPMV_BLOCK_NNZ, SPMV_BLOCK_ROWS);

    for (void *p : owned) dev_free(p);
    owned.clear();
    *out = g;
    return RD_OK;
  } catch (const RdError &e) {
    for (void *p : owned) dev_free(p);
    (void)hipDeviceSynchronize();
    (void)hipGetLastError();
    free_graph_memory(g);
    delete g;
    g_init_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    for (void *p : owned) dev_free(p);
    free_graph_memory(g);
    delete g;
    return RD_E_OOM;
  }
}

rd_status rd_set_weights(rd_graph g, const void *w, int32_t w_dtype, uint32_t flags) {
  if (!g || !w) return RD_E_ARG;
  try {
    g->err.clear();
    RD_REQUIRE(w_dtype == RD_F64 || w_dtype == RD_F32, "w_dtype must be RD_F64 or RD_F32");
    std::vector<void *> owned;
    int32_t *dflags = (int32_t *)dev_alloc(sizeof(int32_t));
    RD_HIP(hipMemset(dflags, 0, sizeof(int32_t)));
    int32_t hf = 0;
    try {
      bool dp = flags & RD_DEVICE_PTRS;
      if (w_dtype == RD_F64) {
        const double *dw = to_device((const double *)w, g->m, dp, owned);
        hipLaunchKernelGGL(k_check_weights<double>, dim3(grid_for(g->m, 256)), dim3(256), 0, 0, g->m,
                           dw, dflags);
      } else {
        const float *dw = to_device((const float *)w, g->m, dp, owned);
        hipLaunchKernelGGL(k_check_weights<float>, dim3(grid_for(g->m, 256)), dim3(256), 0, 0, g->m,
                           dw, dflags);
      }
      RD_HIP(hipGetLastError());
      RD_HIP(hipMemcpy(&hf, dflags, sizeof(int32_t), hipMemcpyDeviceToHost));
    } catch (...) {
      for (void *p : owned) dev_free(p);
      dev_free(dflags);
      throw;
    }
    for (void *p : owned) dev_free(p);
    dev_free(dflags);
    RD_REQUIRE(!(hf & BAD_WEIGHT), "edge weights must be finite and > 0");
    set_weights_impl(g, w, w_dtype, flags);
    return RD_OK;
  } catch (const RdError &e) {
    g->err = e.msg;
    return e.code;
  }
}

void rd_free_graph(rd_graph g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  free_graph_memory(g);
  delete g;
}

}  // extern "C"
