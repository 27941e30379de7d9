// Lanczos Push (Algorithm 4): the subset Lanczos recurrence
//   beta_{i+1} v_{i+1} = AMV(calA, v_i) - alpha_i v_i|S_i - beta_i v_{i-1}|S_{i-1}
// run locally: one workgroup per pair keeps the nonzero entries of v_i as a
// list (the frontier) over per-slot node arrays, and only touched entries are
// read or written, so the work follows the pushed edges, not the graph size.
//
// Per iteration i (block barriers between the phases):
//   targets  each frontier node u (a thread, or a wavefront for rows longer
//            than 64 entries) marks every neighbour v with |v_i(u)| >
//            eps sqrt(d_u d_v) (Definition of AMV); each first mark appends v to
//            the candidate list C (flag array); the nodes of
//            S_{i-1} = {u : |v_{i-1}(u)| > eps d_u} and S_i join C;
//   sums     each candidate v pulls AMV(calA, v_i)(v) = sum over its pushing
//            neighbours u of w_uv v_i(u) / sqrt(d_u d_v), in adjacency order, and
//            subtracts beta_i v_{i-1}(v) when v is in S_{i-1};
//   alpha    alpha_i = <v_{i+1}, v_i> over C;
//   update   v_{i+1} -= alpha_i v_i on S_i; beta_{i+1}^2 = sum over C;
//   rotate   v_{i+1} / beta_{i+1} on the nonzero entries of C becomes the next
//            frontier; the arrays of v_{i-1}, the sums and the flags are
//            cleared over the entries that were used.
// The output r' = (1/d_s + 1/d_t) v_1^T V (I - T)^{-1} e_1 needs
// <v_1, v_j> = v_1(s) v_j(s) + v_1(t) v_j(t) per iteration and a k x k
// tridiagonal solve at the end (thread 0).
//
// Every per-node sum runs in adjacency order and alpha, beta^2 are summed in
// fixed point (integer words), so the order of the lists, which the atomics
// that build them decide, changes nothing: runs are bitwise reproducible.

#include <algorithm>
#include <cmath>
#include <vector>

#include "lanczos_common.h"

namespace {

constexpr int PUSH_THREADS = 1024;
constexpr int PUSH_WAVES = PUSH_THREADS / 64;

// Order-independent sums: a term x (|x| < 2^20) is split into integer words in
// units of 2^-40 and 2^-80; integer addition does not depend on the order in
// which the threads and lists deliver the terms.
__device__ __forceinline__ void fx_add(double x, long long &hi, long long &lo) {
  const double sx = x * 0x1p40;
  const double h = floor(sx);
  hi += (long long)h;
  lo += (long long)rint((sx - h) * 0x1p40);
}

// Block total of the two words (every thread gets it), as a double.
__device__ __forceinline__ double fx_block_total(long long hi, long long lo, long long *sm) {
  for (int off = 32; off > 0; off >>= 1) {
    hi += __shfl_xor(hi, off, 64);
    lo += __shfl_xor(lo, off, 64);
  }
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    sm[2 * wid] = hi;
    sm[2 * wid + 1] = lo;
  }
  __syncthreads();
  long long th = 0, tl = 0;
  for (int wv = 0; wv < PUSH_WAVES; ++wv) {
    th += sm[2 * wv];
    tl += sm[2 * wv + 1];
  }
  return (double)th * 0x1p-40 + (double)tl * 0x1p-80;
}

template <bool WEIGHTED>
__global__ __launch_bounds__(PUSH_THREADS) void k_push(
    int32_t n, const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    const double *__restrict__ w, const double *__restrict__ deg, int32_t npairs,
    const int32_t *__restrict__ ps, const int32_t *__restrict__ pt, int32_t k, double eps,
    double *va_all, double *vb_all, double *y_all, int32_t *flag_all, int32_t *la_all, int32_t *lb_all,
    int32_t *lc_all, double *hist_all, rd_result *__restrict__ out) {
  __shared__ long long red[2 * PUSH_WAVES];
  __shared__ int32_t cnt_c, cnt_next;
  const size_t off = (size_t)blockIdx.x * n;
  double *vcur = va_all + off, *vprev = vb_all + off, *y = y_all + off;
  int32_t *flag = flag_all + off;
  int32_t *fcur = la_all + off, *fprev = lb_all + off, *cand = lc_all + off;
  double *hist = hist_all + (size_t)blockIdx.x * 4 * k;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;

  for (int32_t pair = blockIdx.x; pair < npairs; pair += gridDim.x) {
    const int32_t s = ps[pair], t = pt[pair];
    if (s == t) {
      if (threadIdx.x == 0) out[pair] = rd_result{0.0, 0.0, 0, RD_OK};
      continue;
    }
    const double c = 1.0 / deg[s] + 1.0 / deg[t];
    const double v1s = 1.0 / sqrt(deg[s]) / sqrt(c), v1t = -1.0 / sqrt(deg[t]) / sqrt(c);
    if (threadIdx.x == 0) {
      vcur[s] = v1s;
      vcur[t] = v1t;
      fcur[0] = s;
      fcur[1] = t;
    }
    int32_t nf = 2, nfp = 0;
    double beta = 0.0;
    int32_t kk = 0;
    __syncthreads();
    for (int32_t i = 0; i < k; ++i) {
      if (threadIdx.x == 0) {
        cnt_c = 0;
        cnt_next = 0;
        hist[2 * k + i] = v1s * vcur[s] + v1t * vcur[t];
      }
      __syncthreads();
      // targets: every neighbour v that receives a push (|v_i(u)| >
      // eps sqrt(d_u d_v)) joins the candidates; a thread per frontier node with
      // at most 64 entries, a wavefront (lanes over the entries) per longer row
      for (int32_t idx = threadIdx.x; idx < nf; idx += PUSH_THREADS) {
        const int32_t u = fcur[idx];
        const int32_t pb = row_ptr[u], pe = row_ptr[u + 1];
        if (pe - pb > 64) continue;
        const double val = fabs(vcur[u]), su = sqrt(deg[u]);
        for (int32_t p = pb; p < pe; ++p) {
          const int32_t v = col[p];
          if (val > eps * (su * sqrt(deg[v])) && atomicExch(&flag[v], 1) == 0) cand[atomicAdd(&cnt_c, 1)] = v;
        }
      }
      for (int32_t idx = wid; idx < nf; idx += PUSH_WAVES) {
        const int32_t u = fcur[idx];
        const int32_t pb = row_ptr[u], pe = row_ptr[u + 1];
        if (pe - pb <= 64) continue;
        const double val = fabs(vcur[u]), su = sqrt(deg[u]);
        for (int32_t p = pb + lane; p < pe; p += 64) {
          const int32_t v = col[p];
          if (val > eps * (su * sqrt(deg[v])) && atomicExch(&flag[v], 1) == 0) cand[atomicAdd(&cnt_c, 1)] = v;
        }
      }
      // restrict: beta_i v_{i-1} on S_{i-1}; S_{i-1} and S_i join the candidates
      for (int32_t idx = threadIdx.x; idx < nfp; idx += PUSH_THREADS) {
        const int32_t u = fprev[idx];
        if (fabs(vprev[u]) > eps * deg[u] && atomicExch(&flag[u], 1) == 0) cand[atomicAdd(&cnt_c, 1)] = u;
      }
      for (int32_t idx = threadIdx.x; idx < nf; idx += PUSH_THREADS) {
        const int32_t u = fcur[idx];
        if (fabs(vcur[u]) > eps * deg[u] && atomicExch(&flag[u], 1) == 0) cand[atomicAdd(&cnt_c, 1)] = u;
      }
      __syncthreads();
      const int32_t nc = cnt_c;
      // each candidate's sum, pulled in adjacency order (deterministic): AMV,
      // then - beta_i v_{i-1} on S_{i-1}; alpha_i in fixed point
      long long ah = 0, al = 0;
      for (int32_t idx = threadIdx.x; idx < nc; idx += PUSH_THREADS) {
        const int32_t v = cand[idx];
        const double sv = sqrt(deg[v]);
        double acc = 0.0;
        const int32_t pe = row_ptr[v + 1];
        for (int32_t p = row_ptr[v]; p < pe; ++p) {
          const int32_t u = col[p];
          const double val = vcur[u];
          if (val == 0.0) continue;
          const double sq = sqrt(deg[u]) * sv;
          if (fabs(val) > eps * sq) acc += (WEIGHTED ? w[p] : 1.0) * val / sq;
        }
        const double vp = vprev[v];
        if (fabs(vp) > eps * deg[v]) acc -= beta * vp;
        y[v] = acc;
        fx_add(acc * vcur[v], ah, al);
      }
      const double alpha = fx_block_total(ah, al, red);
      long long bh = 0, bl = 0;
      for (int32_t idx = threadIdx.x; idx < nc; idx += PUSH_THREADS) {
        const int32_t v = cand[idx];
        double x = y[v];
        if (fabs(vcur[v]) > eps * deg[v]) {
          x -= alpha * vcur[v];
          y[v] = x;
        }
        fx_add(x * x, bh, bl);
      }
      const double bnext = sqrt(fx_block_total(bh, bl, red));
      if (threadIdx.x == 0) {
        hist[i] = alpha;
        hist[k + i] = bnext;
      }
      kk = i + 1;
      const bool last = i == k - 1 || bnext == 0.0;
      // v_{i-1} is no longer needed
      for (int32_t idx = threadIdx.x; idx < nfp; idx += PUSH_THREADS) vprev[fprev[idx]] = 0.0;
      __syncthreads();
      // the next frontier from the nonzero candidates, into the freed arrays
      for (int32_t idx = threadIdx.x; idx < nc; idx += PUSH_THREADS) {
        const int32_t v = cand[idx];
        const double x = y[v];
        if (!last && x != 0.0) {
          vprev[v] = x / bnext;
          fprev[atomicAdd(&cnt_next, 1)] = v;
        }
        y[v] = 0.0;
        flag[v] = 0;
      }
      __syncthreads();
      if (last) break;
      {
        double *tv = vprev;
        vprev = vcur;
        vcur = tv;
        int32_t *tl = fprev;
        fprev = fcur;
        fcur = tl;
      }
      nfp = nf;
      nf = cnt_next;
      beta = bnext;
      __syncthreads();
    }
    // clear what is left of the pair's vectors
    for (int32_t idx = threadIdx.x; idx < nf; idx += PUSH_THREADS) vcur[fcur[idx]] = 0.0;
    for (int32_t idx = threadIdx.x; idx < nfp; idx += PUSH_THREADS) vprev[fprev[idx]] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      // (I - T) z = e_1 (diagonal 1 - alpha_j, off-diagonal -beta_{j+2} between
      // rows j and j+1) by the Thomas algorithm, then r' = c sum_j <v_1, v_j> z_j
      double *piv = hist;          // pivots, over alpha (read before written)
      double *fw = hist + 3 * k;   // forward values of e_1
      piv[0] = 1.0 - hist[0];
      fw[0] = 1.0;
      for (int32_t j = 1; j < kk; ++j) {
        const double b = hist[k + j - 1];
        fw[j] = b / piv[j - 1] * fw[j - 1];
        piv[j] = (1.0 - hist[j]) - b * b / piv[j - 1];
      }
      double r = 0.0, znext = 0.0;
      for (int32_t j = kk - 1; j >= 0; --j) {
        const double b = j + 1 < kk ? hist[k + j] : 0.0;
        const double z = (fw[j] + b * znext) / piv[j];
        r += hist[2 * k + j] * z;
        znext = z;
      }
      out[pair] = rd_result{c * r, 0.0, kk, RD_OK};
    }
    __syncthreads();
  }
}

}  // namespace

static void push_run(rd_graph g, int32_t npairs, const int32_t *ps, const int32_t *pt, int32_t k, double eps,
              hipStream_t st, rd_result *out) {
  if (npairs <= 0) return;
  const size_t n = (size_t)g->n;
  const size_t per_slot = n * (3 * sizeof(double) + 4 * sizeof(int32_t));
  const size_t budget = (size_t)48 << 30;  // of the 288 GB HBM
  int32_t slots = (int32_t)std::min<size_t>({(size_t)npairs, (size_t)512, std::max<size_t>(1, budget / per_slot)});
  // every buffer is freed on return and on an exception alike
  struct Bufs {
    std::vector<void *> p;
    ~Bufs() {
      (void)hipDeviceSynchronize();  // no launch may still use them
      for (void *x : p) dev_free(x);
    }
    void *get(size_t bytes) {
      p.push_back(nullptr);
      p.back() = dev_alloc(bytes);
      return p.back();
    }
  } bufs;
  const size_t sn = (size_t)slots * n;
  double *va = (double *)bufs.get(sn * sizeof(double));
  double *vb = (double *)bufs.get(sn * sizeof(double));
  double *yv = (double *)bufs.get(sn * sizeof(double));
  int32_t *fl = (int32_t *)bufs.get(sn * sizeof(int32_t));
  int32_t *la = (int32_t *)bufs.get(sn * sizeof(int32_t));
  int32_t *lb = (int32_t *)bufs.get(sn * sizeof(int32_t));
  int32_t *lc = (int32_t *)bufs.get(sn * sizeof(int32_t));
  double *hist = (double *)bufs.get((size_t)slots * 4 * k * sizeof(double));
  RD_HIP(hipMemsetAsync(va, 0, sn * sizeof(double), st));
  RD_HIP(hipMemsetAsync(vb, 0, sn * sizeof(double), st));
  RD_HIP(hipMemsetAsync(yv, 0, sn * sizeof(double), st));
  RD_HIP(hipMemsetAsync(fl, 0, sn * sizeof(int32_t), st));
  if (g->unit)
    hipLaunchKernelGGL((k_push<false>), dim3(slots), dim3(PUSH_THREADS), 0, st, g->n, g->row_ptr, g->col,
                       (const double *)nullptr, g->deg, npairs, ps, pt, k, eps, va, vb, yv, fl, la, lb, lc,
                       hist, out);
  else
    hipLaunchKernelGGL((k_push<true>), dim3(slots), dim3(PUSH_THREADS), 0, st, g->n, g->row_ptr, g->col,
                       (const double *)g->w64, g->deg, npairs, ps, pt, k, eps, va, vb, yv, fl, la, lb, lc,
                       hist, out);
  RD_HIP(hipGetLastError());
  RD_HIP(hipStreamSynchronize(st));
}

extern "C" rd_status rd_lanczos_push(rd_graph g, int32_t npairs, const int32_t *s, const int32_t *t, int32_t k,
                                     double eps, const rd_options *o, rd_result *out) {
  if (!g || npairs < 0 || k < 1 || !(eps >= 0.0) || (npairs > 0 && (!s || !t || !out))) return RD_E_ARG;
  std::vector<void *> owned;
  try {
    g->err.clear();
    rd_options opt = resolve_options(g, o);
    if (npairs == 0) return RD_OK;
    RD_HIP(hipSetDevice(g->device));
    hipStream_t st = pick_stream(g, o);
    const bool dp = opt.flags & RD_DEVICE_PTRS;
    std::vector<int32_t> hs(npairs), ht(npairs);
    if (dp) {
      RD_HIP(hipMemcpyAsync(hs.data(), s, npairs * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      RD_HIP(hipMemcpyAsync(ht.data(), t, npairs * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      RD_HIP(hipStreamSynchronize(st));
    } else {
      std::copy(s, s + npairs, hs.begin());
      std::copy(t, t + npairs, ht.begin());
    }
    for (int32_t p = 0; p < npairs; ++p) {
      RD_REQUIRE(hs[p] >= 0 && hs[p] < g->n && ht[p] >= 0 && ht[p] < g->n, "pair node ids must be in [0, n)");
      if (g->perm) {
        hs[p] = g->perm_host[hs[p]];
        ht[p] = g->perm_host[ht[p]];
      }
    }
    int32_t *dpair = (int32_t *)dev_alloc(2 * (size_t)npairs * sizeof(int32_t));
    owned.push_back(dpair);
    RD_HIP(hipMemcpyAsync(dpair, hs.data(), npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
    RD_HIP(hipMemcpyAsync(dpair + npairs, ht.data(), npairs * sizeof(int32_t), hipMemcpyHostToDevice, st));
    rd_result *dout = out;
    if (!dp) {
      dout = (rd_result *)dev_alloc((size_t)npairs * sizeof(rd_result));
      owned.push_back(dout);
    }
    push_run(g, npairs, dpair, dpair + npairs, k, eps, st, dout);
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
