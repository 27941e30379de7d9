"""Benchmark: resistance-distance queries per second on one MI355X.

Workload (default): batched queries on a Chung-Lu power-law graph with
n = 4,000,000, degree exponent 2.3, mean degree 32 (about 64M undirected
edges, unit weights, largest connected component), 4,096 (s,t) pairs - half
uniform, half with s among the top 1% nodes by degree - each run to a relative
tolerance of 1e-4 with FP32 sparse products and FP64 Lanczos scalars.

One step = one rd_query_batch call over all pairs, with the graph, the pair
lists and the result array resident in device memory. Printed beside it:
  * the plain single-pair FP64 loop (rd_query) on the same GPU and graph, on
    a sample of the same pairs, and the batched/plain ratio;
  * the roofline of the dominant kernel (the batched short-row sparse
    product), its live duration from HIP events recorded around each launch;
  * the CPU FP64 oracle timed on a bounded sample of pairs;
  * the relative error of the timed GPU results against that oracle sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RD queries/s at 1e-4 rel err (batched FP32 vs plain FP64) + SpMV HBM GB/s"
HBM_PEAK_GBS = 8000.0
EPS = 1e-4

WORKLOADS = {
    "chung_lu_n4M_g2.3_d32_4096pairs": dict(n=4_000_000, gamma=2.3, mean_deg=32.0, seed=4,
                                             pairs=4096, pair_seed=4, hub_seed=40),
    # smaller stand-in for quick checks
    "chung_lu_n500k_g2.3_d32_1024pairs": dict(n=500_000, gamma=2.3, mean_deg=32.0, seed=4,
                                               pairs=1024, pair_seed=4, hub_seed=40),
}
# further workloads, one JSON line each (not the default line)
OTHER_WORKLOADS = ["grid_64x64_100pairs_fp64", "chung_lu_n1M_g2.1_d20_plain_fp64",
                   "road_like_2000x2000_256pairs", "weighted_chung_lu_n1M_grad_256pairs",
                   "grid_64x64_100pairs_power_method", "weighted_chung_lu_n1M_potentials_256pairs",
                   "condition_numbers", "road_like_2000x2000_lanczos_push", "road_like_90x90_power_method"]


def _line(metric_unit, value, steps, warmup, ms_per_step, dtype, config, **extra):
    d = {"metric": METRIC, "value": round(value, 3), "unit": metric_unit, "n_gpus": 1, "steps": steps,
         "warmup": warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
         "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    d.update(extra)
    return d


def _plain_rate(G, rd, s, t, eps, opts):
    """Plain single-pair loop over the given pairs: (q/s, results, launches stats)."""
    import torch
    G.query(int(s[0]), int(t[0]), eps, opts)
    G.kernel_stats(1)
    torch.cuda.synchronize()
    t0 = time.time()
    rs, its = [], []
    for p in range(len(s)):
        r = G.query(int(s[p]), int(t[p]), eps, opts)
        rs.append(r.r)
        its.append(r.iters)
    torch.cuda.synchronize()
    dt = time.time() - t0
    ms, n, b = G.kernel_stats(1)
    avg = ms / max(n, 1)
    roof = {"kernel": "k_spmv (single-pair sparse product)", "bound": "hbm",
            "achieved": round(b / (avg * 1e-3) / 1e9, 1) if n else None, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(b / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if n else None,
            "traffic": None, "avg_launch_ms": round(avg, 4), "launches": n, "alg_bytes_per_launch": b}
    return len(s) / dt, np.array(rs), np.array(its), roof, dt


def _batch_rate(G, rd, s, t, eps, opts, steps=1):
    import torch
    G.query_batch(s[: min(len(s), 64)], t[: min(len(s), 64)], eps, opts)
    log("  warm-up done")
    G.kernel_stats(0)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(steps):
        out = G.query_batch(s, t, eps, opts)
    torch.cuda.synchronize()
    dt = (time.time() - t0) / steps
    ms, n, b = G.kernel_stats(0)
    avg = ms / max(n, 1)
    roof = {"kernel": "k_spmm_short (batched sparse product over the short rows)", "bound": "hbm",
            "achieved": round(b / (avg * 1e-3) / 1e9, 1) if n else None, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(b / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if n else None,
            "traffic": None, "avg_launch_ms": round(avg, 4), "launches": n, "alg_bytes_per_launch": b}
    return len(s) / dt, out, roof, dt


def _oracle_sample(g, s, t, tol, budget_s=20.0, max_iters=None):
    from threadpoolctl import threadpool_limits
    from oracle import lanczos as LZ
    t0 = time.time()
    A, d = LZ.normalized_adjacency(g)
    setup = time.time() - t0
    vals, its, secs = [], [], 0.0
    with threadpool_limits(limits=1):
        for p in range(len(s)):
            t1 = time.time()
            run = LZ.lanczos_rd(g, int(s[p]), int(t[p]), tol=tol, A=A, d=d, max_iters=max_iters)
            secs += time.time() - t1
            vals.append(run.r)
            its.append(run.k)
            if secs > budget_s:
                break
    return np.array(vals), np.array(its), secs, setup


def run_other(name, args):
    """Secondary workloads: one JSON line each."""
    import torch
    torch.cuda.set_device(0)
    from paper_2601_11159_amd import inputs as I
    from paper_2601_11159_amd import rd

    if name == "grid_64x64_100pairs_fp64":
        from oracle import dense as D
        g = I.grid(64, 64)
        s, t = I.uniform_pairs(g.n, 100, seed=1)
        G = rd.RDGraph(g.n, g.u, g.v)
        plain_qps, pr, pit, proof, pdt = _plain_rate(G, rd, s, t, 1e-8, rd.rd_default_options(flags=rd.RD_PROFILE))
        bq, bout, broof, bdt = _batch_rate(G, rd, s, t, 1e-8, rd.rd_default_options(flags=rd.RD_PROFILE), steps=3)
        truth = D.rd_all(g, s, t)
        vals, its, secs, setup = _oracle_sample(g, s, t, 1e-8, budget_s=15.0)
        line = _line("queries/s", plain_qps, 1, 1, pdt * 1e3, "f64",
                     {"workload": name, "n": g.n, "m": g.m, "pairs": 100, "eps_rel": 1e-8,
                      "path": "plain single-pair FP64 (value); batched FP64 beside it"},
                     batched_fp64={"value": round(bq, 2), "unit": "queries/s", "roofline": broof},
                     roofline=dict(proof, note="4,096-node graph: L2-resident, latency-bound"),
                     cpu_baseline={"value": round(len(vals) / secs, 3), "unit": "queries/s", "cores": 1,
                                   "kind": "oracle", "sample": f"{len(vals)} of the 100 pairs, numpy Algorithm 3 at 1e-8"},
                     parity={"plain_max_rel_err_vs_dense": float(np.max(np.abs(pr - truth) / truth)),
                             "batched_max_rel_err_vs_dense": float(np.max(np.abs(bout['r'] - truth) / truth)),
                             "mean_iters": float(pit.mean())})
    elif name == "chung_lu_n1M_g2.1_d20_plain_fp64":
        g = I.chung_lu(1_000_000, 2.1, 20.0, 2)
        s, t = I.uniform_pairs(g.n, 1000, seed=2)
        G = rd.RDGraph(g.n, g.u, g.v, reorder=bool(args.reorder))
        npl = 200
        plain_qps, pr, pit, proof, pdt = _plain_rate(G, rd, s[:npl], t[:npl], 1e-6,
                                                     rd.rd_default_options(flags=rd.RD_PROFILE))
        bq, bout, broof, bdt = _batch_rate(G, rd, s, t, 1e-6, rd.rd_default_options(flags=rd.RD_PROFILE))
        vals, its, secs, setup = _oracle_sample(g, s[:6], t[:6], 1e-6)
        k = len(vals)
        line = _line("queries/s", plain_qps, 1, 1, pdt / npl * 1e3, "f64",
                     {"workload": name, "n": g.n, "m": g.m, "pairs": 1000, "eps_rel": 1e-6,
                      "node_order": "decreasing degree (RD_REORDER)" if args.reorder else "as generated",
                      "path": f"plain single-pair FP64 on {npl} pairs (value); batched FP64 on all 1000 beside it"},
                     batched_fp64={"value": round(bq, 2), "unit": "queries/s", "roofline": broof},
                     roofline=proof,
                     cpu_baseline={"value": round(k / secs, 4), "unit": "queries/s", "cores": 1, "kind": "oracle",
                                   "sample": f"{k} pairs, numpy Algorithm 3 at 1e-6 ({secs:.1f}s after a {setup:.1f}s build)"},
                     parity={"plain_max_rel_err_vs_oracle": float(np.max(np.abs(pr[:k] - vals) / vals)),
                             "batched_max_rel_err_vs_oracle": float(np.max(np.abs(bout['r'][:k] - vals) / vals)),
                             "mean_iters": float(pit.mean())})
    elif name == "road_like_2000x2000_256pairs":
        g = I.road_like(2000, seed=3)
        s, t = I.uniform_pairs(g.n, 256, seed=3)
        G = rd.RDGraph(g.n, g.u, g.v)
        ref = np.array([G.query(int(s[p]), int(t[p]), 1e-10, rd.rd_default_options(max_iters=100000)).r
                        for p in range(8)])
        log("reference values at eps 1e-10 done")
        npl = 8
        plain_qps, pr, pit, proof, pdt = _plain_rate(G, rd, s[:npl], t[:npl], 1e-4,
                                                     rd.rd_default_options(flags=rd.RD_PROFILE, max_iters=100000))
        o32 = rd.rd_default_options(precision=rd.RD_F32, refine=1, block_width=64, max_iters=100000,
                                    flags=rd.RD_PROFILE)
        log(f"plain FP64: {plain_qps:.3f} q/s")
        bq, bout, broof, bdt = _batch_rate(G, rd, s, t, 1e-5, o32)
        log(f"batched FP32 refined: {bq:.3f} q/s")
        raw = G.query_batch(s[:64], t[:64], 1e-4, rd.rd_default_options(precision=rd.RD_F32, block_width=64,
                                                                         max_iters=100000))
        # batched FP64 (no refinement) on all pairs at the 1e-4 target
        log("batched FP32 unrefined (64 pairs) done")
        w64 = G.tune_width(rd.RD_F64, len(s))
        sched = G.batch_schedule()
        o64 = rd.rd_default_options(precision=rd.RD_F64, block_width=w64, max_iters=100000, flags=rd.RD_PROFILE)
        b64q, b64out, b64roof, b64dt = _batch_rate(G, rd, s, t, 1e-4, o64)
        log(f"batched FP64 (width {w64}, schedule {sched}): {b64q:.3f} q/s")
        # CPU oracle: a bounded number of iterations of one pair, scaled to a query
        from threadpoolctl import threadpool_limits
        from oracle import lanczos as LZ
        A, d = LZ.normalized_adjacency(g)
        with threadpool_limits(limits=1):
            t1 = time.time()
            LZ.lanczos_rd(g, int(s[0]), int(t[0]), k=300, A=A, d=d)
            per_it = (time.time() - t1) / 300
        # value: the fastest path that meets 1e-4 here (batched FP64); the FP32
        # path stops at ~1.2e-4 on this graph even with the FP64 energy refinement
        line = _line("queries/s", b64q, 1, 1, b64dt * 1e3, "f64",
                     {"workload": name, "n": g.n, "m": g.m, "pairs": 256, "eps_rel": 1e-4,
                      "path": "batched FP64 at eps 1e-4 (value); plain FP64 at 1e-4 on 8 pairs and "
                              "batched FP32 + FP64 energy refinement at eps 1e-5, width 64, beside it",
                      "block_width": w64, "block_width_source": "autotuned",
                      "row_schedule": dict(zip(("wave_nnz", "long_deg"), sched)),
                      "node_order": "as generated (grid order; the degree relabelling breaks the "
                                    "neighbour locality and is slower here)"},
                     plain_fp64={"value": round(plain_qps, 3), "unit": "queries/s", "mean_iters": float(pit.mean()),
                                 "roofline": proof},
                     speedup_batched_fp64_vs_plain_fp64=round(b64q / plain_qps, 2),
                     batched_fp32_refined={"value": round(bq, 3), "unit": "queries/s", "eps_rel": 1e-5,
                                           "max_rel_err": float(np.max(np.abs(bout['r'][:8] - ref) / ref)),
                                           "roofline": dict(broof, note="refinement adds the two potential streams (P, X)"),
                                           "speedup_vs_plain_fp64": round(bq / plain_qps, 2)},
                     roofline=b64roof,
                     cpu_baseline={"value": round(1.0 / (per_it * float(pit.mean())), 6), "unit": "queries/s",
                                   "cores": 1, "kind": "oracle",
                                   "sample": f"300 iterations of numpy Algorithm 3 on one pair ({per_it * 300:.1f}s), "
                                             f"scaled by the mean FP64 iteration count {pit.mean():.0f}"},
                     parity={"reference": "plain FP64 GPU at eps 1e-10 on 8 pairs (the oracle's parity on "
                                          "road-like grids is tested at 300x300)",
                             "batched_fp32_refined_max_rel_err": float(np.max(np.abs(bout['r'][:8] - ref) / ref)),
                             "batched_fp32_unrefined_max_rel_err": float(np.max(np.abs(raw['r'][:8] - ref) / ref)),
                             "batched_fp64_max_rel_err": float(np.max(np.abs(b64out['r'][:8] - ref) / ref)),
                             "plain_fp64_max_rel_err": float(np.max(np.abs(pr - ref) / ref))})
    elif name == "weighted_chung_lu_n1M_grad_256pairs":
        g = I.chung_lu(1_000_000, 2.1, 20.0, 2)
        w = I.lognormal_weights(g.m, 0.0, 1.0, seed=5)
        s, t = I.uniform_pairs(g.n, 256, seed=6)
        G = rd.RDGraph(g.n, g.u, g.v, w, reorder=bool(args.reorder))
        o = rd.rd_default_options(precision=rd.RD_F32, block_width=64, flags=rd.RD_PROFILE)
        G.grad_edges(s[:64], t[:64], None, 1e-6, o)
        torch.cuda.synchronize()
        G.kernel_stats(2)
        t0 = time.time()
        fwd, gw = G.grad_edges(s, t, None, 1e-6, o)
        torch.cuda.synchronize()
        dt = time.time() - t0
        gms, gl, gbytes = G.kernel_stats(2)
        gavg = gms / max(gl, 1)
        groof = {"kernel": "k_grad_edges (edge pass over 64 harvested potentials, FP32)", "bound": "hbm",
                 "achieved": round(gbytes / (gavg * 1e-3) / 1e9, 1) if gl else None, "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": round(gbytes / (gavg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if gl else None,
                 "traffic": None, "avg_launch_ms": round(gavg, 4), "launches": gl, "alg_bytes_per_launch": gbytes}
        t0 = time.time()
        out = G.query_batch(s, t, 1e-6, rd.rd_default_options(precision=rd.RD_F32, block_width=64))
        torch.cuda.synchronize()
        fdt = time.time() - t0
        euler = float(np.dot(w.astype(np.float64), gw.astype(np.float64)))
        gw_graph = I.Graph(g.n, g.u, g.v, w)
        vals, its, secs, setup = _oracle_sample(gw_graph, s[:2], t[:2], 1e-6)
        line = _line("pairs/s (forward + edge gradient)", len(s) / dt, 1, 1, dt * 1e3, "f32",
                     {"workload": name, "n": g.n, "m": g.m, "pairs": 256, "eps_rel": 1e-6,
                      "path": "rd_grad_edges, FP32 vectors, width 64",
                      "node_order": "decreasing degree (RD_REORDER)" if args.reorder else "as generated"},
                     forward_only={"value": round(len(s) / fdt, 2), "unit": "queries/s"},
                     roofline=groof,
                     cpu_baseline={"value": round(len(vals) / secs, 4), "unit": "queries/s (forward only)",
                                   "cores": 1, "kind": "oracle",
                                   "sample": f"{len(vals)} pairs, numpy Algorithm 3 forward at 1e-6"},
                     parity={"euler_identity_rel_err": abs(euler + float(fwd['r'].sum())) / float(fwd['r'].sum()),
                             "forward_max_rel_err_vs_oracle": float(np.max(np.abs(fwd['r'][:len(vals)] - vals) / vals))})
    elif name == "weighted_chung_lu_n1M_potentials_256pairs":
        # electric potentials (Section 6.3) of C5's pairs, left in device memory
        g = I.chung_lu(1_000_000, 2.1, 20.0, 2)
        w = I.lognormal_weights(g.m, 0.0, 1.0, seed=5)
        s, t = I.uniform_pairs(g.n, 256, seed=6)
        G = rd.RDGraph(g.n, g.u, g.v, w, reorder=True)
        eps = 1e-6
        opts = rd.rd_default_options(precision=rd.RD_F32, block_width=64, flags=rd.RD_PROFILE)
        ds = torch.tensor(s, dtype=torch.int32, device="cuda")
        dt = torch.tensor(t, dtype=torch.int32, device="cuda")
        out = torch.zeros(24 * len(s), dtype=torch.uint8, device="cuda")
        phi = torch.empty((len(s), g.n), dtype=torch.float64, device="cuda")
        G.potentials(ds[:64], dt[:64], eps, opts, out=out[: 24 * 64], phi=phi[:64])
        G.kernel_stats(0)
        steps = max(1, args.steps)
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(steps):
            G.potentials(ds, dt, eps, opts, out=out, phi=phi)
        torch.cuda.synchronize()
        pdt = (time.time() - t0) / steps
        ms, nl, b = G.kernel_stats(0)
        avg = ms / max(nl, 1)
        res = np.frombuffer(out.cpu().numpy().tobytes(), dtype=rd.RESULT_DTYPE)
        # cpu_baseline: the oracle's Lanczos potentials (Algorithm 5's estimate) at the same
        # iteration counts, on a sample of the pairs, against the GPU's
        from threadpoolctl import threadpool_limits
        from oracle import lanczos as LZ
        gw = I.Graph(g.n, g.u, g.v, w)
        A, d = LZ.normalized_adjacency(gw)
        perr, secs, k = [], 0.0, 0
        with threadpool_limits(limits=1):
            for p in range(2):
                t1 = time.time()
                run = LZ.lanczos_rd(gw, int(s[p]), int(t[p]), k=int(res["iters"][p]), keep_vectors=True, A=A, d=d)
                ph = LZ.potentials_lanczos(gw, int(s[p]), int(t[p]), run, d)
                secs += time.time() - t1
                ph = ph - ph.mean()
                gp = phi[p].cpu().numpy()
                perr.append(float(np.abs(gp - ph).max() / np.abs(ph).max()))
                k += 1
        line = _line("pairs/s (potentials)", len(s) / pdt, steps, 1, pdt * 1e3, "f32",
                     {"workload": name, "n": g.n, "m": g.m, "pairs": 256, "eps_rel": eps,
                      "path": "rd_potentials, FP32 vectors, width 64, harvest mode with refill, phi (FP64, "
                              "256 x n) left in device memory",
                      "node_order": "decreasing degree (RD_REORDER)"},
                     roofline={"kernel": "k_spmm_short (batched FP32 sparse product over the short rows)",
                               "bound": "hbm", "achieved": round(b / (avg * 1e-3) / 1e9, 1) if nl else None,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(b / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if nl else None,
                               "traffic": None, "avg_launch_ms": round(avg, 4), "launches": nl,
                               "alg_bytes_per_launch": b},
                     cpu_baseline={"value": round(k / secs, 4), "unit": "pairs/s", "cores": 1, "kind": "oracle",
                                   "sample": f"{k} pairs, numpy Algorithm 3 with its vectors kept and the potential "
                                             "of Algorithm 5, at the GPU's iteration counts"},
                     parity={"phi_max_rel_err_vs_oracle": max(perr), "mean_iters": float(res["iters"].mean())})
    elif name == "road_like_2000x2000_lanczos_push":
        # Lanczos Push (Algorithm 4) on the road-like graph: k = 200 iterations at
        # eps = 1e-4, beside batched Lanczos (Algorithm 3) at the same k
        g = I.road_like(2000, seed=3)
        s, t = I.uniform_pairs(g.n, 256, seed=3)
        G = rd.RDGraph(g.n, g.u, g.v)
        k, eps = 200, 1e-4
        G.lanczos_push(s[:4], t[:4], k, eps)
        torch.cuda.synchronize()
        t0 = time.time()
        out = G.lanczos_push(s, t, k, eps)
        torch.cuda.synchronize()
        pdt = time.time() - t0
        lo = rd.rd_default_options(precision=rd.RD_F64, block_width=256, fixed_k=k, max_iters=k)
        G.query_batch(s[:4], t[:4], 1e-4, lo)
        torch.cuda.synchronize()
        t0 = time.time()
        lz = G.query_batch(s, t, 1e-4, lo)
        torch.cuda.synchronize()
        ldt = time.time() - t0
        # cpu_baseline: the oracle's Algorithm 4 on two of the pairs, with the
        # share of nodes it touched and of edges it pushed along
        from threadpoolctl import threadpool_limits
        from oracle import push as LPO
        W, d = LPO._adjacency(g)
        perr, touched, pushes, raw_pushes, secs = [], [], [], [], 0.0
        with threadpool_limits(limits=1):
            for p in range(2):
                t1 = time.time()
                run = LPO.lanczos_push(g, int(s[p]), int(t[p]), k, eps, W=W, d=d)
                secs += time.time() - t1
                perr.append(abs(out["r"][p] - run.r) / abs(run.r))
                touched.append(run.touched / g.n)
                pushes.append(run.pushes / (k * 2.0 * g.m))
                raw_pushes.append(run.pushes)
        line = _line("queries/s", len(s) / pdt, 1, 1, pdt * 1e3, "f64",
                     {"workload": name, "n": g.n, "m": g.m, "pairs": 256, "k": k, "eps_push": eps,
                      "path": "rd_lanczos_push: one workgroup per pair, frontier lists over per-slot node arrays"},
                     lanczos_fixed_k={"value": round(len(s) / ldt, 3), "unit": "queries/s",
                                      "path": "rd_query_batch FP64, width 256, fixed k = 200"},
                     push_vs_lanczos_same_k={"max_rel_diff": float(np.max(np.abs(out["r"] - lz["r"]) / lz["r"])),
                                             "median_rel_diff": float(np.median(np.abs(out["r"] - lz["r"]) / lz["r"]))},
                     locality={"nodes_touched_share": touched, "edge_pushes_share_of_k_full_products": pushes},
                     roofline={"kernel": "k_push (one 1024-thread workgroup per pair, all k iterations)",
                               "bound": "hbm",
                               "achieved": round(len(s) * float(np.mean(raw_pushes)) * 36.0 / pdt / 1e9, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(len(s) * float(np.mean(raw_pushes)) * 36.0 / pdt / 1e9 / HBM_PEAK_GBS, 5),
                               "traffic": None, "avg_launch_ms": round(pdt * 1e3, 3), "launches": 1,
                               "note": "algorithmic bytes: 36 per edge push (index, degree and flag in the target "
                                       "pass; index, value and degree in the pull), pushes per pair estimated "
                                       "from the oracle's counts on the sample pairs; random accesses, bound by "
                                       "their latency and the barriers between phases"},
                     cpu_baseline={"value": round(2 / secs, 4), "unit": "queries/s", "cores": 1, "kind": "oracle",
                                   "sample": "2 pairs, numpy Algorithm 4 with the same k and eps"},
                     parity={"max_rel_err_vs_oracle": float(max(perr))})
    elif name == "condition_numbers":
        # kappa_hat = 2 / (1 - theta_max) from the extreme Ritz value of a k-step
        # deflated Lanczos run (a lower bound that rises to kappa), per graph
        graphs = [("grid_64x64", lambda: (I.grid(64, 64), None), 400, False),
                  ("chung_lu_n1M_g2.1_d20", lambda: (I.chung_lu(1_000_000, 2.1, 20.0, 2), None), 100, True),
                  ("road_like_2000x2000", lambda: (I.road_like(2000, seed=3), None), 3000, False),
                  ("chung_lu_n4M_g2.3_d32", lambda: (I.chung_lu(4_000_000, 2.3, 32.0, 4), None), 100, True),
                  ("weighted_chung_lu_n1M", lambda: (I.chung_lu(1_000_000, 2.1, 20.0, 2), "w"), 100, True)]
        rows = {}
        t_all = time.time()
        for gname, make, k, reorder in graphs:
            g, wflag = make()
            w = I.lognormal_weights(g.m, 0.0, 1.0, seed=5) if wflag else None
            G = rd.RDGraph(g.n, g.u, g.v, w, reorder=reorder)
            s, t = I.uniform_pairs(g.n, 1, seed=7)
            t0 = time.time()
            lo, hi, it = G.ritz_bounds(int(s[0]), int(t[0]), k, rd.rd_default_options(flags=rd.RD_PROFILE))
            dt = time.time() - t0
            _, hi2, _ = G.ritz_bounds(int(s[0]), int(t[0]), k // 2)
            ms, nl, b = G.kernel_stats(1)
            if gname == "road_like_2000x2000":
                road_stats = (ms, nl, b)
            rows[gname] = {"k": it, "theta_min": lo, "theta_max": hi, "kappa_hat": round(2.0 / (1.0 - hi), 2),
                           "kappa_hat_at_k_over_2": round(2.0 / (1.0 - hi2), 2), "seconds": round(dt, 3),
                           "k_spmv_avg_ms": round(ms / max(nl, 1), 4)}
            log(f"  {gname}: kappa_hat {rows[gname]['kappa_hat']} (k = {it})")
            G.close()
        total = time.time() - t_all
        # the oracle's deflated Lanczos on the 64x64 grid at the same k
        from threadpoolctl import threadpool_limits
        from oracle import lanczos as LZ
        g = I.grid(64, 64)
        s, t = I.uniform_pairs(g.n, 1, seed=7)
        A, d = LZ.normalized_adjacency(g)
        with threadpool_limits(limits=1):
            t0 = time.time()
            run = LZ.lanczos_rd(g, int(s[0]), int(t[0]), k=400, A=A, d=d, reorth=1)
            th = LZ.ritz_values(run)
            osec = time.time() - t0
        c1 = rows["grid_64x64"]
        line = _line("kappa (lower bound, road-like 2000x2000)", rows["road_like_2000x2000"]["kappa_hat"], 1, 0,
                     total * 1e3, "f64",
                     {"workload": name, "graphs": rows,
                      "path": "rd_ritz_bounds: k-step FP64 Lanczos from the pair (e_s, e_t) start vector with "
                              "the null direction deflated, extreme eigenvalues of T_k by Sturm bisection"},
                     roofline={"kernel": "k_spmv (the plain FP64 product; road-like 2000x2000 run)", "bound": "hbm",
                               "achieved": round(road_stats[2] / (road_stats[0] / road_stats[1] * 1e-3) / 1e9, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(road_stats[2] / (road_stats[0] / road_stats[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "traffic": None, "avg_launch_ms": round(road_stats[0] / road_stats[1], 4),
                               "launches": road_stats[1], "alg_bytes_per_launch": road_stats[2]},
                     cpu_baseline={"value": round(1.0 / osec, 3), "unit": "runs/s (64x64 grid, k = 400)", "cores": 1,
                                   "kind": "oracle", "sample": "one deflated numpy Algorithm 3 run with its Ritz values"},
                     parity={"grid_theta_max_abs_diff_vs_oracle": abs(c1["theta_max"] - float(th[-1])),
                             "grid_theta_min_abs_diff_vs_oracle": abs(c1["theta_min"] - float(th[0]))})
    elif name == "road_like_90x90_power_method":
        # the Power Method against Lanczos at equal error on a road-like graph
        # (the paper's high-kappa case), at the configs' 1e-4 tolerance; 90 x 90
        # so that both FP64 vectors fit in LDS (single-workgroup path)
        g = I.road_like(90, seed=3)
        s, t = I.uniform_pairs(g.n, 64, seed=3)
        G = rd.RDGraph(g.n, g.u, g.v)
        f64 = dict(precision=rd.RD_F64, block_width=64)
        ref = G.query_batch(s, t, 1e-12, rd.rd_default_options(**f64))["r"]
        target = 1e-4

        def pm_err(l):
            r = G.power_method(s, t, l, rd.rd_default_options(**f64))["r"]
            e = float(np.max(np.abs(r - ref) / ref))
            log(f"  l = {l}: max rel err {e:.3g}")
            return e

        hi = 8192
        while pm_err(hi) > target and hi < (1 << 22):
            hi *= 2
        lo = hi // 2
        while hi - lo > max(16, hi // 64):
            mid = (lo + hi) // 2
            if pm_err(mid) > target:
                lo = mid
            else:
                hi = mid
        l_pm = hi
        log(f"  Power Method reaches {target:g} at l = {l_pm}")
        opts = rd.rd_default_options(flags=rd.RD_PROFILE, **f64)
        G.kernel_stats(0)
        torch.cuda.synchronize()
        t0 = time.time()
        out = G.power_method(s, t, l_pm, opts)
        torch.cuda.synchronize()
        pdt = time.time() - t0
        ms, nl, b = G.kernel_stats(0)
        avg = ms / max(nl, 1)
        lz = G.query_batch(s, t, target, rd.rd_default_options(**f64))
        bq, bout, broof, bdt = _batch_rate(G, rd, s, t, target, rd.rd_default_options(**f64), steps=2)
        _, th, _ = G.ritz_bounds(int(s[0]), int(t[0]), 3000)
        kappa = 2.0 / (1.0 - th)
        from threadpoolctl import threadpool_limits
        from oracle import power as PMO
        P, d = PMO.transition_matrix(g)
        with threadpool_limits(limits=1):
            t1 = time.time()
            v0 = PMO.power_method(g, int(s[0]), int(t[0]), l_pm, P=P, d=d)
            osec = time.time() - t1
        line = _line("queries/s", len(s) / pdt, 1, 1, pdt * 1e3, "f64",
                     {"workload": name, "n": g.n, "m": g.m, "pairs": 64, "eps_rel": target,
                      "path": f"rd_power_method, FP64, one workgroup per pair (k_pm_small), l = {l_pm} products per pair "
                              f"(the least l, to within {max(16, l_pm // 64)}, whose results are all within "
                              f"{target:g} of batched Lanczos at 1e-12)"},
                     iterations={"power_method_l": l_pm, "lanczos_mean_k": float(lz["iters"].mean()),
                                 "lanczos_max_k": int(lz["iters"].max()),
                                 "ratio_l_over_k": round(l_pm / float(lz["iters"].mean()), 1),
                                 "kappa_hat_k3000": round(kappa, 1), "sqrt_kappa_hat": round(float(np.sqrt(kappa)), 1)},
                     lanczos_batched_fp64={"value": round(bq, 2), "unit": "queries/s",
                                           "speedup_over_power_method": round(bq * pdt / len(s), 1)},
                     roofline={"kernel": "k_pm_small (all steps of a pair in one workgroup, vectors in LDS)",
                               "bound": "alu",
                               "achieved": round(len(s) * l_pm * (4.0 * g.m + 3.0 * g.n) / pdt / 1e12, 4),
                               "peak": 78.6, "unit": "TFLOP/s",
                               "frac": round(len(s) * l_pm * (4.0 * g.m + 3.0 * g.n) / pdt / 1e12 / 78.6, 5),
                               "traffic": None, "avg_launch_ms": round(pdt * 1e3, 3), "launches": 1,
                               "note": "FP64 flops per step and pair: 2 per adjacency entry, 3 per node, against "
                                       "the FP64 vector peak; LDS-resident, bound by LDS latency and the "
                                       "per-step barrier, not by arithmetic"},
                     cpu_baseline={"value": round(1.0 / osec, 4), "unit": "queries/s", "cores": 1, "kind": "oracle",
                                   "sample": "1 pair, numpy Algorithm 1 with the same l"},
                     parity={"max_rel_err_vs_oracle": abs(float(out["r"][0]) - v0) / v0,
                             "max_rel_err_vs_lanczos_1e-12": float(np.max(np.abs(out["r"] - ref) / ref))})
    elif name == "grid_64x64_100pairs_power_method":
        # the Power Method (Algorithm 1) against Lanczos at equal error (1e-8)
        import scipy.sparse as sps
        import scipy.sparse.linalg as spl
        g = I.grid(64, 64)
        s, t = I.uniform_pairs(g.n, 100, seed=1)
        G = rd.RDGraph(g.n, g.u, g.v)
        f64 = dict(precision=rd.RD_F64, block_width=128)
        ref = G.query_batch(s, t, 1e-12, rd.rd_default_options(**f64))["r"]
        target = 1e-8

        def pm_err(l):
            r = G.power_method(s, t, l, rd.rd_default_options(**f64))["r"]
            return float(np.max(np.abs(r - ref) / ref))

        hi = 1024
        while pm_err(hi) > target:
            hi *= 2
        lo = hi // 2
        while hi - lo > max(16, hi // 64):
            mid = (lo + hi) // 2
            if pm_err(mid) > target:
                lo = mid
            else:
                hi = mid
        l_pm = hi
        log(f"  Power Method reaches {target:g} at l = {l_pm}")
        # value: the single-workgroup path (vectors and CSR in LDS, all steps in one launch)
        G.power_method(s[:8], t[:8], 64, rd.rd_default_options(**f64))
        torch.cuda.synchronize()
        t0 = time.time()
        out = G.power_method(s, t, l_pm, rd.rd_default_options(**f64))
        torch.cuda.synchronize()
        pdt = time.time() - t0
        # beside it: the same l on the batched product kernels (k_spmm_short timed)
        gopts = rd.rd_default_options(flags=rd.RD_PROFILE | rd.RD_GENERAL_PATH, **f64)
        G.power_method(s[:8], t[:8], 64, gopts)
        G.kernel_stats(0)
        torch.cuda.synchronize()
        t0 = time.time()
        gout = G.power_method(s, t, l_pm, gopts)
        torch.cuda.synchronize()
        gdt = time.time() - t0
        ms, nl, b = G.kernel_stats(0)
        avg = ms / max(nl, 1)
        lz = G.query_batch(s, t, target, rd.rd_default_options(**f64))
        bq, bout, broof, bdt = _batch_rate(G, rd, s, t, target, rd.rd_default_options(**f64), steps=3)
        # kappa = 2 / mu_2 of the normalised Laplacian (shift-invert for the two smallest eigenvalues)
        w = np.ones(g.m)
        W = sps.coo_matrix((np.concatenate([w, w]), (np.concatenate([g.u, g.v]), np.concatenate([g.v, g.u]))),
                           shape=(g.n, g.n)).tocsr()
        isd = 1.0 / np.sqrt(np.asarray(W.sum(axis=1)).ravel())
        Ln = sps.identity(g.n) - sps.diags(isd) @ W @ sps.diags(isd)
        mu = np.sort(spl.eigsh(Ln.tocsc(), k=3, sigma=-1e-3, which="LM", return_eigenvectors=False))
        kappa = 2.0 / mu[1]
        # cpu_baseline: the oracle's Algorithm 1 at the same l on a sample of the pairs
        from threadpoolctl import threadpool_limits
        from oracle import power as PMO
        P, d = PMO.transition_matrix(g)
        vals, secs = [], 0.0
        with threadpool_limits(limits=1):
            for p in range(len(s)):
                t1 = time.time()
                vals.append(PMO.power_method(g, int(s[p]), int(t[p]), l_pm, P=P, d=d))
                secs += time.time() - t1
                if secs > 15.0:
                    break
        k = len(vals)
        line = _line("queries/s", len(s) / pdt, 1, 1, pdt * 1e3, "f64",
                     {"workload": name, "n": g.n, "m": g.m, "pairs": 100, "eps_rel": target,
                      "path": f"rd_power_method, FP64, one workgroup per pair (k_pm_small), l = {l_pm} "
                              f"products per pair (the least l, to within {max(16, l_pm // 64)}, whose results "
                              f"are all within {target:g} of batched Lanczos at 1e-12)"},
                     batched_product_path={"value": round(len(s) / gdt, 3), "unit": "queries/s",
                                           "max_abs_diff_vs_value_path": float(np.max(np.abs(gout["r"] - out["r"]))),
                                           "roofline": {"kernel": "k_spmm_short (width 128)", "bound": "hbm",
                                                        "achieved": round(b / (avg * 1e-3) / 1e9, 1) if nl else None,
                                                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                                        "avg_launch_ms": round(avg, 4), "launches": nl,
                                                        "alg_bytes_per_launch": b,
                                                        "note": "4,096-node graph: L2-resident; 64 wavefronts per "
                                                                "product launch, latency-bound"}},
                     iterations={"power_method_l": l_pm, "lanczos_mean_k": float(lz["iters"].mean()),
                                 "lanczos_max_k": int(lz["iters"].max()),
                                 "ratio_l_over_k": round(l_pm / float(lz["iters"].mean()), 1),
                                 "kappa": round(kappa, 1), "sqrt_kappa": round(float(np.sqrt(kappa)), 1)},
                     lanczos_batched_fp64={"value": round(bq, 2), "unit": "queries/s",
                                           "speedup_over_power_method": round(bq * pdt / len(s), 1)},
                     roofline={"kernel": "k_pm_small (all steps of a pair in one workgroup, vectors in LDS)",
                               "bound": "alu",
                               "achieved": round(len(s) * l_pm * (4.0 * g.m + 3.0 * g.n) / pdt / 1e12, 4),
                               "peak": 78.6, "unit": "TFLOP/s",
                               "frac": round(len(s) * l_pm * (4.0 * g.m + 3.0 * g.n) / pdt / 1e12 / 78.6, 5),
                               "traffic": None, "avg_launch_ms": round(pdt * 1e3, 3), "launches": 1,
                               "note": "FP64 flops per step and pair: 2 per adjacency entry, 3 per node, against "
                                       "the FP64 vector peak; LDS-resident, bound by LDS latency and the "
                                       "per-step barrier, not by arithmetic"},
                     cpu_baseline={"value": round(k / secs, 3), "unit": "queries/s", "cores": 1, "kind": "oracle",
                                   "sample": f"{k} of the 100 pairs, numpy Algorithm 1 with the same l"},
                     parity={"max_rel_err_vs_oracle": float(np.max(np.abs(out["r"][:k] - np.array(vals)) / np.array(vals))),
                             "max_rel_err_vs_lanczos_1e-12": float(np.max(np.abs(out["r"] - ref) / ref))})
    else:
        raise SystemExit(f"unknown workload {name}")
    print(json.dumps(line), flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the source text of k_spmm_short and the helpers it inlines
    (everything from the block-partials helper to the long-row kernel)."""
    p = os.path.join(ROOT, "paper_2601_11159_amd", "csrc", "lanczos_batch.hip")
    src = open(p).read()
    a = src.index("// Fold the per-lane column partials")
    b = src.index("// Rows longer than long_deg")
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def copy_bandwidth_gbs(torch, gib: int = 1, reps: int = 5) -> float:
    """Achievable device bandwidth on this GPU: a torch device-to-device copy
    of `gib` GiB (bytes read + bytes written per second), HIP events on the
    current stream."""
    n = gib * 256 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2.0 * gib * 2**30 / (ms * 1e-3) / 1e9


def load_traffic(workload: str, width: int):
    """Measured HBM bytes per launch of k_spmm_short for this workload and
    width, from the committed counter summary, when the kernel source is
    unchanged since it was taken."""
    p = os.path.join(ROOT, "profiles", "spmm_short_traffic.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    e = d.get(f"{workload}/B{width}")
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_baseline(g, s, t, budget_s: float = 20.0):
    """The CPU FP64 oracle (literal Algorithm 3, numpy/scipy) on a bounded
    sample of the same pairs, single thread."""
    from threadpoolctl import threadpool_limits
    from oracle import lanczos as LZ

    t0 = time.time()
    A, d = LZ.normalized_adjacency(g)
    setup = time.time() - t0
    vals, times = [], []
    with threadpool_limits(limits=1):
        for p in range(len(s)):
            t1 = time.time()
            run = LZ.lanczos_rd(g, int(s[p]), int(t[p]), tol=EPS, A=A, d=d)
            times.append(time.time() - t1)
            vals.append(run.r)
            if sum(times) > budget_s:
                break
    return np.array(vals), float(sum(times)), setup


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chung_lu_n4M_g2.3_d32_4096pairs",
                    choices=sorted(WORKLOADS) + OTHER_WORKLOADS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--plain-pairs", type=int, default=128)
    ap.add_argument("--width", type=int, default=0, help="block width (0: autotuned)")
    ap.add_argument("--reorder", type=int, default=1, choices=[0, 1],
                    help="1 (default): build the graph with RD_REORDER (internal ids by decreasing "
                         "degree); 0: ids as generated")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device three times (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        torch.cuda.set_device(0)
        x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copied 1 GiB three times")
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(pairs would shard across GPUs with no per-step communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.workload in OTHER_WORKLOADS:
        run_other(args.workload, args)
        return
    from paper_2601_11159_amd import inputs as I
    from paper_2601_11159_amd import rd

    wl = WORKLOADS[args.workload]
    t0 = time.time()
    g = I.chung_lu(wl["n"], wl["gamma"], wl["mean_deg"], wl["seed"])
    half = wl["pairs"] // 2
    s1, t1 = I.uniform_pairs(g.n, half, wl["pair_seed"])
    s2, t2 = I.hub_pairs(g, wl["pairs"] - half, wl["hub_seed"])
    s = np.concatenate([s1, s2]).astype(np.int32)
    t = np.concatenate([t1, t2]).astype(np.int32)
    log(f"graph n={g.n} m={g.m} generated in {time.time() - t0:.1f}s")

    t0 = time.time()
    G = rd.RDGraph(g.n, torch.from_numpy(g.u).cuda(), torch.from_numpy(g.v).cuda(),
                   reorder=bool(args.reorder))
    torch.cuda.synchronize()
    log(f"rd_init_graph {time.time() - t0:.2f}s")
    ds = torch.from_numpy(s).cuda()
    dt = torch.from_numpy(t).cuda()
    dout = torch.zeros(len(s) * 24, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream

    # autotune the width once (kept on the handle), then warm up
    t0 = time.time()
    width = args.width or G.tune_width(rd.RD_F32, len(s), stream)
    opts_prof = rd.rd_default_options(precision=rd.RD_F32, stream=stream, flags=rd.RD_PROFILE,
                                      block_width=width)
    for _ in range(args.warmup):
        G.query_batch(ds, dt, EPS, opts_prof, out=dout)
    torch.cuda.synchronize()
    G.kernel_stats(0)  # reset counters
    log(f"autotune (width {width}) + warmup {time.time() - t0:.1f}s")

    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        G.query_batch(ds, dt, EPS, opts_prof, out=dout)
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    k_ms, k_launches, k_bytes = G.kernel_stats(0)
    res = np.frombuffer(dout.cpu().numpy().tobytes(), dtype=rd.RESULT_DTYPE).copy()
    value = len(s) * args.steps / elapsed
    ms_per_step = elapsed / args.steps * 1e3
    iters = res["iters"]
    log(f"batched: {value:.1f} q/s, {ms_per_step:.1f} ms/step, iters mean {iters.mean():.2f} "
        f"max {iters.max()}, statuses {np.unique(res['status'])}")

    # plain single-pair FP64 loop on a sample of the same pairs (half uniform, half hub)
    npl = min(args.plain_pairs, len(s))
    idx = np.concatenate([np.arange(npl // 2), half + np.arange(npl - npl // 2)])
    popts = rd.rd_default_options(precision=rd.RD_F64, flags=rd.RD_PROFILE)
    G.query(int(s[0]), int(t[0]), EPS, popts)
    G.kernel_stats(1)
    torch.cuda.synchronize()
    t0 = time.time()
    plain_r = np.zeros(npl)
    plain_it = np.zeros(npl, dtype=np.int64)
    for j, p in enumerate(idx):
        rr = G.query(int(s[p]), int(t[p]), EPS, popts)
        plain_r[j] = rr.r
        plain_it[j] = rr.iters
    torch.cuda.synchronize()
    plain_elapsed = time.time() - t0
    plain_value = npl / plain_elapsed
    pk_ms, pk_launches, pk_bytes = G.kernel_stats(1)
    log(f"plain fp64: {plain_value:.1f} q/s, iters mean {plain_it.mean():.2f}")

    # roofline of the dominant kernel
    avg_ms = k_ms / max(k_launches, 1)
    achieved = k_bytes / (avg_ms * 1e-3) / 1e9 if k_launches else None
    wave, long_deg = G.batch_schedule()
    traffic = load_traffic(args.workload + ("/reordered" if args.reorder else "") + f"/w{wave}_l{long_deg}",
                           width) if width else None
    copy_gbs = copy_bandwidth_gbs(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s")
    roofline = {
        "kernel": "k_spmm_short (batched FP32 sparse product over the short rows)",
        "bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": traffic, "avg_launch_ms": round(avg_ms, 4), "launches": k_launches,
        "alg_bytes_per_launch": k_bytes,
        # achievable stream rate on this machine (1 GiB torch copy, read + write),
        # and the rate of the measured bytes against the peak
        "copy_gbs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4) if achieved else None,
        "traffic_frac": round(traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
    }
    plain_avg_ms = pk_ms / max(pk_launches, 1)
    plain_roof = {
        "kernel": "k_spmv (single-pair FP64 sparse product)",
        "achieved": round(pk_bytes / (plain_avg_ms * 1e-3) / 1e9, 1) if pk_launches else None,
        "avg_launch_ms": round(plain_avg_ms, 4), "launches": pk_launches,
    }

    cpu = None
    parity = None
    if not args.no_cpu:
        sample = np.array([0, 1, half, half + 1])
        vals, secs, setup = cpu_baseline(g, s[sample], t[sample])
        done = len(vals)
        cpu = {"value": round(done / secs, 4), "unit": "queries/s", "cores": 1, "kind": "oracle",
               "sample": f"{done} of the {len(s)} pairs (2 uniform, 2 hub-source), literal "
                         f"Algorithm 3 in numpy/scipy FP64 at the same 1e-4 tolerance, "
                         f"{secs:.1f}s after a {setup:.1f}s operator build"}
        gpu_b = res["r"][sample[:done]]
        gpu_p = plain_r[[0, 1, npl // 2, npl // 2 + 1][:done]] if npl >= 4 else None
        parity = {"pairs": int(done),
                  "batched_fp32_max_rel_err_vs_oracle": float(np.max(np.abs(gpu_b - vals) / vals)),
                  "plain_fp64_max_rel_err_vs_oracle":
                      float(np.max(np.abs(gpu_p - vals) / vals)) if gpu_p is not None else None}
        log(f"cpu oracle: {cpu['value']} q/s; parity {parity}")

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "pairs": len(s), "eps_rel": EPS,
                   "precision": "FP32 vectors and sparse products, FP64 Lanczos scalars",
                   "block_width": width, "block_width_source": "fixed" if args.width else "autotuned",
                   "row_schedule": dict(zip(("wave_nnz", "long_deg"), G.batch_schedule())),
                   "node_order": "decreasing degree (RD_REORDER)" if args.reorder else "as generated",
                   "first_iterations": "iteration 1 from the rows of s and t; iteration 2 from the "
                                       "support of q_2 where that scatter costs less than a dense column "
                                       "(RD_NO_SPARSE2 off)",
                   "mean_iters": round(float(iters.mean()), 3)},
        "plain_fp64": {"value": round(plain_value, 2), "unit": "queries/s", "pairs_timed": npl,
                       "mean_iters": round(float(plain_it.mean()), 3), "roofline": plain_roof,
                       "first_iterations": "iteration 1 from the rows of s and t; iteration 2 from the "
                                           "support of q_2 where that scatter has at most nnz/64 entries"},
        "speedup_batched_vs_plain_fp64": round(value / plain_value, 2),
        "roofline": roofline, "cpu_baseline": cpu, "parity": parity,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
