"""Lanczos Push for resistance distance (paper Algorithm 4), FP64.

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.

The steps follow Section 4.1 in the paper's order and notation; vectors are
held dense here (the oracle need not be local), but every entry outside the
pushed set stays exactly zero, so the sets the algorithm touches are those of
the paper:

* v_0 = 0, v_1 = (e_s / sqrt(d_s) - e_t / sqrt(d_t)) / sqrt(1/d_s + 1/d_t)
  (sign -1, the reading of Algorithms 3 and 4; the worked example of
  Section 4 uses +1), beta_1 = 0;
* per iteration i = 1..k:
  - S_i = {u : |v_i(u)| > eps_s d_u} (Definition of the restricted vector;
    eps_s = eps unless given);
  - AMV: for every u with v_i(u) != 0 and every neighbour v with
    |v_i(u)| > eps sqrt(d_u d_v), add w_uv v_i(u) / sqrt(d_u d_v) to v_{i+1}(v)
    (Definition of AMV; weighted graphs use the edge weight, Section 2.1);
  - v_{i+1} -= beta_i v_{i-1} on S_{i-1};
  - alpha_i = <v_{i+1}, v_i>;
  - v_{i+1} -= alpha_i v_i on S_i;
  - beta_{i+1} = ||v_{i+1}||, v_{i+1} /= beta_{i+1}
  (the subset Lanczos recurrence, Eq. subset_lz_recurrence);
* output r' = (1/d_s + 1/d_t) v_1^T V (I - T)^{-1} e_1 with V = [v_1..v_k] and
  T the tridiagonal matrix of alpha_1..alpha_k and beta_2..beta_k. The vectors
  are not orthogonal, so v_1^T V is not e_1^T in general.

With eps = 0 every nonzero entry pushes along every edge and S_i is the
support of v_i, so the recurrence is Algorithm 3's and r' its r_hat_k.
Exact breakdown (beta_{i+1} = 0) ends the run with the iterations done.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class PushRun:
    alpha: list = field(default_factory=list)
    beta: list = field(default_factory=list)  # beta_2, beta_3, ...
    V: list = field(default_factory=list)     # v_1, v_2, ...
    touched: int = 0                          # nodes ever given a nonzero entry
    pushes: int = 0                           # edge pushes made
    r: float = 0.0


def _adjacency(g):
    w = np.ones(g.m) if g.w is None else np.asarray(g.w, dtype=np.float64)
    u = np.asarray(g.u, dtype=np.int64)
    v = np.asarray(g.v, dtype=np.int64)
    W = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([u, v]), np.concatenate([v, u]))),
                      shape=(g.n, g.n)).tocsr()
    d = np.asarray(W.sum(axis=1)).ravel()
    return W, d


def lanczos_push(g, s: int, t: int, k: int, eps: float, eps_s=None, sign: float = -1.0, W=None, d=None):
    """Algorithm 4 for k iterations with push threshold eps and restriction
    threshold eps_s (default eps); sign is that of the e_t term of v_1."""
    if W is None:
        W, d = _adjacency(g)
    eps_s = eps if eps_s is None else eps_s
    n = g.n
    c = 1.0 / d[s] + 1.0 / d[t]
    v1 = np.zeros(n)
    v1[s] += 1.0 / np.sqrt(d[s])
    v1[t] += sign / np.sqrt(d[t])
    v1 /= np.sqrt(c)
    run = PushRun()
    v_prev = np.zeros(n)
    S_prev = np.zeros(n, dtype=bool)
    v = v1
    beta = 0.0
    ever = v != 0.0
    sq = np.sqrt(d)
    for i in range(k):
        run.V.append(v)
        S = np.abs(v) > eps_s * d
        y = np.zeros(n)
        for u in np.flatnonzero(v):
            lo, hi = W.indptr[u], W.indptr[u + 1]
            nb = W.indices[lo:hi]
            wt = W.data[lo:hi]
            keep = np.abs(v[u]) > eps * sq[u] * sq[nb]
            y[nb[keep]] += wt[keep] * v[u] / (sq[u] * sq[nb[keep]])
            run.pushes += int(keep.sum())
        y[S_prev] -= beta * v_prev[S_prev]
        alpha = float(y @ v)
        y[S] -= alpha * v[S]
        run.alpha.append(alpha)
        beta_next = float(np.linalg.norm(y))
        ever |= y != 0.0
        if i == k - 1 or beta_next == 0.0:
            break
        run.beta.append(beta_next)
        v_prev, S_prev = v, S
        v = y / beta_next
        beta = beta_next
    kk = len(run.alpha)
    T = np.diag(run.alpha[:kk])
    off = np.asarray(run.beta[: kk - 1])
    T += np.diag(off, 1) + np.diag(off, -1)
    e1 = np.zeros(kk)
    e1[0] = 1.0
    y = np.linalg.solve(np.eye(kk) - T, e1)
    Vk = np.stack(run.V[:kk], axis=1)
    run.r = float(c * (v1 @ Vk) @ y)
    run.touched = int(ever.sum())
    return run
