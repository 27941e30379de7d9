"""Power Method for resistance distance (paper Algorithm 1), FP64.

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.

The steps follow Section 2.2 (existing methods, Algorithm 1) in the paper's
order and notation:

* P = A D^{-1}, the probability transition matrix (Section 2.2; weighted
  graphs use W and weighted degrees, Section 2.1);
* r_bar = 0 and the vector r = e_s - e_t;
* for i = 0, 1, ..., l: r_bar += r(s) / (2 d_s) - r(t) / (2 d_t), then
  r = (I/2 + P/2) r, the lazy random-walk step;
* output r_bar, which equals the truncated Taylor series
  (1/2) b^T sum_{k=0}^{l} D^{-1} (I/2 + P/2)^k b with b = e_s - e_t
  (Eq. er_laylor_expansion cut after l + 1 terms).

The Power Method guarantee (the theorem after Algorithm 1) states that
l = 2 kappa log(kappa / eps) gives |r_bar - r| <= eps, with kappa = 2 / mu_2
the condition number of the normalised Laplacian (Section 2.1).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def transition_matrix(g):
    """P = W D^{-1} as a scipy CSR matrix, and the weighted degrees d."""
    w = np.ones(g.m) if g.w is None else np.asarray(g.w, dtype=np.float64)
    u = np.asarray(g.u, dtype=np.int64)
    v = np.asarray(g.v, dtype=np.int64)
    W = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([u, v]), np.concatenate([v, u]))),
                      shape=(g.n, g.n)).tocsr()
    d = np.asarray(W.sum(axis=1)).ravel()
    return (W @ sp.diags(1.0 / d)).tocsr(), d


def power_method(g, s: int, t: int, l: int, P=None, d=None, terms: bool = False):
    """Algorithm 1: r_bar after the iterations i = 0..l (l + 1 terms).

    terms=True also returns the list of the l + 1 added terms."""
    if P is None:
        P, d = transition_matrix(g)
    r = np.zeros(g.n)
    r[s] += 1.0
    r[t] -= 1.0
    r_bar = 0.0
    added = []
    for _ in range(l + 1):
        term = r[s] / (2.0 * d[s]) - r[t] / (2.0 * d[t])
        r_bar += term
        added.append(term)
        r = 0.5 * r + 0.5 * (P @ r)
    return (r_bar, added) if terms else r_bar


def iterations_for(kappa: float, eps: float) -> int:
    """l = 2 kappa log(kappa / eps), the iteration count of the Power Method
    guarantee (natural logarithm)."""
    return int(np.ceil(2.0 * kappa * np.log(kappa / eps)))
