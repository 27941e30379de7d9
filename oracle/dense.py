"""Dense FP64 truth for resistance distance, potentials and edge gradients.

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product path
never does.

Everything here is the plain definition written out with numpy/scipy dense
linear algebra, for graphs up to a few thousand nodes:

* Laplacian L = D - W with d_u = sum_v w_uv (paper Section 2.1, definition of
  RD; weighted graphs by the direct generalisation the same section states).
* L^+ = sum_{i>=2} u_i u_i^T / lambda_i (Section 2.1), from a symmetric
  eigendecomposition.
* r(s,t) = (e_s - e_t)^T L^+ (e_s - e_t) (Definition of RD, Section 2.1).
* phi = L^+ (e_s - e_t), f(e) = phi(u) - phi(v) (Definition of potential and
  electric flow, Section 6.3).
* dr/dw_uv = -(phi_u - phi_v)^2 (derivative of the quadratic form b^T L^+ b
  along L = sum_e w_e b_e b_e^T; not stated in the paper).

Two more routes to the same numbers serve as cross-checks: the grounded
Laplacian (delete one node, Cholesky) and (L + J/n)^{-1}.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _weights(g) -> np.ndarray:
    return np.ones(g.m) if g.w is None else np.asarray(g.w, dtype=np.float64)


def laplacian(g) -> np.ndarray:
    """Dense L = D - W in FP64."""
    n = g.n
    w = _weights(g)
    L = np.zeros((n, n))
    u = np.asarray(g.u, dtype=np.int64)
    v = np.asarray(g.v, dtype=np.int64)
    np.add.at(L, (u, v), -w)
    np.add.at(L, (v, u), -w)
    np.add.at(L, (u, u), w)
    np.add.at(L, (v, v), w)
    return L


def pinv(L: np.ndarray) -> np.ndarray:
    """L^+ = sum over non-zero eigenpairs of u u^T / lambda (Section 2.1).

    Eigenvalues below n * eps_mach * lambda_max are treated as the null space
    (exactly one for a connected graph)."""
    lam, U = np.linalg.eigh(L)
    tau = L.shape[0] * np.finfo(np.float64).eps * max(lam[-1], 1.0)
    keep = lam > tau
    Uk = U[:, keep]
    return (Uk / lam[keep]) @ Uk.T


def rd_from_pinv(Lp: np.ndarray, s, t) -> np.ndarray:
    """r(s,t) = (e_s - e_t)^T L^+ (e_s - e_t) for arrays of pairs."""
    s = np.asarray(s)
    t = np.asarray(t)
    return Lp[s, s] + Lp[t, t] - 2.0 * Lp[s, t]


def rd_grounded(L: np.ndarray, s: int, t: int, ground: int) -> float:
    """Same quantity through the grounded Laplacian: delete row/column
    `ground`, solve L_g x = b_g by Cholesky, r = b_g^T x."""
    n = L.shape[0]
    keep = np.array([i for i in range(n) if i != ground])
    b = np.zeros(n)
    b[s] += 1.0
    b[t] -= 1.0
    Lg = L[np.ix_(keep, keep)]
    x = sla.cho_solve(sla.cho_factor(Lg), b[keep])
    return float(b[keep] @ x)


def rd_shifted(L: np.ndarray, s: int, t: int) -> float:
    """Same quantity through (L + J/n)^{-1} (J the all-ones matrix)."""
    n = L.shape[0]
    M = L + np.ones((n, n)) / n
    b = np.zeros(n)
    b[s] += 1.0
    b[t] -= 1.0
    return float(b @ np.linalg.solve(M, b))


def potentials(Lp: np.ndarray, s: int, t: int) -> np.ndarray:
    """phi = L^+ (e_s - e_t) (Definition of electric flow, Section 6.3)."""
    return Lp[:, s] - Lp[:, t]


def flows(g, phi: np.ndarray) -> np.ndarray:
    """f(e) = phi(u) - phi(v) for every edge e = (u, v) (Section 6.3)."""
    return phi[g.u] - phi[g.v]


def grad_edges(g, Lp: np.ndarray, s, t, gbar=None) -> np.ndarray:
    """d(sum_p gbar_p r(s_p, t_p)) / d w_e = -sum_p gbar_p f_p(e)^2, edge order."""
    s = np.atleast_1d(s)
    t = np.atleast_1d(t)
    gbar = np.ones(len(s)) if gbar is None else np.asarray(gbar, dtype=np.float64)
    out = np.zeros(g.m)
    for p in range(len(s)):
        f = flows(g, potentials(Lp, int(s[p]), int(t[p])))
        out -= gbar[p] * f * f
    return out


def rd_all(g, s, t) -> np.ndarray:
    """Convenience: dense truth for arrays of pairs on graph g."""
    return rd_from_pinv(pinv(laplacian(g)), s, t)
