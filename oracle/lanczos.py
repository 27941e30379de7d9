"""Literal Lanczos iteration for resistance distance (paper Algorithm 3), FP64.

Test infrastructure: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.

The steps follow Section 3 in the paper's order and notation:

* normalised adjacency calA = D^{-1/2} A D^{-1/2} (Section 2.2; weighted
  graphs use W and weighted degrees, Section 2.1);
* v_0 = 0, v_1 = (e_s/sqrt(d_s) - e_t/sqrt(d_t)) / sqrt(1/d_s + 1/d_t),
  beta_1 = 0;
* per iteration i: w = calA v_i - beta_i v_{i-1}; alpha_i = <w, v_i>;
  w = w - alpha_i v_i; beta_{i+1} = ||w||; v_{i+1} = w / beta_{i+1}
  (the three-term recurrence, Eq. lz_recurrence);
* output r_hat = (1/d_s + 1/d_t) e_1^T (I - T)^{-1} e_1 with T the k x k
  tridiagonal matrix of alpha_1..alpha_k and beta_2..beta_k (Eq.
  approx_formula). Here the k x k tridiagonal system is solved directly
  (LAPACK banded solver) after every iteration.

The paper runs a fixed number k of iterations. For a tolerance-driven run the
oracle applies the stopping rule `stop_rule` below, which the paper does not
state (it is this implementation's reading, documented with it), evaluated
after each iteration on the sequence r_hat_1, r_hat_2, ...

Exact breakdown (beta_{i+1} = 0, the Krylov space is invariant) ends the run
with r_hat exact; the test is beta_{i+1} <= 1e-13 (|alpha_i| + beta_i).

Optional re-orthogonalisation (`reorth`, not part of Algorithm 3; the paper
relies on v_1 being exactly orthogonal to u_1 = D^{1/2} 1 / sqrt(vol), the
eigenvector of calA for eigenvalue 1, Section 3): after w = w - alpha_i v_i,
with coefficients all taken from that w (one classical Gram-Schmidt step),
  reorth = 1: w -= (u_1^T w) u_1;
  reorth = 2: w -= (u_1^T w) u_1 + (v_i^T w) v_i + (v_{i-1}^T w) v_{i-1}.
In exact arithmetic every coefficient is zero and the run is unchanged.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

BREAKDOWN_REL = 1e-13


def normalized_adjacency(g):
    """calA = D^{-1/2} W D^{-1/2} as a scipy CSR matrix, and the degrees d."""
    w = np.ones(g.m) if g.w is None else np.asarray(g.w, dtype=np.float64)
    u = np.asarray(g.u, dtype=np.int64)
    v = np.asarray(g.v, dtype=np.int64)
    W = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([u, v]), np.concatenate([v, u]))),
                      shape=(g.n, g.n)).tocsr()
    d = np.asarray(W.sum(axis=1)).ravel()
    isd = 1.0 / np.sqrt(d)
    A = sp.diags(isd) @ W @ sp.diags(isd)
    return A.tocsr(), d


def tridiag_solve_e1(alpha, beta) -> float:
    """e_1^T (I - T)^{-1} e_1 with T = tridiag(beta[1:], alpha, beta[1:]).

    `alpha` holds alpha_1..alpha_k, `beta` holds beta_1..beta_k (beta[0] = beta_1
    = 0 is unused). The k x k system (I - T) y = e_1 is solved directly by
    LAPACK's banded solver (the matrix is tridiagonal), so long runs stay
    O(k) per step."""
    k = len(alpha)
    ab = np.zeros((3, k))
    ab[1] = 1.0 - np.asarray(alpha, dtype=np.float64)
    if k > 1:
        off = -np.asarray(beta[1:k], dtype=np.float64)
        ab[0, 1:] = off
        ab[2, :-1] = off
    e1 = np.zeros(k)
    e1[0] = 1.0
    return float(sla.solve_banded((1, 1), ab, e1)[0])


def stop_rule(rhat, tol: float, delay: int) -> tuple:
    """Relative stopping test on the sequence r_hat_1..r_hat_k.

    The paper runs a fixed k; this rule is this implementation's reading of
    a tolerance-driven run. The Lanczos value for a quadratic form of
    (I - calA)^+ is a Gauss quadrature value, so r_hat_k increases towards r.
    With window d = min(delay, k - 2) (k >= 3 is required):

        inc_now  = r_hat_k - r_hat_{k-1}
        inc_prev = r_hat_{k-1} - r_hat_{k-2}
        inc_then = r_hat_{k-d} - r_hat_{k-d-1}
        q        = (inc_now / inc_then)^(1/d)     (mean per-step contraction)

    If both inc_now and inc_then are positive: q >= 1 gives no estimate
    (infinite); otherwise q is capped at 0.9999 and the remaining error is
    estimated by eight times the geometric tail of the latest increment,
    est = max(8 inc_now q / (1 - q), inc_now). If either increment is not
    positive the sequence has reached its rounding floor and
    est = |inc_now| + |inc_prev|. The run stops once est <= tol * r_hat_k.
    Returns (stop, est)."""
    k = len(rhat)
    if k < 3:
        return False, np.inf
    d = min(delay, k - 2)
    inc_now = rhat[-1] - rhat[-2]
    inc_prev = rhat[-2] - rhat[-3]
    inc_then = rhat[-1 - d] - rhat[-2 - d]
    if inc_now <= 0.0 or inc_then <= 0.0:
        est = abs(inc_now) + abs(inc_prev)
    else:
        q = (inc_now / inc_then) ** (1.0 / d)
        if q >= 1.0:
            return False, np.inf
        q = min(q, 0.9999)
        est = max(8.0 * inc_now * q / (1.0 - q), inc_now)
    return est <= tol * rhat[-1], est


@dataclass
class LanczosRun:
    r: float
    k: int
    alpha: list = field(default_factory=list)
    beta: list = field(default_factory=list)  # beta_1..beta_{k+1}
    rhat: list = field(default_factory=list)  # r_hat_1..r_hat_k
    err_est: float = np.inf
    breakdown: bool = False
    converged: bool = False
    V: list = field(default_factory=list)  # v_1..v_k when keep_vectors


def lanczos_rd(g, s: int, t: int, k: int | None = None, tol: float | None = None, delay: int = 8,
               max_iters: int | None = None, keep_vectors: bool = False, A=None, d=None,
               reorth: int = 0) -> LanczosRun:
    """Algorithm 3 for the pair (s, t): fixed k iterations when `k` is given,
    otherwise iterate until `stop_rule(tol, delay)` holds or `max_iters`.
    `reorth` in {0, 1, 2} as in the module docstring."""
    if A is None:
        A, d = normalized_adjacency(g)
    if s == t:
        return LanczosRun(r=0.0, k=0, converged=True)
    n = g.n
    c = 1.0 / d[s] + 1.0 / d[t]
    v_prev = np.zeros(n)
    v = np.zeros(n)
    v[s] = 1.0 / np.sqrt(d[s])
    v[t] = -1.0 / np.sqrt(d[t])
    v /= np.sqrt(c)
    beta_i = 0.0
    u1 = np.sqrt(d) / np.sqrt(d.sum())
    run = LanczosRun(r=0.0, k=0, beta=[0.0])
    limit = k if k is not None else (max_iters if max_iters is not None else n)
    for i in range(1, limit + 1):
        if keep_vectors:
            run.V.append(v.copy())
        w = A @ v - beta_i * v_prev
        alpha_i = float(w @ v)
        w = w - alpha_i * v
        if reorth >= 1:
            corr = (u1 @ w) * u1
            if reorth == 2:
                corr = corr + (v @ w) * v + (v_prev @ w) * v_prev
            w = w - corr
        beta_next = float(np.linalg.norm(w))
        run.alpha.append(alpha_i)
        run.beta.append(beta_next)
        run.rhat.append(c * tridiag_solve_e1(run.alpha, run.beta))
        run.k = i
        if beta_next <= BREAKDOWN_REL * (abs(alpha_i) + beta_i):
            run.breakdown = True
            run.converged = True
            run.err_est = 0.0
            break
        if k is None and tol is not None:
            stop, est = stop_rule(run.rhat, tol, delay)
            run.err_est = est
            if stop:
                run.converged = True
                break
        v_prev, v = v, w / beta_next
        beta_i = beta_next
    run.r = run.rhat[-1]
    return run


def tridiag_matrix(alpha, beta) -> np.ndarray:
    k = len(alpha)
    T = np.diag(np.asarray(alpha, dtype=np.float64))
    if k > 1:
        off = np.asarray(beta[1:k], dtype=np.float64)
        T += np.diag(off, 1) + np.diag(off, -1)
    return T


def ritz_values(run: LanczosRun) -> np.ndarray:
    """Eigenvalues of T_k (diagonal alpha_1..alpha_k, off-diagonal
    beta_2..beta_k), the Ritz values of the run (Section 3), ascending."""
    k = run.k
    return sla.eigvalsh_tridiagonal(np.asarray(run.alpha[:k], dtype=np.float64),
                                    np.asarray(run.beta[1:k], dtype=np.float64))


def potentials_lanczos(g, s: int, t: int, run: LanczosRun, d) -> np.ndarray:
    """phi_hat = sqrt(1/d_s + 1/d_t) D^{-1/2} V (I - T)^{-1} e_1, the potential
    estimate of Algorithm 5, from a run made with keep_vectors=True."""
    k = run.k
    c = 1.0 / d[s] + 1.0 / d[t]
    T = tridiag_matrix(run.alpha[:k], run.beta[:k])
    e1 = np.zeros(k)
    e1[0] = 1.0
    y = np.linalg.solve(np.eye(k) - T, e1)
    V = np.stack(run.V[:k], axis=1)
    return np.sqrt(c) * (V @ y) / np.sqrt(d)
