"""Pins of the Power Method oracle (Algorithm 1) against results fixed
independently of the iteration: the eigendecomposition form of the truncated
series, the exact value on a single edge, the guarantee of the Power Method
theorem against the dense pseudo-inverse, and monotonicity."""

import numpy as np
import pytest

from paper_2601_11159_amd import inputs as I
from oracle import dense as D
from oracle import power as PM


def _spectral_partial_sum(g, s, t, l):
    """(1/2) sum_{k<=l} b^T D^{-1} (I/2 + P/2)^k b from the eigenpairs of the
    normalised adjacency: with y = D^{-1/2} b and calA = U diag(lam) U^T the
    sum is (1/2) sum_j (u_j^T y)^2 (1 - nu_j^(l+1)) / (1 - nu_j),
    nu_j = (1 + lam_j) / 2 (the term nu = 1 has u_j^T y = 0 on a connected
    graph)."""
    w = np.ones(g.m) if g.w is None else np.asarray(g.w, dtype=np.float64)
    W = np.zeros((g.n, g.n))
    W[g.u, g.v] = w
    W[g.v, g.u] = w
    d = W.sum(axis=1)
    isd = 1.0 / np.sqrt(d)
    lam, U = np.linalg.eigh(isd[:, None] * W * isd[None, :])
    y = np.zeros(g.n)
    y[s] += isd[s]
    y[t] -= isd[t]
    c2 = (U.T @ y) ** 2
    nu = (1.0 + lam) / 2.0
    keep = nu < 1.0 - 1e-12
    total = np.where(keep, (1.0 - nu ** (l + 1)) / np.where(keep, 1.0 - nu, 1.0), 0.0)
    return 0.5 * float(np.sum(c2 * total)), lam


def _graphs():
    return [I.grid(6, 5), I.random_connected(40, 60, seed=11, weighted=True),
            I.random_tree(25, seed=3, weighted=True), I.path(12)]


@pytest.mark.parametrize("gi", range(4))
@pytest.mark.parametrize("l", [0, 1, 2, 7, 60])
def test_power_method_equals_spectral_partial_sum(gi, l):
    g = _graphs()[gi]
    for s, t in [(0, g.n - 1), (1, g.n // 2)]:
        want, _ = _spectral_partial_sum(g, s, t, l)
        got = PM.power_method(g, s, t, l)
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (gi, l, s, t, got, want)


def test_single_edge_is_exact_after_the_first_term():
    g = I.path(2)
    for l in [0, 1, 5]:
        assert PM.power_method(g, 0, 1, l) == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("gi", range(3))
def test_theorem_iteration_count_meets_eps(gi):
    g = _graphs()[gi]
    eps = 1e-6
    _, lam = _spectral_partial_sum(g, 0, 1, 0)
    mu2 = 1.0 - np.sort(lam)[-2]  # smallest non-zero eigenvalue of the normalised Laplacian
    kappa = 2.0 / mu2
    l = PM.iterations_for(kappa, eps)
    Lp = D.pinv(D.laplacian(g))
    for s, t in [(0, g.n - 1), (2, g.n // 2)]:
        r = float(D.rd_from_pinv(Lp, s, t))
        assert abs(PM.power_method(g, s, t, l) - r) <= eps


def test_terms_are_nonnegative_and_partial_sums_stay_below_r():
    g = I.random_connected(50, 80, seed=5, weighted=True)
    r = float(D.rd_all(g, 3, 41))
    r_bar, terms = PM.power_method(g, 3, 41, 400, terms=True)
    assert min(terms) >= -1e-15
    assert np.all(np.cumsum(terms) <= r + 1e-12)
    assert abs(r_bar - r) < 1e-3 * r


def test_same_node_is_zero():
    g = I.grid(4, 4)
    assert PM.power_method(g, 5, 5, 10) == 0.0
