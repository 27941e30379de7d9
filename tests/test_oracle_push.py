"""Pins of the Lanczos Push oracle (Algorithm 4): eps = 0 reduces to
Algorithm 3 (whose oracle is pinned separately), a threshold that blocks
every push gives r' = 1/d_s + 1/d_t exactly, the first iteration of the
paper's worked example, and locality (fewer touched nodes for larger eps,
convergence to Algorithm 3 as eps -> 0). The later values of the worked
example (alpha_2 = 0.0281, r = 3.218) are parity unpinned: no reading of the
algorithm reproduces them."""

import os

import numpy as np
import pytest

from oracle import lanczos as LZ
from oracle import push as LP
from paper_2601_11159_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_lanczos_push_example.txt")


def _read_example():
    edges, vals = [], {}
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        key, *rest = line.split()
        if key == "edge":
            edges.append((int(rest[0]) - 1, int(rest[1]) - 1))
        else:
            vals[key] = np.array([float(x) for x in rest])
    return edges, vals


@pytest.mark.parametrize("gi", [0, 1, 2])
def test_eps_zero_is_algorithm_3(gi):
    g = [I.grid(9, 7), I.random_connected(80, 150, seed=61, weighted=True),
         I.chung_lu(3000, 2.3, 8.0, seed=62)][gi]
    A, d = LZ.normalized_adjacency(g)
    s, t = 1, g.n // 2 + 3
    for k in [1, 2, 5, 12]:
        pr = LP.lanczos_push(g, s, t, k, 0.0)
        lr = LZ.lanczos_rd(g, s, t, k=k, A=A, d=d)
        assert len(pr.alpha) == lr.k == k
        np.testing.assert_allclose(pr.alpha, lr.alpha[:k], rtol=0, atol=1e-12)
        np.testing.assert_allclose(pr.beta, lr.beta[1:k], rtol=1e-12, atol=0)
        assert abs(pr.r - lr.rhat[-1]) <= 1e-12 * lr.rhat[-1]


def test_blocked_pushes_give_the_first_order_value():
    g = I.random_connected(60, 100, seed=63, weighted=True)
    s, t = 4, 50
    W, d = LP._adjacency(g)
    pr = LP.lanczos_push(g, s, t, 5, eps=1e6)
    assert pr.pushes == 0 and len(pr.alpha) == 1
    assert pr.r == pytest.approx(1.0 / d[s] + 1.0 / d[t], rel=1e-15)


def test_worked_example_first_iteration():
    edges, vals = _read_example()
    g = I.Graph(4, np.array([e[0] for e in edges], np.int32), np.array([e[1] for e in edges], np.int32))
    pr = LP.lanczos_push(g, 0, 3, 2, eps=0.25, eps_s=0.0, sign=+1.0)
    np.testing.assert_allclose(pr.V[0], vals["v1"], atol=1e-15)
    assert pr.alpha[0] == pytest.approx(vals["alpha1"][0], abs=1e-15)
    assert pr.beta[0] == pytest.approx(vals["beta2"][0], abs=1e-15)
    np.testing.assert_allclose(pr.V[1], vals["v2"], atol=1e-15)


def test_locality_and_convergence_in_eps():
    g = I.grid(30, 30)
    A, d = LZ.normalized_adjacency(g)
    s, t = 40, 500
    k = 20
    lr = LZ.lanczos_rd(g, s, t, k=k, A=A, d=d)
    touched, errs = [], []
    for eps in [1e-1, 1e-2, 1e-3, 1e-5, 1e-9]:
        pr = LP.lanczos_push(g, s, t, k, eps)
        touched.append(pr.touched)
        errs.append(abs(pr.r - lr.rhat[-1]) / lr.rhat[-1])
    assert all(a <= b for a, b in zip(touched, touched[1:]))
    assert touched[0] < touched[-1]
    assert errs[-1] <= 1e-8


def test_worked_example_with_the_definitions_restriction():
    # S_1 = {u : |v_1(u)| > eps d_u} = {4} (node 1: 1/2 > 0.25 * 3 fails), so
    # only node 4 loses alpha_1 v_1: by hand, v_2 before normalisation is
    # [1/2, 0, 0, 1/(2 sqrt 3) - sqrt(3)/4] = [1/2, 0, 0, -sqrt(3)/12] and
    # beta_2 = sqrt(1/4 + 1/48) = sqrt(13/48)
    edges, _ = _read_example()
    g = I.Graph(4, np.array([e[0] for e in edges], np.int32), np.array([e[1] for e in edges], np.int32))
    pr = LP.lanczos_push(g, 0, 3, 2, eps=0.25, sign=+1.0)
    assert pr.alpha[0] == pytest.approx(0.5, abs=1e-15)
    assert pr.beta[0] == pytest.approx(np.sqrt(13.0 / 48.0), abs=1e-15)
    np.testing.assert_allclose(pr.V[1] * pr.beta[0], [0.5, 0.0, 0.0, -np.sqrt(3.0) / 12.0], atol=1e-15)


def test_empty_restriction_is_normalised_power_iteration():
    # eps = 0 pushes everything; eps_s = inf keeps S empty, so nothing is
    # subtracted and v_{i+1} = calA v_i / ||calA v_i||
    g = I.random_connected(40, 70, seed=64, weighted=True)
    A, d = LZ.normalized_adjacency(g)
    pr = LP.lanczos_push(g, 2, 30, 4, eps=0.0, eps_s=np.inf)
    x = pr.V[0]
    for i in range(1, 4):
        x = A @ x
        np.testing.assert_allclose(pr.V[i], x / np.linalg.norm(x), atol=1e-13)


def test_worked_example_output_under_the_definitions():
    # the example's run (eps = 0.25, "+" sign) with the definition's thresholds,
    # worked by hand to four digits: S_2 = {1, 4}; node 1 pushes to 2, 3, 4,
    # node 4 (|v_2| = 0.277 < 0.25 sqrt(3)) does not; alpha_2 = -0.02885;
    # v_1 . v_2 = 0.24019; (I - T)^{-1} e_1 = [4.2237, 2.1365];
    # r' = (4/3)(4.2237 + 0.24019 * 2.1365) = 6.3158. Using e_1 in place of
    # v_1^T V would give 5.6316.
    edges, _ = _read_example()
    g = I.Graph(4, np.array([e[0] for e in edges], np.int32), np.array([e[1] for e in edges], np.int32))
    pr = LP.lanczos_push(g, 0, 3, 2, eps=0.25, sign=+1.0)
    assert pr.alpha[1] == pytest.approx(-0.02885, abs=5e-5)
    assert pr.r == pytest.approx(6.3158, abs=5e-4)
