"""GPU parity of the sparse second iteration of the batched path: pairs whose
second product touches few adjacency entries compute it from the support of
q_2 (a fixed-point scatter over N(S)) instead of a dense product over the
block. The results must agree with the dense FP64 oracle, with the same run
under RD_NO_SPARSE2 (dense second products) to rounding, and with themselves
bit for bit from run to run."""

import numpy as np
import pytest

from oracle import dense as D
from paper_2601_11159_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2601_11159_amd import rd  # noqa: E402


def _graphs():
    return {
        "grid": I.grid(30, 30),
        "power_law": I.chung_lu(3000, 2.3, 8.0, seed=41),
        "weighted": I.random_connected(800, extra=4000, seed=42, weighted=True),
        "tree": I.random_tree(600, seed=43, weighted=True),
        "star": I.star(300),
    }


GRAPHS = _graphs()


def _pairs(g, count, seed):
    s, t = I.uniform_pairs(g.n, count, seed)
    s, t = s.copy(), t.copy()
    # adjacent pairs, a pair at a degree-1 node and a repeated node
    u, v = int(g.u[0]), int(g.v[0])
    s[0], t[0] = u, v
    s[1], t[1] = v, u
    deg = np.bincount(np.concatenate([g.u, g.v]), minlength=g.n)
    leaf = int(np.argmin(deg))
    s[2] = leaf
    if t[2] == leaf:
        t[2] = (leaf + 1) % g.n
    t[3] = s[3]
    return s.astype(np.int32), t.astype(np.int32)


def _run(G, s, t, tol, flags=0, **kw):
    o = rd.rd_default_options(flags=rd.RD_GENERAL_PATH | flags, **kw)
    return G.query_batch(s, t, tol, o)


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("prec,tol,bar", [(rd.RD_F64, 1e-10, 1e-8), (rd.RD_F32, 1e-5, 2e-3)])
def test_sparse2_against_oracle(name, prec, tol, bar):
    g = GRAPHS[name]
    s, t = _pairs(g, 150, seed=44)
    mask = s != t
    truth = np.zeros(len(s))
    truth[mask] = D.rd_all(g, s[mask], t[mask])
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    out = _run(G, s, t, tol, precision=prec, block_width=32)
    assert np.all(out["status"] == rd.RD_OK)
    assert out["r"][3] == 0.0 and out["iters"][3] == 0
    err = np.abs(out["r"][mask] - truth[mask]) / truth[mask]
    assert err.max() <= bar, (name, err.max())


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("k", [1, 2, 3, 4, 9])
def test_sparse2_matches_dense_second_product(name, k):
    # the same number of iterations on both paths: r_hat_k agrees to rounding
    g = GRAPHS[name]
    s, t = _pairs(g, 100, seed=45)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    a = _run(G, s, t, 1e-6, fixed_k=k, block_width=32)
    b = _run(G, s, t, 1e-6, rd.RD_NO_SPARSE2, fixed_k=k, block_width=32)
    mask = s != t
    # a Krylov space exhausted before k stops both runs early, at the same step
    np.testing.assert_array_equal(a["iters"], b["iters"])
    assert np.all(a["iters"][mask] <= k)
    np.testing.assert_allclose(a["r"][mask], b["r"][mask], rtol=1e-11)


def test_sparse2_is_taken_and_repeatable():
    # on a 60x60 grid every pair's scatter (about 40 entries) is far below the
    # cost cap (nnz * 4 / 256 = 221 entries in FP32 at an explicit width)
    g = I.grid(60, 60)
    s, t = I.uniform_pairs(g.n, 300, seed=46)
    G = rd.RDGraph(g.n, g.u, g.v, reorder=True)
    o = dict(precision=rd.RD_F32, fixed_k=3, block_width=64)
    runs = [_run(G, s, t, 1e-6, **o) for _ in range(2)]
    dense = _run(G, s, t, 1e-6, rd.RD_NO_SPARSE2, **o)
    assert runs[0].tobytes() == runs[1].tobytes()
    # in FP32 the dense second product rounds y_2 to FP32 and the sparse step
    # does not, so the bits differ wherever the sparse step was taken
    assert np.count_nonzero(runs[0]["r"] != dense["r"]) > len(s) // 2
    np.testing.assert_allclose(runs[0]["r"], dense["r"], rtol=1e-6)


@pytest.mark.parametrize("prec", [rd.RD_F64, rd.RD_F32])
@pytest.mark.parametrize("width", [16, 64, 256])
def test_sparse2_refill_and_compaction(prec, width):
    # many more pairs than columns: refills at every iteration, then the tail
    # narrows the block; hub pairs mix dense and sparse second iterations
    g = GRAPHS["power_law"]
    s1, t1 = I.uniform_pairs(g.n, 400, seed=47)
    s2, t2 = I.hub_pairs(g, 200, seed=48)
    s = np.concatenate([s1, s2]).astype(np.int32)
    t = np.concatenate([t1, t2]).astype(np.int32)
    mask = s != t
    Lp = D.pinv(D.laplacian(g))
    truth = np.zeros(len(s))
    truth[mask] = D.rd_from_pinv(Lp, s[mask], t[mask])
    G = rd.RDGraph(g.n, g.u, g.v, reorder=True)
    tol, bar = (1e-10, 1e-8) if prec == rd.RD_F64 else (1e-5, 2e-3)
    out = _run(G, s, t, tol, precision=prec, block_width=width)
    assert np.all(out["status"] == rd.RD_OK)
    err = np.abs(out["r"][mask] - truth[mask]) / truth[mask]
    assert err.max() <= bar


def test_sparse2_weighted_after_set_weights():
    g = GRAPHS["weighted"]
    s, t = _pairs(g, 80, seed=49)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    _run(G, s, t, 1e-10, block_width=16)
    w2 = np.asarray(g.w, dtype=np.float64) * np.linspace(0.5, 2.0, g.m)
    G.set_weights(w2)
    g2 = I.Graph(g.n, g.u, g.v, w2, "reweighted")
    mask = s != t
    truth = D.rd_all(g2, s[mask], t[mask])
    out = _run(G, s, t, 1e-10, block_width=16)
    np.testing.assert_allclose(out["r"][mask], truth, rtol=1e-8)


@pytest.mark.parametrize("prec,tol,rtol", [(rd.RD_F64, 1e-10, 1e-9), (rd.RD_F32, 1e-5, 2e-4)])
def test_sparse2_gradient_and_refine(prec, tol, rtol):
    # potentials take their second term from the sparse step: the edge
    # gradient and the refined energy match the dense-second-product runs and
    # the dense oracle
    g = GRAPHS["weighted"]
    s, t = _pairs(g, 120, seed=50)
    s, t = s[s != t], t[s != t]
    gbar = np.linspace(0.5, 1.5, len(s))
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    o = dict(precision=prec, block_width=32, flags=rd.RD_GENERAL_PATH)
    fa, ga = G.grad_edges(s, t, gbar, tol, rd.rd_default_options(**o))
    o2 = dict(o, flags=rd.RD_GENERAL_PATH | rd.RD_NO_SPARSE2)
    fb, gb = G.grad_edges(s, t, gbar, tol, rd.rd_default_options(**o2))
    if prec == rd.RD_F64:
        np.testing.assert_array_equal(fa["iters"], fb["iters"])
    assert np.linalg.norm(ga - gb) / np.linalg.norm(gb) <= rtol
    Lp = D.pinv(D.laplacian(g))
    ref = D.grad_edges(g, Lp, s, t, gbar)
    assert np.linalg.norm(ga - ref) / np.linalg.norm(ref) <= (1e-6 if prec == rd.RD_F64 else 2e-3)
    ra = G.query_batch(s, t, tol, rd.rd_default_options(refine=1, **o))
    rb = G.query_batch(s, t, tol, rd.rd_default_options(refine=1, **o2))
    np.testing.assert_allclose(ra["r"], rb["r"], rtol=rtol)
    np.testing.assert_allclose(ra["r"], D.rd_from_pinv(Lp, s, t), rtol=1e-8 if prec == rd.RD_F64 else 2e-4)


def test_sparse2_gradient_stops_at_second_iteration():
    # fixed_k = 2: the run stops at the sparse step; the potential keeps its
    # second term, as on the dense path
    g = GRAPHS["power_law"]
    s, t = I.uniform_pairs(g.n, 70, seed=51)
    s, t = s[s != t], t[s != t]
    G = rd.RDGraph(g.n, g.u, g.v)
    o = dict(block_width=16, fixed_k=2)
    fa, ga = G.grad_edges(s, t, None, 1e-6, rd.rd_default_options(**o))
    fb, gb = G.grad_edges(s, t, None, 1e-6, rd.rd_default_options(flags=rd.RD_NO_SPARSE2, **o))
    assert np.all(fa["iters"] <= 2)
    np.testing.assert_array_equal(fa["iters"], fb["iters"])
    np.testing.assert_allclose(fa["r"], fb["r"], rtol=1e-11)
    assert np.linalg.norm(ga - gb) / np.linalg.norm(gb) <= 1e-9


def _double_star(leaves):
    # centres 0 and 1 joined by an edge, each with `leaves` leaves: every edge
    # is a bridge, so r adds up along the path (1 per edge)
    n = 2 + 2 * leaves
    u = np.concatenate([[0], np.zeros(leaves, np.int64), np.ones(leaves, np.int64)])
    v = np.concatenate([[1], 2 + np.arange(leaves), 2 + leaves + np.arange(leaves)])
    return I.Graph(n, u.astype(np.int32), v.astype(np.int32), None, f"double_star_{leaves}")


@pytest.mark.parametrize("flags", [0, rd.RD_NO_SPARSE2])
def test_sparse2_list_capacity_fallback(flags):
    # deg(0) + deg(1) + 2 = 66,004 list slots exceed the 65,535 a column's list
    # holds: the pair (0, 1) takes the dense second product, the others the
    # sparse one or the dense one by cost; closed-form resistances
    leaves = 33000
    g = _double_star(leaves)
    a, b = 2, 2 + leaves  # a leaf of each centre
    s = np.array([0, a, a, 0, a, a + 1], np.int32)
    t = np.array([1, b, 1, b, a + 1, 0], np.int32)
    truth = np.array([1.0, 3.0, 2.0, 2.0, 2.0, 1.0])
    G = rd.RDGraph(g.n, g.u, g.v)
    out = _run(G, s, t, 1e-10, flags, block_width=16)
    assert np.all(out["status"] == rd.RD_OK)
    np.testing.assert_allclose(out["r"], truth, rtol=1e-9)


def test_sparse2_handle_reused_across_widths():
    # the sparse-step buffers grow with the width (16 -> 256) and are reused
    # (-> 64); every run agrees with the dense oracle
    g = GRAPHS["power_law"]
    s, t = I.uniform_pairs(g.n, 200, seed=52)
    mask = s != t
    truth = np.zeros(len(s))
    truth[mask] = D.rd_all(g, s[mask], t[mask])
    G = rd.RDGraph(g.n, g.u, g.v, reorder=True)
    for width in (16, 256, 64, 16):
        out = _run(G, s, t, 1e-10, block_width=width)
        assert np.all(out["status"] == rd.RD_OK)
        err = np.abs(out["r"][mask] - truth[mask]) / truth[mask]
        assert err.max() <= 1e-8, (width, err.max())


def test_sparse2_iteration_cap_at_the_sparse_step():
    # max_iters = 2: runs that need more stop as not converged right after the
    # sparse step, with the same r_hat_2 and status as the dense path
    g = GRAPHS["grid"]
    s, t = _pairs(g, 60, seed=53)
    G = rd.RDGraph(g.n, g.u, g.v)
    a = _run(G, s, t, 1e-12, block_width=16, max_iters=2)
    b = _run(G, s, t, 1e-12, rd.RD_NO_SPARSE2, block_width=16, max_iters=2)
    np.testing.assert_array_equal(a["status"], b["status"])
    np.testing.assert_array_equal(a["iters"], b["iters"])
    assert np.any(a["status"] == rd.RD_E_NOT_CONVERGED)
    mask = s != t
    np.testing.assert_allclose(a["r"][mask], b["r"][mask], rtol=1e-11)


@pytest.mark.parametrize("name", ["grid", "power_law", "weighted", "tree"])
@pytest.mark.parametrize("prec,tol,bar", [(rd.RD_F64, 1e-10, 1e-8), (rd.RD_F32, 1e-5, 2e-3)])
def test_sparse2_single_pair_path(name, prec, tol, bar):
    # rd_query takes the sparse second iteration too: against the dense truth,
    # and against the same query with a dense second product (fixed k)
    g = GRAPHS[name]
    s, t = _pairs(g, 12, seed=54)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    o = dict(precision=prec, flags=rd.RD_GENERAL_PATH)
    od = dict(precision=prec, flags=rd.RD_GENERAL_PATH | rd.RD_NO_SPARSE2)
    for p in range(len(s)):
        a = G.query(int(s[p]), int(t[p]), tol, rd.rd_default_options(**o))
        if s[p] == t[p]:
            assert a.r == 0.0
            continue
        truth = D.rd_all(g, s[p:p + 1], t[p:p + 1])[0]
        assert a.status == rd.RD_OK
        assert abs(a.r - truth) / truth <= bar
        for k in (2, 3, 6):
            x = G.query(int(s[p]), int(t[p]), tol, rd.rd_default_options(fixed_k=k, **o))
            y = G.query(int(s[p]), int(t[p]), tol, rd.rd_default_options(fixed_k=k, **od))
            assert x.iters == y.iters
            assert x.r == pytest.approx(y.r, rel=1e-11 if prec == rd.RD_F64 else 1e-5)
