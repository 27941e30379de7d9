"""GPU parity of the single-pair Lanczos path (rd_query / rd_query_trace)
against the CPU FP64 oracle, through the C ABI."""

import numpy as np
import pytest

from oracle import dense as D
from oracle import lanczos as LZ
from paper_2601_11159_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2601_11159_amd import rd  # noqa: E402

F64 = rd.rd_default_options()
F32 = rd.rd_default_options(precision=rd.RD_F32)
# small graphs take the single-workgroup path by default; RD_GENERAL_PATH
# forces the multi-workgroup kernels on the same inputs
PATHS = {"small": 0, "general": rd.RD_GENERAL_PATH}


def _graph(g):
    return rd.RDGraph(g.n, g.u, g.v, g.w)


@pytest.mark.parametrize("path", sorted(PATHS))
def test_grid64_all_pairs_fp64(path):
    # 64x64 grid, 100 seeded pairs, tolerance 1e-8; parity 1e-6 against the
    # dense pseudoinverse, and the tolerance itself is met.
    g = I.grid(64, 64)
    s, t = I.uniform_pairs(g.n, 100, seed=1)
    truth = D.rd_all(g, s, t)
    G = _graph(g)
    opts = rd.rd_default_options(flags=PATHS[path])
    errs = []
    for p in range(len(s)):
        res = G.query(int(s[p]), int(t[p]), 1e-8, opts)
        assert res.status == rd.RD_OK
        errs.append(abs(res.r - truth[p]) / truth[p])
    errs = np.array(errs)
    print(f"grid64 fp64: max rel err {errs.max():.3e}", flush=True)
    assert errs.max() <= 1e-6
    assert np.mean(errs <= 1e-8) >= 0.95


@pytest.mark.parametrize("path", sorted(PATHS))
def test_grid64_step_parity_with_literal_algorithm(path):
    # alpha_i, beta_{i+1}, r_hat_i of the first 50 iterations against the
    # numpy transcription of Algorithm 3.
    g = I.grid(64, 64)
    G = _graph(g)
    for s, t in [(0, 4095), (1000, 1234), (77, 3000)]:
        a, b, r = G.query_trace(s, t, 50, rd.rd_default_options(flags=PATHS[path]))
        run = LZ.lanczos_rd(g, s, t, k=50)
        np.testing.assert_allclose(a, run.alpha, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(b, run.beta[1:51], rtol=1e-9)
        np.testing.assert_allclose(r, run.rhat, rtol=1e-10)


def test_closed_forms():
    cases = [
        (I.path(40), 3, 31, 28.0),
        (I.cycle(30), 0, 11, 11 * 19 / 30),
        (I.complete(12), 2, 9, 2.0 / 12),
        (I.complete_bipartite(5, 9), 0, 5, (5 + 9 - 1) / (5 * 9)),
    ]
    for g, s, t, r in cases:
        G = _graph(g)
        res = G.query(s, t, 1e-12, F64)
        assert res.r == pytest.approx(r, rel=1e-9), g.name
    g, s, t = I.bridged_expanders(200, seed=4)
    assert _graph(g).query(s, t, 1e-12, F64).r == pytest.approx(1.0, rel=1e-8)


def test_weighted_tree_and_random_weighted_graph():
    g = I.random_tree(300, seed=7, weighted=True)
    Lp = D.pinv(D.laplacian(g))
    G = _graph(g)
    for s, t in [(0, 299), (17, 150)]:
        assert G.query(s, t, 1e-12, F64).r == pytest.approx(D.rd_from_pinv(Lp, s, t), rel=1e-8)
    g = I.random_connected(500, extra=3000, seed=8, weighted=True)
    Lp = D.pinv(D.laplacian(g))
    G = _graph(g)
    for s, t in [(0, 499), (123, 321), (5, 6)]:
        assert G.query(s, t, 1e-10, F64).r == pytest.approx(D.rd_from_pinv(Lp, s, t), rel=1e-8)
    # float32 weights: the graph is the float32 values
    g32 = I.Graph(g.n, g.u, g.v, g.w.astype(np.float32))
    Lp32 = D.pinv(D.laplacian(g32))
    G32 = _graph(g32)
    assert G32.query(0, 499, 1e-10, F64).r == pytest.approx(D.rd_from_pinv(Lp32, 0, 499), rel=1e-8)


def test_complete_graph_breaks_down_after_one_step():
    g = I.complete(16)
    res = _graph(g).query(1, 7, 1e-10, F64)
    assert res.iters == 1 and res.status == rd.RD_OK
    assert res.r == pytest.approx(2.0 / 16, rel=1e-13)


def test_paper_toy_graph():
    g = I.paper_toy_graph()
    res = _graph(g).query(0, 3, 1e-12, F64)
    assert res.iters == 2
    assert res.r == pytest.approx(1.0, rel=1e-13)
    a, b, r = _graph(g).query_trace(0, 3, 5, F64)
    assert len(r) == 2 and r[-1] == pytest.approx(1.0, rel=1e-13)


@pytest.mark.parametrize("path", sorted(PATHS))
def test_fixed_k_matches_oracle_fixed_k(path):
    g = I.road_like(40, seed=9)
    s, t = I.uniform_pairs(g.n, 3, seed=2)
    G = _graph(g)
    for p in range(3):
        res = G.query(int(s[p]), int(t[p]), 0.0, rd.rd_default_options(fixed_k=30, flags=PATHS[path]))
        run = LZ.lanczos_rd(g, int(s[p]), int(t[p]), k=30)
        assert res.iters == 30
        assert res.r == pytest.approx(run.r, rel=1e-10)


@pytest.mark.parametrize("path", sorted(PATHS))
def test_iteration_cap_reports_not_converged(path):
    g = I.grid(20, 20)
    res = _graph(g).query(0, 399, 1e-12, rd.rd_default_options(max_iters=3, flags=PATHS[path]))
    assert res.status == rd.RD_E_NOT_CONVERGED and res.iters == 3
    run = LZ.lanczos_rd(g, 0, 399, k=3)
    assert res.r == pytest.approx(run.r, rel=1e-12)


def test_same_node_and_argument_errors():
    g = I.grid(8, 8)
    G = _graph(g)
    res = G.query(5, 5, 1e-6, F64)
    assert res.r == 0.0 and res.iters == 0
    with pytest.raises(rd.RdError) as e:
        G.query(-1, 3, 1e-6, F64)
    assert e.value.code == rd.RD_E_ARG
    with pytest.raises(rd.RdError):
        G.query(0, 64, 1e-6, F64)
    with pytest.raises(rd.RdError):
        G.query(0, 5, 0.0, F64)  # no tolerance and no fixed k


def test_invalid_graphs_rejected():
    with pytest.raises(rd.RdError) as e:
        rd.RDGraph(4, np.array([0, 1], np.int32), np.array([1, 1], np.int32))
    assert e.value.code == rd.RD_E_ARG  # self-loop
    with pytest.raises(rd.RdError) as e:
        rd.RDGraph(4, np.array([0, 1, 0], np.int32), np.array([1, 2, 1], np.int32))
    assert e.value.code == rd.RD_E_ARG  # duplicate
    with pytest.raises(rd.RdError) as e:
        rd.RDGraph(4, np.array([0, 1], np.int32), np.array([1, 7], np.int32))
    assert e.value.code == rd.RD_E_ARG  # out of range
    with pytest.raises(rd.RdError) as e:
        rd.RDGraph(4, np.array([0, 2], np.int32), np.array([1, 3], np.int32))
    assert e.value.code == rd.RD_E_NOT_CONNECTED
    with pytest.raises(rd.RdError) as e:
        rd.RDGraph(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1.0, -2.0]))
    assert e.value.code == rd.RD_E_ARG  # bad weight
    with pytest.raises(rd.RdError) as e:
        rd.RDGraph(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1.0, np.nan]))
    assert e.value.code == rd.RD_E_ARG


def test_fp32_grid_within_1e4():
    g = I.grid(64, 64)
    s, t = I.uniform_pairs(g.n, 20, seed=1)
    truth = D.rd_all(g, s, t)
    G = _graph(g)
    for p in range(len(s)):
        res = G.query(int(s[p]), int(t[p]), 1e-5, F32)
        assert abs(res.r - truth[p]) / truth[p] <= 1e-4


def test_repeatable_bitwise():
    g = I.chung_lu(50000, 2.1, 20, seed=2)
    G = _graph(g)
    a1, b1, r1 = G.query_trace(3, 40000, 12, F64)
    a2, b2, r2 = G.query_trace(3, 40000, 12, F64)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2) and np.array_equal(r1, r2)


def test_chung_lu_200k_against_oracle():
    g = I.chung_lu(200000, 2.1, 20, seed=2)
    A, d = LZ.normalized_adjacency(g)
    s, t = I.uniform_pairs(g.n, 6, seed=5)
    G = _graph(g)
    for p in range(len(s)):
        run = LZ.lanczos_rd(g, int(s[p]), int(t[p]), tol=1e-6, A=A, d=d)
        res = G.query(int(s[p]), int(t[p]), 1e-6, F64)
        assert res.iters == run.k
        assert res.r == pytest.approx(run.r, rel=1e-10)
        resf = G.query(int(s[p]), int(t[p]), 1e-6, F32)
        assert resf.r == pytest.approx(run.r, rel=1e-5)


@pytest.mark.parametrize("ro", [1, 2])
@pytest.mark.parametrize("prec", [rd.RD_F64, rd.RD_F32])
def test_reorth_plain_matches_oracle_steps_and_truth(ro, prec):
    g = I.grid(40, 40)
    G = _graph(g)
    A, d = LZ.normalized_adjacency(g)
    # step parity with the oracle's re-orthogonalised loop
    o = rd.rd_default_options(precision=prec, reorth=ro)
    a, b, r = G.query_trace(3, 1500, 60, o)
    ref = LZ.lanczos_rd(g, 3, 1500, k=60, A=A, d=d, reorth=ro)
    tol = 1e-10 if prec == rd.RD_F64 else 1e-4
    np.testing.assert_allclose(a, ref.alpha, rtol=0, atol=tol)
    np.testing.assert_allclose(b, ref.beta[1:61], rtol=0, atol=tol)
    # converged values against the dense truth
    s, t = I.uniform_pairs(g.n, 6, seed=51)
    truth = D.rd_all(g, s, t)
    eps = 1e-10 if prec == rd.RD_F64 else 1e-5
    bar = 1e-8 if prec == rd.RD_F64 else 1e-3
    for p in range(len(s)):
        res = G.query(int(s[p]), int(t[p]), eps, o)
        assert res.status == rd.RD_OK
        assert res.r == pytest.approx(truth[p], rel=bar)


@pytest.mark.parametrize("ro", [1, 2])
def test_reorth_long_run_past_convergence_stays_at_the_truth(ro):
    # 3n iterations, far beyond convergence: the estimate stays at |s - t|
    g = I.path(200)
    G = _graph(g)
    out = G.query(3, 150, 1.0, rd.rd_default_options(fixed_k=600, reorth=ro))
    assert out.iters == 600
    assert out.r == pytest.approx(147.0, rel=1e-8)


def test_single_workgroup_variants():
    # the one-workgroup kernel stages the CSR in LDS when it fits beside the two
    # vectors and keeps degrees in registers when n <= 4096; each combination
    # against closed forms or the oracle, plain and batched
    cases = [
        (I.grid(64, 64), rd.RD_F64),     # CSR in LDS, degrees in registers
        (I.random_tree(5000, seed=83), rd.RD_F64),  # CSR in LDS, n > 4096
        (I.grid(80, 80), rd.RD_F64),     # neither (CSR does not fit)
        (I.random_tree(3000, seed=81, weighted=True), rd.RD_F64),  # weights in LDS
    ]
    for g, prec in cases:
        G = _graph(g)
        s, t = I.uniform_pairs(g.n, 6, seed=82)
        A, d = LZ.normalized_adjacency(g)
        truth = np.array([LZ.lanczos_rd(g, int(a), int(b), tol=1e-13, A=A, d=d).r for a, b in zip(s, t)])
        eps, bar = 1e-10, 1e-8
        o = rd.rd_default_options(precision=prec, max_iters=100000)
        res = np.array([G.query(int(a), int(b), eps, o).r for a, b in zip(s, t)])
        assert np.max(np.abs(res - truth) / truth) <= bar, g.name
        out = G.query_batch(s, t, eps, o)
        assert np.max(np.abs(out["r"] - truth) / truth) <= bar, g.name
