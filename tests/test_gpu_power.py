"""GPU parity of the Power Method (rd_power_method, Algorithm 1) against the
CPU FP64 oracle, through the C ABI.

Bars: FP64 1e-11 relative (the two sides differ only in summation order, a
few ulps per step, and the lazy step contracts the error of x); FP32 1e-4
relative (x is rounded to FP32 after every product)."""

import functools

import numpy as np
import pytest

from oracle import dense as D
from oracle import power as PM
from paper_2601_11159_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2601_11159_amd import rd  # noqa: E402


def _oracle(g, s, t, l):
    P, d = PM.transition_matrix(g)
    return np.array([PM.power_method(g, int(a), int(b), l, P=P, d=d) for a, b in zip(s, t)])


@functools.lru_cache(maxsize=None)
def _oracle_cached(name, seed, count, l):
    g = _graphs()[name]
    s, t = I.uniform_pairs(g.n, count, seed=seed)
    return _oracle(g, s, t, l)


@functools.lru_cache(maxsize=None)
def _graphs():
    return {
        "grid": I.grid(24, 17),
        "weighted": I.random_connected(3000, extra=12000, seed=21, weighted=True),
        "tree": I.random_tree(800, seed=4, weighted=True),
        "powerlaw": I.chung_lu(20000, 2.1, 12.0, seed=9),
    }


@pytest.mark.parametrize("name", ["grid", "weighted", "tree", "powerlaw"])
@pytest.mark.parametrize("width", [16, 64, 256])
def test_fp64_matches_oracle(name, width):
    g = _graphs()[name]
    s, t = I.uniform_pairs(g.n, 70, seed=31)  # two groups at width 64, a ragged second one
    t[5] = s[5]
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    for l in [0, 1, 6, 150]:
        out = G.power_method(s, t, l, rd.rd_default_options(precision=rd.RD_F64, block_width=width,
                                                             flags=rd.RD_GENERAL_PATH))
        want = _oracle_cached(name, 31, 70, l).copy()
        want[5] = 0.0
        assert np.all(out["status"] == rd.RD_OK) and np.all(out["iters"] == l)
        assert out["r"][5] == 0.0
        m = s != t
        err = np.abs(out["r"][m] - want[m]) / want[m]
        assert err.max() <= 1e-11, (name, width, l, err.max())


@pytest.mark.parametrize("name", ["grid", "weighted", "powerlaw"])
@pytest.mark.parametrize("flags", [0, 1])
def test_fp32_matches_oracle(name, flags):
    g = _graphs()[name]
    s, t = I.uniform_pairs(g.n, 40, seed=32)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    l = 300
    out = G.power_method(s, t, l, rd.rd_default_options(precision=rd.RD_F32, block_width=64,
                                                         flags=rd.RD_GENERAL_PATH if flags else 0))
    want = _oracle_cached(name, 32, 40, l)
    err = np.abs(out["r"] - want) / want
    assert err.max() <= 1e-4, (name, err.max())


@pytest.mark.parametrize("flags", [0, 1])
def test_last_term_and_monotone_limit(flags):
    # err_est is the last term added; the sums increase with l and stay below r
    g = I.random_connected(500, extra=900, seed=8, weighted=True)
    s, t = I.uniform_pairs(g.n, 20, seed=9)
    truth = D.rd_all(g, s, t)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    o = rd.rd_default_options(precision=rd.RD_F64, block_width=32, flags=rd.RD_GENERAL_PATH if flags else 0)
    prev = np.zeros(len(s))
    for l in [0, 3, 30, 300]:
        out = G.power_method(s, t, l, o)
        _, terms = PM.power_method(g, int(s[0]), int(t[0]), l, terms=True)
        assert abs(out["err_est"][0] - terms[-1]) <= 1e-12 * abs(out["r"][0])
        assert np.all(out["r"] >= prev - 1e-15) and np.all(out["r"] <= truth * (1 + 1e-12))
        prev = out["r"]


def test_theorem_iteration_count_reaches_eps_on_gpu():
    g = I.grid(12, 10)
    L = D.laplacian(g)
    d = np.diag(L)
    lam = np.linalg.eigvalsh(L / np.sqrt(np.outer(d, d)))
    kappa = 2.0 / lam[1]
    eps = 1e-6
    l = PM.iterations_for(kappa, eps)
    s, t = I.uniform_pairs(g.n, 30, seed=2)
    truth = D.rd_all(g, s, t)
    G = rd.RDGraph(g.n, g.u, g.v)
    out = G.power_method(s, t, l, rd.rd_default_options(precision=rd.RD_F64, block_width=32))
    assert np.abs(out["r"] - truth).max() <= eps


@pytest.mark.parametrize("name", ["grid", "weighted", "tree"])
@pytest.mark.parametrize("prec,bar", [(rd.RD_F64, 1e-11), (rd.RD_F32, 1e-4)])
def test_single_workgroup_path_matches_oracle(name, prec, bar):
    # graphs whose two vectors fit in LDS: one workgroup runs all steps of a pair
    g = _graphs()[name]
    s, t = I.uniform_pairs(g.n, 70, seed=31)
    t[5] = s[5]
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    for l in [0, 1, 6, 150]:
        out = G.power_method(s, t, l, rd.rd_default_options(precision=prec))
        want = _oracle_cached(name, 31, 70, l).copy()
        assert np.all(out["status"] == rd.RD_OK) and np.all(out["iters"] == l)
        assert out["r"][5] == 0.0
        m = s != t
        err = np.abs(out["r"][m] - want[m]) / want[m]
        assert err.max() <= bar, (name, prec, l, err.max())


def test_grid_64x64_at_the_benchmark_configuration():
    # the 64x64 grid, 100 pairs, FP64, the l that reaches 1e-8 there: sampled
    # pairs against the oracle's Algorithm 1 at the same l
    g = I.grid(64, 64)
    s, t = I.uniform_pairs(g.n, 100, seed=1)
    G = rd.RDGraph(g.n, g.u, g.v)
    l = 57344
    out = G.power_method(s, t, l, rd.rd_default_options(precision=rd.RD_F64))
    idx = [0, 37, 99]
    want = _oracle(g, s[idx], t[idx], l)
    assert np.abs(out["r"][idx] - want).max() <= 1e-11 * want.max()
    truth = D.rd_all(g, s, t)
    assert np.max(np.abs(out["r"] - truth) / truth) <= 1e-8


def test_node_order_and_device_pointers():
    g = I.chung_lu(30000, 2.3, 10.0, seed=12)
    s, t = I.uniform_pairs(g.n, 50, seed=13)
    o = rd.rd_default_options(precision=rd.RD_F64, block_width=64)
    plain = rd.RDGraph(g.n, g.u, g.v).power_method(s, t, 40, o)
    G = rd.RDGraph(g.n, g.u, g.v, reorder=True)
    ordered = G.power_method(s, t, 40, o)
    assert np.abs(ordered["r"] - plain["r"]).max() <= 1e-12 * plain["r"].max()
    ds = torch.tensor(s, dtype=torch.int32, device="cuda")
    dt = torch.tensor(t, dtype=torch.int32, device="cuda")
    buf = torch.zeros(24 * len(s), dtype=torch.uint8, device="cuda")
    G.power_method(ds, dt, 40, o, out=buf)
    dev = np.frombuffer(buf.cpu().numpy().tobytes(), dtype=rd.RESULT_DTYPE)
    assert np.array_equal(dev["r"], ordered["r"])


def test_autotuned_width_and_empty_input():
    g = I.chung_lu(20000, 2.1, 12.0, seed=9)
    G = rd.RDGraph(g.n, g.u, g.v)
    s, t = I.uniform_pairs(g.n, 10, seed=3)
    out = G.power_method(s, t, 12, rd.rd_default_options(precision=rd.RD_F64))
    want = _oracle(g, s, t, 12)
    assert np.abs(out["r"] - want).max() <= 1e-11 * want.max()
    empty = G.power_method(np.zeros(0, np.int32), np.zeros(0, np.int32), 5)
    assert len(empty) == 0


def test_argument_errors():
    g = I.grid(8, 8)
    G = rd.RDGraph(g.n, g.u, g.v)
    s = np.array([0, 1], np.int32)
    t = np.array([5, 9], np.int32)
    with pytest.raises(rd.RdError):
        G.power_method(s, t, -1)
    with pytest.raises(rd.RdError):
        G.power_method(s, np.array([5, 64], np.int32), 3)
    with pytest.raises(rd.RdError):
        G.power_method(s, t, 3, rd.rd_default_options(block_width=48))
    # the handle still works afterwards
    out = G.power_method(s, t, 3, rd.rd_default_options(block_width=16))
    assert np.all(out["status"] == rd.RD_OK)
