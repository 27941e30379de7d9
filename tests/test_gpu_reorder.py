"""GPU parity of graphs built with RD_REORDER (internal numbering by decreasing
degree): every entry point keeps the caller's node ids and edge order, and
the results agree with the dense FP64 oracle and with the same graph built
without the relabelling."""

import numpy as np
import pytest

from oracle import dense as D
from paper_2601_11159_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2601_11159_amd import rd  # noqa: E402


@pytest.fixture(scope="module")
def power_law():
    # heterogeneous degrees, so the relabelling is far from the identity
    g = I.chung_lu(3000, 2.3, 8.0, seed=31)
    Lp = D.pinv(D.laplacian(g))
    return g, Lp


PATHS = [0, rd.RD_GENERAL_PATH]


@pytest.mark.parametrize("flags", PATHS)
def test_plain_query_reordered(power_law, flags):
    g, Lp = power_law
    s, t = I.uniform_pairs(g.n, 12, seed=32)
    truth = D.rd_from_pinv(Lp, s, t)
    A = rd.RDGraph(g.n, g.u, g.v)
    R = rd.RDGraph(g.n, g.u, g.v, reorder=True)
    o = rd.rd_default_options(flags=flags)
    for p in range(len(s)):
        a = A.query(int(s[p]), int(t[p]), 1e-10, o)
        b = R.query(int(s[p]), int(t[p]), 1e-10, o)
        assert b.status == rd.RD_OK
        assert b.r == pytest.approx(truth[p], rel=1e-8)
        # Krylov iterations are invariant under relabelling in exact arithmetic
        assert abs(a.iters - b.iters) <= 1


def test_trace_reordered_matches_unreordered(power_law):
    g, _ = power_law
    A = rd.RDGraph(g.n, g.u, g.v)
    R = rd.RDGraph(g.n, g.u, g.v, reorder=True)
    o = rd.rd_default_options(flags=rd.RD_GENERAL_PATH)
    a1, b1, r1 = A.query_trace(5, 2000, 12, o)
    a2, b2, r2 = R.query_trace(5, 2000, 12, o)
    assert len(a1) == len(a2) == 12
    # the same recurrence up to the order of the roundings
    np.testing.assert_allclose(a2, a1, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(b2, b1, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r2, r1, rtol=1e-9)


@pytest.mark.parametrize("prec,tol,bar", [(rd.RD_F64, 1e-10, 1e-8), (rd.RD_F32, 1e-5, 1e-3)])
@pytest.mark.parametrize("flags", PATHS)
def test_batch_reordered(power_law, prec, tol, bar, flags):
    g, Lp = power_law
    s, t = I.uniform_pairs(g.n, 150, seed=33)
    t[4] = s[4]
    mask = s != t
    truth = np.zeros(len(s))
    truth[mask] = D.rd_from_pinv(Lp, s[mask], t[mask])
    R = rd.RDGraph(g.n, g.u, g.v, reorder=True)
    out = R.query_batch(s, t, tol, rd.rd_default_options(precision=prec, block_width=32, flags=flags))
    assert np.all(out["status"] == rd.RD_OK)
    assert out["r"][4] == 0.0
    err = np.abs(out["r"][mask] - truth[mask]) / truth[mask]
    assert err.max() <= bar, err.max()


def test_batch_reordered_device_pointers(power_law):
    g, Lp = power_law
    s, t = I.uniform_pairs(g.n, 64, seed=34)
    truth = D.rd_from_pinv(Lp, s, t)
    R = rd.RDGraph(g.n, torch.from_numpy(g.u).cuda(), torch.from_numpy(g.v).cuda(), reorder=True)
    out = torch.zeros(64 * 24, dtype=torch.uint8, device="cuda")
    opts = rd.rd_default_options(block_width=64, flags=rd.RD_GENERAL_PATH,
                                 stream=torch.cuda.current_stream().cuda_stream)
    R.query_batch(torch.from_numpy(s).cuda(), torch.from_numpy(t).cuda(), 1e-10, opts, out=out)
    res = np.frombuffer(out.cpu().numpy().tobytes(), dtype=rd.RESULT_DTYPE)
    assert np.max(np.abs(res["r"] - truth) / truth) <= 1e-8


def test_gradient_reordered_in_caller_edge_order():
    g = I.random_connected(900, extra=5000, seed=35, weighted=True)
    s, t = I.uniform_pairs(g.n, 40, seed=36)
    gbar = np.linspace(0.5, 1.5, 40)
    Lp = D.pinv(D.laplacian(g))
    ref = D.grad_edges(g, Lp, s, t, gbar)
    R = rd.RDGraph(g.n, g.u, g.v, g.w, reorder=True)
    fwd, gw = R.grad_edges(s, t, gbar, 1e-12, rd.rd_default_options(block_width=16))
    np.testing.assert_allclose(fwd["r"], D.rd_from_pinv(Lp, s, t), rtol=1e-9)
    assert np.linalg.norm(gw - ref) / np.linalg.norm(ref) <= 1e-6


def test_reorder_with_set_weights_and_ties():
    # a cycle has all degrees equal: the relabelling is the identity (ties by id)
    g = I.cycle(40)
    R = rd.RDGraph(g.n, g.u, g.v, reorder=True)
    assert R.query(0, 20, 1e-12).r == pytest.approx(10.0, rel=1e-10)
    # weights replaced after the build stay in caller edge order
    w = np.linspace(1.0, 3.0, g.m)
    R.set_weights(w)
    gw = I.Graph(g.n, g.u, g.v, w, "cycle_w")
    truth = D.rd_all(gw, np.array([0, 3]), np.array([20, 31]))
    out = R.query_batch(np.array([0, 3], np.int32), np.array([20, 31], np.int32), 1e-12,
                        rd.rd_default_options(flags=rd.RD_GENERAL_PATH, block_width=16))
    np.testing.assert_allclose(out["r"], truth, rtol=1e-9)
