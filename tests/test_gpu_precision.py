"""Precision split on high-condition-number graphs: FP32 sparse products with
FP64 Lanczos scalars, with and without the FP64 energy refinement, against
the FP64 oracle (road-like grids, the stand-in for road networks)."""

import numpy as np
import pytest

from oracle import lanczos as LZ
from paper_2601_11159_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2601_11159_amd import rd  # noqa: E402


@pytest.fixture(scope="module")
def road300():
    g = I.road_like(300, seed=3)
    s, t = I.uniform_pairs(g.n, 64, seed=3)
    A, d = LZ.normalized_adjacency(g)
    truth = np.array([LZ.lanczos_rd(g, int(s[p]), int(t[p]), tol=1e-11, A=A, d=d, max_iters=20000).r
                      for p in range(6)])
    return g, s, t, truth


def test_fp64_plain_meets_tolerance(road300):
    g, s, t, truth = road300
    G = rd.RDGraph(g.n, g.u, g.v)
    for p in range(6):
        res = G.query(int(s[p]), int(t[p]), 1e-6)
        assert res.status == rd.RD_OK
        assert abs(res.r - truth[p]) / truth[p] <= 1e-6


def test_fp32_refined_within_1e4(road300):
    g, s, t, truth = road300
    G = rd.RDGraph(g.n, g.u, g.v)
    o = rd.rd_default_options(precision=rd.RD_F32, block_width=32, refine=1)
    out = G.query_batch(s, t, 1e-5, o)
    err = np.abs(out["r"][:6] - truth) / truth
    raw = G.query_batch(s, t, 1e-5, rd.rd_default_options(precision=rd.RD_F32, block_width=32))
    err_raw = np.abs(raw["r"][:6] - truth) / truth
    print(f"road300 fp32: raw max rel err {err_raw.max():.2e}, refined {err.max():.2e}")
    assert err.max() <= 1e-4
    # the energy is a lower bound of r up to rounding
    assert np.all(out["r"][:6] <= truth * (1 + 1e-6))


def test_fp64_refine_equals_quadrature_value(road300):
    # in FP64 the energy of the potential and the Gauss quadrature value agree
    g, s, t, truth = road300
    G = rd.RDGraph(g.n, g.u, g.v)
    a = G.query_batch(s[:16], t[:16], 1e-8, rd.rd_default_options(block_width=16, refine=1))
    b = G.query_batch(s[:16], t[:16], 1e-8, rd.rd_default_options(block_width=16))
    np.testing.assert_allclose(a["r"], b["r"], rtol=1e-7)
    np.testing.assert_array_equal(a["iters"], b["iters"])


def test_weighted_refine():
    g = I.random_connected(3000, extra=6000, seed=41, weighted=True)
    from oracle import dense as D
    Lp = D.pinv(D.laplacian(g))
    s, t = I.uniform_pairs(g.n, 48, seed=42)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    out = G.query_batch(s, t, 1e-6, rd.rd_default_options(precision=rd.RD_F32, block_width=64, refine=1))
    ref = D.rd_from_pinv(Lp, s, t)
    assert np.max(np.abs(out["r"] - ref) / ref) <= 1e-4
