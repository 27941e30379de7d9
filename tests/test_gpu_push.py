"""GPU parity of Lanczos Push (rd_lanczos_push, Algorithm 4) against the CPU
FP64 oracle, through the C ABI.

Bar: 1e-10 relative on r' (FP64 on both sides; the GPU pulls each node's AMV
sum in adjacency order and sums alpha and beta^2 in fixed point, which changes
only the rounding of those sums)."""

import numpy as np
import pytest

from oracle import lanczos as LZ
from oracle import push as LP
from paper_2601_11159_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2601_11159_amd import rd  # noqa: E402

GRAPHS = {
    "grid": lambda: I.grid(30, 30),
    "weighted": lambda: I.random_connected(2000, extra=5000, seed=71, weighted=True),
    "powerlaw": lambda: I.chung_lu(20000, 2.3, 8.0, seed=72),
}


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("eps", [0.0, 1e-6, 1e-4, 1e-3])
def test_matches_oracle(name, eps):
    g = GRAPHS[name]()
    W, d = LP._adjacency(g)
    s, t = I.uniform_pairs(g.n, 6, seed=73)
    t[3] = s[3]
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    for k in [1, 2, 7, 25]:
        out = G.lanczos_push(s, t, k, eps)
        assert out["r"][3] == 0.0
        for p in range(len(s)):
            if s[p] == t[p]:
                continue
            want = LP.lanczos_push(g, int(s[p]), int(t[p]), k, eps, W=W, d=d)
            assert out["iters"][p] == len(want.alpha)
            assert abs(out["r"][p] - want.r) <= 1e-10 * abs(want.r), (name, eps, k, p, out["r"][p], want.r)


def test_eps_zero_is_the_lanczos_estimate():
    g = GRAPHS["weighted"]()
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    s, t = I.uniform_pairs(g.n, 6, seed=74)
    for k in [3, 15]:
        out = G.lanczos_push(s, t, k, 0.0)
        for p in range(len(s)):
            _, _, rhat = G.query_trace(int(s[p]), int(t[p]), k)
            assert len(rhat) == k
            assert abs(out["r"][p] - rhat[-1]) <= 1e-10 * rhat[-1]


def test_blocked_pushes_give_the_first_order_value():
    g = GRAPHS["weighted"]()
    W, d = LP._adjacency(g)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    s, t = I.uniform_pairs(g.n, 5, seed=75)
    out = G.lanczos_push(s, t, 10, 1e6)
    np.testing.assert_allclose(out["r"], 1.0 / d[s] + 1.0 / d[t], rtol=1e-14)
    assert np.all(out["iters"] == 1)


def test_more_pairs_than_slots_and_node_order():
    g = I.chung_lu(3000, 2.1, 6.0, seed=76)
    W, d = LP._adjacency(g)
    s, t = I.uniform_pairs(g.n, 600, seed=77)
    a = rd.RDGraph(g.n, g.u, g.v).lanczos_push(s, t, 6, 1e-4)
    b = rd.RDGraph(g.n, g.u, g.v, reorder=True).lanczos_push(s, t, 6, 1e-4)
    assert np.max(np.abs(a["r"] - b["r"]) / np.abs(a["r"])) <= 1e-10
    for p in [0, 299, 599]:
        want = LP.lanczos_push(g, int(s[p]), int(t[p]), 6, 1e-4, W=W, d=d)
        assert abs(a["r"][p] - want.r) <= 1e-10 * abs(want.r)


def test_road_like_2000_full_size():
    # the road-like 2000 x 2000 graph (4M nodes): two pairs against the oracle
    g = I.road_like(2000, seed=3)
    W, d = LP._adjacency(g)
    s, t = I.uniform_pairs(g.n, 2, seed=3)
    G = rd.RDGraph(g.n, g.u, g.v)
    out = G.lanczos_push(s, t, 60, 1e-5)
    for p in range(2):
        want = LP.lanczos_push(g, int(s[p]), int(t[p]), 60, 1e-5, W=W, d=d)
        assert out["iters"][p] == len(want.alpha)
        assert abs(out["r"][p] - want.r) <= 1e-10 * abs(want.r)


def test_argument_errors():
    g = I.grid(8, 8)
    G = rd.RDGraph(g.n, g.u, g.v)
    s = np.array([0], np.int32)
    t = np.array([5], np.int32)
    for args in [(s, t, 0, 1e-3), (s, t, 5, -1.0), (s, np.array([64], np.int32), 5, 1e-3)]:
        with pytest.raises(rd.RdError):
            G.lanczos_push(*args)
    out = G.lanczos_push(s, t, 5, 1e-3)
    assert out["status"][0] == rd.RD_OK


def test_bitwise_repeatable():
    # the lists' order depends on scheduling; the per-node sums (adjacency
    # order) and the fixed-point alpha and beta do not
    g = I.chung_lu(30000, 2.1, 8.0, seed=78)
    G = rd.RDGraph(g.n, g.u, g.v)
    s, t = I.uniform_pairs(g.n, 300, seed=79)
    a = G.lanczos_push(s, t, 12, 1e-5)
    b = G.lanczos_push(s, t, 12, 1e-5)
    c = G.lanczos_push(s[:7], t[:7], 12, 1e-5)  # other slot counts, other list orders
    assert np.array_equal(a["r"], b["r"]) and np.array_equal(a["r"][:7], c["r"])
