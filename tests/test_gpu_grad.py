"""GPU parity of the edge-weight gradient (rd_grad_edges and the autograd
Function) against the dense FP64 oracle, central finite differences and the
homogeneity identity."""

import numpy as np
import pytest

from oracle import dense as D
from paper_2601_11159_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2601_11159_amd import rd  # noqa: E402
from paper_2601_11159_amd.autograd import resistance_distance  # noqa: E402


def _opts(**kw):
    return rd.rd_default_options(**kw)


@pytest.mark.parametrize("width", [16, 64])
def test_gradient_matches_dense_pseudoinverse(width):
    g = I.random_connected(800, extra=5000, seed=21, weighted=True)
    s, t = I.uniform_pairs(g.n, 40, seed=22)
    gbar = np.linspace(0.5, 1.5, 40)
    Lp = D.pinv(D.laplacian(g))
    ref = D.grad_edges(g, Lp, s, t, gbar)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    fwd, gw = G.grad_edges(s, t, gbar, 1e-12, _opts(block_width=width))
    np.testing.assert_allclose(fwd["r"], D.rd_from_pinv(Lp, s, t), rtol=1e-9)
    rel = np.linalg.norm(gw - ref) / np.linalg.norm(ref)
    print(f"width {width}: grad rel err {rel:.2e}")
    assert rel <= 1e-6
    assert np.max(np.abs(gw - ref)) <= 1e-6 * np.max(np.abs(ref)) + 1e-7


def test_gradient_fp32():
    g = I.random_connected(1000, extra=6000, seed=23, weighted=True)
    s, t = I.uniform_pairs(g.n, 64, seed=24)
    ref = D.grad_edges(g, D.pinv(D.laplacian(g)), s, t)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    fwd, gw = G.grad_edges(s, t, None, 1e-6, _opts(block_width=64, precision=rd.RD_F32))
    rel = np.linalg.norm(gw - ref) / np.linalg.norm(ref)
    print(f"fp32 grad rel err {rel:.2e}")
    assert rel <= 1e-3


def test_gradient_more_pairs_than_width_and_degenerate_pairs():
    g = I.random_connected(500, extra=2500, seed=25, weighted=True)
    s, t = I.uniform_pairs(g.n, 70, seed=26)
    t[3] = s[3]  # r = 0, contributes nothing
    ref = D.grad_edges(g, D.pinv(D.laplacian(g)), s, t)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    fwd, gw = G.grad_edges(s, t, None, 1e-12, _opts(block_width=32))
    assert fwd["r"][3] == 0.0
    assert np.linalg.norm(gw - ref) / np.linalg.norm(ref) <= 1e-6


def test_gradient_on_bfs_ball_of_weighted_chung_lu():
    # Dense check on the induced subgraph of a 2000-node BFS ball of a weighted
    # Chung-Lu graph (lognormal weights), run as its own graph.
    big = I.chung_lu(100000, 2.1, 20, seed=5)
    w = I.lognormal_weights(big.m, 0.0, 1.0, seed=5)
    adj = [[] for _ in range(big.n)]
    for a, b in zip(big.u.tolist(), big.v.tolist()):
        adj[a].append(b)
        adj[b].append(a)
    root = int(np.argsort(big.degrees())[big.n // 2])
    seen = {root: 0}
    frontier = [root]
    while frontier and len(seen) < 2000:
        nxt = []
        for x in frontier:
            for y in adj[x]:
                if y not in seen and len(seen) < 2000:
                    seen[y] = len(seen)
                    nxt.append(y)
        frontier = nxt
    keep = np.array([(a in seen and b in seen) for a, b in zip(big.u.tolist(), big.v.tolist())])
    uu = np.array([seen[a] for a in big.u[keep].tolist()], np.int32)
    vv = np.array([seen[b] for b in big.v[keep].tolist()], np.int32)
    sub = I._canon(len(seen), np.stack([uu, vv], 1), w[keep].astype(np.float64))
    sub = I.Graph(sub.n, sub.u, sub.v, sub.w.astype(np.float32))
    # the BFS ball is connected by construction
    s, t = I.uniform_pairs(sub.n, 32, seed=27)
    Lp = D.pinv(D.laplacian(sub))
    ref = D.grad_edges(sub, Lp, s, t)
    G = rd.RDGraph(sub.n, sub.u, sub.v, sub.w)
    fwd, gw = G.grad_edges(s, t, None, 1e-12, _opts(block_width=32))
    assert np.linalg.norm(gw - ref) / np.linalg.norm(ref) <= 1e-5
    fwd32, gw32 = G.grad_edges(s, t, None, 1e-6, _opts(block_width=32, precision=rd.RD_F32))
    assert np.linalg.norm(gw32 - ref) / np.linalg.norm(ref) <= 1e-3


def test_central_differences_and_euler_identity_weighted_chung_lu():
    g = I.chung_lu(200000, 2.1, 20, seed=5)
    w = I.lognormal_weights(g.m, 0.0, 1.0, seed=5).astype(np.float64)
    s, t = I.uniform_pairs(g.n, 64, seed=6)
    G = rd.RDGraph(g.n, g.u, g.v, w)
    opts = _opts(block_width=64)
    fwd, gw = G.grad_edges(s, t, None, 1e-11, opts)
    # homogeneity of degree -1: sum_e w_e dL/dw_e = -L
    euler = float(np.dot(w, gw.astype(np.float64)))
    assert euler == pytest.approx(-fwd["r"].sum(), rel=1e-5)
    rng = np.random.default_rng(7)
    edges = rng.choice(g.m, size=12, replace=False)
    # include the edges with the largest gradient magnitude (well above FD noise)
    edges = np.concatenate([edges, np.argsort(np.abs(gw))[-8:]])
    for e in edges:
        h = 1e-3 * w[e]
        wp = w.copy()
        wp[e] += h
        G.set_weights(wp)
        rp = G.query_batch(s, t, 1e-12, opts)["r"].sum()
        wm = w.copy()
        wm[e] -= h
        G.set_weights(wm)
        rm = G.query_batch(s, t, 1e-12, opts)["r"].sum()
        fd = (rp - rm) / (2 * h)
        assert gw[e] == pytest.approx(fd, rel=1e-3, abs=1e-6 * np.abs(gw).max())
    G.set_weights(w)


def test_autograd_function_matches_dense():
    g = I.random_connected(600, extra=3000, seed=28, weighted=True)
    s, t = I.uniform_pairs(g.n, 24, seed=29)
    Lp = D.pinv(D.laplacian(g))
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    w = torch.tensor(g.w, dtype=torch.float64, device="cuda", requires_grad=True)
    ds = torch.from_numpy(s).cuda()
    dt = torch.from_numpy(t).cuda()
    r = resistance_distance(w, G, ds, dt, eps=1e-12, block_width=32)
    np.testing.assert_allclose(r.detach().cpu().numpy(), D.rd_from_pinv(Lp, s, t), rtol=1e-9)
    coef = torch.linspace(0.1, 1.0, len(s), dtype=torch.float64, device="cuda")
    (r * coef).sum().backward()
    ref = D.grad_edges(g, Lp, s, t, coef.cpu().numpy())
    got = w.grad.cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-6
    # float32 weights
    w32 = torch.tensor(g.w, dtype=torch.float32, device="cuda", requires_grad=True)
    r32 = resistance_distance(w32, G, ds, dt, eps=1e-6, precision=rd.RD_F32, block_width=32)
    r32.sum().backward()
    assert w32.grad.dtype == torch.float32
    assert torch.isfinite(w32.grad).all()


def _hub_graph():
    # node 0 joined to every other node: its row holds ~1000 upper entries,
    # cut into many edge chunks with a ragged last one
    rng = np.random.default_rng(41)
    n = 1003
    edges = {(0, i) for i in range(1, n)}
    while len(edges) < n - 1 + 2500:
        a, b = (int(x) for x in rng.integers(1, n, size=2))
        if a != b:
            edges.add((min(a, b), max(a, b)))
    pairs = sorted(edges)
    return I._canon(n, pairs, rng.uniform(0.25, 4.0, size=len(pairs)), "hub_1003")


@pytest.mark.parametrize("width", [16, 32, 64, 128, 256])
def test_gradient_and_refinement_on_hub_rows(width):
    g = _hub_graph()
    s, t = I.uniform_pairs(g.n, 50, seed=42)
    s[0], t[0] = 0, 7  # the hub itself
    t[5] = s[5]
    Lp = D.pinv(D.laplacian(g))
    ref = D.grad_edges(g, Lp, s, t)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    fwd, gw = G.grad_edges(s, t, None, 1e-12, _opts(block_width=width))
    assert np.linalg.norm(gw - ref) / np.linalg.norm(ref) <= 1e-6
    assert np.max(np.abs(gw - ref)) <= 1e-6 * np.max(np.abs(ref))
    mask = s != t
    truth = D.rd_from_pinv(Lp, s[mask], t[mask])
    out = G.query_batch(s, t, 1e-10, _opts(block_width=width, refine=1))
    assert out["r"][5] == 0.0
    np.testing.assert_allclose(out["r"][mask], truth, rtol=1e-9)


def test_gradient_degenerate_inputs():
    g = I.random_connected(300, extra=900, seed=91, weighted=True)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    # every pair has s == t: r = 0 and a zero gradient
    s = np.arange(20, dtype=np.int32)
    fwd, gw = G.grad_edges(s, s.copy(), None, 1e-8, _opts(block_width=16))
    assert np.all(fwd["r"] == 0.0) and np.all(fwd["iters"] == 0)
    assert np.all(gw == 0.0)
    # no pairs at all
    fwd0, gw0 = G.grad_edges(np.zeros(0, np.int32), np.zeros(0, np.int32), None, 1e-8, _opts(block_width=16))
    assert len(fwd0) == 0 and np.all(gw0 == 0.0)
    # the same pair many times: the gradient is the single-pair gradient times the count
    s1 = np.full(37, 5, np.int32)
    t1 = np.full(37, 250, np.int32)
    f1, g1 = G.grad_edges(s1[:1], t1[:1], None, 1e-12, _opts(block_width=16))
    fn, gn = G.grad_edges(s1, t1, None, 1e-12, _opts(block_width=16))
    np.testing.assert_allclose(gn, 37 * g1, rtol=1e-5)
    np.testing.assert_allclose(fn["r"], f1["r"][0], rtol=1e-12)
