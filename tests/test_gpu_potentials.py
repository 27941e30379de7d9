"""GPU parity of the electric potentials (rd_potentials; Section 6.3, the
potential estimate of Algorithm 5) against the CPU FP64 oracle, through the
C ABI.

Bars: at a fixed iteration count k the GPU and the oracle compute the same
phi_hat (FP64: 1e-9 of max |phi|, the bar of the alpha/beta step parity); run
to eps = 1e-12 the estimate meets the dense L^+ b to 1e-5 of max |phi| (the
error of phi is of the order of the square root of r's); FP32 storage stays
within 1e-4 of FP64 at the same k."""

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


def _oracle_phi(g, s, t, k):
    A, d = LZ.normalized_adjacency(g)
    out = []
    for a, b in zip(s, t):
        run = LZ.lanczos_rd(g, int(a), int(b), k=k, keep_vectors=True, A=A, d=d)
        phi = LZ.potentials_lanczos(g, int(a), int(b), run, d)
        out.append(phi - phi.mean())
    return np.array(out)


GRAPHS = {
    "grid": lambda: I.grid(20, 20),
    "weighted": lambda: I.random_connected(400, extra=1200, seed=41, weighted=True),
    "powerlaw": lambda: I.chung_lu(5000, 2.3, 10.0, seed=7),
}


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("k", [1, 3, 12])
def test_fixed_k_matches_oracle(name, k):
    g = GRAPHS[name]()
    s, t = I.uniform_pairs(g.n, 40, seed=17)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    o = rd.rd_default_options(precision=rd.RD_F64, block_width=16, fixed_k=k, max_iters=k)
    res, phi = G.potentials(s, t, 1e-12, o)
    want = _oracle_phi(g, s, t, k)
    scale = np.abs(want).max(axis=1, keepdims=True)
    err = np.abs(phi - want) / scale
    assert err.max() <= 1e-9, (name, k, err.max())
    assert np.all(res["iters"] == k)
    assert np.abs(phi.sum(axis=1)).max() <= 1e-9 * scale.max()


@pytest.mark.parametrize("name", list(GRAPHS))
def test_converged_potentials_and_flows_match_dense(name):
    g = GRAPHS[name]()
    s, t = I.uniform_pairs(g.n, 70, seed=18)  # three groups at width 32, the last ragged
    t[9] = s[9]
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    res, phi = G.potentials(s, t, 1e-12, rd.rd_default_options(precision=rd.RD_F64, block_width=32))
    Lp = D.pinv(D.laplacian(g))
    m = s != t
    assert np.all(phi[9] == 0.0) and res["r"][9] == 0.0
    w = np.ones(g.m) if g.w is None else np.asarray(g.w)
    for p in np.flatnonzero(m):
        ref = D.potentials(Lp, int(s[p]), int(t[p]))
        sc = np.abs(ref).max()
        assert np.abs(phi[p] - ref).max() <= 1e-5 * sc, (name, p)
        f = w * D.flows(g, phi[p])
        fr = w * D.flows(g, ref)
        assert np.abs(f - fr).max() <= 1e-5 * np.abs(fr).max()
    truth = D.rd_from_pinv(Lp, s[m], t[m])
    assert np.max(np.abs(res["r"][m] - truth) / truth) <= 1e-10


def test_fp32_storage_against_fp64():
    g = GRAPHS["powerlaw"]()
    s, t = I.uniform_pairs(g.n, 40, seed=19)
    G = rd.RDGraph(g.n, g.u, g.v)
    k = 8
    _, p64 = G.potentials(s, t, 1e-12, rd.rd_default_options(precision=rd.RD_F64, block_width=64,
                                                             fixed_k=k, max_iters=k))
    _, p32 = G.potentials(s, t, 1e-12, rd.rd_default_options(precision=rd.RD_F32, block_width=64,
                                                             fixed_k=k, max_iters=k))
    sc = np.abs(p64).max(axis=1, keepdims=True)
    assert (np.abs(p32 - p64) / sc).max() <= 1e-4


def test_node_order_gives_the_same_potentials():
    g = I.chung_lu(20000, 2.1, 12.0, seed=23)
    s, t = I.uniform_pairs(g.n, 24, seed=24)
    o = rd.rd_default_options(precision=rd.RD_F64, block_width=32, fixed_k=6, max_iters=6)
    _, a = rd.RDGraph(g.n, g.u, g.v).potentials(s, t, 1e-12, o)
    _, b = rd.RDGraph(g.n, g.u, g.v, reorder=True).potentials(s, t, 1e-12, o)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_weighted_chung_lu_1M_current_balance_and_energy():
    # full-size weighted power-law graph (1M nodes, lognormal FP32 weights): the
    # potentials satisfy Kirchhoff's current law L phi = e_s - e_t and their
    # energy is r, properties that hold at any size
    g0 = I.chung_lu(1_000_000, 2.1, 20.0, 2)
    w = I.lognormal_weights(g0.m, 0.0, 1.0, seed=5)
    g = I.Graph(g0.n, g0.u, g0.v, w)
    s, t = I.uniform_pairs(g.n, 4, seed=6)
    G = rd.RDGraph(g.n, g.u, g.v, w, reorder=True)
    res, phi = G.potentials(s, t, 1e-10, rd.rd_default_options(precision=rd.RD_F64, block_width=16))
    wd = np.asarray(w, dtype=np.float64)
    for p in range(len(s)):
        f = wd * (phi[p][g.u] - phi[p][g.v])
        net = np.bincount(g.u, f, g.n) - np.bincount(g.v, f, g.n)
        b = np.zeros(g.n)
        b[s[p]] = 1.0
        b[t[p]] = -1.0
        assert np.abs(net - b).max() <= 1e-3, p
        energy = float(np.sum(wd * (phi[p][g.u] - phi[p][g.v]) ** 2))
        assert abs(energy - res["r"][p]) <= 1e-6 * res["r"][p]


def test_argument_errors():
    g = I.grid(8, 8)
    G = rd.RDGraph(g.n, g.u, g.v)
    with pytest.raises(rd.RdError):
        G.potentials(np.array([0], np.int32), np.array([64], np.int32), 1e-6)
    with pytest.raises(rd.RdError):
        G.potentials(np.array([0], np.int32), np.array([5], np.int32), 0.0)
    res, phi = G.potentials(np.array([0], np.int32), np.array([5], np.int32), 1e-8,
                            rd.rd_default_options(block_width=16))
    assert res["status"][0] == rd.RD_OK and phi.shape == (1, 64)
