"""GPU parity of the batched Lanczos path (rd_query_batch) against the CPU
FP64 oracle, through the C ABI."""

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


def _opts(**kw):
    # these tests exercise the block-column kernels, also on graphs small
    # enough for the single-workgroup path (tested separately below)
    kw.setdefault("flags", rd.RD_GENERAL_PATH)
    return rd.rd_default_options(**kw)


@pytest.mark.parametrize("prec,tol,bar", [(rd.RD_F64, 1e-10, 1e-8), (rd.RD_F32, 1e-6, 1e-4)])
def test_single_workgroup_path_batch(prec, tol, bar):
    # graphs whose two vectors fit in LDS run one workgroup per pair
    for g in [I.grid(64, 64), I.random_connected(2000, extra=9000, seed=13, weighted=True)]:
        s, t = I.uniform_pairs(g.n, 120, seed=14)
        t[7] = s[7]
        mask = s != t
        truth = np.zeros(len(s))
        truth[mask] = D.rd_all(g, s[mask], t[mask])
        G = rd.RDGraph(g.n, g.u, g.v, g.w)
        out = G.query_batch(s, t, tol, rd.rd_default_options(precision=prec))
        assert np.all(out["status"] == rd.RD_OK)
        assert out["r"][7] == 0.0 and out["iters"][7] == 0
        err = np.abs(out["r"][mask] - truth[mask]) / truth[mask]
        assert err.max() <= bar, (g.name, err.max())
        gen = G.query_batch(s, t, tol, _opts(precision=prec, block_width=32))
        assert np.all(np.abs(out["iters"] - gen["iters"]) <= 1)


@pytest.mark.parametrize("width", [16, 32, 64, 128, 256])
def test_grid64_batch_fp64_all_widths(width):
    g = I.grid(64, 64)
    s, t = I.uniform_pairs(g.n, 100, seed=1)
    truth = D.rd_all(g, s, t)
    G = rd.RDGraph(g.n, g.u, g.v)
    out = G.query_batch(s, t, 1e-8, _opts(block_width=width))
    assert np.all(out["status"] == rd.RD_OK)
    err = np.abs(out["r"] - truth) / truth
    print(f"width {width}: max rel err {err.max():.3e} iters {out['iters'].min()}..{out['iters'].max()}")
    assert err.max() <= 1e-6
    assert np.mean(err <= 1e-8) >= 0.95
    # same stopping decisions as the single-pair path up to rounding
    for p in range(0, 100, 17):
        single = G.query(int(s[p]), int(t[p]), 1e-8)
        assert abs(int(single.iters) - int(out["iters"][p])) <= 1
        assert out["r"][p] == pytest.approx(single.r, rel=1e-9)


def test_batch_matches_literal_algorithm_fixed_k():
    g = I.road_like(60, seed=9)
    s, t = I.uniform_pairs(g.n, 40, seed=3)
    G = rd.RDGraph(g.n, g.u, g.v)
    out = G.query_batch(s, t, 0.0, _opts(block_width=32, fixed_k=25))
    A, d = LZ.normalized_adjacency(g)
    for p in range(len(s)):
        run = LZ.lanczos_rd(g, int(s[p]), int(t[p]), k=25, A=A, d=d)
        assert out["iters"][p] == 25
        assert out["r"][p] == pytest.approx(run.r, rel=1e-10)


def test_refill_with_uneven_pairs_and_degenerate_entries():
    # 300 pairs through 32 slots: pairs differ in length (near and far pairs
    # on a grid), some pairs repeat a node (r = 0), all must come back.
    g = I.grid(40, 40)
    s, t = I.uniform_pairs(g.n, 300, seed=4)
    t[::7] = s[::7] + 1  # neighbours: short runs
    t[5::50] = s[5::50]  # s == t
    truth = np.where(s == t, 0.0, 0.0)
    mask = s != t
    truth[mask] = D.rd_all(g, s[mask], t[mask])
    G = rd.RDGraph(g.n, g.u, g.v)
    out = G.query_batch(s, t, 1e-9, _opts(block_width=32))
    assert np.all(out["status"] == rd.RD_OK)
    assert np.all(out["r"][~mask] == 0.0) and np.all(out["iters"][~mask] == 0)
    err = np.abs(out["r"][mask] - truth[mask]) / truth[mask]
    assert err.max() <= 1e-7
    assert out["iters"][mask].min() < out["iters"][mask].max()


def test_weighted_batch():
    g = I.random_connected(600, extra=4000, seed=8, weighted=True)
    Lp = D.pinv(D.laplacian(g))
    s, t = I.uniform_pairs(g.n, 70, seed=6)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    for prec, tol, bar in [(rd.RD_F64, 1e-10, 1e-8), (rd.RD_F32, 1e-6, 1e-4)]:
        out = G.query_batch(s, t, tol, _opts(block_width=64, precision=prec))
        err = np.abs(out["r"] - D.rd_from_pinv(Lp, s, t)) / D.rd_from_pinv(Lp, s, t)
        assert err.max() <= bar, (prec, err.max())


def test_chung_lu_fp32_batch_with_long_rows():
    # power-law graph with rows longer than the short-row limit (1024)
    g = I.chung_lu(300000, 2.1, 20, seed=2)
    assert g.degrees().max() > 2048
    A, d = LZ.normalized_adjacency(g)
    s, t = I.uniform_pairs(g.n, 200, seed=7)
    hs, ht = I.hub_pairs(g, 56, seed=8)
    s = np.concatenate([s, hs])
    t = np.concatenate([t, ht])
    G = rd.RDGraph(g.n, g.u, g.v)
    out = G.query_batch(s, t, 1e-4, _opts(precision=rd.RD_F32))
    assert np.all(out["status"] == rd.RD_OK)
    idx = list(range(0, len(s), 16)) + list(range(200, 256, 8))
    for p in idx:
        run = LZ.lanczos_rd(g, int(s[p]), int(t[p]), tol=1e-10, A=A, d=d)
        assert abs(out["r"][p] - run.r) / run.r <= 1e-4
    out64 = G.query_batch(s[:64], t[:64], 1e-8, _opts(precision=rd.RD_F64, block_width=64))
    for p in range(0, 64, 9):
        run = LZ.lanczos_rd(g, int(s[p]), int(t[p]), tol=1e-8, A=A, d=d)
        assert out64["r"][p] == pytest.approx(run.r, rel=1e-9)


def test_device_pointer_batch():
    g = I.grid(32, 32)
    s, t = I.uniform_pairs(g.n, 50, seed=9)
    truth = D.rd_all(g, s, t)
    G = rd.RDGraph(g.n, torch.from_numpy(g.u).cuda(), torch.from_numpy(g.v).cuda())
    ds = torch.from_numpy(s).cuda()
    dt = torch.from_numpy(t).cuda()
    out = torch.zeros(50 * 24, dtype=torch.uint8, device="cuda")
    opts = _opts(block_width=32, stream=torch.cuda.current_stream().cuda_stream)
    G.query_batch(ds, dt, 1e-10, opts, out=out)
    res = np.frombuffer(out.cpu().numpy().tobytes(), dtype=rd.RESULT_DTYPE)
    assert np.max(np.abs(res["r"] - truth) / truth) <= 1e-8


def test_batch_argument_errors():
    g = I.grid(8, 8)
    G = rd.RDGraph(g.n, g.u, g.v)
    with pytest.raises(rd.RdError) as e:
        G.query_batch(np.array([0, 1], np.int32), np.array([5, 64], np.int32), 1e-6)
    assert e.value.code == rd.RD_E_ARG
    with pytest.raises(rd.RdError):
        G.query_batch(np.array([0], np.int32), np.array([5], np.int32), 1e-6, _opts(block_width=48))
    assert len(G.query_batch(np.zeros(0, np.int32), np.zeros(0, np.int32), 1e-6)) == 0


def test_autotuned_width_and_schedule(tmp_path, monkeypatch):
    # rows longer than 512 entries exist, so the long-row threshold matters
    g = I.chung_lu(50000, 2.3, 32, seed=4)
    assert np.bincount(np.r_[g.u, g.v]).max() > 512
    s, t = I.uniform_pairs(g.n, 300, seed=2)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("RD_AUTOTUNE_CACHE", str(cache))
    G = rd.RDGraph(g.n, g.u, g.v)
    assert G.batch_schedule() == (256, 1024)  # the default before tuning
    width = G.tune_width(rd.RD_F32, len(s))
    wave, long_deg = G.batch_schedule()
    assert width in (32, 64, 128, 256)
    assert wave in (128, 256, 512) and long_deg in (512, 1024, 2048)
    out = G.query_batch(s, t, 1e-4, _opts(precision=rd.RD_F32))
    A, d = LZ.normalized_adjacency(g)
    for p in range(0, 300, 50):
        run = LZ.lanczos_rd(g, int(s[p]), int(t[p]), tol=1e-10, A=A, d=d)
        assert abs(out["r"][p] - run.r) / run.r <= 1e-4
    # a new handle on the same graph reads the choice back from the cache file
    fields = cache.read_text().split()
    assert fields[-4:-1] == [str(width), str(wave), str(long_deg)]
    assert float(fields[-1]) > 0.0  # product time per column (ms)
    G2 = rd.RDGraph(g.n, g.u, g.v)
    assert G2.tune_width(rd.RD_F32, len(s)) == width
    assert G2.batch_schedule() == (wave, long_deg)
    # a line without the time (four fields) is still read
    cache.write_text(" ".join(fields[:-1]) + "\n")
    G3 = rd.RDGraph(g.n, g.u, g.v)
    assert G3.tune_width(rd.RD_F32, len(s)) == width
    out3 = G3.query_batch(s, t, 1e-4, _opts(precision=rd.RD_F32))
    np.testing.assert_allclose(out3["r"], out["r"], rtol=2e-4)


@pytest.mark.parametrize("ro", [1, 2])
@pytest.mark.parametrize("prec,eps,bar", [(rd.RD_F64, 1e-10, 1e-8), (rd.RD_F32, 1e-5, 1e-3)])
def test_reorth_batch_matches_truth_and_plain(ro, prec, eps, bar):
    # uneven pairs with refill (more pairs than columns) and s == t entries
    g = I.chung_lu(4000, 2.3, 8.0, seed=61)
    s, t = I.uniform_pairs(g.n, 90, seed=62)
    t[11] = s[11]
    mask = s != t
    truth = np.zeros(len(s))
    truth[mask] = D.rd_all(g, s[mask], t[mask])
    G = rd.RDGraph(g.n, g.u, g.v)
    out = G.query_batch(s, t, eps, _opts(precision=prec, block_width=32, reorth=ro))
    assert np.all(out["status"] == rd.RD_OK)
    assert out["r"][11] == 0.0
    err = np.abs(out["r"][mask] - truth[mask]) / truth[mask]
    assert err.max() <= bar, err.max()
    if prec == rd.RD_F64:
        o = rd.rd_default_options(reorth=ro, flags=rd.RD_GENERAL_PATH)
        for p in range(0, 90, 13):
            if s[p] == t[p]:
                continue
            single = G.query(int(s[p]), int(t[p]), eps, o)
            assert abs(single.iters - out["iters"][p]) <= 1
            assert single.r == pytest.approx(out["r"][p], rel=1e-9)


def test_reorth_gradient_matches_dense():
    g = I.random_connected(700, extra=4000, seed=63, weighted=True)
    s, t = I.uniform_pairs(g.n, 40, seed=64)
    ref = D.grad_edges(g, D.pinv(D.laplacian(g)), s, t)
    G = rd.RDGraph(g.n, g.u, g.v, g.w)
    fwd, gw = G.grad_edges(s, t, None, 1e-12, _opts(block_width=32, reorth=2))
    assert np.linalg.norm(gw - ref) / np.linalg.norm(ref) <= 1e-6


@pytest.mark.parametrize("prec,width,eps,bar", [(rd.RD_F64, 64, 1e-10, 1e-8), (rd.RD_F32, 256, 1e-5, 1e-3)])
def test_tail_compaction_matches_fixed_width(prec, width, eps, bar):
    # uneven iteration counts (road-like grid): once the queue is empty the
    # running columns move to narrower blocks, repeatedly down to 16
    g = I.road_like(60, seed=9)
    s, t = I.uniform_pairs(g.n, width + 40, seed=71)
    t[3] = s[3]
    mask = s != t
    truth = np.zeros(len(s))
    truth[mask] = D.rd_all(g, s[mask], t[mask])
    G = rd.RDGraph(g.n, g.u, g.v)
    flags = rd.RD_GENERAL_PATH | rd.RD_PROFILE
    G.kernel_stats(0)
    comp = G.query_batch(s, t, eps, rd.rd_default_options(precision=prec, block_width=width, flags=flags))
    _, n_c, bytes_c = G.kernel_stats(0)
    fixed = G.query_batch(s, t, eps, rd.rd_default_options(precision=prec, block_width=width,
                                                           flags=flags | rd.RD_NO_COMPACT))
    _, n_f, bytes_f = G.kernel_stats(0)
    assert np.all(comp["status"] == rd.RD_OK) and np.all(fixed["status"] == rd.RD_OK)
    assert comp["r"][3] == 0.0
    # narrower launches carry fewer algorithmic bytes: compaction happened
    print(f"mean bytes per launch: {bytes_c:.4g} with compaction, {bytes_f:.4g} without")
    assert bytes_c < bytes_f
    for out in (comp, fixed):
        err = np.abs(out["r"][mask] - truth[mask]) / truth[mask]
        assert err.max() <= bar, err.max()
    assert np.all(np.abs(comp["iters"] - fixed["iters"]) <= 1)
    if prec == rd.RD_F64:
        np.testing.assert_allclose(comp["r"], fixed["r"], rtol=1e-11)


def test_batched_runs_are_bitwise_repeatable():
    # refill, tail compaction, degree order and the gradient harvest all hand
    # out pairs and slots in a fixed order and sum partials in a fixed order
    g = I.road_like(50, seed=11)
    s, t = I.uniform_pairs(g.n, 90, seed=12)
    G = rd.RDGraph(g.n, g.u, g.v, reorder=True)
    o = _opts(precision=rd.RD_F32, block_width=32)
    a = G.query_batch(s, t, 1e-5, o)
    b = G.query_batch(s, t, 1e-5, o)
    assert a.tobytes() == b.tobytes()
    w = np.linspace(0.5, 2.0, g.m)
    Gw = rd.RDGraph(g.n, g.u, g.v, w)
    f1, g1 = Gw.grad_edges(s, t, None, 1e-6, _opts(block_width=16))
    f2, g2 = Gw.grad_edges(s, t, None, 1e-6, _opts(block_width=16))
    assert f1.tobytes() == f2.tobytes() and g1.tobytes() == g2.tobytes()
