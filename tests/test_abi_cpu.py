"""Host-side checks of the C ABI library and the input generators (no GPU)."""

import os
import re

import numpy as np
import pytest

from paper_2601_11159_amd import inputs as I
from paper_2601_11159_amd import rd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "rd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rd_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = rd.load()
    declared = _declared_symbols()
    assert len(declared) >= 11
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in rd.h but not exported"
    assert sorted(rd.EXPORTED) == declared


def test_header_constants_match_binding():
    txt = open(os.path.join(ROOT, "include", "rd.h")).read()
    defs = dict(re.findall(r"#define (RD_[A-Z0-9_]+) (0x[0-9a-f]+|\d+)u?", txt))
    assert set(defs) >= {"RD_DEVICE_PTRS", "RD_PROFILE", "RD_GENERAL_PATH", "RD_REORDER", "RD_NO_COMPACT",
                         "RD_NO_SPARSE2", "RD_F64", "RD_F32"}
    for name, val in defs.items():
        assert getattr(rd, name) == int(val, 0), name


def test_status_strings_without_gpu():
    assert rd.rd_status_string(rd.RD_OK) == "ok"
    assert "connected" in rd.rd_status_string(rd.RD_E_NOT_CONNECTED)


def test_default_options_layout():
    o = rd.rd_default_options()
    assert o.precision == rd.RD_F64 and o.delay == 8 and o.fixed_k == 0 and o.flags == 0 and o.refine == 0


def test_generators_deterministic_and_simple():
    a = I.chung_lu(20000, 2.1, 20, seed=2)
    b = I.chung_lu(20000, 2.1, 20, seed=2)
    assert a.n == b.n and np.array_equal(a.u, b.u) and np.array_equal(a.v, b.v)
    assert np.all(a.u < a.v)
    key = a.u.astype(np.int64) * a.n + a.v
    assert np.all(np.diff(key) > 0)  # sorted, no duplicates
    c = I.chung_lu(20000, 2.1, 20, seed=3)
    assert not (c.m == a.m and np.array_equal(c.u, a.u))


def test_grid_sizes():
    g = I.grid(64, 64)
    assert g.n == 4096 and g.m == 8064
    d = g.degrees()
    assert set(np.unique(d)) == {2, 3, 4}


def test_road_like_shape():
    g = I.road_like(200, seed=3)
    d = g.degrees()
    assert 0.9 * 200 * 200 < g.n <= 200 * 200
    assert 3.2 < d.mean() < 3.7
    assert np.all(g.u < g.v)


def test_chung_lu_degree_shape():
    g = I.chung_lu(100000, 2.1, 20, seed=2)
    d = g.degrees()
    assert abs(d.mean() - 20) < 1.0
    assert d.max() > 1000  # heavy tail
    assert g.n > 0.98 * 100000


def test_lognormal_weights():
    w = I.lognormal_weights(200000, 0.0, 1.0, seed=5)
    lw = np.log(w.astype(np.float64))
    assert abs(lw.mean()) < 0.01 and abs(lw.std() - 1.0) < 0.01
    assert np.array_equal(w, I.lognormal_weights(200000, 0.0, 1.0, seed=5))


def test_bench_traffic_lookup_hashes_the_kernel_source():
    # the committed counter summary is keyed by workload, schedule and width
    # and is used only while the kernel source is unchanged
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    h = bench.kernel_source_hash()
    assert len(h) == 16
    import json
    d = json.load(open(os.path.join(ROOT, "profiles", "spmm_short_traffic.json")))
    for key, e in d.items():
        workload, width = key.rsplit("/B", 1)
        got = bench.load_traffic(workload, int(width))
        assert (got is not None) == (e["source_hash"] == h)


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: a request for more exits at once with a message, before any GPU use
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)


def test_bench_lists_every_workload_it_runs():
    import importlib.util
    import inspect
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    src = inspect.getsource(bench.run_other)
    for name in bench.OTHER_WORKLOADS:
        assert f'name == "{name}"' in src, name
