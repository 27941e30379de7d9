"""Seeded synthetic inputs: graphs and (s, t) query pairs.

This module builds graphs and draws query pairs only; it holds none of the
resistance-distance arithmetic. Both the CPU oracle and the GPU path take their
inputs from here.

Large graphs come from the compiled generator ``graphgen.cpp`` (counter-based
random numbers, so results do not depend on the thread count); the small
closed-form families are plain numpy.

Every graph is returned as ``Graph(n, u, v, w)`` with int32 canonical edges
``u < v`` (one record per undirected edge) and ``w`` either ``None`` (unit
weights) or a float array aligned with the edges.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_graphgen.so")
_lib = None


@dataclass
class Graph:
    n: int
    u: np.ndarray  # int32 [m]
    v: np.ndarray  # int32 [m]
    w: Optional[np.ndarray] = None  # float32/float64 [m] or None for unit weights
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.u.shape[0])

    def degrees(self) -> np.ndarray:
        """Unweighted degree (neighbour count) of every node."""
        return np.bincount(self.u, minlength=self.n) + np.bincount(self.v, minlength=self.n)


def build_graphgen(verbose: bool = False) -> str:
    """Compile graphgen.cpp into _graphgen.so (g++, OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "graphgen.cpp")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"graph generator library missing: {_LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(vp)]
    lib.gg_road_like.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                 ctypes.c_uint64, ctypes.POINTER(vp)]
    lib.gg_chung_lu.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                ctypes.POINTER(vp)]
    lib.gg_lognormal.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, vp]
    for f in (lib.gg_grid, lib.gg_road_like, lib.gg_chung_lu, lib.gg_lognormal):
        f.restype = ctypes.c_int
    lib.gg_num_nodes.argtypes = [vp]
    lib.gg_num_nodes.restype = ctypes.c_int64
    lib.gg_num_edges.argtypes = [vp]
    lib.gg_num_edges.restype = ctypes.c_int64
    lib.gg_copy_edges.argtypes = [vp, vp, vp]
    lib.gg_copy_edges.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_free.restype = None
    _lib = lib
    return lib


def _take(h: ctypes.c_void_p, name: str) -> Graph:
    lib = _load()
    try:
        n = int(lib.gg_num_nodes(h))
        m = int(lib.gg_num_edges(h))
        u = np.empty(m, dtype=np.int32)
        v = np.empty(m, dtype=np.int32)
        lib.gg_copy_edges(h, u.ctypes.data, v.ctypes.data)
    finally:
        lib.gg_free(h)
    return Graph(n, u, v, None, name)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"{what}: generator returned {rc}")


def grid(nx: int, ny: int) -> Graph:
    """nx-by-ny four-neighbour grid, node id y*nx + x, unit weights."""
    h = ctypes.c_void_p()
    _check(_load().gg_grid(nx, ny, ctypes.byref(h)), "grid")
    return _take(h, f"grid_{nx}x{ny}")


def road_like(N: int, p_del: float = 0.15, frac_short: float = 0.01, max_len: int = 5,
              seed: int = 3) -> Graph:
    """N x N grid with i.i.d. edge deletions and short random shortcuts (LCC)."""
    h = ctypes.c_void_p()
    _check(_load().gg_road_like(N, p_del, frac_short, max_len, seed, ctypes.byref(h)), "road_like")
    return _take(h, f"road_like_{N}x{N}")


def chung_lu(n: int, gamma: float, mean_deg: float, seed: int) -> Graph:
    """Chung-Lu power-law graph (largest connected component, unit weights)."""
    h = ctypes.c_void_p()
    _check(_load().gg_chung_lu(n, gamma, mean_deg, seed, ctypes.byref(h)), "chung_lu")
    return _take(h, f"chung_lu_n{n}_g{gamma}_d{mean_deg}")


def lognormal_weights(m: int, mu: float = 0.0, sigma: float = 1.0, seed: int = 5) -> np.ndarray:
    out = np.empty(m, dtype=np.float32)
    _check(_load().gg_lognormal(m, mu, sigma, seed, out.ctypes.data), "lognormal")
    return out


# ----------------------------------------------------------------------------
# Small closed-form families (numpy)
# ----------------------------------------------------------------------------

def _canon(n, pairs, w=None, name="") -> Graph:
    a = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    u = np.minimum(a[:, 0], a[:, 1])
    v = np.maximum(a[:, 0], a[:, 1])
    order = np.lexsort((v, u))
    ww = None if w is None else np.asarray(w, dtype=np.float64)[order]
    return Graph(n, u[order].astype(np.int32), v[order].astype(np.int32), ww, name)


def path(n: int, w=None) -> Graph:
    return _canon(n, [(i, i + 1) for i in range(n - 1)], w, f"path_{n}")


def cycle(n: int) -> Graph:
    return _canon(n, [(i, (i + 1) % n) for i in range(n)], None, f"cycle_{n}")


def complete(n: int) -> Graph:
    return _canon(n, [(i, j) for i in range(n) for j in range(i + 1, n)], None, f"complete_{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    """K_{a,b}: nodes 0..a-1 on one side, a..a+b-1 on the other."""
    return _canon(a + b, [(i, a + j) for i in range(a) for j in range(b)], None, f"K_{a}_{b}")


def star(n: int) -> Graph:
    return _canon(n, [(0, i) for i in range(1, n)], None, f"star_{n}")


def random_tree(n: int, seed: int, weighted: bool = False) -> Graph:
    """Random recursive tree: node i attaches to a uniform earlier node."""
    rng = np.random.default_rng(seed)
    pairs = [(int(rng.integers(0, i)), i) for i in range(1, n)]
    w = rng.uniform(0.5, 2.0, size=n - 1) if weighted else None
    return _canon(n, pairs, w, f"tree_{n}")


def random_connected(n: int, extra: int, seed: int, weighted: bool = False) -> Graph:
    """A random tree plus `extra` random non-duplicate chords."""
    rng = np.random.default_rng(seed)
    edges = {(int(rng.integers(0, i)), i) for i in range(1, n)}
    edges = {(min(a, b), max(a, b)) for a, b in edges}
    tries = 0
    while len(edges) < n - 1 + extra and tries < 100 * (extra + 1):
        a, b = (int(x) for x in rng.integers(0, n, size=2))
        tries += 1
        if a != b:
            edges.add((min(a, b), max(a, b)))
    pairs = sorted(edges)
    w = rng.uniform(0.25, 4.0, size=len(pairs)) if weighted else None
    return _canon(n, pairs, w, f"rand_{n}_{extra}")


def random_regular3(n: int, rng: np.random.Generator) -> list:
    """Simple connected 3-regular graph on n (even) nodes by the configuration
    model with rejection of loops / multi-edges / disconnected samples."""
    assert n % 2 == 0 and n >= 4
    for _ in range(10000):
        stubs = np.repeat(np.arange(n), 3)
        rng.shuffle(stubs)
        pr = stubs.reshape(-1, 2)
        if np.any(pr[:, 0] == pr[:, 1]):
            continue
        canon = {(int(min(a, b)), int(max(a, b))) for a, b in pr}
        if len(canon) != len(pr):
            continue
        # connectivity
        adj = [[] for _ in range(n)]
        for a, b in canon:
            adj[a].append(b)
            adj[b].append(a)
        seen = {0}
        stack = [0]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y not in seen:
                    seen.add(y)
                    stack.append(y)
        if len(seen) == n:
            return sorted(canon)
    raise RuntimeError("could not sample a simple connected 3-regular graph")


def bridged_expanders(half: int, seed: int) -> tuple:
    """Two random 3-regular graphs on `half` nodes each, joined by one edge
    between node 0 of the first and node 0 of the second (ids 0 and half).
    The joining edge is a bridge, so r(0, half) = 1. Returns (Graph, s, t)."""
    rng = np.random.default_rng(seed)
    e1 = random_regular3(half, rng)
    e2 = [(a + half, b + half) for a, b in random_regular3(half, rng)]
    pairs = e1 + e2 + [(0, half)]
    return _canon(2 * half, pairs, None, f"bridged_expanders_{half}"), 0, half


def paper_toy_graph() -> Graph:
    """The four-node example graph of the paper's Section 4 worked example:
    V = {1,2,3,4}, E = {(1,2),(1,3),(1,4),(2,3)}, relabelled to 0..3."""
    return _canon(4, [(0, 1), (0, 2), (0, 3), (1, 2)], None, "paper_toy")


# ----------------------------------------------------------------------------
# Query pairs
# ----------------------------------------------------------------------------

def uniform_pairs(n: int, count: int, seed: int) -> tuple:
    """`count` pairs with s, t uniform over [0, n), s != t (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, size=count)
    t = rng.integers(0, n, size=count)
    bad = s == t
    while np.any(bad):
        t[bad] = rng.integers(0, n, size=int(bad.sum()))
        bad = s == t
    return s.astype(np.int32), t.astype(np.int32)


def hub_pairs(g: Graph, count: int, seed: int, top_frac: float = 0.01) -> tuple:
    """`count` pairs with s uniform over the top ceil(top_frac n) nodes by
    degree (ties broken by smaller id) and t uniform over all nodes, s != t."""
    deg = g.degrees()
    k = int(np.ceil(top_frac * g.n))
    order = np.lexsort((np.arange(g.n), -deg))
    top = order[:k]
    rng = np.random.default_rng(seed)
    s = top[rng.integers(0, k, size=count)]
    t = rng.integers(0, g.n, size=count)
    bad = s == t
    while np.any(bad):
        t[bad] = rng.integers(0, g.n, size=int(bad.sum()))
        bad = s == t
    return s.astype(np.int32), t.astype(np.int32)
