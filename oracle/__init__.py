"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded reference for what the GPU traversal path computes:
BFS, min-ID connected components, FP64 PageRank, multi-source BFS,
single-source betweenness, k-core, greedy MIS and colouring, the approximate
densest subgraph, low-diameter decomposition, the selector MLP (``mlp.py``)
and batch edge updates (``updates.py``). Only the test suite, the smoke check
and the benchmark's CPU baseline leg may import this package. It shares no
code with the product library: ``oracle.c`` is compiled on its own by gcc,
and ``mlp.py`` and ``updates.py`` are numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c (plain C, -O2, no OpenMP: the oracle is single-threaded)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_graph_new.argtypes = [i64, i64, i32p, i32p]
        lib.oracle_graph_new.restype = vp
        lib.oracle_graph_free.argtypes = [vp]
        lib.oracle_graph_free.restype = None
        lib.oracle_num_vertices.argtypes = [vp]
        lib.oracle_num_vertices.restype = i64
        lib.oracle_num_edges.argtypes = [vp]
        lib.oracle_num_edges.restype = i64
        lib.oracle_degree.argtypes = [vp, i64]
        lib.oracle_degree.restype = i64
        lib.oracle_neighbors.argtypes = [vp, i64, i32p, i64]
        lib.oracle_neighbors.restype = i64
        lib.oracle_export.argtypes = [vp, i64p, i32p]
        lib.oracle_export.restype = None
        lib.oracle_bfs.argtypes = [vp, i64, i32p, i32p]
        lib.oracle_bfs.restype = ctypes.c_int
        lib.oracle_cc.argtypes = [vp, i32p]
        lib.oracle_cc.restype = ctypes.c_int
        lib.oracle_pagerank.argtypes = [vp, ctypes.c_double, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_double)]
        lib.oracle_pagerank.restype = ctypes.c_int
        lib.oracle_msbfs.argtypes = [vp, i64p, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_msbfs.restype = ctypes.c_int
        dblp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_bc_definition.argtypes = [vp, i64, dblp]
        lib.oracle_bc_definition.restype = ctypes.c_int
        lib.oracle_bc.argtypes = [vp, i64, dblp, dblp, i32p]
        lib.oracle_bc.restype = ctypes.c_int
        lib.oracle_mis.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_mis.restype = ctypes.c_int
        lib.oracle_coloring.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), i32p]
        lib.oracle_coloring.restype = ctypes.c_int
        lib.oracle_densest.argtypes = [vp, ctypes.c_double, i64p, i64p, ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_densest.restype = i64
        lib.oracle_ldd.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32p]
        lib.oracle_ldd.restype = ctypes.c_int
        lib.oracle_ldd_definition.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32p]
        lib.oracle_ldd_definition.restype = ctypes.c_int
        lib.oracle_kcore_definition.argtypes = [vp, i32p]
        lib.oracle_kcore_definition.restype = ctypes.c_int
        lib.oracle_kcore.argtypes = [vp, i32p]
        lib.oracle_kcore.restype = ctypes.c_int
        lib.oracle_check_bfs.argtypes = [vp, i64, i32p, i32p]
        lib.oracle_check_bfs.restype = i64
        _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class Graph:
    """Neighbour-set graph built from raw pairs (symmetrised, simple)."""

    def __init__(self, n: int, src: np.ndarray, dst: np.ndarray):
        lib = _load()
        src = np.ascontiguousarray(src, np.int32)
        dst = np.ascontiguousarray(dst, np.int32)
        self._h = lib.oracle_graph_new(int(n), int(src.shape[0]), _p(src, ctypes.c_int32),
                                       _p(dst, ctypes.c_int32))
        if not self._h:
            raise ValueError("oracle graph build failed (vertex out of range or no memory)")
        self.n = int(lib.oracle_num_vertices(self._h))
        self.m = int(lib.oracle_num_edges(self._h))

    @classmethod
    def from_pairs(cls, pairs):
        return cls(pairs.n, pairs.src, pairs.dst)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().oracle_graph_free(h)
            self._h = None

    def degree(self, v: int) -> int:
        return int(_load().oracle_degree(self._h, v))

    def neighbors(self, v: int) -> np.ndarray:
        d = self.degree(v)
        out = np.empty(max(d, 1), np.int32)
        _load().oracle_neighbors(self._h, v, _p(out, ctypes.c_int32), d)
        return out[:d]

    def export(self):
        off = np.empty(self.n + 1, np.int64)
        nbr = np.empty(max(self.m, 1), np.int32)
        _load().oracle_export(self._h, _p(off, ctypes.c_int64), _p(nbr, ctypes.c_int32))
        return off, nbr[: self.m]

    def degrees(self) -> np.ndarray:
        off, _ = self.export()
        return np.diff(off)

    def bfs(self, src: int):
        depth = np.empty(self.n, np.int32)
        parent = np.empty(self.n, np.int32)
        rc = _load().oracle_bfs(self._h, int(src), _p(depth, ctypes.c_int32), _p(parent, ctypes.c_int32))
        if rc != 0:
            raise ValueError(f"oracle_bfs failed ({rc})")
        return depth, parent

    def cc(self) -> np.ndarray:
        label = np.empty(self.n, np.int32)
        if _load().oracle_cc(self._h, _p(label, ctypes.c_int32)) != 0:
            raise MemoryError("oracle_cc failed")
        return label

    def pagerank(self, damping: float = 0.85, iters: int = 20) -> np.ndarray:
        rank = np.empty(max(self.n, 1), np.float64)
        if _load().oracle_pagerank(self._h, float(damping), int(iters), _p(rank, ctypes.c_double)) != 0:
            raise ValueError("oracle_pagerank failed")
        return rank[: self.n]

    def msbfs(self, srcs) -> np.ndarray:
        srcs = np.ascontiguousarray(srcs, np.int64)
        k = int(srcs.shape[0])
        depth = np.empty(max(self.n * k, 1), np.uint8)
        rc = _load().oracle_msbfs(self._h, _p(srcs, ctypes.c_int64), k, _p(depth, ctypes.c_uint8))
        if rc != 0:
            raise ValueError(f"oracle_msbfs failed ({rc})")
        return depth[: self.n * k].reshape(self.n, k)

    def bc(self, src: int):
        """Brandes' recurrence: (sigma, delta, dist) from src, FP64."""
        sigma = np.empty(max(self.n, 1), np.float64)
        delta = np.empty(max(self.n, 1), np.float64)
        dist = np.empty(max(self.n, 1), np.int32)
        rc = _load().oracle_bc(self._h, int(src), _p(sigma, ctypes.c_double), _p(delta, ctypes.c_double),
                               _p(dist, ctypes.c_int32))
        if rc != 0:
            raise ValueError(f"oracle_bc failed ({rc})")
        return sigma[: self.n], delta[: self.n], dist[: self.n]

    def bc_definition(self, src: int) -> np.ndarray:
        """The pairwise definition of the dependencies (small graphs only)."""
        delta = np.empty(max(self.n, 1), np.float64)
        if _load().oracle_bc_definition(self._h, int(src), _p(delta, ctypes.c_double)) != 0:
            raise ValueError("oracle_bc_definition failed")
        return delta[: self.n]

    def mis(self, prio) -> np.ndarray:
        """Greedy maximal independent set in (prio, id) order: uint8 membership."""
        prio = np.ascontiguousarray(prio, np.uint64)
        assert prio.shape[0] >= self.n
        out = np.empty(max(self.n, 1), np.uint8)
        if _load().oracle_mis(self._h, _p(prio, ctypes.c_uint64), _p(out, ctypes.c_uint8)) != 0:
            raise MemoryError("oracle_mis failed")
        return out[: self.n]

    def coloring(self, prio) -> np.ndarray:
        """Greedy colouring in (prio, id) order: int32 colours from 0."""
        prio = np.ascontiguousarray(prio, np.uint64)
        assert prio.shape[0] >= self.n
        out = np.empty(max(self.n, 1), np.int32)
        if _load().oracle_coloring(self._h, _p(prio, ctypes.c_uint64), _p(out, ctypes.c_int32)) != 0:
            raise MemoryError("oracle_coloring failed")
        return out[: self.n]

    def densest(self, eps: float = 0.001):
        """Peeling rounds: (best |E(S)|, best |S|, rounds, membership of that S)."""
        be, bv = ctypes.c_int64(), ctypes.c_int64()
        inb = np.empty(max(self.n, 1), np.uint8)
        r = _load().oracle_densest(self._h, float(eps), ctypes.byref(be), ctypes.byref(bv), _p(inb, ctypes.c_uint8))
        if r < 0:
            raise MemoryError("oracle_densest failed")
        return be.value, bv.value, int(r), inb[: self.n]

    def ldd(self, delta, definition: bool = False) -> np.ndarray:
        """Shifted clustering: cluster[v] = argmin_u dist(u, v) - delta[u] (ties: smaller u)."""
        delta = np.ascontiguousarray(delta, np.float64)
        assert delta.shape[0] >= self.n
        out = np.empty(max(self.n, 1), np.int32)
        fn = _load().oracle_ldd_definition if definition else _load().oracle_ldd
        if fn(self._h, _p(delta, ctypes.c_double), _p(out, ctypes.c_int32)) != 0:
            raise MemoryError("oracle_ldd failed")
        return out[: self.n]

    def kcore(self) -> np.ndarray:
        """Coreness of every vertex by bucketed peeling."""
        core = np.empty(max(self.n, 1), np.int32)
        if _load().oracle_kcore(self._h, _p(core, ctypes.c_int32)) != 0:
            raise MemoryError("oracle_kcore failed")
        return core[: self.n]

    def kcore_definition(self) -> np.ndarray:
        """Coreness from the definition (small graphs only)."""
        core = np.empty(max(self.n, 1), np.int32)
        if _load().oracle_kcore_definition(self._h, _p(core, ctypes.c_int32)) != 0:
            raise MemoryError("oracle_kcore_definition failed")
        return core[: self.n]

    def check_bfs(self, src: int, depth: np.ndarray, parent: np.ndarray) -> int:
        depth = np.ascontiguousarray(depth, np.int32)
        parent = np.ascontiguousarray(parent, np.int32)
        return int(_load().oracle_check_bfs(self._h, int(src), _p(depth, ctypes.c_int32),
                                            _p(parent, ctypes.c_int32)))
