"""Seeded synthetic graph inputs (raw vertex pairs), shared by the HIP path and the oracle.

Nothing here performs traversal arithmetic: the functions only draw pairs and
sources. Shapes follow the paper's synthetic datasets (Section 6.2): uniform
Erdos-Renyi pairs, Graph500-style RMAT/Kronecker sampling with (a, b, c, d), and
a road-like lattice with random edge deletions. The sampler is the C file
``gen.c`` (SplitMix64 in counter mode), built with gcc and loaded through ctypes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libbyogen.so")
_lib = None

STREAM_PARAMS = 6
GRAPH500_ABCD = (0.57, 0.19, 0.19, 0.05)


def build(force: bool = True) -> str:
    """Compile gen.c into libbyogen.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u64, i64, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
        lib.byogen_draw.argtypes = [u64, u64, u64]
        lib.byogen_draw.restype = u64
        lib.byogen_unit.argtypes = [u64, u64, u64]
        lib.byogen_unit.restype = dbl
        lib.byogen_er.argtypes = [u64, i64, i64, i32p, i32p]
        lib.byogen_er.restype = ctypes.c_int
        lib.byogen_rmat.argtypes = [u64, ctypes.c_int, i64, dbl, dbl, dbl, ctypes.c_int, i32p, i32p]
        lib.byogen_rmat.restype = ctypes.c_int
        lib.byogen_grid_edges.argtypes = [i64, i64]
        lib.byogen_grid_edges.restype = i64
        lib.byogen_grid.argtypes = [u64, i64, i64, i64, i32p, i32p]
        lib.byogen_grid.restype = i64
        lib.byogen_pick_sources.argtypes = [u64, i64, i64, i32p, i32p, i64, i64p]
        lib.byogen_pick_sources.restype = i64
        _lib = lib
    return _lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


@dataclass
class Pairs:
    """Raw undirected pair sample: n vertices and (src[i], dst[i]) draws.

    Pairs may repeat and may be self-loops; consumers symmetrise, drop
    self-loops and deduplicate.
    """
    n: int
    src: np.ndarray
    dst: np.ndarray
    name: str = ""

    @property
    def npairs(self) -> int:
        return int(self.src.shape[0])


def draw(seed: int, stream: int, i: int) -> int:
    return int(_load().byogen_draw(seed, stream, i))


def unit(seed: int, stream: int, i: int) -> float:
    return float(_load().byogen_unit(seed, stream, i))


def er_pairs(n: int, avg_degree: float, seed: int = 1) -> Pairs:
    """Erdos-Renyi: round(n * avg_degree / 2) uniform pairs over [0, n)."""
    npairs = int(round(n * avg_degree / 2.0))
    src = np.empty(npairs, np.int32)
    dst = np.empty(npairs, np.int32)
    if _load().byogen_er(seed, n, npairs, _p32(src), _p32(dst)) != 0:
        raise ValueError("bad ER parameters")
    return Pairs(n, src, dst, f"er-n{n}-d{avg_degree:g}-s{seed}")


def rmat_pairs(scale: int, edge_factor: int = 16, abcd=GRAPH500_ABCD, seed: int = 1,
               permute: bool = True) -> Pairs:
    """RMAT/Kronecker: edge_factor * 2^scale sampled pairs over 2^scale vertices."""
    a, b, c, d = abcd
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("RMAT probabilities must sum to 1")
    n = 1 << scale
    npairs = edge_factor * n
    src = np.empty(npairs, np.int32)
    dst = np.empty(npairs, np.int32)
    if _load().byogen_rmat(seed, scale, npairs, a, b, c, int(permute), _p32(src), _p32(dst)) != 0:
        raise ValueError("bad RMAT parameters")
    return Pairs(n, src, dst, f"rmat-s{scale}-ef{edge_factor}-s{seed}")


def grid_pairs(rows: int, cols: int, delete_frac: float = 0.1, seed: int = 1) -> Pairs:
    """rows x cols 4-neighbour lattice with floor(delete_frac * E) edges removed."""
    lib = _load()
    E = int(lib.byogen_grid_edges(rows, cols))
    ndel = int(math.floor(delete_frac * E + 1e-9))
    src = np.empty(max(E - ndel, 0), np.int32)
    dst = np.empty(max(E - ndel, 0), np.int32)
    w = lib.byogen_grid(seed, rows, cols, ndel, _p32(src), _p32(dst))
    if w != E - ndel:
        raise ValueError("grid generation failed")
    return Pairs(rows * cols, src, dst, f"grid-{rows}x{cols}-del{delete_frac:g}-s{seed}")


def grid_edge_count(rows: int, cols: int) -> int:
    return int(_load().byogen_grid_edges(rows, cols))


def pick_sources(p: Pairs, k: int, seed: int = 2) -> np.ndarray:
    """k distinct uniformly drawn non-isolated vertices (fewer if not enough exist)."""
    out = np.empty(max(k, 1), np.int64)
    got = _load().byogen_pick_sources(seed, p.n, p.npairs, _p32(p.src), _p32(p.dst), k, _p64(out))
    if got < 0:
        raise MemoryError("source picker failed")
    return out[:got].copy()


def batch_specs(count: int = 64, seed: int = 3, log2_lo: float = 10.0, log2_hi: float = 18.0,
                deg_lo: float = 4.0, deg_hi: float = 32.0):
    """(n, avg_degree, graph_seed) per graph: n log-uniform on [2^lo, 2^hi], degree uniform."""
    specs = []
    for g in range(count):
        un = unit(seed, STREAM_PARAMS, 3 * g)
        ud = unit(seed, STREAM_PARAMS, 3 * g + 1)
        n = int(round(2.0 ** (log2_lo + (log2_hi - log2_lo) * un)))
        d = deg_lo + (deg_hi - deg_lo) * ud
        specs.append((n, d, int(draw(seed, STREAM_PARAMS, 3 * g + 2) & 0x7FFFFFFF)))
    return specs


def batch_pairs(count: int = 64, seed: int = 3, **kw):
    return [er_pairs(n, d, s) for (n, d, s) in batch_specs(count, seed, **kw)]
