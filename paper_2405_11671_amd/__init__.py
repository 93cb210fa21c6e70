"""MI355X (gfx950) edgeMap traversal library: Python binding.

Thin wrapper over the C ABI (include/byo.h): it converts arguments, allocates
outputs as torch tensors on the current HIP device and passes the current
stream. All traversal work runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (FORM_GROUPED_SORT, FORM_SEMISORT, FORM_SORT, API_CONFIGS, API_NO_DEGREE, API_NO_EARLY_EXIT, API_NO_NUM_EDGES, API_NO_PAR_EARLY_EXIT,
                   API_NO_PAR_MAP, ByoError, F_BFS, F_CC_MIN, F_PR_ACC, NUM_VARIANTS, SEL_FIXED, SEL_HEURISTIC, SEL_MLP,
                   V_PULL_THREAD, V_PULL_WAVE, V_PUSH_BUCKET, V_PUSH_EDGE, V_PUSH_THREAD, V_PUSH_WAVE, VARIANTS,
                   default_opts)

__all__ = ["Graph", "VSet", "bfs", "bfs_noalloc", "batch_order", "cc", "pagerank", "edge_map", "csr_from_pairs", "default_opts", "ByoError",
           "VARIANTS", "NUM_VARIANTS", "API_CONFIGS"]


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, need: int = 0, size: int | None = None):
    """Device pointer of a tensor the library will read or write, checked
    first: a host tensor, a non-contiguous view, a wrong element size or fewer
    than `need` elements raise ValueError here instead of reaching a kernel."""
    if not getattr(t, "is_cuda", False):
        raise ValueError("buffers passed to the library must be device (cuda) tensors")
    if not t.is_contiguous():
        raise ValueError("buffers passed to the library must be contiguous")
    if size is not None and t.element_size() != size:
        raise ValueError(f"buffer elements of {t.element_size()} bytes where {size} are needed")
    if t.numel() < need:
        raise ValueError(f"buffer of {t.numel()} elements where {need} are needed")
    return ctypes.c_void_p(t.data_ptr())


def csr_from_pairs(n: int, src: np.ndarray, dst: np.ndarray):
    """Host CSR (int64 offsets, int32 sorted unique neighbours) from raw pairs."""
    lib = _lib.load()
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    off = np.empty(n + 1, np.int64)
    nbr = np.empty(max(2 * src.shape[0], 1), np.int32)
    m = ctypes.c_int64(0)
    _lib.check(lib.byo_csr_from_pairs(src.ctypes.data, dst.ctypes.data, src.shape[0], n, off.ctypes.data,
                                      nbr.ctypes.data, ctypes.byref(m)))
    return off, nbr[: m.value]


class Graph:
    """CSR GraphContainer on the current device (num_vertices, num_edges, degree, map_neighbors)."""

    def __init__(self, handle, n, m, keep=None):
        self._h = handle
        self.n = n
        self.m = m
        self._keep = keep

    @classmethod
    def from_csr(cls, off: np.ndarray, nbr: np.ndarray, validate: bool = False):
        lib = _lib.load()
        off = np.ascontiguousarray(off, np.int64)
        nbr = np.ascontiguousarray(nbr, np.int32)
        n = off.shape[0] - 1
        m = int(off[-1]) if n >= 0 else 0
        h = ctypes.c_void_p()
        flags = _lib.HOST_INPUT | (_lib.VALIDATE if validate else 0)
        _lib.check(lib.byo_graph_from_csr(off.ctypes.data, nbr.ctypes.data if nbr.size else None, n, m, flags,
                                          _stream(), ctypes.byref(h)))
        return cls(h, n, m)

    @classmethod
    def from_device_csr(cls, off_t, nbr_t, borrow: bool = True, validate: bool = False):
        lib = _lib.load()
        n = off_t.shape[0] - 1
        m = nbr_t.shape[0]
        h = ctypes.c_void_p()
        flags = (_lib.DEVICE_BORROW if borrow else _lib.DEVICE_COPY) | (_lib.VALIDATE if validate else 0)
        _lib.check(lib.byo_graph_from_csr(_ptr(off_t), _ptr(nbr_t), n, m, flags, _stream(), ctypes.byref(h)))
        return cls(h, n, m, keep=(off_t, nbr_t) if borrow else None)

    @classmethod
    def from_pairs(cls, pairs, validate: bool = False):
        off, nbr = csr_from_pairs(pairs.n, pairs.src, pairs.dst)
        g = cls.from_csr(off, nbr, validate=validate)
        return g

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().byo_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def num_vertices(self) -> int:
        return int(_lib.load().byo_num_vertices(self._h))

    def num_edges(self) -> int:
        return int(_lib.load().byo_num_edges(self._h))

    def degree(self, v: int) -> int:
        out = ctypes.c_int64()
        _lib.check(_lib.load().byo_degree(self._h, v, ctypes.byref(out)))
        return out.value

    def neighbors(self, v: int) -> np.ndarray:
        cnt = ctypes.c_int64()
        d = self.degree(v)
        buf = np.empty(max(d, 1), np.int32)
        _lib.check(_lib.load().byo_get_neighbors(self._h, v, buf.ctypes.data, d, ctypes.byref(cnt)))
        return buf[: cnt.value]

    def stats(self):
        mx, iso = ctypes.c_int64(), ctypes.c_int64()
        mean, cv = ctypes.c_double(), ctypes.c_double()
        _lib.check(_lib.load().byo_graph_stats(self._h, ctypes.byref(mx), ctypes.byref(iso), ctypes.byref(mean),
                                               ctypes.byref(cv)))
        return {"max_degree": mx.value, "isolated": iso.value, "mean_degree": mean.value, "cv_degree": cv.value}

    def cz_build(self):
        """Build the byte-coded lists (once per graph)."""
        _lib.check(_lib.load().byo_cz_build(self._h, _stream()))

    def cz_arrays(self):
        """(offsets int64[n+1], stream uint8[bytes]) of the byte-coded lists, on the host."""
        lib = _lib.load()
        self.cz_build()
        nb = ctypes.c_int64()
        _lib.check(lib.byo_cz_bytes(self._h, ctypes.byref(nb)))
        off = np.empty(self.n + 1, np.int64)
        data = np.empty(max(nb.value, 1), np.uint8)
        _lib.check(lib.byo_cz_copy(self._h, off.ctypes.data, data.ctypes.data))
        return off, data[: nb.value]

    def cz_decode(self, v: int):
        """v's neighbours decoded from the byte-coded lists on the device (int32 tensor)."""
        torch = _torch()
        out = torch.empty(max(self.degree(v), 1), dtype=torch.int32, device="cuda")
        _lib.check(_lib.load().byo_cz_decode(self._h, int(v), _ptr(out), _stream()))
        return out[: self.degree(v)]

    def csr(self):
        """Host copies (off int64[n+1], nbr int32[m]) of the current CSR."""
        m = self.num_edges()
        off = np.empty(self.n + 1, np.int64)
        nbr = np.empty(max(m, 1), np.int32)
        _lib.check(_lib.load().byo_graph_copy(self._h, off.ctypes.data, nbr.ctypes.data))
        return off, nbr[:m]

    def _update(self, fn, src, dst):
        k = int(src.numel())
        if int(dst.numel()) != k:
            raise ValueError("source and target batches differ in length")
        changed = ctypes.c_int64()
        _lib.check(fn(self._h, _ptr(src, k, 4) if k else None, _ptr(dst, k, 4) if k else None, k, _stream(),
                      ctypes.byref(changed)))
        self.m = self.num_edges()
        return changed.value

    def insert_batch(self, src, dst) -> int:
        """Insert the undirected edges {src[i], dst[i]} (int32 device tensors);
        returns the number of directed entries added."""
        return self._update(_lib.load().byo_graph_insert_batch, src, dst)

    def delete_batch(self, src, dst) -> int:
        """Delete the undirected edges {src[i], dst[i]}; returns the number of
        directed entries removed."""
        return self._update(_lib.load().byo_graph_delete_batch, src, dst)

    def device_arrays(self):
        """(off, nbr, deg) device pointers as ints."""
        o, nb, d = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _lib.check(_lib.load().byo_graph_arrays(self._h, ctypes.byref(o), ctypes.byref(nb), ctypes.byref(d)))
        return o.value, nb.value, d.value


class VSet:
    """vertexSubset over a graph: sparse ID list and/or dense bitmap on the device."""

    def __init__(self, g: Graph):
        self.g = g
        h = ctypes.c_void_p()
        _lib.check(_lib.load().byo_vset_create(g.handle, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                _lib.load().byo_vset_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def set_ids(self, ids_t):
        _lib.check(_lib.load().byo_vset_from_ids(self._h, _ptr(ids_t) if ids_t.numel() else None, ids_t.numel(),
                                                 _stream()))
        return self

    def set_bitmap(self, bits_t):
        _lib.check(_lib.load().byo_vset_from_bitmap(self._h, _ptr(bits_t, (self.g.n + 63) // 64, 8), _stream()))
        return self

    def fill(self):
        _lib.check(_lib.load().byo_vset_fill(self._h, _stream()))
        return self

    def size(self) -> int:
        out = ctypes.c_int64()
        _lib.check(_lib.load().byo_vset_size(self._h, ctypes.byref(out), _stream()))
        return out.value

    def ids(self):
        torch = _torch()
        k = self.size()
        out = torch.empty(max(k, 1), dtype=torch.int32, device="cuda")
        got = ctypes.c_int64()
        _lib.check(_lib.load().byo_vset_to_ids(self._h, _ptr(out), out.numel(), ctypes.byref(got), _stream()))
        return out[: got.value]

    def bitmap(self):
        torch = _torch()
        words = (self.g.n + 63) // 64
        out = torch.empty(max(words, 1), dtype=torch.int64, device="cuda")
        _lib.check(_lib.load().byo_vset_to_bitmap(self._h, _ptr(out), _stream()))
        return out[:words]


def _opts(opts, kw):
    if opts is None:
        opts = default_opts(**kw)
    elif kw:
        for k, v in kw.items():
            setattr(opts, k, int(v))
    return opts


def bfs(g: Graph, src: int, opts=None, depth=None, parent=None, **kw):
    """BFS from src: (depth, parent, stats) as int32 device tensors."""
    torch = _torch()
    o = _opts(opts, kw)
    depth = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") if depth is None else depth
    parent = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") if parent is None else parent
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_bfs(g.handle, int(src), _ptr(depth, g.n, 4), _ptr(parent, g.n, 4), ctypes.byref(o),
                                   _stream(),
                                   ctypes.byref(stt)))
    return depth[: g.n], parent[: g.n], stt.as_dict()


def batch_order(src, dst, n: int, form: int):
    """The batch (int32 device tensors) in one of the three batch forms
    (FORM_SORT, FORM_SEMISORT, FORM_GROUPED_SORT): new (src, dst) tensors."""
    torch = _torch()
    k = int(src.numel())
    out_s = torch.empty(max(k, 1), dtype=torch.int32, device="cuda")
    out_d = torch.empty(max(k, 1), dtype=torch.int32, device="cuda")
    if k:
        _lib.check(_lib.load().byo_batch_order(_ptr(src, k, 4), _ptr(dst, k, 4), k, int(n), int(form), _ptr(out_s),
                                               _ptr(out_d), _stream()))
    return out_s[:k], out_d[:k]


def bfs_noalloc(g: Graph, src: int, depth, parent, opts=None, **kw):
    """BFS that allocates nothing (byo_bfs_noalloc) into caller-owned int32
    device tensors of at least n elements; returns the run statistics."""
    o = _opts(opts, kw)
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_bfs_noalloc(g.handle, int(src), _ptr(depth, g.n, 4), _ptr(parent, g.n, 4),
                                           ctypes.byref(o), _stream(), ctypes.byref(stt)))
    return stt.as_dict()


def cc(g: Graph, opts=None, label=None, **kw):
    """Min-ID component labels (int32 device tensor) and stats."""
    torch = _torch()
    o = _opts(opts, kw)
    label = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") if label is None else label
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_cc(g.handle, _ptr(label, g.n, 4), ctypes.byref(o), _stream(), ctypes.byref(stt)))
    return label[: g.n], stt.as_dict()


def pagerank(g: Graph, damping: float = 0.85, iters: int = 20, opts=None, rank=None, **kw):
    """FP32 PageRank after `iters` steps (float32 device tensor)."""
    torch = _torch()
    o = _opts(opts, kw)
    rank = torch.empty(max(g.n, 1), dtype=torch.float32, device="cuda") if rank is None else rank
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_pagerank(g.handle, float(damping), int(iters), _ptr(rank, g.n, 4), ctypes.byref(o),
                                        _stream(), ctypes.byref(stt)))
    return rank[: g.n], stt.as_dict()


def bc(g: Graph, src: int, opts=None, delta=None, sigma=None, depth=None, **kw):
    """Single-source betweenness from src: (delta, sigma, depth, stats); delta and sigma float64,
    depth int32, device tensors."""
    torch = _torch()
    o = _opts(opts, kw)
    n1 = max(g.n, 1)
    delta = torch.empty(n1, dtype=torch.float64, device="cuda") if delta is None else delta
    sigma = torch.empty(n1, dtype=torch.float64, device="cuda") if sigma is None else sigma
    depth = torch.empty(n1, dtype=torch.int32, device="cuda") if depth is None else depth
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_bc(g.handle, int(src), _ptr(delta, g.n, 8), _ptr(sigma, g.n, 8), _ptr(depth, g.n, 4),
                                  ctypes.byref(o),
                                  _stream(), ctypes.byref(stt)))
    return delta[: g.n], sigma[: g.n], depth[: g.n], stt.as_dict()


def kcore(g: Graph, opts=None, core=None, **kw):
    """Coreness of every vertex (int32 device tensor) and stats."""
    torch = _torch()
    o = _opts(opts, kw)
    core = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") if core is None else core
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_kcore(g.handle, _ptr(core, g.n, 4), ctypes.byref(o), _stream(), ctypes.byref(stt)))
    return core[: g.n], stt.as_dict()


def mis(g: Graph, prio, opts=None, in_set=None, **kw):
    """Greedy maximal independent set in (prio, id) order: (uint8 device tensor, stats).
    prio: uint64 priorities, a device tensor (int64 dtype holding the bits) or a numpy array."""
    torch = _torch()
    o = _opts(opts, kw)
    if isinstance(prio, np.ndarray):
        prio = torch.from_numpy(np.ascontiguousarray(prio, np.uint64).view(np.int64)).to("cuda")
    assert prio.numel() >= g.n and prio.element_size() == 8
    in_set = torch.empty(max(g.n, 1), dtype=torch.uint8, device="cuda") if in_set is None else in_set
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_mis(g.handle, _ptr(prio, g.n, 8), _ptr(in_set, g.n, 1), ctypes.byref(o), _stream(),
                                   ctypes.byref(stt)))
    return in_set[: g.n], stt.as_dict()


def coloring(g: Graph, prio, opts=None, color=None, **kw):
    """Greedy colouring in (prio, id) order: (int32 device tensor, stats). prio as for mis()."""
    torch = _torch()
    o = _opts(opts, kw)
    if isinstance(prio, np.ndarray):
        prio = torch.from_numpy(np.ascontiguousarray(prio, np.uint64).view(np.int64)).to("cuda")
    assert prio.numel() >= g.n and prio.element_size() == 8
    color = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda") if color is None else color
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_coloring(g.handle, _ptr(prio, g.n, 8), _ptr(color, g.n, 4), ctypes.byref(o), _stream(),
                                        ctypes.byref(stt)))
    return color[: g.n], stt.as_dict()


def densest(g: Graph, eps: float = 0.001, opts=None, in_best=None, **kw):
    """Approximate densest subgraph by peeling: (best |E(S)|, best |S|, uint8 membership tensor, stats)."""
    torch = _torch()
    o = _opts(opts, kw)
    in_best = torch.empty(max(g.n, 1), dtype=torch.uint8, device="cuda") if in_best is None else in_best
    be, bv = ctypes.c_int64(), ctypes.c_int64()
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_densest(g.handle, float(eps), _ptr(in_best, g.n, 1), ctypes.byref(be), ctypes.byref(bv),
                                       ctypes.byref(o), _stream(), ctypes.byref(stt)))
    return be.value, bv.value, in_best[: g.n], stt.as_dict()


def edge_map(g: Graph, U: VSet, fn: int, state, out: VSet, variant: int = -1, opts=None, **kw) -> int:
    """edgeMap(G, U, F) into `out`; returns the variant that ran."""
    o = _opts(opts, kw)
    used = ctypes.c_int32(-1)
    _lib.check(_lib.load().byo_edge_map(g.handle, U.handle, int(fn), ctypes.byref(state), out.handle, int(variant),
                                        ctypes.byref(o), _stream(), ctypes.byref(used)))
    return used.value


def bfs_fn_state(parent_t, depth_t, visited_t, level: int):
    return _lib.BfsFn(_ptr(parent_t, 0, 4).value, _ptr(depth_t, 0, 4).value, _ptr(visited_t, 0, 8).value, int(level))


def cc_fn_state(label_t):
    return _lib.CcFn(_ptr(label_t, 0, 4).value)


def pr_fn_state(contrib_t, acc_t):
    return _lib.PrFn(_ptr(contrib_t, 0, 4).value, _ptr(acc_t, 0, 4).value)


def msbfs(g: Graph, srcs, opts=None, depth=None, **kw):
    """Multi-source BFS from up to 256 sources: uint8 depths [n, k] (255 = unreached) and stats."""
    torch = _torch()
    o = _opts(opts, kw)
    srcs = np.ascontiguousarray(np.asarray(srcs, np.int64))
    k = int(srcs.shape[0])
    depth = torch.empty(max(g.n * k, 1), dtype=torch.uint8, device="cuda") if depth is None else depth
    stt = _lib.RunStats()
    _lib.check(_lib.load().byo_msbfs(g.handle, srcs.ctypes.data, k, _ptr(depth, g.n * k, 1), ctypes.byref(o), _stream(),
                                     ctypes.byref(stt)))
    return depth[: g.n * k].view(g.n, k), stt.as_dict()


def trace_enable(on: bool = True):
    _lib.check(_lib.load().byo_trace_enable(1 if on else 0))


def trace_read():
    lib = _lib.load()
    cnt = ctypes.c_int64()
    _lib.check(lib.byo_trace_pending(ctypes.byref(cnt)))
    buf = (_lib.LevelRecord * max(cnt.value, 1))()
    got = ctypes.c_int64()
    _lib.check(lib.byo_trace_read(buf, cnt.value, ctypes.byref(got)))
    return [buf[i].as_dict() for i in range(got.value)]


def ktimer_enable(on: bool = True):
    _lib.check(_lib.load().byo_ktimer_enable(1 if on else 0))


def ktimer_select(families=None):
    """Record only these families (names or ids) while timing is on; None = all."""
    if families is None:
        mask = 0xFFFFFFFF
    else:
        mask = 0
        for f in families:
            mask |= 1 << (_lib.K_FAMILIES.index(f) if isinstance(f, str) else int(f))
    _lib.check(_lib.load().byo_ktimer_select(ctypes.c_uint32(mask)))


def ktimer_reset():
    _lib.check(_lib.load().byo_ktimer_reset())


def ktimer_read(family):
    """(launches, total device ms) for a kernel family name or id."""
    fid = _lib.K_FAMILIES.index(family) if isinstance(family, str) else int(family)
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _lib.check(_lib.load().byo_ktimer_read(fid, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


class Batch:
    """Many graphs traversed together (laid out as one disjoint-union CSR on the device)."""

    def __init__(self, csrs):
        """csrs: list of (off int64[n+1], nbr int32[m]) host arrays."""
        lib = _lib.load()
        self._keep = [(np.ascontiguousarray(o, np.int64), np.ascontiguousarray(nb, np.int32)) for o, nb in csrs]
        cnt = len(self._keep)
        offs = (ctypes.c_void_p * cnt)(*[o.ctypes.data for o, _ in self._keep])
        nbrs = (ctypes.c_void_p * cnt)(*[nb.ctypes.data if nb.size else None for _, nb in self._keep])
        ns = np.array([o.shape[0] - 1 for o, _ in self._keep], np.int64)
        h = ctypes.c_void_p()
        _lib.check(lib.byo_batch_create(cnt, offs, nbrs, ns.ctypes.data, _stream(), ctypes.byref(h)))
        self._h = h
        self.count = cnt
        tn, tm = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(lib.byo_batch_info(h, ctypes.byref(tn), ctypes.byref(tm)))
        self.n, self.m = tn.value, tm.value
        self.voff = []
        for i in range(cnt + 1):
            x = ctypes.c_int64()
            _lib.check(lib.byo_batch_vertex_offset(h, i, ctypes.byref(x)))
            self.voff.append(x.value)

    @classmethod
    def from_pairs(cls, pairs_list):
        return cls([csr_from_pairs(p.n, p.src, p.dst) for p in pairs_list])

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                _lib.load().byo_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def bfs(self, srcs, opts=None, depth=None, parent=None, **kw):
        torch = _torch()
        o = _opts(opts, kw)
        srcs = np.ascontiguousarray(np.asarray(srcs, np.int64))
        depth = torch.empty(self.n, dtype=torch.int32, device="cuda") if depth is None else depth
        parent = torch.empty(self.n, dtype=torch.int32, device="cuda") if parent is None else parent
        stt = _lib.RunStats()
        _lib.check(_lib.load().byo_batch_bfs(self._h, srcs.ctypes.data, _ptr(depth, self.n, 4), _ptr(parent, self.n, 4),
                                             ctypes.byref(o),
                                             _stream(), ctypes.byref(stt)))
        return depth, parent, stt.as_dict()

    def cc(self, opts=None, label=None, **kw):
        torch = _torch()
        o = _opts(opts, kw)
        label = torch.empty(self.n, dtype=torch.int32, device="cuda") if label is None else label
        stt = _lib.RunStats()
        _lib.check(_lib.load().byo_batch_cc(self._h, _ptr(label, self.n, 4), ctypes.byref(o), _stream(),
                                            ctypes.byref(stt)))
        return label, stt.as_dict()

    def split(self, t):
        """Per-graph views of a concatenated result."""
        return [t[self.voff[i]:self.voff[i + 1]] for i in range(self.count)]
