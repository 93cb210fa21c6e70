"""Batch updates of the graph container -- TEST INFRASTRUCTURE ONLY.

Plain numpy statement of what a dynamic container computes when it applies a
batch of edge insertions or deletions (Section 4, the batch-update interface),
for the test suite to check a device implementation against. It shares no code
with the product library.

Readings (the paper leaves these open):
- An update batch is a list of vertex pairs. Each pair (u, v) with u != v
  names the undirected edge {u, v}, so both directions change together, and
  the result stays symmetric and simple, like the static container. Pairs
  with u == v change nothing, and repeated pairs act once (set semantics).
- The vertex count is fixed; a pair naming a vertex outside [0, n) is an error.
- The three batch forms of the paper: a global sort, in ascending (source,
  target) order; a semisort, which only puts equal sources next to each other;
  and a semisort whose groups are each sorted by target. A semisort has many
  correct results, so the last two are given as validity checks.
"""
from __future__ import annotations

import numpy as np

from . import Graph


def _pairs(n: int, src, dst):
    src = np.asarray(src, np.int64).ravel()
    dst = np.asarray(dst, np.int64).ravel()
    if src.shape != dst.shape:
        raise ValueError("source and target lists differ in length")
    if src.size and (min(src.min(), dst.min()) < 0 or max(src.max(), dst.max()) >= n):
        raise ValueError("batch names a vertex outside [0, n)")
    return src, dst


def edge_keys(g: Graph) -> np.ndarray:
    """Every directed edge of g as the key u * n + v, ascending."""
    off, nbr = g.export()
    u = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(off))
    return np.sort(u * g.n + nbr.astype(np.int64))


def _batch_keys(n: int, src, dst) -> np.ndarray:
    """The batch's undirected edges, both directions, as keys u * n + v."""
    src, dst = _pairs(n, src, dst)
    keep = src != dst
    s, d = src[keep], dst[keep]
    return np.unique(np.concatenate([s * n + d, d * n + s]))


def _from_keys(n: int, keys: np.ndarray) -> Graph:
    return Graph(n, (keys // max(n, 1)).astype(np.int32), (keys % max(n, 1)).astype(np.int32))


def insert_batch(g: Graph, src, dst) -> Graph:
    """The graph whose edge set is that of g together with the batch's edges."""
    return _from_keys(g.n, np.union1d(edge_keys(g), _batch_keys(g.n, src, dst)))


def delete_batch(g: Graph, src, dst) -> Graph:
    """The graph whose edge set is that of g without the batch's edges."""
    return _from_keys(g.n, np.setdiff1d(edge_keys(g), _batch_keys(g.n, src, dst)))


def sort_batch(src, dst):
    """The global sort: the pairs in ascending (source, target) order. Equal
    pairs are interchangeable, so the result is unique."""
    src = np.asarray(src, np.int64).ravel()
    dst = np.asarray(dst, np.int64).ravel()
    order = np.lexsort((dst, src))
    return src[order], dst[order]


def _same_multiset(src_in, dst_in, src_out, dst_out) -> bool:
    a = sort_batch(src_in, dst_in)
    b = sort_batch(src_out, dst_out)
    return a[0].shape == b[0].shape and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def is_semisorted(src_in, dst_in, src_out, dst_out) -> bool:
    """True when the output holds the input's pairs, each as often, with all
    pairs of one source next to each other (in any order of sources)."""
    if not _same_multiset(src_in, dst_in, src_out, dst_out):
        return False
    s = np.asarray(src_out, np.int64).ravel()
    if s.size == 0:
        return True
    starts = np.concatenate([[True], s[1:] != s[:-1]])
    return np.unique(s[starts]).size == int(starts.sum())   # each source opens exactly one run


def is_grouped_sorted(src_in, dst_in, src_out, dst_out) -> bool:
    """A semisort in which each source's group is in ascending target order."""
    if not is_semisorted(src_in, dst_in, src_out, dst_out):
        return False
    s = np.asarray(src_out, np.int64).ravel()
    d = np.asarray(dst_out, np.int64).ravel()
    same = s[1:] == s[:-1]
    return bool(np.all(d[1:][same] >= d[:-1][same]))
