"""Brute-force and closed-form checkers used to pin the oracle on tiny graphs.

Independent of both the oracle and the HIP path: dense matrices, Floyd-Warshall,
union-find and library routines (scipy.sparse.csgraph, numpy.linalg).
"""
from __future__ import annotations

import numpy as np


def simple_edges(n, src, dst):
    """Set of undirected edges {u, v}, u != v, as sorted tuples (plain Python)."""
    E = set()
    for u, v in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
        if u != v:
            E.add((min(u, v), max(u, v)))
    return E


def adjacency_matrix(n, src, dst):
    A = np.zeros((n, n), np.int64)
    for u, v in simple_edges(n, src, dst):
        A[u, v] = A[v, u] = 1
    return A


def floyd_warshall_hops(A):
    n = A.shape[0]
    INF = 10 ** 9
    D = np.where(A > 0, 1, INF).astype(np.int64)
    np.fill_diagonal(D, 0)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    D[D >= INF] = -1
    return D


def union_find_min_labels(n, src, dst):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u, v in simple_edges(n, src, dst):
        ru, rv = find(u), find(v)
        if ru != rv:
            parent[max(ru, rv)] = min(ru, rv)
    roots = [find(v) for v in range(n)]
    best = {}
    for v in range(n):
        best.setdefault(roots[v], v)
        best[roots[v]] = min(best[roots[v]], v)
    return np.array([best[roots[v]] for v in range(n)], np.int64)


def pagerank_matrix(A, d):
    """Column-stochastic Google matrix G with p_{t+1} = G p_t (dangling mass spread uniformly)."""
    n = A.shape[0]
    deg = A.sum(axis=0).astype(np.float64)
    M = np.zeros((n, n))
    nz = deg > 0
    M[:, nz] = A[:, nz] / deg[nz]
    z = (~nz).astype(np.float64)
    return d * (M + np.outer(np.ones(n), z) / n) + (1.0 - d) / n * np.ones((n, n))


def pagerank_power(A, d, T):
    n = A.shape[0]
    G = pagerank_matrix(A, d)
    return np.linalg.matrix_power(G, T) @ np.full(n, 1.0 / n)


def pagerank_fixed_point(A, d):
    n = A.shape[0]
    deg = A.sum(axis=0).astype(np.float64)
    M = np.zeros((n, n))
    nz = deg > 0
    M[:, nz] = A[:, nz] / deg[nz]
    z = (~nz).astype(np.float64)
    lhs = np.eye(n) - d * (M + np.outer(np.ones(n), z) / n)
    return np.linalg.solve(lhs, np.full(n, (1.0 - d) / n))


def all_shortest_paths(n, src, dst, s):
    """Every shortest path from s, enumerated explicitly: {t: [path, ...]} with
    paths as vertex tuples (plain Python breadth-first path extension)."""
    adj = {v: set() for v in range(n)}
    for u, v in simple_edges(n, src, dst):
        adj[u].add(v)
        adj[v].add(u)
    paths = {s: [(s,)]}
    frontier = [s]
    seen = {s}
    while frontier:
        nxt = {}
        for u in frontier:
            for p in paths[u]:
                for w in adj[u]:
                    if w not in seen:
                        nxt.setdefault(w, []).append(p + (w,))
        for w, ps in nxt.items():
            paths[w] = ps
        seen |= set(nxt)
        frontier = list(nxt)
    return paths


def dependency_by_enumeration(n, src, dst, s):
    """delta_s(v) = sum over t != s, v of (shortest s-t paths through v) / (shortest s-t paths),
    counted on the enumerated paths with exact fractions."""
    from fractions import Fraction
    paths = all_shortest_paths(n, src, dst, s)
    delta = [Fraction(0)] * n
    for t, ps in paths.items():
        if t == s:
            continue
        for v in range(n):
            if v in (s, t):
                continue
            through = sum(1 for p in ps if v in p)
            if through:
                delta[v] += Fraction(through, len(ps))
    return delta, {t: len(ps) for t, ps in paths.items()}
