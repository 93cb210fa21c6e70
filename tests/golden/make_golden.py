"""Write exact-arithmetic fixtures for a small hand-made graph.

The paper prints no worked example, so these values come from the definitions
evaluated in exact rational arithmetic (fractions) and by hand-checkable hop
counting; nothing here calls the GPU path. Run: python tests/golden/make_golden.py
"""
import json
import os
from fractions import Fraction

# 9 vertices: a 4-cycle 0-1-2-3, a tail 3-4-5, a triangle 6-7-8, and a self-pair (5, 5)
N = 9
PAIRS = [(0, 1), (1, 2), (2, 3), (3, 0), (3, 4), (4, 5), (6, 7), (7, 8), (8, 6), (5, 5), (1, 0)]


def neighbours():
    nb = {v: set() for v in range(N)}
    for u, v in PAIRS:
        if u != v:
            nb[u].add(v)
            nb[v].add(u)
    return {v: sorted(s) for v, s in nb.items()}


def hops(src, nb):
    dist = {src: 0}
    layer = [src]
    while layer:
        nxt = []
        for u in layer:
            for v in nb[u]:
                if v not in dist:
                    dist[v] = dist[u] + 1
                    nxt.append(v)
        layer = nxt
    return [dist.get(v, -1) for v in range(N)]


def pagerank_exact(nb, d, T):
    p = [Fraction(1, N)] * N
    for _ in range(T):
        D = sum((p[u] for u in range(N) if not nb[u]), Fraction(0))
        p = [(1 - d) / N + d * (sum((p[u] / len(nb[u]) for u in nb[v]), Fraction(0)) + D / N) for v in range(N)]
    return p


def main():
    nb = neighbours()
    d = Fraction(85, 100)
    out = {
        "source": "hand-made graph; exact rational evaluation of the definitions",
        "n": N,
        "pairs": PAIRS,
        "bfs_depth_from_0": hops(0, nb),
        "bfs_depth_from_6": hops(6, nb),
        "cc_min_label": [min(v2 for v2 in range(N) if hops(v, nb)[v2] >= 0) for v in range(N)],
        "pagerank_d085_T3": [str(x) for x in pagerank_exact(nb, d, 3)],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_graph.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
