"""The per-level frontier statistics the level loop feeds to its variant
choice: |U|, sum deg(U) and the largest degree in U, as traced for each BFS
level, against the frontiers the oracle's BFS layers define (depth == level)."""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")

CASES = [
    ("rmat15", lambda: gen.rmat_pairs(15, 16, seed=4)),
    ("grid64", lambda: gen.grid_pairs(64, 64, 0.1, seed=4)),
    ("two_hubs", lambda: graphs.two_hubs()),
    ("star", lambda: graphs.star(5000)),
]


# the threshold rule, then each variant on every level
CHOICES = [dict()] + [dict(selector=byo.SEL_FIXED, fixed_variant=v) for v in range(6)]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("choice", CHOICES, ids=["heuristic"] + [f"fixed{v}" for v in range(6)])
def test_traced_frontier_max_degree(name, make, choice):
    p = make()
    g = byo.Graph.from_pairs(p)
    og = oracle.Graph.from_pairs(p)
    deg = og.degrees()
    src = int(gen.pick_sources(p, 1, seed=9)[0])
    want_depth, _ = og.bfs(src)
    byo.trace_enable(True)
    try:
        byo.trace_read()
        # host-driven levels only: the device-resident loop does not trace
        depth, _, _ = byo.bfs(g, src, small_frontier=0, persistent=0, **choice)
        recs = [r for r in byo.trace_read() if r["algo"] == 0]
    finally:
        byo.trace_enable(False)
    assert np.array_equal(depth.cpu().numpy(), want_depth)
    assert recs
    known = 0
    for r in recs:
        U = np.flatnonzero(want_depth == r["level"])
        assert r["k"] == U.size, (name, r["level"])
        assert r["degsum"] == int(deg[U].sum()), (name, r["level"])
        if r["max_deg_u"] >= 0:
            assert r["max_deg_u"] == int(deg[U].max()), (name, r["level"])
            known += 1
    # every host-driven BFS level knows it
    assert known == len(recs)
