"""GPU parity of single-source BFS in one persistent launch (option
persistent = 2): depths equal to the oracle's BFS, parents a valid BFS tree,
and the same level count, reached set size and edge total as the host loop."""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")

SHAPES = [
    ("rmat16", lambda: gen.rmat_pairs(16, 16, seed=12)),
    ("star", lambda: graphs.star(70000)),
    ("path", lambda: graphs.path(3000)),
    ("grid", lambda: gen.grid_pairs(200, 150, 0.1, seed=3)),
    ("er", lambda: gen.er_pairs(50000, 12, 5)),
]


def first_non_isolated(og):
    nz = np.flatnonzero(og.degrees())
    return int(nz[0]) if nz.size else 0


@pytest.mark.parametrize("divisor", [20, 1, 1 << 30])
@pytest.mark.parametrize("name,mk", SHAPES, ids=[x[0] for x in SHAPES])
def test_single_source_persistent(name, mk, divisor):
    p = mk()
    og = oracle.Graph.from_pairs(p)
    g = byo.Graph.from_pairs(p)
    src = first_non_isolated(og)
    want, _ = og.bfs(src)
    for _ in range(2):  # the launch resets what it reads: a second call gives the same
        depth, parent, st = byo.bfs(g, src, persistent=2, dense_divisor=divisor)
        d, par = depth.cpu().numpy(), parent.cpu().numpy()
        assert np.array_equal(d, want)
        assert og.check_bfs(src, d, par) == 0
    _, _, st0 = byo.bfs(g, src, persistent=0, dense_divisor=divisor)
    assert st["reached"] == st0["reached"] == int((want >= 0).sum())
    assert st["edges"] == st0["edges"] and st["levels"] == st0["levels"]


def test_single_source_persistent_level_cap():
    g = byo.Graph.from_pairs(graphs.path(100))
    with pytest.raises(byo.ByoError, match="ELIMIT"):
        byo.bfs(g, 0, persistent=2, max_levels=10)
    depth, _, st = byo.bfs(g, 0, persistent=2)
    assert np.array_equal(depth.cpu().numpy(), np.arange(100, dtype=np.int32))
