"""GPU parity of batched execution: each graph of a batch equals its own oracle run."""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")


def first_non_isolated(og):
    deg = og.degrees()
    nz = np.flatnonzero(deg)
    return int(nz[0]) if nz.size else 0


def check_batch(plist, **kw):
    B = byo.Batch.from_pairs(plist)
    ogs = [oracle.Graph.from_pairs(p) for p in plist]
    srcs = [first_non_isolated(og) for og in ogs]
    depth, parent, st = B.bfs(srcs, **kw)
    label, _ = B.cc(**kw)
    D, P, L = B.split(depth.cpu().numpy()), B.split(parent.cpu().numpy()), B.split(label.cpu().numpy())
    reached = 0
    for i, og in enumerate(ogs):
        want, _ = og.bfs(srcs[i])
        assert np.array_equal(D[i], want), i
        assert og.check_bfs(srcs[i], D[i], P[i]) == 0, i
        assert np.array_equal(L[i], og.cc()), i
        reached += int((want >= 0).sum())
    assert st["reached"] == reached
    return st


def test_batch_config_64_er_graphs():
    """The full batch: 64 ER graphs, n log-uniform in [2^10, 2^18], degree in
    [4, 32]; one persistent launch (the default) and the host level loop."""
    st = check_batch(gen.batch_pairs(64, seed=3))
    assert st["levels"] >= 2 and st["device_levels"] == st["levels"]
    st_host = check_batch(gen.batch_pairs(64, seed=3), persistent=0)
    assert st_host["levels"] == st["levels"] and st_host["reached"] == st["reached"]


@pytest.mark.parametrize("variant", list(range(6)))
def test_batch_fixed_variants(variant):
    plist = gen.batch_pairs(12, seed=7, log2_hi=13.0)
    check_batch(plist, selector=byo.SEL_FIXED, fixed_variant=variant, persistent=0)


SHAPES = [
    ("rmat16", lambda: [gen.rmat_pairs(16, 16, seed=12)]),
    ("star", lambda: [graphs.star(70000)]),
    ("path", lambda: [graphs.path(3000)]),
    ("grid", lambda: [gen.grid_pairs(200, 150, 0.1, seed=3)]),
    ("mixed", lambda: [graphs.star(5000), graphs.path(300), graphs.pairs(1, [], [], "single"),
                       gen.grid_pairs(30, 40, 0.1, seed=2), gen.rmat_pairs(12, 8, seed=9), graphs.empty(70)]),
]


@pytest.mark.parametrize("divisor", [20, 1, 1 << 30])
@pytest.mark.parametrize("name,mk", SHAPES, ids=[x[0] for x in SHAPES])
def test_batch_persistent_launch(name, mk, divisor):
    """Every level in one persistent launch, on skewed, long-path and mixed
    graphs; divisor 1 keeps every level a push, 2^30 makes every level a
    pull. Depths exact, parents valid, and the same counts as the host loop."""
    plist = mk()
    st = check_batch(plist, dense_divisor=divisor)
    st_host = check_batch(plist, dense_divisor=divisor, persistent=0)
    assert st["reached"] == st_host["reached"] and st["edges"] == st_host["edges"]
    assert st["levels"] == st_host["levels"], (st, st_host)
    pushes, pulls = st["variant_count"]["push_bucket"], st["variant_count"]["pull_thread"]
    assert pushes + pulls == st["levels"]
    if divisor == 1:
        assert pulls == 0
    if divisor == 1 << 30:
        assert pushes == 0


def test_batch_persistent_level_cap():
    B = byo.Batch.from_pairs([graphs.path(100)])
    with pytest.raises(byo.ByoError, match="ELIMIT"):
        B.bfs([0], max_levels=10)
    # the launch state left by a capped search does not leak into the next one
    depth, parent, st = B.bfs([0])
    assert np.array_equal(depth.cpu().numpy(), np.arange(100, dtype=np.int32))
    assert st["levels"] == 100


@pytest.mark.parametrize("count", [63, 64, 65, 130])
def test_batch_persistent_many_sources(count):
    """Up to 64 sources travel in the persistent launch's arguments, more are
    copied to the device first: both sides of that boundary, twice in a row
    (the launch resets everything it reads)."""
    plist = gen.batch_pairs(count, seed=11, log2_hi=12.0)
    st = check_batch(plist)
    assert st["device_levels"] == st["levels"]
    st2 = check_batch(plist)
    assert st2["reached"] == st["reached"] and st2["levels"] == st["levels"]
    st_host = check_batch(plist, persistent=0)
    assert st_host["reached"] == st["reached"] and st_host["levels"] == st["levels"]


def test_batch_mixed_shapes():
    plist = [graphs.star(5000), graphs.path(300), graphs.pairs(1, [], [], "single"),
             gen.grid_pairs(30, 40, 0.1, seed=2), gen.rmat_pairs(12, 8, seed=9), graphs.empty(70)]
    check_batch(plist)


def test_batch_rejects_bad_input():
    with pytest.raises(byo.ByoError):
        byo.Batch([(np.array([0, 1], np.int64), np.array([5], np.int32))])   # neighbour out of range
    B = byo.Batch.from_pairs([graphs.path(10), graphs.path(5)])
    with pytest.raises(byo.ByoError):
        B.bfs([0, 5])                                                         # source outside graph 1


def test_batch_graph_mode_matches_eager():
    plist = gen.batch_pairs(64, seed=3)
    B = byo.Batch.from_pairs(plist)
    ogs = [oracle.Graph.from_pairs(p) for p in plist]
    srcs = [first_non_isolated(og) for og in ogs]
    for rep in range(3):
        depth, parent, st = B.bfs(srcs, use_graph=1)
        D, P = B.split(depth.cpu().numpy()), B.split(parent.cpu().numpy())
        for i, og in enumerate(ogs):
            want, _ = og.bfs(srcs[i])
            assert np.array_equal(D[i], want), (rep, i)
            assert og.check_bfs(srcs[i], D[i], P[i]) == 0


@pytest.mark.parametrize("cap", [1024, 8192])
def test_batch_device_resident_loop(cap):
    """Batched BFS with small frontiers in the device-resident loop (64
    sources in one frontier; hand-back to the host loop when it grows)."""
    plist = gen.batch_pairs(64, seed=3)
    B = byo.Batch.from_pairs(plist)
    ogs = [oracle.Graph.from_pairs(p) for p in plist]
    srcs = [first_non_isolated(og) for og in ogs]
    depth, parent, st = B.bfs(srcs, small_frontier=cap, persistent=0)
    D, P = B.split(depth.cpu().numpy()), B.split(parent.cpu().numpy())
    for i, og in enumerate(ogs):
        want, _ = og.bfs(srcs[i])
        assert np.array_equal(D[i], want), i
        assert og.check_bfs(srcs[i], D[i], P[i]) == 0
    assert st["device_levels"] >= 1
