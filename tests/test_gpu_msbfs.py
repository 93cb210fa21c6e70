"""GPU parity of multi-source BFS (bit-parallel, up to 256 sources) vs the oracle."""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")

_cache = {}


def build(p):
    if p.name not in _cache:
        _cache[p.name] = (byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p))
    return _cache[p.name]


SUITE = [p for p in graphs.small_suite() if not p.name.startswith("path")]


@pytest.mark.parametrize("k", [1, 7, 64, 65, 200, 256])
@pytest.mark.parametrize("p", SUITE, ids=[p.name for p in SUITE])
def test_msbfs_matches_single_source_oracle(p, k):
    g, og = build(p)
    rng = np.random.default_rng(k)
    srcs = rng.integers(0, og.n, k)
    srcs[0] = srcs[-1]          # a repeated source is allowed
    want = og.msbfs(srcs)
    reached = int((want != 255).sum())
    for tiled in (1, 0):        # the default (tiles where the graph qualifies) and the CSR levels
        D, st = byo.msbfs(g, srcs, tiled=tiled)
        assert np.array_equal(D.cpu().numpy(), want), (p.name, k, tiled)
        assert st["reached"] == reached


@pytest.mark.parametrize("variant", [byo.V_PUSH_THREAD, byo.V_PUSH_WAVE, byo.V_PUSH_BUCKET, byo.V_PUSH_EDGE,
                                     byo.V_PULL_WAVE])
def test_msbfs_fixed_variants(variant):
    p = gen.rmat_pairs(13, 16, seed=4)
    g, og = build(p)
    srcs = gen.pick_sources(p, 130, seed=5)
    D, _ = byo.msbfs(g, srcs, selector=byo.SEL_FIXED, fixed_variant=variant)
    assert np.array_equal(D.cpu().numpy(), og.msbfs(srcs))


TILED = [gen.rmat_pairs(16, 16, seed=12), gen.er_pairs(70001, 10, seed=5), gen.rmat_pairs(17, 4, seed=7),
         graphs.hub_over_er()]


@pytest.mark.parametrize("k", [1, 7, 64, 65, 150, 200, 256])
@pytest.mark.parametrize("pi", range(len(TILED)))
def test_msbfs_tiled_matches_oracle(pi, k):
    """Tile-layout levels (degree-relabelled, 2^12-vertex tiles, several
    chunks per hub tile, ragged last tile, isolated vertices)."""
    p = TILED[pi]
    g, og = build(p)
    rng = np.random.default_rng(100 + k)
    srcs = rng.integers(0, og.n, k)
    srcs[0] = srcs[-1]
    D, st = byo.msbfs(g, srcs, tiled=1)
    want = og.msbfs(srcs)
    assert np.array_equal(D.cpu().numpy(), want), (pi, k)
    assert st["reached"] == int((want != 255).sum())
    D2, st2 = byo.msbfs(g, srcs, tiled=0)
    assert np.array_equal(D2.cpu().numpy(), want)
    assert st2["edges"] == st["edges"] and st2["reached"] == st["reached"]


@pytest.mark.parametrize("k", [16, 150, 256])
def test_msbfs_tiled_many_levels(k):
    """A king-move lattice from sources near its middle: about 200 levels, far
    more than the frontier-history slots, so the depth rows are built from the
    history partway and the later levels write their depths on top."""
    p = graphs.king_lattice()
    g, og = build(p)
    assert g.m >= 4 * g.n >= 4 * 65536
    rows, cols = 200, 400
    rng = np.random.default_rng(7 + k)
    r = rng.integers(90, 110, k)
    c = rng.integers(190, 210, k)
    srcs = r * cols + c
    D, st = byo.msbfs(g, srcs, tiled=1)
    want = og.msbfs(srcs)
    assert st["levels"] > 100
    assert np.array_equal(D.cpu().numpy(), want), k
    # the Chebyshev distance is the closed form on this lattice
    vr, vc = np.divmod(np.arange(g.n), cols)
    j = k - 1
    cheb = np.maximum(np.abs(vr - r[j]), np.abs(vc - c[j]))
    assert np.array_equal(want.reshape(g.n, k)[:, j], cheb)


@pytest.mark.parametrize("hist", [2, 3, 5])
def test_msbfs_tiled_history_cap(hist):
    """Fewer frontier-history slots than levels: the depth rows are built at the
    level that would need one slot more, and the later levels write their
    depths directly, at the smallest caps too."""
    rng = np.random.default_rng(40 + hist)
    for p, ks in ((TILED[0], (64, 150, 256)), (graphs.king_lattice(), (16,))):
        g, og = build(p)
        for k in ks:
            if p.name.startswith("king"):  # near the middle: every distance stays below 255
                srcs = rng.integers(90, 110, k) * 400 + rng.integers(190, 210, k)
            else:
                srcs = rng.integers(0, og.n, k)
            D, st = byo.msbfs(g, srcs, tiled=1, ms_history=hist)
            assert st["levels"] > hist
            assert np.array_equal(D.cpu().numpy(), og.msbfs(srcs)), (p.name, k, hist)


def test_msbfs_tiled_history_cap_range():
    g, _ = build(TILED[0])
    for bad in (1, 17, -1):
        with pytest.raises(byo.ByoError) as e:
            byo.msbfs(g, [0, 1], tiled=1, ms_history=bad)
        assert e.value.status == -1


@pytest.mark.parametrize("p", SUITE, ids=[p.name for p in SUITE])
def test_msbfs_tiled_falls_back_below_size_cut(p):
    """tiled = 1 on graphs the layout does not take runs over the CSR."""
    g, og = build(p)
    srcs = np.random.default_rng(3).integers(0, og.n, 65)
    D, _ = byo.msbfs(g, srcs, tiled=1)
    assert np.array_equal(D.cpu().numpy(), og.msbfs(srcs))


def test_msbfs_tiled_after_pagerank_layout_change():
    """PageRank with another tile size builds a second layout next to the
    multi-source run's 2^12 one; both keep giving exact results, in either
    order."""
    p = TILED[0]
    g, og = build(p)
    srcs = gen.pick_sources(p, 100, seed=3)
    byo.pagerank(g, 0.85, 2, pr_blocked=14)
    D, _ = byo.msbfs(g, srcs, tiled=1)
    assert np.array_equal(D.cpu().numpy(), og.msbfs(srcs))
    r, _ = byo.pagerank(g, 0.85, 5, pr_blocked=1)
    r64 = og.pagerank(0.85, 5)
    assert np.max(np.abs(r.cpu().numpy() - r64)) / np.max(np.abs(r64)) < 1e-5


def test_msbfs_depth_limit():
    p = graphs.path(400)
    g, og = build(p)
    with pytest.raises(byo.ByoError) as e:
        byo.msbfs(g, [0, 5])                 # distance 399 does not fit in uint8
    assert e.value.status == -4
    D, _ = byo.msbfs(g, [200, 210])      # every distance <= 210
    assert np.array_equal(D.cpu().numpy(), og.msbfs(np.array([200, 210])))


def test_msbfs_rejects_bad_arguments():
    g, _ = build(SUITE[0])
    with pytest.raises(byo.ByoError):
        byo.msbfs(g, list(range(257)))
    with pytest.raises(byo.ByoError):
        byo.msbfs(g, [g.n])
