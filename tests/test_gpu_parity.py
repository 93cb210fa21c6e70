"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

BFS depths and min-ID CC labels must match exactly for every edgeMap variant;
BFS parents must form a valid BFS tree (several are correct); PageRank in FP32
must be within 1e-5 relative L-infinity (max |p32 - p64| / max |p64|) of the
FP64 oracle after the same number of steps.
"""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")

PR_TOL = 1e-5
ALL_VARIANTS = list(range(byo.NUM_VARIANTS))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


_cache = {}


def build(p):
    key = p.name
    if key not in _cache:
        _cache[key] = (byo.Graph.from_pairs(p, validate=True), oracle.Graph.from_pairs(p))
    return _cache[key]


SUITE = graphs.small_suite()
IDS = [p.name for p in SUITE]


def sources(p, og, k=3):
    deg = og.degrees()
    nz = np.flatnonzero(deg)
    out = [0]
    if nz.size:
        out += [int(nz[len(nz) // 2]), int(nz[np.argmax(deg[nz])])]
    return sorted(set(out))[:k]


@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_container_queries(p):
    g, og = build(p)
    assert g.num_vertices() == og.n and g.num_edges() == og.m
    for v in sorted({0, og.n // 2, og.n - 1}):
        assert g.degree(v) == og.degree(v)
        assert g.neighbors(v).tolist() == og.neighbors(v).tolist()


@pytest.mark.parametrize("variant", [None] + ALL_VARIANTS)
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_bfs(p, variant):
    g, og = build(p)
    kw = {} if variant is None else {"selector": byo.SEL_FIXED, "fixed_variant": variant}
    for s in sources(p, og):
        depth, parent, st = byo.bfs(g, s, **kw)
        d = depth.cpu().numpy()
        par = parent.cpu().numpy()
        want, _ = og.bfs(s)
        print(p.name, variant, s, st["levels"])
        assert np.array_equal(d, want), (p.name, variant, s)
        assert og.check_bfs(s, d, par) == 0
        assert st["reached"] == int((want >= 0).sum())


@pytest.mark.parametrize("variant", [None] + ALL_VARIANTS)
@pytest.mark.parametrize("shortcut", [1, 0])
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_cc(p, variant, shortcut):
    g, og = build(p)
    kw = {"cc_shortcut": shortcut}
    if variant is not None:
        # a fixed variant runs the CSR rounds (the tile layout, the default for
        # graphs that qualify, has its own passes)
        kw.update(selector=byo.SEL_FIXED, fixed_variant=variant, tiled=0)
    label, st = byo.cc(g, **kw)
    assert np.array_equal(label.cpu().numpy(), og.cc()), (p.name, variant, shortcut)


@pytest.mark.parametrize("iters", [0, 1, 20])
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_pagerank(p, iters):
    g, og = build(p)
    r64 = og.pagerank(0.85, iters)
    for layout in (1, 0):   # the default (tiles where the graph qualifies) and the CSR pull
        r32, _ = byo.pagerank(g, 0.85, iters, pr_blocked=layout)
        r = r32.cpu().numpy().astype(np.float64)
        err = np.max(np.abs(r - r64)) / np.max(np.abs(r64))
        assert err < PR_TOL, (p.name, iters, layout, err)
        assert abs(r.sum() - 1.0) < 1e-4


@pytest.mark.parametrize("layout", [1, 12, 13, 14])
@pytest.mark.parametrize("iters", [1, 20])
def test_pagerank_tiled_layout(layout, iters):
    """Destination-tiled PageRank: several tiles, chunks per tile and a ragged last tile."""
    p = gen.rmat_pairs(16, 16, seed=12)
    g, og = build(p)
    assert g.n >= 1 << 16 and g.m >= 4 * g.n
    r32, st = byo.pagerank(g, 0.85, iters, pr_blocked=layout)
    r64 = og.pagerank(0.85, iters)
    r = r32.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(r - r64)) / np.max(np.abs(r64)) < PR_TOL
    assert abs(r.sum() - 1.0) < 1e-4
    # graph with n not a multiple of the tile and isolated vertices
    q = gen.er_pairs(70001, 10, seed=5)
    g2, og2 = build(q)
    r32, _ = byo.pagerank(g2, 0.85, iters, pr_blocked=layout)
    r64 = og2.pagerank(0.85, iters)
    assert np.max(np.abs(r32.cpu().numpy() - r64)) / np.max(np.abs(r64)) < PR_TOL


TILED = [gen.rmat_pairs(16, 16, seed=12), gen.er_pairs(70001, 10, seed=5), gen.rmat_pairs(17, 4, seed=7),
         graphs.hub_over_er()]


@pytest.mark.parametrize("shift", [0, 13, 14])
@pytest.mark.parametrize("shortcut", [1, 0])
@pytest.mark.parametrize("pi", range(len(TILED)))
def test_cc_tiled_matches_oracle(pi, shortcut, shift):
    """Connectivity over the tile layout: minimum original ID per component
    (many components and isolated vertices in the sparse RMAT), with the tile
    size chosen from n and at 2^13 and 2^14 (a layout of its own per size)."""
    p = TILED[pi]
    g, og = build(p)
    lab, st = byo.cc(g, tiled=1, cc_shortcut=shortcut, tile_shift=shift)
    want = og.cc()
    assert np.array_equal(lab.cpu().numpy(), want), (pi, shortcut, shift)
    assert st["levels"] >= 1


@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_tiled_options_fall_back_below_size_cut(p):
    """tiled / pr_blocked on graphs the layout does not take (n < 2^16 or
    m < 4n) run over the CSR and stay exact."""
    g, og = build(p)
    if g.n >= 1 << 16 and g.m >= 4 * g.n:
        pytest.skip("graph qualifies for the layout")
    lab, _ = byo.cc(g, tiled=1)
    assert np.array_equal(lab.cpu().numpy(), og.cc())
    r, _ = byo.pagerank(g, 0.85, 5, pr_blocked=1)
    r64 = og.pagerank(0.85, 5)
    assert np.max(np.abs(r.cpu().numpy() - r64)) / np.max(np.abs(r64)) < PR_TOL


def test_cc_tiled_round_cap():
    g, _ = build(TILED[2])
    with pytest.raises(byo.ByoError) as e:
        byo.cc(g, tiled=1, max_levels=1, cc_shortcut=0)
    assert e.value.status == -4


def test_bfs_repeat_deterministic_depths():
    p = SUITE[1]
    g, og = build(p)
    want, _ = og.bfs(5)
    for _ in range(5):
        d, par, _ = byo.bfs(g, 5, selector=byo.SEL_FIXED, fixed_variant=byo.V_PUSH_EDGE)
        assert np.array_equal(d.cpu().numpy(), want)
        assert og.check_bfs(5, d.cpu().numpy(), par.cpu().numpy()) == 0


def test_vset_roundtrip():
    p = SUITE[0]
    g, og = build(p)
    rng = np.random.default_rng(3)
    ids = np.unique(rng.integers(0, og.n, 3000)).astype(np.int32)
    rng.shuffle(ids)
    U = byo.VSet(g).set_ids(torch.from_numpy(ids).cuda())
    assert U.size() == ids.size
    assert U.ids().cpu().numpy().tolist() == sorted(ids.tolist())
    bits = U.bitmap().cpu().numpy().view(np.uint64)
    unpacked = np.flatnonzero(np.unpackbits(bits.view(np.uint8), bitorder="little")[: og.n])
    assert unpacked.tolist() == sorted(ids.tolist())
    V = byo.VSet(g).set_bitmap(torch.from_numpy(bits.view(np.int64)).cuda())
    assert V.size() == ids.size
    assert V.ids().cpu().numpy().tolist() == sorted(ids.tolist())
    W = byo.VSet(g).fill()
    assert W.size() == og.n
    assert W.ids().cpu().numpy().tolist() == list(range(og.n))


@pytest.mark.parametrize("variant", ALL_VARIANTS)
def test_edge_map_bfs_step(variant):
    """One edgeMap from the level-L frontier emits exactly the level-(L+1) set."""
    p = SUITE[1]
    g, og = build(p)
    src = sources(p, og)[-1]
    want, _ = og.bfs(src)
    n = og.n
    for L in range(0, int(want.max())):
        depth = torch.from_numpy(np.where((want >= 0) & (want <= L), want, -1).astype(np.int32)).cuda()
        # any valid parents up to level L (oracle tree)
        _, opar = og.bfs(src)
        parent = torch.from_numpy(np.where((want >= 0) & (want <= L), opar, -1).astype(np.int32)).cuda()
        vis = np.zeros(((n + 63) // 64) * 64, bool)
        vis[:n] = (want >= 0) & (want <= L)
        vis[n:] = True
        visited = torch.from_numpy(np.packbits(vis, bitorder="little").view(np.int64).copy()).cuda()
        U = byo.VSet(g).set_ids(torch.from_numpy(np.flatnonzero(want == L).astype(np.int32)).cuda())
        out = byo.VSet(g)
        st = byo.bfs_fn_state(parent, depth, visited, L)
        used = byo.edge_map(g, U, byo.F_BFS, st, out, variant=variant)
        assert used == variant
        got = out.ids().cpu().numpy()
        assert got.tolist() == np.flatnonzero(want == L + 1).tolist()
        d = depth.cpu().numpy()
        assert np.array_equal(d[want == L + 1], np.full((want == L + 1).sum(), L + 1))


@pytest.mark.parametrize("variant", ALL_VARIANTS)
def test_edge_map_cc_step_bounds(variant):
    """One min-label edgeMap from the full set. Updates inside one call may chain
    (a lowered label can be read again in the same call), so the result lies
    between the synchronous one-hop minimum and the component minimum, and
    every new label is the initial label of a vertex in the same component."""
    p = SUITE[0]
    g, og = build(p)
    off, nbr = og.export()
    n = og.n
    rng = np.random.default_rng(9)
    lab0 = rng.permutation(n).astype(np.int32)
    label = torch.from_numpy(lab0.copy()).cuda()
    U = byo.VSet(g).fill()
    out = byo.VSet(g)
    byo.edge_map(g, U, byo.F_CC_MIN, byo.cc_fn_state(label), out, variant=variant)
    got = label.cpu().numpy()
    one = lab0.copy()
    for v in range(n):
        nb = nbr[off[v]:off[v + 1]]
        if nb.size:
            one[v] = min(one[v], lab0[nb].min())
    comp = og.cc()
    cmin = np.full(n, np.iinfo(np.int32).max, np.int64)
    np.minimum.at(cmin, comp, lab0)
    owner = np.empty(n, np.int64)
    owner[lab0] = np.arange(n)
    assert np.all(got <= one)
    assert np.all(got >= cmin[comp])
    assert np.array_equal(comp[owner[got]], comp)
    changed = np.flatnonzero(got < lab0)
    assert out.ids().cpu().numpy().tolist() == changed.tolist()


def test_edge_map_pr_accumulate():
    p = SUITE[4]
    g, og = build(p)
    off, nbr = og.export()
    rng = np.random.default_rng(2)
    contrib = rng.random(og.n).astype(np.float32)
    acc = torch.zeros(og.n, dtype=torch.float32, device="cuda")
    U = byo.VSet(g).fill()
    out = byo.VSet(g)
    byo.edge_map(g, U, byo.F_PR_ACC, byo.pr_fn_state(torch.from_numpy(contrib).cuda(), acc), out)
    want = np.array([contrib[nbr[off[v]:off[v + 1]]].astype(np.float64).sum() for v in range(og.n)])
    got = acc.cpu().numpy()
    assert np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-30)) < 1e-5


def test_validation_rejects_bad_csr():
    off = np.array([0, 1, 2], np.int64)
    nbr = np.array([1, 1], np.int32)          # (1,1) is a self-loop, (0,1) lacks (1,0)? no: row1 = [1]
    with pytest.raises(byo.ByoError):
        byo.Graph.from_csr(off, nbr, validate=True)
    off = np.array([0, 1, 1], np.int64)
    nbr = np.array([1], np.int32)             # asymmetric
    with pytest.raises(byo.ByoError):
        byo.Graph.from_csr(off, nbr, validate=True)
    off = np.array([0, 2, 1], np.int64)       # decreasing offsets
    nbr = np.array([1], np.int32)
    with pytest.raises(byo.ByoError):
        byo.Graph.from_csr(off, nbr, validate=True)
    off = np.array([0, 1, 2], np.int64)
    nbr = np.array([1, 0], np.int32)          # valid
    byo.Graph.from_csr(off, nbr, validate=True)


def test_bfs_level_cap_and_bad_source():
    p = graphs.path(300)
    g, og = build(p)
    with pytest.raises(byo.ByoError) as e:
        byo.bfs(g, 0, max_levels=10)
    assert e.value.status == -4
    with pytest.raises(byo.ByoError) as e:
        byo.bfs(g, 300)
    assert e.value.status == -1


@pytest.mark.parametrize("cap", [1, 64, 1000, 8192])
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_bfs_device_resident_small_frontier(p, cap):
    """Levels run in the device-resident loop while |U| <= cap; results stay exact."""
    g, og = build(p)
    for s in sources(p, og):
        depth, parent, st = byo.bfs(g, s, small_frontier=cap)
        want, _ = og.bfs(s)
        d = depth.cpu().numpy()
        assert np.array_equal(d, want), (p.name, cap, s)
        assert og.check_bfs(s, d, parent.cpu().numpy()) == 0
        assert st["reached"] == int((want >= 0).sum())
        assert st["levels"] == int(want.max()) + 1 if (want >= 0).sum() > 1 else True


def test_small_frontier_runs_on_device_for_lattices():
    from paper_2405_11671_amd import gen
    p = gen.grid_pairs(300, 200, 0.1, seed=4)
    g, og = build(p)
    depth, _, st = byo.bfs(g, 0, small_frontier=4096)
    want, _ = og.bfs(0)
    assert np.array_equal(depth.cpu().numpy(), want)
    assert st["device_levels"] >= st["levels"] - 2 and st["device_levels"] > 100
    # the level cap still holds inside the device loop
    with pytest.raises(byo.ByoError) as e:
        byo.bfs(g, 0, small_frontier=4096, max_levels=50)
    assert e.value.status == -4


@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_bfs_graph_mode(p):
    """Device-side level control replayed from a captured hipGraph; several
    replays per run on deep graphs, with the eager result as reference."""
    g, og = build(p)
    for s in sources(p, og):
        for rep in range(2):                                  # the cached graph is replayed
            depth, parent, st = byo.bfs(g, s, use_graph=1)
            want, _ = og.bfs(s)
            d = depth.cpu().numpy()
            assert np.array_equal(d, want), (p.name, s, rep)
            assert og.check_bfs(s, d, parent.cpu().numpy()) == 0
            assert st["reached"] == int((want >= 0).sum())
        d2, _, _ = byo.bfs(g, s)                              # eager run in between
        assert np.array_equal(d2.cpu().numpy(), want)


def test_bfs_graph_mode_level_cap():
    p = graphs.path(300)
    g, og = build(p)
    with pytest.raises(byo.ByoError) as e:
        byo.bfs(g, 0, use_graph=1, max_levels=40)
    assert e.value.status == -4
    d, _, st = byo.bfs(g, 0, use_graph=1)
    assert np.array_equal(d.cpu().numpy(), og.bfs(0)[0]) and st["levels"] == 300
