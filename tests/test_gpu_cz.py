"""GPU: the byte-coded CSR (byo_cz_build) and the traversals that decode it.

The device-built stream must equal, byte for byte, the reference encoder of
tests/czcode.py run on the oracle's neighbour lists; lists decoded on the
device must equal the oracle's; BFS depths and connectivity labels over the
byte-coded lists must equal the oracle's exactly (parents a valid BFS tree),
and PageRank must stay within 1e-5 relative L-infinity of the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen
from tests import czcode, graphs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")

PR_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


_cache = {}


def build(p):
    if p.name not in _cache:
        _cache[p.name] = (byo.Graph.from_pairs(p, validate=True), oracle.Graph.from_pairs(p))
    return _cache[p.name]


SUITE = graphs.small_suite() + [gen.rmat_pairs(16, 16, seed=12)]
IDS = [p.name for p in SUITE]


def sources(og):
    deg = og.degrees()
    nz = np.flatnonzero(deg)
    out = [0]
    if nz.size:
        out += [int(nz[len(nz) // 2]), int(nz[np.argmax(deg[nz])])]
    return sorted(set(out))


@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_stream_matches_reference_encoder(p):
    g, og = build(p)
    off, data = g.cz_arrays()
    want_off, want = czcode.encode([og.neighbors(v) for v in range(og.n)])
    assert np.array_equal(off, want_off)
    assert np.array_equal(data, want)
    if og.m:
        print(p.name, "bytes per edge", round(len(data) / og.m, 3))


@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_decode_back(p):
    g, og = build(p)
    deg = og.degrees()
    vs = {0, og.n - 1, og.n // 2}
    if og.m:
        vs.add(int(np.argmax(deg)))
    for v in sorted(vs):
        got = g.cz_decode(v).cpu().numpy()
        assert got.tolist() == og.neighbors(v).tolist(), v


@pytest.mark.parametrize("variant", [None, 0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_bfs_compressed(p, variant):
    g, og = build(p)
    kw = {} if variant is None else {"selector": byo.SEL_FIXED, "fixed_variant": variant}
    for s in sources(og):
        depth, parent, st = byo.bfs(g, s, compressed=1, **kw)
        want, _ = og.bfs(s)
        d = depth.cpu().numpy()
        assert np.array_equal(d, want), (p.name, variant, s)
        assert og.check_bfs(s, d, parent.cpu().numpy()) == 0
        assert st["reached"] == int((want >= 0).sum())
        used = {k for k, c in st["variant_count"].items() if c}
        assert "push_bucket" not in used, used


@pytest.mark.parametrize("variant", [None, 0, 1, 4, 5])
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_cc_compressed(p, variant):
    g, og = build(p)
    kw = {} if variant is None else {"selector": byo.SEL_FIXED, "fixed_variant": variant}
    want = og.cc()
    for shortcut in (1, 0):
        label, _ = byo.cc(g, compressed=1, cc_shortcut=shortcut, **kw)
        assert np.array_equal(label.cpu().numpy(), want), (p.name, variant, shortcut)


@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_pagerank_compressed(p):
    g, og = build(p)
    for iters in (0, 1, 20):
        r32, _ = byo.pagerank(g, 0.85, iters, compressed=1)
        r64 = og.pagerank(0.85, iters)
        r = r32.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(r - r64)) / np.max(np.abs(r64)) < PR_TOL, (p.name, iters)


def test_compressed_with_api_omit_is_rejected():
    g, _ = build(SUITE[0])
    for call in (lambda: byo.bfs(g, 0, compressed=1, api_omit=1), lambda: byo.cc(g, compressed=1, api_omit=4),
                 lambda: byo.pagerank(g, 0.85, 3, compressed=1, api_omit=8)):
        with pytest.raises(byo.ByoError):
            call()


def test_compressed_ignores_tiled_and_graph_paths():
    g, og = build(SUITE[-1])
    want, _ = og.bfs(5)
    depth, _, st = byo.bfs(g, 5, compressed=1, use_graph=1, small_frontier=8192)
    assert np.array_equal(depth.cpu().numpy(), want) and st["device_levels"] == 0
    label, _ = byo.cc(g, compressed=1, tiled=1)
    assert np.array_equal(label.cpu().numpy(), og.cc())
    r32, _ = byo.pagerank(g, 0.85, 20, compressed=1, pr_blocked=1)
    r64 = og.pagerank(0.85, 20)
    assert np.max(np.abs(r32.cpu().numpy() - r64)) / np.max(np.abs(r64)) < PR_TOL


def spread_hub():
    """A hub whose 66 neighbours lie 2.1M ids apart in a graph of 140M
    vertices: its first block is 64 values of 4 bytes (256 bytes), and two
    1-byte lists before it leave that block off 4-byte alignment, so the
    wavefront decoder needs a second pass."""
    n, hub = 140_000_000, 70_000_000
    leaves = [1000 + i * 2_100_000 for i in range(66)]
    src = [1] + [hub] * len(leaves)
    dst = [2] + leaves
    return graphs.pairs(n, src, dst, "spread_hub")


def test_wave_decoder_second_pass():
    p = spread_hub()
    g, og = build(p)
    hub, last = 70_000_000, 1000 + 65 * 2_100_000
    off, data = g.cz_arrays()
    start0 = int(off[hub]) + 4              # block 0 follows the 1-entry offset table
    start1 = int(off[hub]) + int.from_bytes(bytes(data[int(off[hub]):int(off[hub]) + 4]), "little")
    assert start0 % 4 != 0 and start1 - start0 == 256
    assert g.cz_decode(hub).cpu().numpy().tolist() == og.neighbors(hub).tolist()
    for s, variant in ((hub, 1), (hub, 3), (last, 5), (last, 4)):
        depth, parent, _ = byo.bfs(g, s, compressed=1, selector=byo.SEL_FIXED, fixed_variant=variant)
        want, _ = og.bfs(s)
        d = depth.cpu().numpy()
        assert np.array_equal(d, want), (s, variant)
        assert og.check_bfs(s, d, parent.cpu().numpy()) == 0
    label, _ = byo.cc(g, compressed=1)
    assert np.array_equal(label.cpu().numpy(), og.cc())
    _cache.pop(p.name, None)
