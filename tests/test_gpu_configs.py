"""Parity at the sizes of the quoted workloads (paper Section 6.2,
tab:graph-sizes: the KR / ER / RD shapes these synthetic graphs stand in
for), in the launch configurations the benchmark times:

- ER n = 2^14, average degree 8: BFS from vertex 0, connectivity, PageRank
  d = 0.85 for 20 steps (FP32 against the FP64 oracle);
- RMAT scale 20, edge factor 16: BFS from 16 random non-isolated sources,
  connectivity, PageRank 10 steps, threshold heuristic (and the tile layout
  for connectivity and PageRank);
- the 4096 x 4096 lattice with 10% of its edges deleted: BFS from the corner
  and the centre under the heuristic, the learned selector, the
  device-resident small-frontier loop (8192) and hipGraph-replayed levels, and
  connectivity under the heuristic and the learned selector;
- RMAT scale 25 (about 1.07 billion directed entries): four BFS sources,
  tiled connectivity, PageRank 20 steps over 2^14-vertex tiles, and
  multi-source BFS columns from each of the four 64-source words. Its oracle
  takes several minutes, so it runs only when BYO_SLOW=1.

BFS depths and connectivity labels must be bit-exact, parents a valid BFS
tree; PageRank within 1e-5 relative L-infinity.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")

PR_TOL = 1e-5
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


def progress(msg):
    """Progress of the long cases, past pytest's capture."""
    sys.__stderr__.write(f"[configs {time.strftime('%H:%M:%S')}] {msg}\n")
    sys.__stderr__.flush()


def pr_err(a, b):
    return float(np.max(np.abs(a.astype(np.float64) - b)) / np.max(np.abs(b)))


def check_bfs(g, og, src, opts, want=None):
    d, par, st = byo.bfs(g, int(src), opts=opts)
    got = d.cpu().numpy()
    if want is None:
        want, _ = og.bfs(int(src))
    assert np.array_equal(got, want), f"depths differ from the oracle (src {src})"
    assert og.check_bfs(int(src), got, par.cpu().numpy()) == 0, f"parents invalid (src {src})"
    return st


def mlp_opts(**kw):
    from paper_2405_11671_amd import selector as sel
    params, mu, sd, _ = sel.load_weights(os.path.join(ROOT, "paper_2405_11671_amd", "selector_weights.json"))
    sel.install(params, mu, sd)
    return byo.default_opts(selector=byo.SEL_MLP, **kw)


def test_er14_bfs_cc_pagerank():
    p = gen.er_pairs(1 << 14, 8, seed=1)
    g, og = byo.Graph.from_pairs(p, validate=True), oracle.Graph.from_pairs(p)
    assert g.n == 1 << 14 and p.npairs == 65536
    check_bfs(g, og, 0, byo.default_opts())
    lab, _ = byo.cc(g)
    assert np.array_equal(lab.cpu().numpy(), og.cc())
    r, _ = byo.pagerank(g, 0.85, 20)
    got = r.cpu().numpy()
    assert pr_err(got, og.pagerank(0.85, 20)) < PR_TOL
    assert abs(got.astype(np.float64).sum() - 1.0) < 1e-5


def test_rmat20_sixteen_sources_cc_pagerank():
    p = gen.rmat_pairs(20, 16, seed=1)
    g, og = byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p)
    srcs = gen.pick_sources(p, 16, seed=2)
    assert len(srcs) == 16
    heur = byo.default_opts()
    for s in srcs:
        check_bfs(g, og, s, heur)
    want = og.cc()
    for tiled in (0, 1):
        lab, _ = byo.cc(g, tiled=tiled)
        assert np.array_equal(lab.cpu().numpy(), want), tiled
    r64 = og.pagerank(0.85, 10)
    for blocked in (0, 1):
        r, _ = byo.pagerank(g, 0.85, 10, pr_blocked=blocked)
        assert pr_err(r.cpu().numpy(), r64) < PR_TOL, blocked


@pytest.fixture(scope="module")
def lattice4096():
    progress("building the 4096^2 lattice")
    p = gen.grid_pairs(4096, 4096, 0.1, seed=1)
    g, og = byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p)
    assert g.n == 4096 * 4096 and g.m == 60383232
    return g, og


@pytest.mark.parametrize("where", ["corner", "centre"])
def test_lattice4096_bfs_every_level_loop(lattice4096, where):
    g, og = lattice4096
    src = 0 if where == "corner" else 2048 * 4096 + 2048
    want, _ = og.bfs(src)
    cases = {"heuristic": byo.default_opts(), "learned": mlp_opts(),
             "device_loop": byo.default_opts(small_frontier=8192),
             "learned_device_loop": mlp_opts(small_frontier=8192),
             "hipgraph": byo.default_opts(use_graph=1)}
    for name, o in cases.items():
        progress(f"lattice BFS {where} {name}")
        st = check_bfs(g, og, src, o, want)
        if "device_loop" in name:
            assert st["device_levels"] > 0, name


def test_lattice4096_cc(lattice4096):
    g, og = lattice4096
    want = og.cc()
    for name, o in (("heuristic", byo.default_opts()), ("learned", mlp_opts())):
        progress(f"lattice CC {name}")
        lab, _ = byo.cc(g, opts=o)
        assert np.array_equal(lab.cpu().numpy(), want), name


@pytest.mark.skipif(os.environ.get("BYO_SLOW") != "1",
                    reason="RMAT-25 oracle takes minutes; set BYO_SLOW=1 to run it")
def test_rmat25_subset():
    progress("generating RMAT-25")
    p = gen.rmat_pairs(25, 16, seed=1)
    g = byo.Graph.from_pairs(p)
    progress(f"device graph n={g.n} m={g.m}; building the oracle")
    og = oracle.Graph.from_pairs(p)
    srcs = gen.pick_sources(p, 256, seed=2)
    del p
    assert g.m > 1_000_000_000
    for s in srcs[:4]:
        progress(f"BFS {int(s)}")
        check_bfs(g, og, s, byo.default_opts())
    progress("tiled connectivity")
    lab, _ = byo.cc(g, tiled=1, tile_shift=14)
    assert np.array_equal(lab.cpu().numpy(), og.cc())
    del lab
    progress("PageRank, 20 steps over 2^14 tiles")
    r, _ = byo.pagerank(g, 0.85, 20, pr_blocked=14)
    assert pr_err(r.cpu().numpy(), og.pagerank(0.85, 20)) < PR_TOL
    del r
    progress("256-source BFS over the tile layout")
    D, st = byo.msbfs(g, srcs, tiled=1)
    for w in range(4):
        for j in (64 * w + 5, 64 * w + 58):
            progress(f"multi-source column {j}")
            want, _ = og.bfs(int(srcs[j]))
            col = D[:, j].cpu().numpy()
            assert np.array_equal(col, np.where(want < 0, 255, want)), j
