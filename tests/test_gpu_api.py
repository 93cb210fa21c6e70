"""GPU parity of the container-API configurations (Section 4.2, Table
api-components-avg): a run that may not use some optional container functions
does different work but must return the same results as the oracle: exact BFS
depths with a valid parent tree, exact connectivity labels, and PageRank within
1e-5 relative L-infinity of the FP64 oracle.
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
CONFIGS = sorted(byo.API_CONFIGS.items(), key=lambda kv: kv[1])
CFG_IDS = [k for k, _ in CONFIGS]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


_cache = {}


def build(p):
    if p.name not in _cache:
        _cache[p.name] = (byo.Graph.from_pairs(p, validate=True), oracle.Graph.from_pairs(p))
    return _cache[p.name]


SUITE = graphs.small_suite()
IDS = [p.name for p in SUITE]
# graphs whose levels take every direction and push variant
MIXED = [gen.rmat_pairs(14, 16, seed=1), graphs.star(70000), gen.grid_pairs(97, 61, 0.1, seed=1),
         graphs.two_hubs()]
MIXED_IDS = [p.name for p in MIXED]


def sources(og):
    deg = og.degrees()
    nz = np.flatnonzero(deg)
    out = [0]
    if nz.size:
        out += [int(nz[len(nz) // 2]), int(nz[np.argmax(deg[nz])])]
    return sorted(set(out))


def used(st):
    return {k for k, c in st["variant_count"].items() if c}


def check_allowed(st, omit, bfs):
    """The variants a run used are ones its container functions allow."""
    u = used(st)
    if omit & byo.API_NO_PAR_MAP:
        assert not u & {"push_wave", "push_bucket", "push_edge"}, u
        if not bfs:
            assert "pull_wave" not in u, u
    if bfs and omit & byo.API_NO_PAR_EARLY_EXIT:
        assert "pull_wave" not in u, u


@pytest.mark.parametrize("cfg,omit", CONFIGS, ids=CFG_IDS)
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_bfs_api_config(p, cfg, omit):
    g, og = build(p)
    for s in sources(og):
        depth, parent, st = byo.bfs(g, s, api_omit=omit)
        want, _ = og.bfs(s)
        d = depth.cpu().numpy()
        print(p.name, cfg, s, st["levels"], used(st))
        assert np.array_equal(d, want), (p.name, cfg, s)
        assert og.check_bfs(s, d, parent.cpu().numpy()) == 0
        assert st["reached"] == int((want >= 0).sum())
        # edges traversed: the degree sums of every frontier, mapped or not
        _, _, full = byo.bfs(g, s, small_frontier=0, use_graph=0)
        if st["variant_count"] == full["variant_count"]:
            assert st["edges"] == full["edges"]
        check_allowed(st, omit, True)


@pytest.mark.parametrize("cfg,omit", CONFIGS, ids=CFG_IDS)
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_cc_api_config(p, cfg, omit):
    g, og = build(p)
    want = og.cc()
    for shortcut in (1, 0):
        label, st = byo.cc(g, api_omit=omit, cc_shortcut=shortcut)
        assert np.array_equal(label.cpu().numpy(), want), (p.name, cfg, shortcut)
        check_allowed(st, omit, False)


@pytest.mark.parametrize("cfg,omit", CONFIGS, ids=CFG_IDS)
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_pagerank_api_config(p, cfg, omit):
    g, og = build(p)
    for iters in (1, 20):
        r32, _ = byo.pagerank(g, 0.85, iters, api_omit=omit)
        r64 = og.pagerank(0.85, iters)
        r = r32.cpu().numpy().astype(np.float64)
        err = np.max(np.abs(r - r64)) / np.max(np.abs(r64))
        assert err < PR_TOL, (p.name, cfg, iters, err)


@pytest.mark.parametrize("omit", [1, 4, 5, 16, 20, 24, 31])
@pytest.mark.parametrize("variant", range(6))
@pytest.mark.parametrize("p", MIXED, ids=MIXED_IDS)
def test_bfs_forced_variant_under_api(p, variant, omit):
    """Each variant, narrowed by what the container allows."""
    g, og = build(p)
    s = sources(og)[-1]
    depth, parent, st = byo.bfs(g, s, api_omit=omit, selector=byo.SEL_FIXED, fixed_variant=variant)
    want, _ = og.bfs(s)
    d = depth.cpu().numpy()
    assert np.array_equal(d, want), (p.name, variant, omit)
    assert og.check_bfs(s, d, parent.cpu().numpy()) == 0
    check_allowed(st, omit, True)


@pytest.mark.parametrize("omit", [1, 8, 9, 31])
@pytest.mark.parametrize("variant", range(6))
@pytest.mark.parametrize("p", MIXED, ids=MIXED_IDS)
def test_cc_forced_variant_under_api(p, variant, omit):
    g, og = build(p)
    label, st = byo.cc(g, api_omit=omit, selector=byo.SEL_FIXED, fixed_variant=variant)
    assert np.array_equal(label.cpu().numpy(), og.cc()), (p.name, variant, omit)
    check_allowed(st, omit, False)


def test_api_config_bypasses_tiled_and_graph_paths():
    """With functions left out, the tiled, captured and device-loop paths give
    way to the CSR level loop, with the same results."""
    p = gen.rmat_pairs(16, 16, seed=12)
    g, og = build(p)
    want, _ = og.bfs(0)
    depth, parent, st = byo.bfs(g, 0, api_omit=28, use_graph=1, small_frontier=8192)
    assert np.array_equal(depth.cpu().numpy(), want)
    assert st["device_levels"] == 0
    label, st = byo.cc(g, api_omit=9, tiled=1)
    assert np.array_equal(label.cpu().numpy(), og.cc())
    check_allowed(st, 9, False)  # the tiled rounds count as edge-balanced push or wavefront pull
    r32, _ = byo.pagerank(g, 0.85, 20, api_omit=9, pr_blocked=1)
    r64 = og.pagerank(0.85, 20)
    assert np.max(np.abs(r32.cpu().numpy() - r64)) / np.max(np.abs(r64)) < PR_TOL


@pytest.mark.parametrize("cfg,omit", CONFIGS, ids=CFG_IDS)
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_bc_api_config(p, cfg, omit):
    g, og = build(p)
    for s in sources(og):
        delta, sigma, depth, st = byo.bc(g, s, api_omit=omit)
        ws, wd, wdist = og.bc(s)
        assert np.array_equal(depth.cpu().numpy(), wdist), (p.name, cfg, s)
        small = ws < 2.0 ** 53
        assert np.array_equal(sigma.cpu().numpy()[small], ws[small])
        scale = max(1.0, float(np.max(np.abs(wd), initial=0.0)))
        assert np.max(np.abs(delta.cpu().numpy() - wd), initial=0.0) <= 1e-9 * scale
        _, _, _, full = byo.bc(g, s)
        assert st["edges"] == full["edges"]
        if omit & byo.API_NO_PAR_MAP:
            used = {k for k, c in st["variant_count"].items() if c}
            assert used <= {"push_thread", "pull_thread"}, used


@pytest.mark.parametrize("cfg,omit", CONFIGS, ids=CFG_IDS)
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_kcore_api_config(p, cfg, omit):
    g, og = build(p)
    core, st = byo.kcore(g, api_omit=omit)
    assert np.array_equal(core.cpu().numpy(), og.kcore()), (p.name, cfg)
    if omit & byo.API_NO_PAR_MAP:
        assert st["variant_count"]["push_edge"] == 0
    assert sum(st["variant_count"].values()) == st["levels"]
