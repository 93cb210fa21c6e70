"""Parity at the benchmark's own sizes (RMAT-22, the launch configuration bench.py
times) and at a mid size, for both PageRank layouts."""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")

PR_TOL = 1e-5


@pytest.fixture(scope="module")
def rmat22():
    p = gen.rmat_pairs(22, 16, seed=1)
    return p, byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p)


def pr_err(a, b):
    return float(np.max(np.abs(a.astype(np.float64) - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("blocked", [1, 0])
def test_pagerank_rmat21_blocked_and_plain(blocked):
    p = gen.rmat_pairs(21, 16, seed=3)
    g, og = byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p)
    r, _ = byo.pagerank(g, 0.85, 6, pr_blocked=blocked)
    assert pr_err(r.cpu().numpy(), og.pagerank(0.85, 6)) < PR_TOL


def test_pagerank_rmat22_full(rmat22):
    p, g, og = rmat22
    r, _ = byo.pagerank(g, 0.85, 20)
    r64 = og.pagerank(0.85, 20)
    got = r.cpu().numpy()
    assert pr_err(got, r64) < PR_TOL
    assert abs(got.astype(np.float64).sum() - 1.0) < 1e-4
    for layout in (0, 1):
        r2, _ = byo.pagerank(g, 0.85, 20, pr_blocked=layout)
        assert pr_err(r2.cpu().numpy(), r64) < PR_TOL, layout


def test_bfs_cc_rmat22_full(rmat22):
    p, g, og = rmat22
    for s in gen.pick_sources(p, 2, seed=2):
        d, par, _ = byo.bfs(g, int(s))
        want, _ = og.bfs(int(s))
        assert np.array_equal(d.cpu().numpy(), want)
        assert og.check_bfs(int(s), d.cpu().numpy(), par.cpu().numpy()) == 0
    want = og.cc()
    for tiled in (0, 1):
        lab, _ = byo.cc(g, tiled=tiled)
        assert np.array_equal(lab.cpu().numpy(), want), tiled


def test_kcore_rmat22_full(rmat22):
    """Coreness at the benchmark's size (244 distinct values, 768 sub-rounds),
    in one persistent launch and through the host-driven loop."""
    p, g, og = rmat22
    want = og.kcore()
    subs = []
    for persistent in (1, 0):
        core, st = byo.kcore(g, persistent=persistent)
        got = core.cpu().numpy()
        assert np.array_equal(got, want), (persistent, int(np.sum(got != want)))
        subs.append(st["levels"])
    assert subs[0] == subs[1]


# eight columns in each of the four 64-source words of the benchmark's
# 256-source batch (first and last lane of every word included)
MS_COLUMNS = [64 * w + j for w in range(4) for j in (0, 9, 18, 27, 36, 45, 54, 63)]


def test_msbfs_rmat22_sampled_columns(rmat22):
    p, g, og = rmat22
    srcs = gen.pick_sources(p, 256, seed=2)
    assert len(srcs) == 256
    want = {j: og.bfs(int(srcs[j]))[0] for j in MS_COLUMNS}
    for tiled in (1, 0):
        D, st = byo.msbfs(g, srcs, tiled=tiled)
        D = D.cpu().numpy()
        for j in MS_COLUMNS:
            assert np.array_equal(D[:, j], np.where(want[j] < 0, 255, want[j])), (tiled, j)
        assert st["reached"] == int((D != 255).sum())
