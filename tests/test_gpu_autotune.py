"""Autotuner: tuned options keep results exact and never lose to the defaults."""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")
from paper_2405_11671_amd import autotune  # noqa: E402


def test_autotune_bfs_and_batch(tmp_path):
    cache = str(tmp_path / "tune.json")
    p = gen.grid_pairs(256, 256, 0.1, seed=8)
    g, og = byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p)
    srcs = gen.pick_sources(p, 2, seed=2)
    opts, rep = autotune.tune_bfs(g, srcs, repeats=2, cache=cache)
    assert rep["tuned_ms"] <= rep["default_ms"] * 1.05
    for s in srcs:
        d, par, _ = byo.bfs(g, int(s), opts=byo.default_opts(**opts))
        want, _ = og.bfs(int(s))
        assert np.array_equal(d.cpu().numpy(), want)
        assert og.check_bfs(int(s), d.cpu().numpy(), par.cpu().numpy()) == 0
    # cached
    again, rep2 = autotune.tune_bfs(g, srcs, cache=cache)
    assert again == opts and rep2 == rep

    plist = gen.batch_pairs(16, seed=5, log2_hi=14.0)
    B = byo.Batch.from_pairs(plist)
    ogs = [oracle.Graph.from_pairs(q) for q in plist]
    bsrc = [int(np.flatnonzero(o.degrees())[0]) for o in ogs]
    bopts, brep = autotune.tune_batch(B, bsrc, repeats=2, cache=cache)
    depth, _, _ = B.bfs(bsrc, opts=byo.default_opts(**bopts))
    for i, d in enumerate(B.split(depth.cpu().numpy())):
        assert np.array_equal(d, ogs[i].bfs(bsrc[i])[0])
