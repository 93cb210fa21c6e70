"""The BFS entry point that allocates nothing (byo_bfs_noalloc), called
through the C ABI, against byo_bfs: depths bit-exact, parents a valid BFS
tree (several are correct). Two calls in a row share the device scratch
array, the second on a smaller graph, so a value left over from the first
call would show; a third call repeats the first graph after the smaller one.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import _lib, gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


def _noalloc(g, src, depth, parent, opts):
    stt = _lib.RunStats()
    status = _lib.load().byo_bfs_noalloc(g.handle, int(src), ctypes.c_void_p(depth.data_ptr()),
                                         ctypes.c_void_p(parent.data_ptr()), ctypes.byref(opts),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                         ctypes.byref(stt))
    _lib.check(status)
    return stt


# a graph near the scratch limit (RMAT-20 with ef 8: skewed, pull and push
# levels), then a small ER graph, then the first graph again
CASES = [
    ("rmat20", lambda: gen.rmat_pairs(20, 8, seed=5)),
    ("er12", lambda: gen.er_pairs(1 << 12, 6, seed=6)),
]


@pytest.mark.parametrize("selector", [byo.SEL_HEURISTIC, byo.SEL_FIXED])
def test_noalloc_matches_bfs_two_calls_second_smaller(selector):
    graphs = []
    for name, mk in CASES:
        p = mk()
        graphs.append((name, byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p), p))
    order = [0, 1, 0]
    for i in order:
        name, g, og, p = graphs[i]
        srcs = [0] + [int(s) for s in gen.pick_sources(p, 2, seed=7)]
        for src in srcs:
            for variant in ([byo.V_PUSH_EDGE] if selector == byo.SEL_HEURISTIC else [byo.V_PUSH_BUCKET,
                                                                                        byo.V_PULL_WAVE]):
                o = byo.default_opts(selector=selector, fixed_variant=variant)
                print(f"[noalloc] graph={name} n={g.n} src={src} selector={selector} variant={variant}", flush=True)
                # outputs poisoned so that an unwritten entry shows
                d_na = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
                p_na = torch.full((g.n,), 7, dtype=torch.int32, device="cuda")
                st_na = _noalloc(g, src, d_na, p_na, o)
                d_ref, p_ref, st_ref = byo.bfs(g, src, opts=o)
                torch.cuda.synchronize()
                got = d_na.cpu().numpy()
                assert np.array_equal(got, d_ref.cpu().numpy()), f"{name} src {src}: depths differ from byo_bfs"
                assert np.array_equal(got, og.bfs(src)[0]), f"{name} src {src}: depths differ from the oracle"
                assert og.check_bfs(src, got, p_na.cpu().numpy()) == 0, f"{name} src {src}: parents invalid"
                assert st_na.levels == st_ref["levels"] and st_na.reached == st_ref["reached"]
                assert st_na.edges == st_ref["edges"]


def test_noalloc_rejects_what_it_cannot_run():
    small = byo.Graph.from_pairs(gen.er_pairs(1 << 10, 4, seed=8))
    d = torch.empty(small.n, dtype=torch.int32, device="cuda")
    q = torch.empty(small.n, dtype=torch.int32, device="cuda")
    for kw in ({"use_graph": 1}, {"small_frontier": 64}, {"compressed": 1}, {"api_omit": 1}):
        with pytest.raises(byo.ByoError, match="EINVAL"):
            _noalloc(small, 0, d, q, byo.default_opts(**kw))
    with pytest.raises(byo.ByoError, match="EINVAL"):
        _noalloc(small, small.n, d, q, byo.default_opts())
    big = byo.Graph.from_pairs(gen.Pairs(_lib.NOALLOC_MAX_N + 1, np.array([0], np.int32), np.array([1], np.int32),
                                         "over"))
    d2 = torch.empty(big.n, dtype=torch.int32, device="cuda")
    q2 = torch.empty(big.n, dtype=torch.int32, device="cuda")
    with pytest.raises(byo.ByoError, match="EINVAL"):
        _noalloc(big, 0, d2, q2, byo.default_opts())
    # a rejected call leaves the scratch usable
    _noalloc(small, 0, d, q, byo.default_opts())
    og = oracle.Graph.from_pairs(gen.er_pairs(1 << 10, 4, seed=8))
    assert np.array_equal(d.cpu().numpy(), og.bfs(0)[0])
