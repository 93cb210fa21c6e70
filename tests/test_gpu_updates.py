"""Batch updates of the CSR container on the GPU (Section 4.1, the set-level
batch interface and its three batch forms; Section 4.2, the container's
insert_sorted_batch / delete_sorted_batch), against the oracle's set
semantics (oracle/updates.py):

- after an insert or delete the container's CSR equals, array for array, the
  oracle's graph with the batch's undirected edges added or removed; batches
  hold self-pairs, repeated pairs, edges already present and edges absent;
- BFS, connectivity and PageRank on the updated container match the oracle
  on the updated graph (the tile layout and other derived structures are
  rebuilt);
- the three batch forms: the global sort is exact, the semisort and the
  grouped sort are valid by the oracle's checks;
- a batch naming a vertex outside [0, n) is refused and changes nothing.
"""
import numpy as np
import pytest

import oracle
from oracle import updates
from paper_2405_11671_amd import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")

PR_TOL = 1e-5
PAPER_UPDATE_ABCD = (0.5, 0.1, 0.1, 0.3)   # the update batches' generator setting (Section 6.6)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).to("cuda")


def mixed_batch(p, og, k, seed):
    """k pairs: RMAT draws over the graph's vertices, plus self-pairs,
    repeats and edges the graph already has."""
    rng = np.random.default_rng(seed)
    scale = max(1, int(np.ceil(np.log2(max(p.n, 2)))))
    q = gen.rmat_pairs(scale, 1, PAPER_UPDATE_ABCD, seed=seed)
    keep = (q.src < p.n) & (q.dst < p.n)
    s, d = q.src[keep][: k], q.dst[keep][: k]
    off, nbr = og.export()
    if og.m:
        e = rng.integers(0, og.m, max(1, k // 8))
        u = np.searchsorted(off, e, side="right") - 1
        s = np.concatenate([s, u.astype(np.int32)])
        d = np.concatenate([d, nbr[e]])
    v = rng.integers(0, p.n, max(1, k // 16)).astype(np.int32)
    s = np.concatenate([s, v, s[: k // 8]])            # self-pairs and repeats
    d = np.concatenate([d, v, d[: k // 8]])
    perm = rng.permutation(s.size)
    return s[perm].astype(np.int32), d[perm].astype(np.int32)


def same_csr(g, og):
    off, nbr = g.csr()
    want_off, want_nbr = og.export()
    assert g.n == og.n and g.num_edges() == og.m
    assert np.array_equal(off, want_off), "offsets differ from the oracle"
    assert np.array_equal(nbr, want_nbr), "neighbour lists differ from the oracle"


def check_traversals(g, og, srcs):
    for s in srcs:
        d, par, _ = byo.bfs(g, int(s))
        want, _ = og.bfs(int(s))
        assert np.array_equal(d.cpu().numpy(), want)
        assert og.check_bfs(int(s), d.cpu().numpy(), par.cpu().numpy()) == 0
    lab, _ = byo.cc(g, tiled=1)
    assert np.array_equal(lab.cpu().numpy(), og.cc())
    r, _ = byo.pagerank(g, 0.85, 10, pr_blocked=1)
    r64 = og.pagerank(0.85, 10)
    assert float(np.max(np.abs(r.cpu().numpy() - r64)) / np.max(np.abs(r64))) < PR_TOL


CASES = [
    ("er12", lambda: gen.er_pairs(1 << 12, 6, seed=21), 3000, 51),
    ("rmat16", lambda: gen.rmat_pairs(16, 16, seed=22), 40000, 52),
    ("grid", lambda: gen.grid_pairs(60, 50, 0.1, seed=23), 800, 53),
    ("rmat18_big_batch", lambda: gen.rmat_pairs(18, 8, seed=24), 600000, 54),
]


@pytest.mark.parametrize("name,mk,k,seed", CASES, ids=[c[0] for c in CASES])
def test_insert_then_delete_match_the_oracle(name, mk, k, seed):
    p = mk()
    g, og = byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p)
    s, d = mixed_batch(p, og, k, seed=seed)
    m0 = g.m
    added = g.insert_batch(dev(s), dev(d))
    og_ins = updates.insert_batch(og, s, d)
    same_csr(g, og_ins)
    assert added == og_ins.m - m0
    srcs = gen.pick_sources(p, 2, seed=5)
    check_traversals(g, og_ins, srcs)
    # inserting the same batch again changes nothing
    assert g.insert_batch(dev(s), dev(d)) == 0
    same_csr(g, og_ins)
    # delete half of the batch (present edges and now-missing ones mixed)
    h = s.size // 2
    removed = g.delete_batch(dev(s[:h]), dev(d[:h]))
    og_del = updates.delete_batch(og_ins, s[:h], d[:h])
    same_csr(g, og_del)
    assert removed == og_ins.m - og_del.m
    check_traversals(g, og_del, srcs)


def test_insert_into_empty_graph_and_delete_everything():
    n = 5000
    p = gen.Pairs(n, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty")
    g, og = byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p)
    q = gen.er_pairs(n, 8, seed=31)
    g.insert_batch(dev(q.src), dev(q.dst))
    og2 = updates.insert_batch(og, q.src, q.dst)
    same_csr(g, og2)
    st = g.stats()
    assert st["max_degree"] == int(og2.degrees().max()) and st["isolated"] == int((og2.degrees() == 0).sum())
    g.delete_batch(dev(q.src), dev(q.dst))
    same_csr(g, og)
    assert g.stats()["isolated"] == n


def test_batch_outside_the_vertex_range_is_refused():
    p = gen.er_pairs(1 << 10, 4, seed=32)
    g, og = byo.Graph.from_pairs(p), oracle.Graph.from_pairs(p)
    for s, d in (([0, 5, 1 << 10], [1, 6, 0]), ([3, -1], [4, 2])):
        for fn in (g.insert_batch, g.delete_batch):
            with pytest.raises(byo.ByoError, match="EINVAL"):
                fn(dev(s), dev(d))
            same_csr(g, og)


@pytest.mark.parametrize("k", [1, 17, 5000, 300000])
def test_batch_forms(k):
    n = 1 << 16
    q = gen.rmat_pairs(16, 1, PAPER_UPDATE_ABCD, seed=40 + k)
    rng = np.random.default_rng(k)
    idx = rng.integers(0, q.npairs, k)               # with repeats
    s, d = q.src[idx].astype(np.int32), q.dst[idx].astype(np.int32)
    ws, wd = updates.sort_batch(s, d)
    out_s, out_d = byo.batch_order(dev(s), dev(d), n, byo.FORM_SORT)
    assert np.array_equal(out_s.cpu().numpy(), ws) and np.array_equal(out_d.cpu().numpy(), wd)
    out_s, out_d = byo.batch_order(dev(s), dev(d), n, byo.FORM_SEMISORT)
    assert updates.is_semisorted(s, d, out_s.cpu().numpy(), out_d.cpu().numpy())
    out_s, out_d = byo.batch_order(dev(s), dev(d), n, byo.FORM_GROUPED_SORT)
    assert updates.is_grouped_sorted(s, d, out_s.cpu().numpy(), out_d.cpu().numpy())
    with pytest.raises(byo.ByoError, match="EINVAL"):
        bad = s.copy()
        bad[-1] = n
        byo.batch_order(dev(bad), dev(d), n, byo.FORM_SEMISORT)
