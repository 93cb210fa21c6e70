"""Pins for the batch-update oracle (Section 4, the batch-update interface).

The oracle is checked against plain Python sets of undirected edges on tiny
graphs, against the algebra that set insertion and deletion obey at any size
(idempotence, batches that merge, deletion undoing insertion, degree changes
counted edge by edge), and its batch-form checkers against planted invalid
orders.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from oracle import updates
from paper_2405_11671_amd import gen


def undirected(g):
    return {frozenset((v, int(u))) for v in range(g.n) for u in g.neighbors(v)}


def same_graph(g, h):
    return g.n == h.n and np.array_equal(updates.edge_keys(g), updates.edge_keys(h))


graph_and_batch = st.integers(1, 25).flatmap(lambda n: st.tuples(
    st.just(n),
    st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=3 * n),
    st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)), max_size=2 * n)))


@settings(max_examples=80, deadline=None)
@given(graph_and_batch)
def test_updates_match_python_edge_sets(case):
    n, pairs, batch = case
    g = oracle.Graph(n, np.array([p[0] for p in pairs], np.int32), np.array([p[1] for p in pairs], np.int32))
    bs = np.array([p[0] for p in batch], np.int64)
    bd = np.array([p[1] for p in batch], np.int64)
    before = undirected(g)
    change = {frozenset(p) for p in batch if p[0] != p[1]}
    ins = updates.insert_batch(g, bs, bd)
    assert undirected(ins) == before | change
    dele = updates.delete_batch(g, bs, bd)
    assert undirected(dele) == before - change
    for h in (ins, dele):                      # symmetric and simple, like the static container
        for v in range(n):
            nb = h.neighbors(v).tolist()
            assert nb == sorted(set(nb)) and v not in nb


def scale_case(seed=7):
    p = gen.rmat_pairs(12, 8, seed=3)
    g = oracle.Graph.from_pairs(p)
    rng = np.random.default_rng(seed)
    k = 6000
    bs = rng.integers(0, g.n, k)
    bd = rng.integers(0, g.n, k)
    bs[:200] = bd[:200]                         # self-loops change nothing
    bs[200:400], bd[200:400] = bs[400:600], bd[400:600]   # repeated pairs act once
    off, nbr = g.export()
    u = np.repeat(np.arange(g.n), np.diff(off))
    pick = rng.integers(0, nbr.size, 300)       # pairs already in the graph, some reversed
    bs[600:900], bd[600:900] = nbr[pick], u[pick]
    return g, bs, bd


def test_insert_and_delete_algebra_at_scale():
    g, bs, bd = scale_case()
    ins = updates.insert_batch(g, bs, bd)
    assert same_graph(updates.insert_batch(ins, bs, bd), ins)                    # idempotent
    assert same_graph(updates.delete_batch(ins, bs, bd), updates.delete_batch(g, bs, bd))
    assert same_graph(updates.insert_batch(updates.delete_batch(g, bs, bd), bs, bd), ins)
    h = len(bs) // 2                                                               # batches merge
    two = updates.insert_batch(updates.insert_batch(g, bs[:h], bd[:h]), bs[h:], bd[h:])
    assert same_graph(two, ins)
    off, nbr = g.export()
    u = np.repeat(np.arange(g.n), np.diff(off))
    assert same_graph(updates.insert_batch(g, u, nbr), g)                          # own edges: no change
    emptied = updates.delete_batch(g, u, nbr)
    assert emptied.m == 0 and emptied.n == g.n


def test_degree_changes_counted_edge_by_edge():
    g, bs, bd = scale_case(seed=11)
    have = {(v, int(w)) for v in range(g.n) for w in g.neighbors(v)}
    new = {(a, b) for a, b in zip(bs.tolist(), bd.tolist()) if a != b and (a, b) not in have}
    new |= {(b, a) for a, b in new}
    ins = updates.insert_batch(g, bs, bd)
    assert ins.m == g.m + len(new)
    gain = np.zeros(g.n, np.int64)
    for a, _ in new:
        gain[a] += 1
    assert np.array_equal(ins.degrees(), g.degrees() + gain)
    gone = {(a, b) for a, b in zip(bs.tolist(), bd.tolist()) if (a, b) in have}
    gone |= {(b, a) for a, b in gone}
    dele = updates.delete_batch(g, bs, bd)
    assert dele.m == g.m - len(gone)
    loss = np.zeros(g.n, np.int64)
    for a, _ in gone:
        loss[a] += 1
    assert np.array_equal(dele.degrees(), g.degrees() - loss)


def test_batch_forms():
    rng = np.random.default_rng(5)
    s = rng.integers(0, 40, 500)
    d = rng.integers(0, 1000, 500)
    gs, gd = updates.sort_batch(s, d)
    assert list(zip(gs.tolist(), gd.tolist())) == sorted(zip(s.tolist(), d.tolist()))
    assert updates.is_semisorted(s, d, gs, gd) and updates.is_grouped_sorted(s, d, gs, gd)
    # a semisort in a shuffled order of sources, groups left unsorted
    perm = rng.permutation(40)
    order = np.argsort(perm[s], kind="stable")
    ss, sd = s[order], d[order]
    assert updates.is_semisorted(s, d, ss, sd)
    assert not updates.is_grouped_sorted(s, d, ss, sd)
    # the same with each group sorted by target
    order = np.lexsort((d, perm[s]))
    assert updates.is_grouped_sorted(s, d, s[order], d[order])
    # planted faults: a split group, a changed pair, a dropped pair
    split = np.concatenate([ss[1:], ss[:1]]), np.concatenate([sd[1:], sd[:1]])
    if split[0][0] != split[0][-1]:
        assert not updates.is_semisorted(s, d, *split)
    bad = sd.copy()
    bad[7] += 1
    assert not updates.is_semisorted(s, d, ss, bad)
    assert not updates.is_semisorted(s, d, ss[1:], sd[1:])
    assert updates.is_semisorted([], [], [], [])


def test_out_of_range_batch_is_an_error():
    g = oracle.Graph(4, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(ValueError):
        updates.insert_batch(g, [0], [4])
    with pytest.raises(ValueError):
        updates.delete_batch(g, [-1], [0])
