"""Pins for the CPU oracle against mathematics it does not share code with.

Every check compares the oracle with something other than itself: brute force
(Floyd-Warshall, union-find), library routines (scipy.sparse.csgraph,
numpy.linalg.solve, torch.autograd), closed forms (paths, cycles, stars,
cliques, lattices, regular graphs) and invariants (sum of ranks is 1).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
from hypothesis import given, settings, strategies as st

import oracle
from oracle import mlp
from tests import brute


def G(n, pairs):
    a = np.array([p[0] for p in pairs], np.int32)
    b = np.array([p[1] for p in pairs], np.int32)
    return oracle.Graph(n, a, b), a, b


tiny_graphs = st.integers(1, 40).flatmap(
    lambda n: st.tuples(st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)),
                                             max_size=3 * n)))


# ---------------------------------------------------------------- graph build

@settings(max_examples=60, deadline=None)
@given(tiny_graphs)
def test_neighbour_sets_match_edge_set(case):
    n, pairs = case
    g, a, b = G(n, pairs)
    E = brute.simple_edges(n, a, b)
    assert g.m == 2 * len(E)
    for v in range(n):
        want = sorted({y for (x, y) in E if x == v} | {x for (x, y) in E if y == v})
        assert g.neighbors(v).tolist() == want
    off, nbr = g.export()
    assert off[0] == 0 and off[-1] == g.m and np.all(np.diff(off) >= 0)


def test_rejects_out_of_range_pairs():
    with pytest.raises(ValueError):
        oracle.Graph(3, np.array([0], np.int32), np.array([3], np.int32))


# ---------------------------------------------------------------- BFS

@settings(max_examples=80, deadline=None)
@given(tiny_graphs, st.integers(0, 10 ** 6))
def test_bfs_matches_floyd_warshall_and_scipy(case, s):
    n, pairs = case
    g, a, b = G(n, pairs)
    src = s % n
    depth, parent = g.bfs(src)
    A = brute.adjacency_matrix(n, a, b)
    D = brute.floyd_warshall_hops(A)
    assert depth.tolist() == D[src].tolist()
    sd = csg.shortest_path(sp.csr_matrix(A), unweighted=True, indices=src)
    want = np.where(np.isinf(sd), -1, sd).astype(np.int64)
    assert depth.tolist() == want.tolist()
    # parent validity checked independently of the oracle's checker
    for v in range(n):
        if depth[v] < 0:
            assert parent[v] == -1
        elif v == src:
            assert parent[v] == src
        else:
            p = parent[v]
            assert A[p, v] == 1 and depth[p] == depth[v] - 1
    assert g.check_bfs(src, depth, parent) == 0


def test_bfs_closed_forms():
    n = 50
    g, _, _ = G(n, [(i, i + 1) for i in range(n - 1)])          # path
    assert g.bfs(7)[0].tolist() == [abs(v - 7) for v in range(n)]
    g, _, _ = G(n, [(i, (i + 1) % n) for i in range(n)])         # cycle
    assert g.bfs(3)[0].tolist() == [min(abs(v - 3), n - abs(v - 3)) for v in range(n)]
    g, _, _ = G(n, [(0, i) for i in range(1, n)])                # star
    assert g.bfs(0)[0].tolist() == [0] + [1] * (n - 1)
    assert g.bfs(5)[0].tolist() == [1] + [2 if v != 5 else 0 for v in range(1, n)]
    k = 12
    g, _, _ = G(k, [(i, j) for i in range(k) for j in range(i + 1, k)])  # clique
    assert g.bfs(4)[0].tolist() == [0 if v == 4 else 1 for v in range(k)]
    R, C = 9, 13                                                  # full lattice: Manhattan
    pairs = [(r * C + c, r * C + c + 1) for r in range(R) for c in range(C - 1)]
    pairs += [(r * C + c, (r + 1) * C + c) for r in range(R - 1) for c in range(C)]
    g, _, _ = G(R * C, pairs)
    s = 3 * C + 5
    assert g.bfs(s)[0].tolist() == [abs(v // C - 3) + abs(v % C - 5) for v in range(R * C)]
    g, _, _ = G(6, [])                                            # no edges
    d, p = g.bfs(2)
    assert d.tolist() == [-1, -1, 0, -1, -1, -1] and p.tolist() == [-1, -1, 2, -1, -1, -1]


def test_bfs_checker_catches_planted_mistakes():
    # 3 is at depth 2 with two valid parents (1 and 4); 5 only has a self-loop
    g, a, b = G(6, [(0, 1), (1, 2), (1, 3), (0, 4), (4, 3), (5, 5)])
    d, p = g.bfs(0)
    assert d.tolist() == [0, 1, 2, 2, 1, -1]
    assert g.check_bfs(0, d, p) == 0
    bad = d.copy(); bad[3] += 1
    assert g.check_bfs(0, bad, p) > 0                 # wrong depth
    bad = p.copy(); bad[3] = 2                        # 2 is not adjacent to 3
    assert g.check_bfs(0, d, bad) > 0
    bad = p.copy(); bad[2] = 4                        # 4 is not adjacent to 2
    assert g.check_bfs(0, d, bad) > 0
    bad = p.copy(); bad[2] = 2                        # a vertex at the same depth
    assert g.check_bfs(0, d, bad) > 0
    bad = p.copy(); bad[0] = -1                       # root must be its own parent
    assert g.check_bfs(0, d, bad) > 0
    bad = p.copy(); bad[5] = 0                        # unreached must stay -1
    assert g.check_bfs(0, d, bad) > 0
    alt = p.copy(); alt[3] = 4 if p[3] == 1 else 1    # the other valid parent is accepted
    assert g.check_bfs(0, d, alt) == 0


# ---------------------------------------------------------------- CC

@settings(max_examples=80, deadline=None)
@given(tiny_graphs)
def test_cc_matches_union_find_and_scipy(case):
    n, pairs = case
    g, a, b = G(n, pairs)
    lab = g.cc()
    assert lab.tolist() == brute.union_find_min_labels(n, a, b).tolist()
    ncomp, comp = csg.connected_components(sp.csr_matrix(brute.adjacency_matrix(n, a, b)), directed=False)
    mins = {}
    for v in range(n):
        mins.setdefault(comp[v], v)
    assert lab.tolist() == [mins[comp[v]] for v in range(n)]
    assert len(set(lab.tolist())) == ncomp


def test_cc_closed_forms():
    g, _, _ = G(5, [])
    assert g.cc().tolist() == [0, 1, 2, 3, 4]
    # disjoint cliques {7,2,9}, {1,4}, {0,3,5,6,8}
    cl = [[7, 2, 9], [1, 4], [0, 3, 5, 6, 8]]
    pairs = [(c[i], c[j]) for c in cl for i in range(len(c)) for j in range(i + 1, len(c))]
    g, _, _ = G(10, pairs)
    want = [0] * 10
    for c in cl:
        for v in c:
            want[v] = min(c)
    assert g.cc().tolist() == want


# ---------------------------------------------------------------- PageRank

@settings(max_examples=40, deadline=None)
@given(tiny_graphs, st.sampled_from([0.85, 0.5, 0.99]), st.integers(0, 25))
def test_pagerank_matches_dense_power_iteration(case, d, T):
    n, pairs = case
    g, a, b = G(n, pairs)
    p = g.pagerank(d, T)
    want = brute.pagerank_power(brute.adjacency_matrix(n, a, b), d, T)
    assert np.max(np.abs(p - want)) < 1e-13
    assert abs(p.sum() - 1.0) < 1e-12


@settings(max_examples=30, deadline=None)
@given(tiny_graphs)
def test_pagerank_converges_to_linear_solve(case):
    n, pairs = case
    g, a, b = G(n, pairs)
    p = g.pagerank(0.85, 300)
    want = brute.pagerank_fixed_point(brute.adjacency_matrix(n, a, b), 0.85)
    assert np.max(np.abs(p - want)) < 1e-12


def test_pagerank_closed_forms():
    n = 30
    for pairs in ([(i, (i + 1) % n) for i in range(n)],                       # cycle
                  [(i, j) for i in range(n) for j in range(i + 1, n)],         # clique
                  []):                                                          # no edges
        g, _, _ = G(n, pairs)
        assert np.allclose(g.pagerank(0.85, 20), 1.0 / n, rtol=0, atol=1e-15)
    # star K_{1,k}: fixed point of the centre is ((1-d)/n + d) / (1 + d)
    k, d = 9, 0.85
    n = k + 1
    g, _, _ = G(n, [(0, i) for i in range(1, n)])
    p = g.pagerank(d, 400)
    pc = ((1 - d) / n + d) / (1 + d)
    assert abs(p[0] - pc) < 1e-14
    assert np.allclose(p[1:], (1 - pc) / k, rtol=0, atol=1e-14)


def test_pagerank_closed_forms_at_scale():
    """A star is a two-state chain: the centre receives every leaf's whole
    mass and the leaves share the centre's, so from the uniform start
    p_c(t + 1) = (1 - d)/n + d (1 - p_c(t)), that is
    p_c(T) = p* + (1/n - p*)(-d)^T with p* = ((1 - d)/n + d)/(1 + d), and each
    leaf holds (1 - p_c)/k. A 4-regular torus keeps the uniform vector at every
    step. Both at sizes where an indexing or accumulation slip would show."""
    k, d = 200_000, 0.85
    n = k + 1
    g = oracle.Graph(n, np.zeros(k, np.int32), np.arange(1, n, dtype=np.int32))
    ps = ((1 - d) / n + d) / (1 + d)
    # the centre sums k terms of total mass <= 1 in sequence: rounding within
    # (k - 1) u (Higham's bound for recursive summation, u = 2^-53); a dropped
    # or misplaced term would move it by at least 1/n
    tol_c = 2 * k * 2.0 ** -53
    for T in (1, 2, 5, 20):
        p = g.pagerank(d, T)
        pc = ps + (1.0 / n - ps) * (-d) ** T
        assert abs(p[0] - pc) < tol_c, T
        assert np.max(np.abs(p[1:] - (1 - pc) / k)) < 2 * tol_c / k, T
    R, C = 300, 300
    v = np.arange(R * C, dtype=np.int32)
    right = (v // C) * C + (v % C + 1) % C
    down = (v + C) % (R * C)
    t = oracle.Graph(R * C, np.concatenate([v, v]), np.concatenate([right, down]).astype(np.int32))
    assert np.all(t.degrees() == 4)
    assert np.max(np.abs(t.pagerank(d, 20) - 1.0 / (R * C))) < 1e-18


def test_pagerank_one_step_exact_fractions():
    # path 0-1-2 plus isolated 3, one step from 1/4 each, in exact rationals
    g, _, _ = G(4, [(0, 1), (1, 2)])
    d = Fraction(85, 100)
    n = 4
    p0 = Fraction(1, 4)
    D = p0                                    # vertex 3 has degree 0
    base = (1 - d) / n + d * D / n
    want = [base + d * (p0 / 2), base + d * (p0 + p0), base + d * (p0 / 2), base]
    got = g.pagerank(0.85, 1)
    assert np.max(np.abs(got - np.array([float(x) for x in want]))) < 1e-16


# ---------------------------------------------------------------- MS-BFS

@settings(max_examples=30, deadline=None)
@given(tiny_graphs, st.integers(1, 9))
def test_msbfs_columns_are_single_bfs(case, k):
    n, pairs = case
    g, a, b = G(n, pairs)
    srcs = np.array([(7 * j + 3) % n for j in range(k)], np.int64)
    D = g.msbfs(srcs)
    for j in range(k):
        d, _ = g.bfs(int(srcs[j]))
        assert D[:, j].tolist() == np.where(d < 0, 255, d).tolist()


# ---------------------------------------------------------------- MLP

def _params(F, H, K, rng):
    return {k: rng.standard_normal(s) * 0.5 for k, s in mlp.shapes(F, H, K).items()}


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(4)
    F, H, K, N = 5, 7, 4, 11
    p = _params(F, H, K, rng)
    X, Y = rng.standard_normal((N, F)), rng.standard_normal((N, K))
    M = (rng.random((N, K)) < 0.7).astype(float)
    _, g = mlp.loss_and_grads(p, X, Y, M)
    h = 1e-6
    for name in mlp.PARAM_NAMES:
        num = np.zeros_like(p[name])
        for idx in np.ndindex(*p[name].shape):
            old = p[name][idx]
            p[name][idx] = old + h
            lp = mlp.loss(mlp.forward(p, X)[0], Y, M)
            p[name][idx] = old - h
            lm = mlp.loss(mlp.forward(p, X)[0], Y, M)
            p[name][idx] = old
            num[idx] = (lp - lm) / (2 * h)
        rel = np.linalg.norm(num - g[name]) / max(np.linalg.norm(num), 1e-12)
        assert rel < 1e-6, name


def test_mlp_backward_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    F, H, K, N = 12, 32, 7, 64
    p = _params(F, H, K, rng)
    X, Y = rng.standard_normal((N, F)), rng.standard_normal((N, K))
    M = (rng.random((N, K)) < 0.5).astype(float)
    L, g = mlp.loss_and_grads(p, X, Y, M)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    Xt, Yt, Mt = (torch.tensor(a, dtype=torch.float64) for a in (X, Y, M))
    h1 = torch.relu(Xt @ tp["W1"] + tp["b1"])
    h2 = torch.relu(h1 @ tp["W2"] + tp["b2"])
    out = h2 @ tp["W3"] + tp["b3"]
    lt = (Mt * (out - Yt) ** 2).sum() / Mt.sum().clamp(min=1)
    lt.backward()
    assert abs(lt.item() - L) < 1e-12
    for k in mlp.PARAM_NAMES:
        assert np.allclose(tp[k].grad.numpy(), g[k], rtol=1e-11, atol=1e-13), k


def test_adam_first_step_closed_form():
    # with zero moments, bias correction makes the first step lr * g / (|g| + eps)
    rng = np.random.default_rng(6)
    p = _params(3, 4, 2, rng)
    g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
    st_ = mlp.adam_init(p)
    q = mlp.adam_step({k: v.copy() for k, v in p.items()}, g, st_, 1, lr=0.01)
    for k in mlp.PARAM_NAMES:
        assert np.allclose(p[k] - q[k], 0.01 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12, atol=1e-15)


def test_training_fits_a_learnable_target():
    rng = np.random.default_rng(7)
    F, H, K, N = 4, 16, 3, 256
    X = rng.standard_normal((N, F))
    Y = np.stack([X[:, 0] * 2 - X[:, 1], np.abs(X[:, 2]), X[:, 3] ** 2], axis=1)
    M = np.ones_like(Y)
    p0 = _params(F, H, K, rng)
    _, losses = mlp.train(p0, X, Y, M, 1500, lr=3e-3)
    assert losses[-1] < 0.05 * losses[0]


def test_predict_argmin_respects_mask_and_ties():
    p = {k: np.zeros(s) for k, s in mlp.shapes(2, 3, 4).items()}
    p["b3"] = np.array([1.0, 0.5, 0.5, 2.0])
    X = np.zeros((2, 2))
    assert mlp.predict_argmin(p, X).tolist() == [1, 1]
    assert mlp.predict_argmin(p, X, allowed=[[True, False, True, True]] * 2).tolist() == [2, 2]


# ---------------------------------------------------------------- golden fixture

# ---------------------------------------------------------------- single-source betweenness

@settings(max_examples=60, deadline=None)
@given(st.integers(1, 9).flatmap(
    lambda n: st.tuples(st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)),
                                             max_size=2 * n))), st.integers(0, 10 ** 6))
def test_bc_definition_matches_path_enumeration(case, s):
    n, pairs = case
    g, a, b = G(n, pairs)
    s = s % n
    want, counts = brute.dependency_by_enumeration(n, a, b, s)
    got = g.bc_definition(s)
    assert np.allclose(got, [float(x) for x in want], rtol=1e-12, atol=1e-12)
    sigma, delta, dist = g.bc(s)
    for v in range(n):
        assert sigma[v] == counts.get(v, 0)
    assert np.allclose(delta, [float(x) for x in want], rtol=1e-12, atol=1e-12)


@settings(max_examples=40, deadline=None)
@given(tiny_graphs, st.integers(0, 10 ** 6))
def test_bc_recurrence_matches_definition(case, s):
    n, pairs = case
    g, a, b = G(n, pairs)
    s = s % n
    sigma, delta, dist = g.bc(s)
    assert np.allclose(delta, g.bc_definition(s), rtol=1e-12, atol=1e-12)
    want_d, _ = g.bfs(s)
    assert np.array_equal(dist, want_d)
    assert np.all((sigma > 0) == (want_d >= 0))


@pytest.mark.parametrize("shape", ["rmat", "lattice", "star"])
def test_bc_dependencies_sum_to_interior_path_lengths(shape):
    """Summed over v, the dependencies of a source s count, for each reachable
    target t, the average number of interior vertices on a shortest s-t path,
    which is d(s, t) - 1 for every such path. So the sum of delta_s equals the
    sum of d(s, t) - 1 over reachable t != s, with the distances taken here from
    scipy's breadth-first search; the source's own dependency is 0. This holds
    at any size, beyond what path enumeration can reach."""
    from paper_2405_11671_amd import gen
    from tests import graphs
    p = {"rmat": lambda: gen.rmat_pairs(12, 8, seed=3), "lattice": lambda: gen.grid_pairs(40, 50, 0.2, seed=2),
         "star": lambda: graphs.star(500)}[shape]()
    og = oracle.Graph.from_pairs(p)
    n = og.n
    src, dst = np.asarray(p.src), np.asarray(p.dst)
    A = sp.coo_matrix((np.ones(len(src)), (src, dst)), shape=(n, n)).tocsr()
    for s in sorted({0, int(np.argmax(og.degrees())), n // 2}):
        D = csg.shortest_path(A, directed=False, unweighted=True, indices=s)
        reach = np.isfinite(D)
        reach[s] = False
        want = float(np.sum(D[reach] - 1))
        sigma, delta, dist = og.bc(s)
        assert delta[s] == 0.0
        assert abs(float(np.sum(delta)) - want) <= 1e-12 * max(1.0, want), (shape, s)


def test_bc_closed_forms():
    n = 12
    path = [(i, i + 1) for i in range(n - 1)]
    g, _, _ = G(n, path)
    # from one end every vertex v carries the n-1-v targets beyond it
    assert np.allclose(g.bc(0)[1], [0] + [n - 1 - v for v in range(1, n)])
    # from vertex 4: its left side carries v targets, its right side n-1-v
    want = [v for v in range(4)] + [0] + [n - 1 - v for v in range(5, n)]
    assert np.allclose(g.bc(4)[1], want)
    star = [(0, i) for i in range(1, n)]
    g, _, _ = G(n, star)
    assert np.allclose(g.bc(0)[1], 0)
    # from a leaf, the centre carries the other n-2 leaves
    assert np.allclose(g.bc(3)[1], [n - 2] + [0] * (n - 1))
    complete = [(u, v) for u in range(7) for v in range(u + 1, 7)]
    g, _, _ = G(7, complete)
    assert np.allclose(g.bc(2)[1], 0)
    # even cycle C_2k from 0: vertex 1 carries k-2 targets alone and half of the antipode
    k = 6
    cyc = [(i, (i + 1) % (2 * k)) for i in range(2 * k)]
    g, _, _ = G(2 * k, cyc)
    sigma, delta, _ = g.bc(0)
    assert sigma[k] == 2 and delta[1] == pytest.approx(k - 2 + 0.5)
    # disconnected: unreachable vertices keep 0
    g, _, _ = G(5, [(0, 1), (1, 2), (3, 4)])
    sigma, delta, dist = g.bc(0)
    assert delta.tolist() == [0, 1, 0, 0, 0] and sigma.tolist() == [1, 1, 1, 0, 0]


# ---------------------------------------------------------------- maximal independent set

def brute_greedy_mis(n, a, b, prio):
    """Greedy MIS with plain Python sets, vertices in (prio, id) order."""
    E = brute.simple_edges(n, a, b)
    adj = {v: set() for v in range(n)}
    for u, v in E:
        adj[u].add(v)
        adj[v].add(u)
    taken = set()
    for v in sorted(range(n), key=lambda x: (int(prio[x]), x)):
        if not adj[v] & taken:
            taken.add(v)
    return [1 if v in taken else 0 for v in range(n)]


@settings(max_examples=80, deadline=None)
@given(tiny_graphs, st.integers(0, 2 ** 32))
def test_mis_matches_brute_force_and_is_maximal_independent(case, seed):
    n, pairs = case
    g, a, b = G(n, pairs)
    prio = np.random.default_rng(seed).integers(0, 5, n).astype(np.uint64)   # many ties: id decides
    got = g.mis(prio)
    assert got.tolist() == brute_greedy_mis(n, a, b, prio)
    for v in range(n):
        nb = g.neighbors(v)
        if got[v]:
            assert not got[nb].any()            # independent
        else:
            assert got[nb].any()                # maximal


def test_mis_closed_forms():
    def run(n, pairs, prio):
        return G(n, pairs)[0].mis(np.asarray(prio, np.uint64)).tolist()
    path = [(i, i + 1) for i in range(6)]
    assert run(7, path, range(7)) == [1, 0, 1, 0, 1, 0, 1]                  # in id order: every other vertex
    assert run(7, path, [1, 0, 1, 0, 1, 0, 1]) == [0, 1, 0, 1, 0, 1, 0]    # odd vertices first
    star = [(0, i) for i in range(1, 6)]
    assert run(6, star, [0, 1, 1, 1, 1, 1]) == [1, 0, 0, 0, 0, 0]          # centre first
    assert run(6, star, [9, 1, 1, 1, 1, 1]) == [0, 1, 1, 1, 1, 1]          # leaves first
    k5 = [(u, v) for u in range(5) for v in range(u + 1, 5)]
    assert run(5, k5, [3, 2, 0, 4, 1]) == [0, 0, 1, 0, 0]                  # the earliest vertex alone
    assert run(4, [], [0, 0, 0, 0]) == [1, 1, 1, 1]                          # no edges: everything


# ---------------------------------------------------------------- colouring

def brute_greedy_coloring(n, a, b, prio):
    E = brute.simple_edges(n, a, b)
    adj = {v: set() for v in range(n)}
    for u, v in E:
        adj[u].add(v)
        adj[v].add(u)
    color = {}
    for v in sorted(range(n), key=lambda x: (int(prio[x]), x)):
        used = {color[u] for u in adj[v] if u in color}
        c = 0
        while c in used:
            c += 1
        color[v] = c
    return [color[v] for v in range(n)]


@settings(max_examples=80, deadline=None)
@given(tiny_graphs, st.integers(0, 2 ** 32))
def test_coloring_matches_brute_force_and_is_proper(case, seed):
    n, pairs = case
    g, a, b = G(n, pairs)
    prio = np.random.default_rng(seed).integers(0, 4, n).astype(np.uint64)
    got = g.coloring(prio)
    assert got.tolist() == brute_greedy_coloring(n, a, b, prio)
    for v in range(n):
        nb = g.neighbors(v)
        assert not np.any(got[nb] == got[v])            # proper
        assert got[v] <= g.degree(v)                      # at most degree + 1 colours


def _earlier_edges(p, n, prio):
    """Every undirected edge as (later, earlier) in (prio, id) order."""
    src, dst = np.asarray(p.src, np.int64), np.asarray(p.dst, np.int64)
    keep = src != dst
    und = np.unique(np.minimum(src[keep], dst[keep]) * n + np.maximum(src[keep], dst[keep]))
    a, b = und // n, und % n
    pa, pb = prio[a].astype(np.int64), prio[b].astype(np.int64)
    a_first = (pa < pb) | ((pa == pb) & (a < b))
    return np.where(a_first, b, a), np.where(a_first, a, b)


@pytest.mark.parametrize("shape", ["rmat", "lattice"])
def test_mis_and_coloring_local_characterisations_at_scale(shape):
    """Beyond exhaustive sizes, each greedy result is checked by the local
    condition that fixes it uniquely, over an edge list, in numpy:
    - MIS: v is in the set exactly when no neighbour earlier in (prio, id)
      order is (the lexicographically first maximal independent set);
    - colouring: each colour is the least one missing among the earlier
      neighbours' colours, so none of them shares it and the distinct smaller
      colours among them number exactly the colour itself."""
    from paper_2405_11671_amd import gen
    p = gen.rmat_pairs(13, 8, seed=4) if shape == "rmat" else gen.grid_pairs(60, 70, 0.15, seed=3)
    og = oracle.Graph.from_pairs(p)
    n = og.n
    for seed in range(3):
        prio = np.random.default_rng(seed).integers(0, 3, n).astype(np.uint64)   # heavy ties: id decides
        late, early = _earlier_edges(p, n, prio)
        mis = og.mis(prio).astype(bool)
        blocked = np.zeros(n, bool)
        np.logical_or.at(blocked, late, mis[early])
        assert np.array_equal(mis, ~blocked), (shape, seed)
        col = og.coloring(prio).astype(np.int64)
        assert not np.any(col[late] == col[early])
        lower = col[early] < col[late]
        pairs = np.unique(late[lower] * (int(col.max()) + 1) + col[early][lower])
        have = np.bincount(pairs // (int(col.max()) + 1), minlength=n)
        assert np.array_equal(have, col), (shape, seed)


def test_coloring_closed_forms():
    def run(n, pairs, prio):
        return G(n, pairs)[0].coloring(np.asarray(prio, np.uint64)).tolist()
    k5 = [(u, v) for u in range(5) for v in range(u + 1, 5)]
    assert run(5, k5, [3, 2, 0, 4, 1]) == [3, 2, 0, 4, 1]                  # K5: colour = rank in the order
    path = [(i, i + 1) for i in range(6)]
    assert run(7, path, range(7)) == [0, 1, 0, 1, 0, 1, 0]                  # bipartite in id order
    # an order that forces a third colour on a path: v0, v3 take 0, v1 takes 1, v2 (beside 1 and 0) takes 2
    assert run(4, [(0, 1), (1, 2), (2, 3)], [0, 2, 3, 1]) == [0, 1, 2, 0]
    star = [(0, i) for i in range(1, 6)]
    assert run(6, star, [9, 1, 1, 1, 1, 1]) == [1, 0, 0, 0, 0, 0]          # leaves first, centre takes 1
    cyc = [(i, (i + 1) % 5) for i in range(5)]
    assert run(5, cyc, range(5)) == [0, 1, 0, 1, 2]                         # odd cycle needs 3


# ---------------------------------------------------------------- approximate densest subgraph

def brute_max_density(n, a, b):
    """Exact densest subgraph by enumerating every vertex subset (tiny n)."""
    from fractions import Fraction
    E = brute.simple_edges(n, a, b)
    best = Fraction(0)
    for mask in range(1, 1 << n):
        k = bin(mask).count("1")
        e = sum(1 for u, v in E if (mask >> u) & 1 and (mask >> v) & 1)
        best = max(best, Fraction(e, k))
    return best


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 10).flatmap(
    lambda n: st.tuples(st.just(n), st.lists(st.tuples(st.integers(0, n - 1), st.integers(0, n - 1)),
                                             max_size=3 * n))), st.sampled_from([0.001, 0.1, 0.5]))
def test_densest_within_its_bound_of_the_exact_optimum(case, eps):
    from fractions import Fraction
    n, pairs = case
    g, a, b = G(n, pairs)
    be, bv, rounds, inb = g.densest(eps)
    got = Fraction(be, bv)
    opt = brute_max_density(n, a, b)
    assert got <= opt
    assert got * Fraction(2) * (1 + Fraction(eps)) >= opt
    # the reported set has exactly that many vertices and inner edges
    E = brute.simple_edges(n, a, b)
    if be > 0:
        assert int(inb.sum()) == bv
        assert sum(1 for u, v in E if inb[u] and inb[v]) == be


@pytest.mark.parametrize("eps", [0.001, 0.1, 1.0])
@pytest.mark.parametrize("shape", ["rmat", "lattice", "star"])
def test_densest_bracketed_by_the_maximum_core_at_scale(shape, eps):
    """Beyond exhaustive sizes: a densest subgraph has minimum degree at least
    its density rho* (dropping a vertex of smaller degree would raise it), so it
    lies inside the ceil(rho*)-core and rho* <= k_max; the k_max-core has every
    degree >= k_max, so rho* >= k_max / 2. Peeling returns at least
    rho* / (2(1 + eps)). The reported set must also hold exactly the reported
    vertex and inner-edge counts, counted here over the edge list."""
    from paper_2405_11671_amd import gen
    from tests import graphs
    p = {"rmat": lambda: gen.rmat_pairs(12, 8, seed=3), "lattice": lambda: gen.grid_pairs(40, 50, 0.2, seed=2),
         "star": lambda: graphs.star(500)}[shape]()
    og = oracle.Graph.from_pairs(p)
    kmax = int(og.kcore().max())
    be, bv, rounds, inb = og.densest(eps)
    assert kmax * bv <= 4 * (1 + eps) * be + 1e-9 * bv and be <= kmax * bv, (shape, eps, be, bv, kmax)
    src, dst = np.asarray(p.src, np.int64), np.asarray(p.dst, np.int64)
    keep = src != dst
    und = np.unique(np.minimum(src[keep], dst[keep]) * og.n + np.maximum(src[keep], dst[keep]))
    a, b = und // og.n, und % og.n
    assert int(inb.sum()) == bv
    assert int(np.sum(inb[a].astype(bool) & inb[b].astype(bool))) == be


def test_densest_closed_forms():
    k6 = [(u, v) for u in range(6) for v in range(u + 1, 6)]
    be, bv, rounds, _ = G(6, k6)[0].densest(0.001)
    assert (be, bv, rounds) == (15, 6, 1)                  # K6: density 5/2, peeled whole in one round
    k5_tail = [(u, v) for u in range(5) for v in range(u + 1, 5)] + [(4, 5), (5, 6), (6, 7), (7, 8)]
    be, bv, _, inb = G(9, k5_tail)[0].densest(0.001)
    assert be * 5 == bv * 10 or be / bv >= 2.0             # K5's density 2 is reached
    assert be / bv == 2.0 and inb[:5].all() and not inb[6:].any()
    be, bv, rounds, _ = G(4, [])[0].densest(0.1)
    assert be == 0 and rounds == 1
    # eps = 0 on a regular graph: nothing falls below the average, the first round ends the run
    be, bv, rounds, _ = G(8, [(i, (i + 1) % 8) for i in range(8)])[0].densest(0.0)
    assert (be, bv, rounds) == (8, 8, 1)


# ---------------------------------------------------------------- low-diameter decomposition

@settings(max_examples=80, deadline=None)
@given(tiny_graphs, st.integers(0, 2 ** 32), st.sampled_from([0.05, 0.5, 2.0]))
def test_ldd_dijkstra_matches_definition_and_clusters_are_connected(case, seed, beta):
    n, pairs = case
    g, a, b = G(n, pairs)
    delta = np.random.default_rng(seed).exponential(1.0 / beta, n)
    got = g.ldd(delta)
    assert got.tolist() == g.ldd(delta, definition=True).tolist()
    D = brute.floyd_warshall_hops(brute.adjacency_matrix(n, a, b))
    for v in range(n):
        c = int(got[v])
        assert D[c, v] >= 0                               # a centre in v's component
        keys = [(D[u, v] - delta[u], u) for u in range(n) if D[u, v] >= 0]
        assert (D[c, v] - delta[c], c) == min(keys)       # the least shifted distance
        # connected clusters: some neighbour one hop closer to c is in c's cluster
        if c != v:
            assert any(D[c, u] == D[c, v] - 1 and got[u] == c for u in g.neighbors(v))


def test_ldd_closed_forms():
    path = [(i, i + 1) for i in range(9)]
    g, _, _ = G(10, path)
    assert g.ldd(np.zeros(10)).tolist() == list(range(10))              # equal shifts: every vertex alone
    big = np.zeros(10)
    big[4] = 100.0
    assert g.ldd(big).tolist() == [4] * 10                              # one dominant shift takes everything
    two = np.zeros(10)
    two[0], two[9] = 5.0, 5.0
    assert g.ldd(two).tolist() == [0] * 5 + [9] * 5                     # two equal centres split the path
    g2, _, _ = G(6, [(0, 1), (1, 2), (3, 4), (4, 5)])
    assert g2.ldd(np.full(6, 50.0) - np.arange(6)).tolist() == [0, 0, 0, 3, 3, 3]   # per component


@pytest.mark.parametrize("beta", [0.05, 0.2, 1.0])
@pytest.mark.parametrize("shape", ["grid", "rmat"])
def test_ldd_cut_probability_within_the_exponential_shift_bound(shape, beta):
    """With shifts drawn from an exponential distribution of rate beta, an edge
    ends up between two clusters with probability at most 1 - exp(-beta)
    (Miller, Peng and Xu, 2013: the midpoint of an edge keeps one centre
    unless its two least shifted distances lie within 1 of each other, and by
    memorylessness that happens with probability at most 1 - exp(-beta)).
    The mean cut fraction over seeded draws must stay within that bound plus
    three standard errors. Every centre is also its own centre: a vertex u
    that beat c at c would, by the triangle inequality and the smaller-id tie
    rule, also beat c at every vertex that chose c. And since a vertex's
    centre beat the vertex itself, hop(c, v) <= delta_c - delta_v, with the
    hops taken from scipy's breadth-first search."""
    from paper_2405_11671_amd import gen
    p = gen.grid_pairs(60, 60, 0.0, seed=1) if shape == "grid" else gen.rmat_pairs(12, 8, seed=3)
    og = oracle.Graph.from_pairs(p)
    src, dst = np.asarray(p.src), np.asarray(p.dst)
    src, dst = src[src != dst], dst[src != dst]
    A = sp.coo_matrix((np.ones(src.size), (src, dst)), shape=(og.n, og.n)).tocsr()
    fractions = []
    for seed in range(16):
        delta = np.random.default_rng(seed).exponential(1.0 / beta, og.n)
        c = og.ldd(delta)
        assert np.array_equal(c[c], c)
        fractions.append(np.mean(c[src] != c[dst]))
        centres, size = np.unique(c, return_counts=True)
        big = centres[size > 1]                 # a singleton cluster meets the bound with hop 0
        if seed < 2:
            # a centre beat the vertex itself: hop(c, v) <= delta_c - delta_v
            D = csg.shortest_path(A, directed=False, unweighted=True, indices=big)
            vs = np.flatnonzero(np.isin(c, big))
            hop = D[np.searchsorted(big, c[vs]), vs]
            assert np.all(hop <= delta[c[vs]] - delta[vs] + 1e-9), (shape, beta, seed)
    mean = float(np.mean(fractions))
    se = float(np.std(fractions)) / math.sqrt(len(fractions))
    assert mean <= 1.0 - math.exp(-beta) + 3.0 * se, (shape, beta, mean, se)


# ---------------------------------------------------------------- k-core

def brute_kcore(n, a, b):
    """Coreness from the definition with plain Python sets: for each k the
    vertices left after deleting, one at a time, any vertex with fewer than k
    remaining neighbours."""
    E = brute.simple_edges(n, a, b)
    adj = {v: set() for v in range(n)}
    for u, v in E:
        adj[u].add(v)
        adj[v].add(u)
    core = [0] * n
    k = 1
    while True:
        alive = set(range(n))
        stack = [v for v in alive if len(adj[v]) < k]
        while stack:
            v = stack.pop()
            if v not in alive:
                continue
            alive.discard(v)
            for u in adj[v]:
                if u in alive and len(adj[u] & alive) < k:
                    stack.append(u)
        if not alive:
            return core
        for v in alive:
            core[v] = k
        k += 1


@settings(max_examples=80, deadline=None)
@given(tiny_graphs)
def test_kcore_matches_brute_force_and_definition(case):
    n, pairs = case
    g, a, b = G(n, pairs)
    want = brute_kcore(n, a, b)
    assert g.kcore_definition().tolist() == want
    assert g.kcore().tolist() == want


def test_kcore_properties_on_larger_graphs():
    rng = np.random.default_rng(7)
    for n, m in ((300, 1500), (500, 4000)):
        a = rng.integers(0, n, m).astype(np.int32)
        b = rng.integers(0, n, m).astype(np.int32)
        g = oracle.Graph(n, a, b)
        core = g.kcore()
        assert np.array_equal(core, g.kcore_definition())
        # every vertex keeps at least core[v] neighbours of coreness >= core[v],
        # and not core[v] + 1 neighbours of coreness >= core[v] + 1
        for v in range(n):
            nb = g.neighbors(v)
            assert int((core[nb] >= core[v]).sum()) >= core[v]
            assert int((core[nb] >= core[v] + 1).sum()) < core[v] + 1 or core[v] == g.degree(v)


def test_kcore_closed_forms():
    def run(n, pairs):
        return G(n, pairs)[0].kcore().tolist()
    assert run(6, [(u, v) for u in range(6) for v in range(u + 1, 6)]) == [5] * 6          # K6
    assert run(8, [(i, i + 1) for i in range(7)]) == [1] * 8                               # path
    assert run(9, [(0, i) for i in range(1, 9)]) == [1] * 9                                # star
    assert run(10, [(i, (i + 1) % 10) for i in range(10)]) == [2] * 10                     # cycle
    assert run(7, [(u, v) for u in range(3) for v in range(3, 7)]) == [3] * 7              # K_{3,4}
    k4_tail = [(u, v) for u in range(4) for v in range(u + 1, 4)] + [(3, 4), (4, 5)]
    assert run(7, k4_tail) == [3, 3, 3, 3, 1, 1, 0]                                        # K4, tail, isolated


def test_golden_small_graph():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "small_graph.json")
    gold = json.load(open(path))
    g, _, _ = G(gold["n"], [tuple(p) for p in gold["pairs"]])
    assert g.bfs(0)[0].tolist() == gold["bfs_depth_from_0"]
    assert g.bfs(6)[0].tolist() == gold["bfs_depth_from_6"]
    assert g.cc().tolist() == gold["cc_min_label"]
    want = np.array([float(Fraction(x)) for x in gold["pagerank_d085_T3"]])
    assert np.max(np.abs(g.pagerank(0.85, 3) - want)) < 1e-16
    assert sum(Fraction(x) for x in gold["pagerank_d085_T3"]) == 1
