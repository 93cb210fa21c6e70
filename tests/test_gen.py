"""Seeded input generators: determinism, exact counts, ranges."""
import numpy as np

from paper_2405_11671_amd import gen


def test_er_deterministic_and_in_range():
    a = gen.er_pairs(1 << 14, 8, seed=1)
    b = gen.er_pairs(1 << 14, 8, seed=1)
    c = gen.er_pairs(1 << 14, 8, seed=2)
    assert a.npairs == 65536
    assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst)
    assert not np.array_equal(a.src, c.src)
    assert a.src.min() >= 0 and a.src.max() < (1 << 14)
    # uniformity: each half of the ID range gets about half of the endpoints
    lo = np.count_nonzero(a.src < (1 << 13))
    assert abs(lo - a.npairs / 2) < 5 * np.sqrt(a.npairs / 4)


def test_rmat_quadrant_frequencies():
    p = gen.rmat_pairs(10, 16, seed=5, permute=False)
    n = 1 << 10
    top = p.src < n // 2
    left = p.dst < n // 2
    N = p.npairs
    # first level picks quadrant a, b, c, d with probabilities .57, .19, .19, .05
    for mask, q in ((top & left, .57), (top & ~left, .19), (~top & left, .19), (~top & ~left, .05)):
        assert abs(np.count_nonzero(mask) / N - q) < 5 * np.sqrt(q * (1 - q) / N)


def test_rmat_permutation_is_a_relabelling():
    a = gen.rmat_pairs(9, 8, seed=3, permute=False)
    b = gen.rmat_pairs(9, 8, seed=3, permute=True)
    # the same degree multiset (counted over endpoints) under a bijection of IDs
    da = np.bincount(np.concatenate([a.src, a.dst]), minlength=512)
    db = np.bincount(np.concatenate([b.src, b.dst]), minlength=512)
    assert np.array_equal(np.sort(da), np.sort(db))
    perm = {}
    for x, y in zip(np.concatenate([a.src, a.dst]).tolist(), np.concatenate([b.src, b.dst]).tolist()):
        assert perm.setdefault(x, y) == y


def test_grid_exact_counts():
    R, C = 64, 48
    E = 2 * R * C - R - C
    assert gen.grid_edge_count(R, C) == E
    g = gen.grid_pairs(R, C, 0.1, seed=1)
    assert g.npairs == E - int(0.1 * E)
    # every pair is a lattice edge and none repeats
    keys = set()
    for u, v in zip(g.src.tolist(), g.dst.tolist()):
        assert v == u + 1 and u % C != C - 1 or v == u + C
        keys.add((u, v))
    assert len(keys) == g.npairs
    full = gen.grid_pairs(R, C, 0.0)
    assert full.npairs == E
    assert gen.grid_edge_count(4096, 4096) == 33546240


def test_sources_distinct_and_non_isolated():
    p = gen.er_pairs(2000, 1.0, seed=9)
    s = gen.pick_sources(p, 64, seed=2)
    assert len(set(s.tolist())) == 64
    touched = set(p.src[p.src != p.dst].tolist()) | set(p.dst[p.src != p.dst].tolist())
    assert set(s.tolist()) <= touched
    tiny = gen.Pairs(5, np.array([1, 2], np.int32), np.array([2, 2], np.int32))
    assert sorted(gen.pick_sources(tiny, 10).tolist()) == [1, 2]


def test_batch_specs_ranges():
    specs = gen.batch_specs(64, seed=3)
    assert len(specs) == 64
    for n, d, s in specs:
        assert 2 ** 10 - 1 <= n <= 2 ** 18 + 1 and 4 <= d <= 32
    assert specs == gen.batch_specs(64, seed=3)


M64 = (1 << 64) - 1
GAMMA = 0x9e3779b97f4a7c15


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & M64
    z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & M64
    return z ^ (z >> 31)


def _splitmix64(state, k):
    """SplitMix64 (Steele, Lea and Flood, 2014): add the golden gamma, then mix."""
    out = []
    for _ in range(k):
        state = (state + GAMMA) & M64
        out.append(_mix(state))
    return out


def test_draws_are_splitmix64_from_a_per_stream_state():
    """The published SplitMix64 sequence from state 0 begins e220a8397b1dcdaf,
    6e789e6aa1b965f4, 06c45d188009454f; the generator's draw i of a (seed,
    stream) is output i of SplitMix64 started from a state mixed out of the
    seed and stream, so every draw is a pure function of the three."""
    assert _splitmix64(0, 3) == [0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f]
    for seed in (0, 1, 12345, 2 ** 63 + 5):
        for stream in (1, 2, 5):
            state = _mix((seed * GAMMA + stream * 0xd1b54a32d192ed03 + 0x632be59bd9b4e019) & M64)
            assert [gen.draw(seed, stream, i) for i in range(20)] == _splitmix64(state, 20), (seed, stream)
    assert gen.draw(7, 1, 1000) == gen.draw(7, 1, 1000)          # no hidden state between calls
    assert gen.unit(7, 1, 3) == (gen.draw(7, 1, 3) >> 11) / 2.0 ** 53
