"""GPU parity of the maximal independent set (byo_mis): for a given priority
order the greedy MIS is unique, so the GPU's membership must equal the
oracle's greedy scan exactly."""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


SUITE = graphs.small_suite() + [gen.rmat_pairs(16, 16, seed=12), graphs.hub_over_er()]
IDS = [p.name for p in SUITE]


@pytest.mark.parametrize("variant", [None, 0])
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_mis_matches_oracle(p, variant):
    g = byo.Graph.from_pairs(p, validate=True)
    og = oracle.Graph.from_pairs(p)
    kw = {} if variant is None else {"selector": byo.SEL_FIXED, "fixed_variant": variant}
    for seed, hi in ((1, 2 ** 63), (2, 3)):      # distinct priorities, then many ties (ids decide)
        prio = np.random.default_rng(seed).integers(0, hi, max(og.n, 1), dtype=np.uint64)[: og.n]
        got, st = byo.mis(g, prio, **kw)
        want = og.mis(prio)
        assert np.array_equal(got.cpu().numpy(), want), (p.name, seed)
        print(p.name, seed, "rounds", st["levels"], "size", int(want.sum()))


def test_mis_round_cap():
    g = byo.Graph.from_pairs(graphs.path(1000))
    prio = np.arange(1000, dtype=np.uint64)          # id order: a chain of dependencies
    with pytest.raises(byo.ByoError):
        byo.mis(g, prio, max_levels=2)


def dense_hub(n_hub_nbrs=5000):
    """A hub adjacent to a clique-heavy neighbourhood: its earlier neighbours
    hold many distinct colours, past the 64 a lane's mask covers."""
    src, dst = [], []
    k = 90                                   # a 90-clique: colours 0..89 in any order
    for u in range(k):
        for v in range(u + 1, k):
            src.append(u)
            dst.append(v)
    hub = k
    for u in range(k + 1, k + 1 + n_hub_nbrs):
        src.append(hub)
        dst.append(u)
    for u in range(k):
        src.append(hub)
        dst.append(u)
    return graphs.pairs(k + 1 + n_hub_nbrs, src, dst, "clique_hub")


@pytest.mark.parametrize("variant", [None, 0])
@pytest.mark.parametrize("p", SUITE + [dense_hub()], ids=IDS + ["clique_hub"])
def test_coloring_matches_oracle(p, variant):
    g = byo.Graph.from_pairs(p, validate=True)
    og = oracle.Graph.from_pairs(p)
    kw = {} if variant is None else {"selector": byo.SEL_FIXED, "fixed_variant": variant}
    for seed, hi in ((1, 2 ** 63), (2, 3)):
        prio = np.random.default_rng(seed).integers(0, hi, max(og.n, 1), dtype=np.uint64)[: og.n]
        if p.name == "clique_hub":
            prio[90] = 2 ** 63 + 5               # the hub last: it sees all 90 clique colours
        got, st = byo.coloring(g, prio, **kw)
        want = og.coloring(prio)
        assert np.array_equal(got.cpu().numpy(), want), (p.name, seed)
        print(p.name, seed, "rounds", st["levels"], "colours", int(want.max(initial=-1)) + 1)
