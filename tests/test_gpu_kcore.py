"""GPU parity of the k-core decomposition (byo_kcore): coreness must equal the
oracle's bucketed peeling (itself pinned to the definition on the CPU),
exactly, on every graph."""
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


SUITE = graphs.small_suite() + [gen.rmat_pairs(16, 16, seed=12), graphs.hub_over_er(),
                                gen.er_pairs(70001, 10, seed=5),
                                graphs.pairs(7, [0, 0, 0, 1, 1, 2, 3, 4], [1, 2, 3, 2, 3, 3, 4, 5], "k4_tail")]
IDS = [p.name for p in SUITE]


@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_kcore_matches_oracle(p):
    g = byo.Graph.from_pairs(p, validate=True)
    og = oracle.Graph.from_pairs(p)
    core, st = byo.kcore(g)
    want = og.kcore()
    got = core.cpu().numpy()
    assert np.array_equal(got, want), (p.name, int(np.sum(got != want)))
    print(p.name, "max core", int(want.max(initial=0)), "sub-rounds", st["levels"])
    # repeat on the same graph: the workspace is reused
    core2, _ = byo.kcore(g)
    assert np.array_equal(core2.cpu().numpy(), want)


def test_kcore_round_cap():
    g = byo.Graph.from_pairs(graphs.path(1000))
    with pytest.raises(byo.ByoError):
        byo.kcore(g, max_levels=3)


@pytest.mark.parametrize("eps", [0.001, 0.1])
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_densest_matches_oracle(p, eps):
    """Peeling rounds are deterministic: best |E(S)|, |S|, round count and the
    best set equal the oracle's exactly."""
    g = byo.Graph.from_pairs(p, validate=True)
    og = oracle.Graph.from_pairs(p)
    be, bv, inb, st = byo.densest(g, eps)
    we, wv, wr, winb = og.densest(eps)
    assert (be, bv, st["levels"]) == (we, wv, wr), p.name
    assert np.array_equal(inb.cpu().numpy(), winb), p.name
    print(p.name, eps, "density", round(be / bv, 4), "rounds", wr)
