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


# persistent = 1: every phase in one cooperative launch; 0: the host-driven loop
@pytest.mark.parametrize("persistent", [1, 0])
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_kcore_matches_oracle(p, persistent):
    g = byo.Graph.from_pairs(p, validate=True)
    og = oracle.Graph.from_pairs(p)
    core, st = byo.kcore(g, persistent=persistent)
    want = og.kcore()
    got = core.cpu().numpy()
    assert np.array_equal(got, want), (p.name, int(np.sum(got != want)))
    print(p.name, "max core", int(want.max(initial=0)), "sub-rounds", st["levels"])
    # repeat on the same graph: the workspace is reused
    core2, _ = byo.kcore(g, persistent=persistent)
    assert np.array_equal(core2.cpu().numpy(), want)


@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_kcore_persistent_takes_the_same_sub_rounds(p):
    """Both forms remove the same frontier in every sub-round: the sub-round
    count and the edges summed over them agree."""
    g = byo.Graph.from_pairs(p)
    _, a = byo.kcore(g, persistent=1)
    _, b = byo.kcore(g, persistent=0)
    assert a["levels"] == b["levels"], p.name
    assert a["device_levels"] == a["levels"] and b["device_levels"] == 0
    assert a["edges"] == b["edges"] and a["reached"] == b["reached"] == p.n


@pytest.mark.parametrize("persistent", [1, 0])
def test_kcore_round_cap(persistent):
    g = byo.Graph.from_pairs(graphs.path(1000))
    with pytest.raises(byo.ByoError):
        byo.kcore(g, max_levels=3, persistent=persistent)
    # the cap leaves the graph usable
    core, _ = byo.kcore(g, persistent=persistent)
    want = np.ones(1000, np.int32)
    assert np.array_equal(core.cpu().numpy(), want)


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
