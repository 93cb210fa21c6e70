"""GPU parity of single-source betweenness (byo_bc) against the oracle's
Brandes recurrence (itself pinned to the pairwise definition on the CPU).

Depths must match exactly; path counts exactly while below 2^53 (integers in
FP64; above that, to 1e-12 relative); dependencies to 1e-9 of the largest
dependency. The bound: every dependency is a chain of at most `levels` sums of
at most `deg` FP64 terms, each rounding by 2^-53 relative, about
levels * max_deg * 1.1e-16 <= 1e-11 on these graphs; 1e-9 leaves a margin.
"""
import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
byo = pytest.importorskip("paper_2405_11671_amd")

DELTA_TOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")


_cache = {}


def build(p):
    if p.name not in _cache:
        _cache[p.name] = (byo.Graph.from_pairs(p, validate=True), oracle.Graph.from_pairs(p))
    return _cache[p.name]


SUITE = graphs.small_suite() + [gen.rmat_pairs(16, 16, seed=12), graphs.hub_over_er()]
IDS = [p.name for p in SUITE]


def sources(og):
    deg = og.degrees()
    nz = np.flatnonzero(deg)
    out = [0]
    if nz.size:
        out += [int(nz[len(nz) // 2]), int(nz[np.argmax(deg[nz])])]
    return sorted(set(out))


def check(g, og, s, **kw):
    delta, sigma, depth, st = byo.bc(g, s, **kw)
    ws, wd, wdist = og.bc(s)
    d = depth.cpu().numpy()
    assert np.array_equal(d, wdist)
    sg = sigma.cpu().numpy()
    small = ws < 2.0 ** 53
    assert np.array_equal(sg[small], ws[small])
    assert np.allclose(sg[~small], ws[~small], rtol=1e-12, atol=0)
    dl = delta.cpu().numpy()
    scale = max(1.0, float(np.max(np.abs(wd))) if wd.size else 1.0)
    assert np.max(np.abs(dl - wd), initial=0.0) <= DELTA_TOL * scale
    assert dl[s] == 0.0
    assert st["reached"] == int((wdist >= 0).sum())
    return st


@pytest.mark.parametrize("variant", [None, 0, 1, 3, 4, 5])
@pytest.mark.parametrize("p", SUITE, ids=IDS)
def test_bc_matches_oracle(p, variant):
    g, og = build(p)
    kw = {} if variant is None else {"selector": byo.SEL_FIXED, "fixed_variant": variant}
    for s in sources(og):
        st = check(g, og, s, **kw)
        used = {k for k, c in st["variant_count"].items() if c}
        if variant is not None:
            assert used <= {byo.VARIANTS[variant]}, used


def test_bc_heuristic_uses_both_directions():
    p = gen.rmat_pairs(16, 16, seed=12)
    g, og = build(p)
    st = check(g, og, int(np.argmax(og.degrees())))
    used = {k for k, c in st["variant_count"].items() if c}
    assert used & {"push_edge", "push_wave"} and "pull_wave" in used, used


def test_bc_level_cap_and_bad_source():
    p = graphs.path(1000)
    g, _ = build(p)
    with pytest.raises(byo.ByoError):
        byo.bc(g, 0, max_levels=10)
    with pytest.raises(byo.ByoError):
        byo.bc(g, g.n)
