"""CPU checks of the selector's host-side pieces (features, threshold rule,
weight validation, weight files)."""
import ctypes
import math

import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2405_11671_amd import _lib
from paper_2405_11671_amd import selector as sel


def rec(**kw):
    base = dict(algo=0, level=3, variant=0, dense_in=0, n=1 << 20, m=31_000_000, k=1000, degsum=50_000,
                unvisited=600_000, out_count=0, out_degsum=0, max_deg=60_000, cv=4.5, ms=0.0)
    base.update(kw)
    return base


@pytest.mark.parametrize("r", [rec(), rec(k=0, degsum=0, dense_in=1), rec(k=1 << 20, degsum=31_000_000, unvisited=0),
                               rec(n=1, m=0, k=1, degsum=0, max_deg=0, cv=0.0)])
def test_features_match_oracle_definition(r):
    got = sel.features(r)
    want = omlp.selector_features(r["k"], r["degsum"], r["unvisited"], r["n"], r["m"], r["max_deg"], r["cv"],
                                  r["dense_in"])
    assert np.allclose(got, np.array(want, np.float32), rtol=1e-6, atol=1e-7)


def test_features_pinned_to_hand_computed_values():
    """The oracle's feature definition (and the library's) on a level whose
    features are exact by hand: every count one below a power of two, so each
    log2(1 + x) is an integer; a dropped term, swapped argument or wrong
    ratio changes at least one of these literals."""
    r = rec(k=3, degsum=7, unvisited=15, n=31, m=63, max_deg=127, cv=0.5, dense_in=1)
    # log2 4, log2 8, log2 16, log2 32, log2 64, (3+7)/64, 3/32, log2 128, cv,
    # log2(1 + 7/4) = log2 2.75, 15/32, flag
    want = [2.0, 3.0, 4.0, 5.0, 6.0, 0.15625, 0.09375, 7.0, 0.5, math.log2(2.75), 0.46875, 1.0]
    got_oracle = omlp.selector_features(3, 7, 15, 31, 63, 127, 0.5, 1)
    assert got_oracle == pytest.approx(want, rel=0, abs=1e-15)
    assert np.allclose(sel.features(r), np.array(want, np.float32), rtol=0, atol=1e-6)
    # an empty frontier on an edgeless one-vertex graph: every log term is 0
    z = omlp.selector_features(0, 0, 0, 0, 0, 0, 0.0, 0)
    assert z == [0.0] * 12


def test_heuristic_cutoff_and_balance_choices():
    m = 2_000_000
    # exactly at the cutoff stays sparse; one more goes dense (k + degsum > m/20)
    at = rec(m=m, k=10, degsum=m // 20 - 10, max_deg=100, cv=0.5)
    over = rec(m=m, k=11, degsum=m // 20 - 10, max_deg=100, cv=0.5)
    assert sel.heuristic_choice(at) in (0, 1, 2, 3)
    assert sel.heuristic_choice(over) == 4                       # low skew -> thread pull
    assert sel.heuristic_choice(dict(over, cv=3.0)) == 5         # skewed -> wave-assisted pull
    assert sel.heuristic_choice(over, allow_pull=False) in (0, 1, 2, 3)
    assert sel.heuristic_choice(rec(m=m, k=10, degsum=100, max_deg=10, cv=0.1)) == 0
    assert sel.heuristic_choice(rec(m=m, k=10, degsum=5000, max_deg=900, cv=0.1)) == 1
    assert sel.heuristic_choice(rec(m=m, k=10, degsum=5000, max_deg=5000, cv=0.1)) == 3
    # a push looks at the frontier's own longest list when the level knows it
    hub = rec(m=m, k=10, degsum=5000, max_deg=5000, cv=0.1)
    assert sel.heuristic_choice(dict(hub, max_deg_u=512)) == 1      # 8 wavefront rounds
    assert sel.heuristic_choice(dict(hub, max_deg_u=513)) == 3      # longer: edge-balanced
    assert sel.heuristic_choice(dict(hub, max_deg_u=-1)) == 3       # unknown: the graph's 5000
    assert sel.heuristic_choice(rec(m=m, k=400, degsum=3000, max_deg=5000, max_deg_u=8)) == 0
    assert sel.heuristic_choice(rec(m=m, k=400, degsum=3000, max_deg=5000, max_deg_u=9)) == 1
    assert sel.heuristic_choice(rec(m=m, k=10, degsum=70000, max_deg=5000, max_deg_u=100)) == 3
    # ... and a pull keeps the graph's (it scans the lists of unvisited vertices)
    assert sel.heuristic_choice(dict(over, max_deg=1000, max_deg_u=5)) == 5


def test_selector_rejects_non_finite_weights():
    p = sel.init_params(1)
    mu, sd = np.zeros(12, np.float32), np.ones(12, np.float32)
    for bad in (p.copy(), mu.copy(), sd.copy()):
        bad[3] = np.nan
    fp = ctypes.POINTER(ctypes.c_float)
    lib = _lib.load()
    bp = p.copy(); bp[7] = np.nan
    assert lib.byo_selector_set(bp.ctypes.data_as(fp), mu.ctypes.data_as(fp), sd.ctypes.data_as(fp)) == -1
    bs = sd.copy(); bs[0] = 0.0
    assert lib.byo_selector_set(p.ctypes.data_as(fp), mu.ctypes.data_as(fp), bs.ctypes.data_as(fp)) == -1
    bm = mu.copy(); bm[2] = np.inf
    assert lib.byo_selector_set(p.ctypes.data_as(fp), bm.ctypes.data_as(fp), sd.ctypes.data_as(fp)) == -1


def test_weight_file_roundtrip(tmp_path):
    p = sel.init_params(2)
    mu, sd = np.arange(12, dtype=np.float32), np.full(12, 2.0, np.float32)
    path = tmp_path / "w.json"
    sel.save(path, p, mu, sd, {"trained_on": ["x"]})
    p2, mu2, sd2, meta = sel.load_weights(path)
    assert np.array_equal(p, p2) and np.array_equal(mu, mu2) and np.array_equal(sd, sd2)
    assert meta == {"trained_on": ["x"]}
