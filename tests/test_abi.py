"""CPU-side checks of the C ABI: every declared symbol is exported, host-only
entry points work, and argument errors come back as status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2405_11671_amd import _lib, csr_from_pairs, gen
from tests import graphs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(byo_[a-z0-9_]+)\s*\(", text))
    return names


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    bound = set(_lib.SIGNATURES)
    assert declared_functions() == bound


def test_opts_defaults_and_version():
    o = _lib.default_opts()
    assert (o.selector, o.dense_divisor, o.t_wave, o.t_block, o.cc_shortcut) == (0, 20, 32, 4096, 1)
    # the tile layout is the default wherever a graph qualifies
    assert (o.pr_blocked, o.tiled, o.use_graph, o.small_frontier) == (1, 1, 0, 0)
    assert b"gfx950" in _lib.load().byo_version()


def test_argument_errors_are_status_codes():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.byo_graph_from_csr(None, None, 4, 0, _lib.HOST_INPUT, None, ctypes.byref(h)) == -1
    assert b"null" in lib.byo_last_error()
    off = np.array([0, 0], np.int64)
    assert lib.byo_graph_from_csr(off.ctypes.data, None, 1, 0, 0, None, ctypes.byref(h)) == -1
    assert b"exactly one" in lib.byo_last_error()
    assert lib.byo_bfs(None, 0, None, None, None, None, None) == -1
    assert lib.byo_num_vertices(None) == -1
    # the other algorithms and the byte-coded container check their pointers
    # before any device work
    assert lib.byo_bc(None, 0, None, None, None, None, None, None) == -1
    assert lib.byo_kcore(None, None, None, None, None) == -1
    assert lib.byo_mis(None, None, None, None, None, None) == -1
    assert lib.byo_coloring(None, None, None, None, None, None) == -1
    assert lib.byo_densest(None, 0.1, None, None, None, None, None, None) == -1
    assert lib.byo_cz_build(None, None) == -1
    assert lib.byo_cz_bytes(None, None) == -1
    assert lib.byo_cz_copy(None, None, None) == -1
    assert lib.byo_cz_decode(None, 0, None, None) == -1
    assert b"null" in lib.byo_last_error()


NO_HANDLE = {"byo_last_error", "byo_version", "byo_heuristic_choice"}
# no handle, but they switch process-wide state (tracing, kernel timers, the
# loaded selector) that later tests in the same process may rely on
STATEFUL = {"byo_selector_clear", "byo_trace_enable", "byo_ktimer_enable", "byo_ktimer_select", "byo_ktimer_reset"}
DESTROY = {"byo_graph_destroy", "byo_vset_destroy", "byo_batch_destroy"}


def test_every_entry_point_rejects_null_arguments_before_device_work():
    """Each declared function, called with null pointers and zero scalars on a
    host with no GPU, returns the argument-error status (or -1 for the
    counts) with a message, rather than crashing or reaching the device; the
    destroy calls accept null, and the pure calls that take no handle succeed.
    The calls that switch process-wide state are left uncalled."""
    lib = _lib.load()
    sigs = dict(_lib.SIGNATURES)
    h = ctypes.c_void_p()
    off = np.array([0, 0], np.int64)
    for name in sorted(declared_functions() - STATEFUL):
        _, args = sigs[name]
        vals = []
        for a in args:
            if a in (ctypes.c_double, ctypes.c_float):
                vals.append(0.0)
            elif a not in (ctypes.c_void_p, ctypes.c_char_p) and isinstance(a, type) and \
                    issubclass(a, ctypes._SimpleCData):
                vals.append(0)
            else:
                vals.append(None)
        # leave a different message behind, so a stale one cannot pass below
        assert lib.byo_graph_from_csr(off.ctypes.data, None, 1, 0, 0, None, ctypes.byref(h)) == -1
        r = getattr(lib, name)(*vals)
        if name in DESTROY or name == "byo_opts_default":
            assert r is None, name
        elif name in NO_HANDLE:
            assert r is not None and r != -1, (name, r)
        else:
            assert r == -1, (name, r)
            msg = lib.byo_last_error()
            assert b"null" in msg or b"bad argument" in msg, (name, msg)


@pytest.mark.parametrize("p", [gen.er_pairs(1 << 12, 8), gen.rmat_pairs(11), gen.grid_pairs(33, 17, 0.1),
                               graphs.star(500, centre=7), graphs.empty(9)], ids=lambda p: p.name)
def test_host_csr_build_matches_oracle_sets(p):
    off, nbr = csr_from_pairs(p.n, p.src, p.dst)
    ooff, onbr = oracle.Graph.from_pairs(p).export()
    assert np.array_equal(off, ooff) and np.array_equal(nbr, onbr)


def test_host_csr_build_rejects_out_of_range():
    with pytest.raises(_lib.ByoError):
        csr_from_pairs(3, np.array([0], np.int32), np.array([3], np.int32))
