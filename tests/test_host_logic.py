"""CPU checks of host-side logic: the container-API configurations against
the descriptions in Table api-components-avg, and the benchmark's refusal of
more than one GPU."""
import os
import subprocess
import sys

from paper_2405_11671_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DEG, NUM_E, EE, PMAP, PEE = (_lib.API_NO_DEGREE, _lib.API_NO_NUM_EDGES, _lib.API_NO_EARLY_EXIT,
                             _lib.API_NO_PAR_MAP, _lib.API_NO_PAR_EARLY_EXIT)
ALL = DEG | NUM_E | EE | PMAP | PEE


def kept(omit):
    """The optional functions a configuration keeps."""
    names = {DEG: "degree", NUM_E: "num_edges", EE: "map_early_exit", PMAP: "parallel_map",
             PEE: "parallel_map_early_exit"}
    return {name for bit, name in names.items() if not omit & bit}


def test_bits_are_distinct_single_bits():
    bits = [DEG, NUM_E, EE, PMAP, PEE]
    assert len(set(bits)) == 5 and all(b and not b & (b - 1) for b in bits)


def test_configurations_follow_the_table():
    c = _lib.API_CONFIGS
    assert len(c) == 9
    # Min: only the required map_neighbors and num_vertices
    assert kept(c["min"]) == set()
    # Min + degree; Min efficient = Min + degree + num_edges
    assert kept(c["min+degree"]) == {"degree"}
    assert kept(c["min_efficient"]) == {"degree", "num_edges"}
    # Full minus one function
    assert kept(c["full-num_edges"]) == kept(0) - {"num_edges"}
    assert kept(c["full-degree"]) == kept(0) - {"degree"}
    assert kept(c["full-parallel_early_exit"]) == kept(0) - {"parallel_map_early_exit"}
    # Full minus both early-exit maps; full minus both parallel maps
    assert kept(c["no_early_exit"]) == kept(0) - {"map_early_exit", "parallel_map_early_exit"}
    assert kept(c["no_parallel_map"]) == kept(0) - {"parallel_map", "parallel_map_early_exit"}
    assert c["full"] == 0 and c["min"] == ALL


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


class _FakeDeviceTensor:
    """Stands in for a CUDA tensor on a machine without one."""

    def __init__(self, numel, element_size, contiguous=True):
        self._n, self._e, self._c = numel, element_size, contiguous
        self.is_cuda = True

    def is_contiguous(self):
        return self._c

    def element_size(self):
        return self._e

    def numel(self):
        return self._n

    def data_ptr(self):
        return 0x1000


def test_buffers_are_checked_before_they_reach_the_library():
    import pytest
    import torch

    import paper_2405_11671_amd as byo
    with pytest.raises(ValueError, match="device"):
        byo._ptr(torch.zeros(4))                                  # host memory
    with pytest.raises(ValueError, match="contiguous"):
        byo._ptr(_FakeDeviceTensor(8, 4, contiguous=False))
    with pytest.raises(ValueError, match="bytes"):
        byo._ptr(_FakeDeviceTensor(8, 8), 8, 4)                   # int64 where int32 is needed
    with pytest.raises(ValueError, match="elements"):
        byo._ptr(_FakeDeviceTensor(7, 4), 8, 4)                   # too short
    assert byo._ptr(_FakeDeviceTensor(8, 4), 8, 4).value == 0x1000
