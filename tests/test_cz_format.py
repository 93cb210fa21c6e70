"""CPU pins of the reference byte-code encoder used by the GPU tests of the
byte-coded lists: a list worked by hand from the format's definition, the
zig-zag map's first values, byte-code boundaries, and round trips."""
import numpy as np

from tests import czcode


def test_hand_worked_list():
    # v = 5, neighbours 3, 7, 300: zigzag(3 - 5) = 3; gaps 4 and 293 = 0b10_0100101
    assert czcode.encode_list(5, [3, 7, 300]) == bytes([0x03, 0x04, 0xA5, 0x02])


def test_zigzag_and_byte_code_boundaries():
    assert [czcode.zigzag(x) for x in (0, -1, 1, -2, 2)] == [0, 1, 2, 3, 4]
    assert all(czcode.unzigzag(czcode.zigzag(x)) == x for x in range(-1000, 1000))
    assert czcode.byte_code(127) == bytes([0x7F])
    assert czcode.byte_code(128) == bytes([0x80, 0x01])
    assert czcode.byte_code(2 ** 14 - 1) == bytes([0xFF, 0x7F])
    assert czcode.byte_code(2 ** 14) == bytes([0x80, 0x80, 0x01])
    assert len(czcode.byte_code(2 ** 32 - 1)) == 5


def test_block_table_for_long_lists():
    v = 1000
    nbrs = list(range(0, 130 * 3, 3))          # 130 neighbours: 3 blocks
    data = czcode.encode_list(v, nbrs)
    first = int.from_bytes(data[0:4], "little")
    second = int.from_bytes(data[4:8], "little")
    # block 0 starts after the 2-entry table; block 0: zigzag(-1000) = 1999 (2 bytes) + 63 gaps of 3
    assert first == 8 + 2 + 63
    # block 1 starts with zigzag(192 - 1000) = 1615 (2 bytes), then 63 gaps
    assert second == first + 2 + 63
    assert czcode.decode_list(v, len(nbrs), data) == nbrs


def test_round_trip_random_lists():
    rng = np.random.default_rng(3)
    for v in (0, 7, 4095, 10 ** 6):
        for d in (1, 63, 64, 65, 200):
            nbrs = np.unique(rng.integers(0, 2 ** 31 - 1, size=3 * d))[:d].tolist()
            assert czcode.decode_list(v, len(nbrs), czcode.encode_list(v, nbrs)) == nbrs
