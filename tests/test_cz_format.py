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


PASSES = []  # decoding passes per emulated block


def wave_decode_emulated(data, r, rend, v, d, nb, j):
    """Lane-by-lane emulation, on the CPU, of the wavefront block decoder's
    algorithm (one aligned dword per lane, value ends found from bit 7, each
    value assembled from a two-lane byte window, a second pass from the first
    undecoded value): a check of the algorithm's boundary logic on many
    blocks. Returns the block's neighbours."""
    W = 64

    def block_pos(jj):
        if jj == 0:
            return r + 4 * (nb - 1)
        o = r + 4 * (jj - 1)
        return r + int.from_bytes(bytes(data[o:o + 4]), "little")

    def dword(p):
        return int.from_bytes(bytes(data[p:p + 4]).ljust(4, b"\0"), "little")

    start = block_pos(j)
    end = block_pos(j + 1) if j + 1 < nb else rend
    c = min(64, d - 64 * j)
    frm, done, lds = start, 0, [None] * 64
    passes = 0
    while done < c:
        passes += 1
        a0 = frm & ~3
        xs, tms, bms = [], [], []
        for lane in range(W):
            wp = a0 + 4 * lane
            x = dword(wp) if wp < end else 0
            tm = bm = 0
            for k in range(4):
                p = wp + k
                if p < frm:
                    bm |= 1 << k
                elif p < end and not ((x >> (8 * k)) & 0x80):
                    tm |= 1 << k
            xs.append(x)
            tms.append(tm)
            bms.append(bm | tm)
        pre = 0
        for lane in range(W):
            xp = xs[lane - 1] if lane else xs[0]
            bmp = bms[lane - 1] if lane else 0xF
            win = xp | (xs[lane] << 32)
            wb = bmp | (bms[lane] << 4)
            rank = 0
            for k in range(4):
                if (tms[lane] >> k) & 1:
                    q = 4 + k
                    below = wb & ((1 << q) - 1)
                    s0 = below.bit_length() if below else 0
                    val = 0
                    for t in range(s0, q + 1):
                        val |= ((win >> (8 * t)) & 0x7F) << (7 * (t - s0))
                    idx = done + pre + rank
                    if idx < c:
                        lds[idx] = val
                    rank += 1
            pre += bin(tms[lane]).count("1")
        done += pre
        if done < c:
            ll = max(lane for lane in range(W) if tms[lane])
            frm = a0 + 4 * ll + (tms[ll].bit_length() - 1) + 1
    PASSES.append(passes)
    out, u = [], v + czcode.unzigzag(lds[0])
    out.append(u)
    for g in lds[1:c]:
        u += g
        out.append(u)
    return out


def test_wave_decoder_algorithm_on_random_blocks():
    rng = np.random.default_rng(11)
    for trial in range(300):
        v = int(rng.integers(0, 2 ** 31 - 1))
        d = int(rng.integers(1, 200))
        spread = int(rng.choice([2 ** 7, 2 ** 14, 2 ** 21, 2 ** 28, 2 ** 31 - 1, 0]))
        if spread:
            nbrs = np.unique(rng.integers(0, spread, size=d))
        else:
            # gaps in [2^22, 2^23): 4 bytes each, so a full block is 257 bytes (two passes)
            d = min(d, 250)
            nbrs = np.cumsum(rng.integers(2 ** 22, 2 ** 23, size=d))
            nbrs = nbrs[nbrs < 2 ** 31 - 1]
        nbrs = sorted({int(x) for x in nbrs} - {v})
        if not nbrs:
            continue
        pad = int(rng.integers(0, 4))              # the list's start, off 4-byte alignment by 0..3
        lst = czcode.encode_list(v, nbrs)
        data = bytearray(bytes([0x55]) * pad) + bytearray(lst) + bytearray(8)
        r, rend = pad, pad + len(lst)
        nb = (len(nbrs) + 63) // 64
        got = []
        for j in range(nb):
            got += wave_decode_emulated(data, r, rend, v, len(nbrs), nb, j)
        assert got == nbrs, (trial, v, len(nbrs), spread, pad)
    assert max(PASSES) == 2 and PASSES.count(2) >= 5   # blocks over 256 bytes took the second pass
