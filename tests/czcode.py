"""Reference encoder and decoder of the byte-coded lists, written from the
format's definition (byo.h, byo_cz_build): per vertex, blocks of 64 sorted
neighbours; a block's first neighbour as zigzag(u - v), the rest as gaps; each
value a base-128 byte code, low group first, bit 7 = more bytes; lists of
several blocks start with little-endian uint32 offsets of blocks 1 .. nb-1.
Test infrastructure only: it shares nothing with the library."""
import numpy as np

BLOCK = 64


def zigzag(x: int) -> int:
    return 2 * x if x >= 0 else -2 * x - 1


def unzigzag(z: int) -> int:
    return z // 2 if z % 2 == 0 else -(z + 1) // 2


def byte_code(x: int) -> bytes:
    assert x >= 0
    out = bytearray()
    while True:
        low = x & 0x7F
        x >>= 7
        if x:
            out.append(low | 0x80)
        else:
            out.append(low)
            return bytes(out)


def encode_list(v: int, nbrs) -> bytes:
    nbrs = [int(u) for u in nbrs]
    blocks = []
    for j in range(0, len(nbrs), BLOCK):
        part = nbrs[j:j + BLOCK]
        b = bytearray(byte_code(zigzag(part[0] - v)))
        for a, c in zip(part, part[1:]):
            assert c > a
            b += byte_code(c - a)
        blocks.append(bytes(b))
    if not blocks:
        return b""
    table = bytearray()
    pos = 4 * (len(blocks) - 1)
    starts = []
    for b in blocks:
        starts.append(pos)
        pos += len(b)
    for s in starts[1:]:
        table += int(s).to_bytes(4, "little")
    return bytes(table) + b"".join(blocks)


def encode(lists):
    """lists: sequence of (sorted) neighbour arrays, vertex v = index. Returns (off, bytes)."""
    chunks = [encode_list(v, l) for v, l in enumerate(lists)]
    off = np.zeros(len(chunks) + 1, np.int64)
    off[1:] = np.cumsum([len(c) for c in chunks])
    return off, np.frombuffer(b"".join(chunks), dtype=np.uint8)


def decode_list(v: int, d: int, data: bytes) -> list:
    nb = (d + BLOCK - 1) // BLOCK
    out = []
    for j in range(nb):
        pos = 4 * (nb - 1) if j == 0 else int.from_bytes(data[4 * (j - 1):4 * j], "little")
        count = min(BLOCK, d - j * BLOCK)
        vals = []
        while len(vals) < count:
            x, sh = 0, 0
            while True:
                byte = data[pos]
                pos += 1
                x |= (byte & 0x7F) << sh
                sh += 7
                if not byte & 0x80:
                    break
            vals.append(x)
        u = v + unzigzag(vals[0])
        out.append(u)
        for g in vals[1:]:
            u += g
            out.append(u)
    return out
