"""Seeded test graphs (raw pairs) shared by the GPU parity tests."""
import numpy as np

from paper_2405_11671_amd import gen


def pairs(n, src, dst, name):
    return gen.Pairs(n, np.asarray(src, np.int32), np.asarray(dst, np.int32), name)


def star(leaves, centre=0):
    n = leaves + 1
    others = [v for v in range(n) if v != centre]
    return pairs(n, [centre] * leaves, others, f"star{leaves}")


def path(n):
    return pairs(n, np.arange(n - 1), np.arange(1, n), f"path{n}")


def empty(n):
    return pairs(n, [], [], f"empty{n}")


def two_hubs(n=20000, hub_deg=9000, seed=11):
    """Two hubs above every bucket cutoff plus a sparse random background."""
    rng = np.random.default_rng(seed)
    a = [0] * hub_deg + [1] * hub_deg
    b = list(rng.integers(2, n, hub_deg)) + list(rng.integers(2, n, hub_deg))
    bg = gen.er_pairs(n, 2.0, seed=seed)
    return pairs(n, np.concatenate([a, bg.src]), np.concatenate([b, bg.dst]), "two_hubs")


def hub_over_er(leaves=70000, avg_degree=8.0, seed=13):
    """A star with `leaves` leaves on top of an ER graph over the leaves: one
    vertex above the 16-bit tile-local range of entries, and m >= 4n, so the
    degree-ordered tile layout applies."""
    n = leaves + 1
    bg = gen.er_pairs(leaves, avg_degree, seed=seed)
    src = np.concatenate([np.zeros(leaves, np.int64), bg.src.astype(np.int64) + 1])
    dst = np.concatenate([np.arange(1, n), bg.dst.astype(np.int64) + 1])
    return pairs(n, src, dst, f"hub{leaves}_er{avg_degree:g}")


def king_lattice(rows=200, cols=400):
    """rows x cols lattice with the 8 king-move neighbours: average degree
    near 8 (so the tile layout applies) and a diameter of max(rows, cols) - 1,
    for traversals with far more levels than the tiled multi-source run keeps
    frontier history for."""
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    v = (r * cols + c).ravel()
    src, dst = [], []
    for dr, dc in ((0, 1), (1, 0), (1, 1), (1, -1)):
        ok = ((r + dr < rows) & (c + dc >= 0) & (c + dc < cols)).ravel()
        src.append(v[ok])
        dst.append(v[ok] + dr * cols + dc)
    return pairs(rows * cols, np.concatenate(src), np.concatenate(dst), f"king{rows}x{cols}")


def small_suite():
    """Graphs that finish in the oracle in well under a second."""
    return [
        gen.er_pairs(1 << 14, 8, seed=1),                 # the paper-shaped ER case
        gen.rmat_pairs(14, 16, seed=1),                   # skewed, several tiles
        gen.grid_pairs(97, 61, 0.1, seed=1),              # high diameter, ragged n
        star(70000),                                      # one hub above every cutoff
        two_hubs(),
        path(1000),
        empty(130),
        pairs(1, [], [], "single"),
        pairs(64, [0, 63], [63, 0], "one_word"),
        pairs(65, [64, 3], [3, 64], "word_tail"),
    ]
