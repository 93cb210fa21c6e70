"""Train the edgeMap-variant selector on this GPU and write a weight file.

    python -m paper_2405_11671_amd.train_selector --out paper_2405_11671_amd/selector_weights.json

Training data are the library's own per-level timings (every variant timed from
the same saved state, byo_selector_collect) on seeded synthetic graphs shaped
like the paper's inputs: Kronecker/RMAT (0.57, 0.19, 0.19, 0.05), Erdos-Renyi
and road-like lattices with 10% of edges removed. Seeds differ from every
benchmark input. Training runs on the GPU (byo_mlp_train).
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

from . import Graph, gen
from . import selector as sel


def training_set(max_scale: int):
    out = [gen.rmat_pairs(s, 16, seed=100 + s) for s in range(14, max_scale + 1, 2)]
    out += [gen.er_pairs(1 << 17, d, seed=200 + d) for d in (4, 10, 16, 32)]
    out += [gen.er_pairs(1 << 20, d, seed=300 + d) for d in (4, 16)]
    out += [gen.grid_pairs(r, r, 0.1, seed=400 + r) for r in (256, 1024, 2048)]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--max-scale", type=int, default=22)
    ap.add_argument("--sources", type=int, default=2)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=3e-3)
    a = ap.parse_args(argv)
    levels, names = [], []
    for p in training_set(a.max_scale):
        t = time.time()
        g = Graph.from_pairs(p)
        for s in gen.pick_sources(p, a.sources, seed=5):
            lv, _ = sel.collect(g, sel.ALGO_BFS, int(s), repeats=2, tag=p.name)
            levels += lv
        lv, _ = sel.collect(g, sel.ALGO_CC, 0, repeats=2, tag=p.name)
        levels += lv
        names.append(p.name)
        print(f"[train_selector] {p.name}: {len(levels)} levels so far ({time.time() - t:.1f}s)", flush=True)
        del g
    X, Y, M = sel.dataset(levels)
    mu, sd = sel.normaliser(X)
    params, losses = sel.train((X - mu) / sd, Y, M, steps=a.steps, lr=a.lr)
    rep = sel.compare(levels, params, mu, sd)
    print(f"[train_selector] loss {losses[0]:.3f} -> {losses[-1]:.4f}; training tables: heuristic "
          f"{rep['heuristic_ms']:.2f} ms, learned {rep['learned_ms']:.2f} ms, best {rep['best_ms']:.2f} ms",
          flush=True)
    sel.save(a.out, params, mu, sd, {"graphs": names, "levels": len(levels), "steps": a.steps, "lr": a.lr,
                                     "final_loss": float(losses[-1]), "train_report": rep})
    return 0


if __name__ == "__main__":
    sys.exit(main())
