"""Learned edgeMap-variant selector: training data, GPU training, weights I/O.

The library collects per-level timings of every variant (byo_selector_collect),
trains the MLP with its own HIP kernels (byo_mlp_train) and runs inference on
the device inside the level loop (selector mode BYO_SEL_MLP). This module only
arranges the data: one sample per collected level, target = log2 of each
variant's time in ms, mask = which variants were timed.
"""
from __future__ import annotations

import ctypes
import json
from collections import OrderedDict

import numpy as np

from . import _lib

F, H, K = 12, 32, 6
P = F * H + H + H * H + H + H * K + K
ALGO_BFS, ALGO_CC = 0, 1


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def features(rec) -> np.ndarray:
    """Raw features of one level record (the library's host function)."""
    r = _lib.LevelRecord(**{k: rec[k] for k in rec if k in dict(_lib.LevelRecord._fields_)})
    out = (ctypes.c_float * F)()
    _lib.check(_lib.load().byo_selector_features(ctypes.byref(r), out))
    return np.array(out[:], np.float32)


def heuristic_choice(rec, opts=None, allow_pull=True) -> int:
    o = opts if opts is not None else _lib.default_opts()
    return int(_lib.load().byo_heuristic_choice(int(rec["k"]), int(rec["degsum"]), int(rec["m"]),
                                                int(rec["max_deg"]), float(rec["cv"]), ctypes.byref(o),
                                                1 if allow_pull else 0, int(rec.get("max_deg_u", -1))))


def collect(g, algo: int = ALGO_BFS, src: int = 0, repeats: int = 2, opts=None, tag: str = ""):
    """Time every variant at every level of one run; returns a list of level dicts."""
    torch = _torch()
    from . import trace_read
    trace_read()  # drop anything pending
    out = torch.empty(max(g.n, 1), dtype=torch.int32, device="cuda")
    o = opts if opts is not None else _lib.default_opts()
    _lib.check(_lib.load().byo_selector_collect(g.handle, int(algo), int(src), int(repeats),
                                                ctypes.c_void_p(out.data_ptr()), ctypes.byref(o), _stream()))
    recs = trace_read()
    levels = OrderedDict()
    for r in recs:
        key = (tag, r["algo"], r["level"])
        lv = levels.setdefault(key, {"rec": r, "ms": np.full(K, np.nan), "tag": tag})
        lv["ms"][r["variant"]] = r["ms"]
    return list(levels.values()), out[: g.n]


def dataset(levels):
    """X raw features [N, F], Y log2 ms [N, K], M mask [N, K]."""
    X = np.stack([features(lv["rec"]) for lv in levels]).astype(np.float32)
    ms = np.stack([lv["ms"] for lv in levels])
    M = np.isfinite(ms).astype(np.float32)
    Y = np.where(M > 0, np.log2(np.maximum(np.nan_to_num(ms, nan=1.0), 1e-4)), 0.0).astype(np.float32)
    return X, Y, M


def normaliser(X):
    mu = X.mean(axis=0).astype(np.float32)
    sd = np.maximum(X.std(axis=0), 1e-3).astype(np.float32)
    return mu, sd


def init_params(seed: int = 4) -> np.ndarray:
    """He-uniform weights, zero biases, packed W1 b1 W2 b2 W3 b3."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((F, H), (H, H), (H, K)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, (fan_in, fan_out)).astype(np.float32).ravel())
        parts.append(np.zeros(fan_out, np.float32))
    return np.concatenate(parts)


def unpack(params):
    """Packed vector -> dict W1 b1 W2 b2 W3 b3 (views)."""
    p = np.asarray(params)
    out, i = {}, 0
    for name, shape in (("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, K)), ("b3", (K,))):
        sz = int(np.prod(shape))
        out[name] = p[i:i + sz].reshape(shape)
        i += sz
    return out


def train(X, Y, M, steps: int = 3000, lr: float = 3e-3, params=None, seed: int = 4):
    """Full-batch Adam on the GPU. X must already be normalised. Returns (params, losses)."""
    torch = _torch()
    p = torch.from_numpy(np.ascontiguousarray(init_params(seed) if params is None else params, np.float32)).cuda()
    Xd, Yd, Md = (torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda() for a in (X, Y, M))
    losses = torch.zeros(max(steps, 1), dtype=torch.float32, device="cuda")
    _lib.check(_lib.load().byo_mlp_train(ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(Xd.data_ptr()),
                                         ctypes.c_void_p(Yd.data_ptr()), ctypes.c_void_p(Md.data_ptr()),
                                         int(X.shape[0]), int(steps), float(lr),
                                         ctypes.c_void_p(losses.data_ptr()), _stream()))
    torch.cuda.synchronize()
    return p.cpu().numpy(), losses.cpu().numpy()[:steps]


def install(params, mu, sd):
    fp = ctypes.POINTER(ctypes.c_float)
    a, b, c = (np.ascontiguousarray(x, np.float32) for x in (params, mu, sd))
    _lib.check(_lib.load().byo_selector_set(a.ctypes.data_as(fp), b.ctypes.data_as(fp), c.ctypes.data_as(fp)))


def clear():
    _lib.check(_lib.load().byo_selector_clear())


def loaded() -> bool:
    x = ctypes.c_int32()
    _lib.check(_lib.load().byo_selector_loaded(ctypes.byref(x)))
    return bool(x.value)


def predict(raw_features, allow_pull=True):
    """Device inference with the installed weights: (predictions[K], variant)."""
    fp = ctypes.POINTER(ctypes.c_float)
    f = np.ascontiguousarray(raw_features, np.float32)
    pred = (ctypes.c_float * K)()
    v = ctypes.c_int32()
    _lib.check(_lib.load().byo_selector_predict(f.ctypes.data_as(fp), 1 if allow_pull else 0, pred, ctypes.byref(v)))
    return np.array(pred[:], np.float32), v.value


def save(path, params, mu, sd, meta=None):
    with open(path, "w") as f:
        json.dump({"format": "byo-selector-v1", "F": F, "H": H, "K": K, "params": np.asarray(params).tolist(),
                   "mu": np.asarray(mu).tolist(), "sd": np.asarray(sd).tolist(), "meta": meta or {}}, f)


def load_weights(path):
    with open(path) as f:
        d = json.load(f)
    if d.get("format") != "byo-selector-v1" or (d["F"], d["H"], d["K"]) != (F, H, K):
        raise ValueError("unsupported selector weight file")
    return (np.array(d["params"], np.float32), np.array(d["mu"], np.float32), np.array(d["sd"], np.float32),
            d.get("meta", {}))


def evaluate(levels, choose):
    """Total time (sum of the timed ms) of the variants `choose(level)` picks."""
    tot = 0.0
    for lv in levels:
        v = choose(lv)
        t = lv["ms"][v]
        if not np.isfinite(t):
            t = np.nanmax(lv["ms"])
        tot += float(t)
    return tot


def forward(params, Xn):
    """Predictions [N, K] of the network on normalised features [N, F], by the
    library's forward kernel (byo_mlp_forward)."""
    torch = _torch()
    Xn = np.ascontiguousarray(Xn, np.float32)
    N = int(Xn.shape[0])
    p = torch.from_numpy(np.ascontiguousarray(params, np.float32)).cuda()
    Xd = torch.from_numpy(Xn).cuda()
    out = torch.empty((max(N, 1), K), dtype=torch.float32, device="cuda")
    _lib.check(_lib.load().byo_mlp_forward(ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(Xd.data_ptr()), N,
                                           ctypes.c_void_p(out.data_ptr()), _stream()))
    return out[:N].cpu().numpy()


def compare(levels, params, mu, sd, opts=None):
    """Sum of timed ms per policy over the levels: heuristic, learned, best."""
    X, _, _ = dataset(levels)
    pred = forward(params, (X - mu) / sd)
    learned = {id(lv): int(np.argmin(pred[i])) for i, lv in enumerate(levels)}
    return {
        "heuristic_ms": evaluate(levels, lambda lv: heuristic_choice(lv["rec"], opts)),
        "learned_ms": evaluate(levels, lambda lv: learned[id(lv)]),
        "best_ms": evaluate(levels, lambda lv: int(np.nanargmin(lv["ms"]))),
        "levels": len(levels),
    }
