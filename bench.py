"""Benchmark: GTEPS of the edgeMap hot path on RMAT scale 22 (one MI355X).

One step = multi-source BFS from 256 sources (bit-parallel batch) + PageRank
(20 steps, FP32) + connectivity, all on the same HBM-resident graph. TEPS
conventions:
  BFS: undirected edges in the reached component, summed over sources (Graph500),
  PageRank: iterations x m directed edges, connectivity: m/2 undirected edges.
value = all traversed edges of the timed steps / their wall time.
PageRank, the multi-source BFS and connectivity run over the degree-ordered
tile layout, built once per graph on first use and kept with it like the CSR
(its build time is reported in "detail"; `--no-tiles` runs them over the CSR
instead, connectivity then with the learned variant selector).
Single-source BFS from 16 sources is timed separately, with the threshold
heuristic ("plain") and with the learned selector, and reported in "detail"
next to the batched rate.

Prints ONE JSON line. `--probe pr|ms|cc|all` instead runs a few tiled
PageRank steps, multi-source BFS or connectivity calls and a plain 512 MiB
device copy, for hardware-counter runs (bytes per dispatch).
`--ablation` instead replays the container-API configurations of the paper's
Table api-components-avg, `--compression` compares the byte-coded CSR with
the CSR (one JSON line of per-case times and slowdowns each), and `--inserts`
measures batch-insert throughput against batch size.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
PR_SOURCE = os.path.join(ROOT, "paper_2405_11671_amd", "csrc", "pagerank_tile.hip")


def pr_kernels(n):
    """Names of the tiled PageRank step's kernels: the library takes tiles of
    2^12 vertices up to n = 2^22, 2^13 up to 2^23 and 2^14 beyond."""
    s = min(14, max(12, (max(n, 1) - 1).bit_length() - 10))
    return f"pr_tile_kernel<{s}> + pr_tile_apply_kernel<{s}> (one PageRank step)"


def source_tag(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:12]


def counter_traffic(kernel_tag):
    """HBM bytes per PageRank step (both tile kernels) from the committed
    counter summary, or None when it is missing or was taken on other source."""
    path = os.path.join(PROFILES, "pr_tile_rmat22_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ": " in line and line.startswith("- "):
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("pagerank_tile.hip sha256[:12]") != kernel_tag:
        return None
    try:
        return float(vals["scaled HBM bytes per step"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(pairs, srcs, args):
    """The oracle (single-threaded C) on a bounded sample of the same workload:
    single-source BFS from the first few of the multi-source batch's sources
    (the oracle's multi-source BFS is one BFS per source), a few PageRank
    steps and one connectivity run, counted like the GPU step."""
    import oracle
    og = oracle.Graph.from_pairs(pairs)
    ks = list(srcs[: args.cpu_sample_sources])
    t = time.perf_counter()
    depths = [og.bfs(int(s))[0] for s in ks]
    og.pagerank(0.85, args.cpu_sample_pr_iters)
    og.cc()
    el = time.perf_counter() - t
    deg = og.degrees()
    bfs_e = sum(int(deg[d >= 0].sum()) // 2 for d in depths)
    edges = bfs_e + args.cpu_sample_pr_iters * og.m + og.m // 2
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": round(edges / el / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "host": f"{model}; {os.cpu_count()} logical CPUs visible; the oracle uses one thread",
            "sample": f"BFS from {len(ks)} of the {args.ms_sources} multi-source BFS sources + "
                      f"{args.cpu_sample_pr_iters} PageRank steps (FP64) + CC on the same rmat-{args.scale} graph; "
                      f"{el:.1f} s"}


def grid_workload(byo, gen, mlp_opts, side):
    """Road-like lattice (side x side, 10% of edges deleted): BFS from the corner
    and connectivity under the threshold heuristic, the learned selector and the
    device-resident small-frontier loop (median of 3 runs each, ms)."""
    import torch
    p = gen.grid_pairs(side, side, 0.1, seed=1)
    g = byo.Graph.from_pairs(p)
    depth = torch.empty(g.n, dtype=torch.int32, device="cuda")
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    label = torch.empty(g.n, dtype=torch.int32, device="cuda")

    def timed(fn):
        fn()
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        return float(np.median(ts)), st

    res = {"n": g.n, "m": g.m}
    cases = {"heuristic": byo.default_opts(), "learned": mlp_opts,
             "heuristic_device_loop": byo.default_opts(small_frontier=8192),
             "learned_device_loop": byo.default_opts(selector=byo.SEL_MLP, small_frontier=8192)}
    for name, o in cases.items():
        ms, st = timed(lambda: byo.bfs(g, 0, opts=o, depth=depth, parent=parent)[2])
        res[f"bfs_{name}_ms"] = round(ms, 3)
        res["bfs_levels"] = st["levels"]
    centre = (side // 2) * side + side // 2
    for name in ("heuristic", "heuristic_device_loop"):
        ms, stc = timed(lambda: byo.bfs(g, centre, opts=cases[name], depth=depth, parent=parent)[2])
        res[f"bfs_centre_{name}_ms"] = round(ms, 3)
        res["bfs_centre_levels"] = stc["levels"]
    res["bfs_gteps_best"] = round(st["edges"] / 2 / (min(res[f"bfs_{c}_ms"] for c in cases) * 1e-3) / 1e9, 4)
    for name, o in (("heuristic", byo.default_opts()), ("learned", mlp_opts)):
        ms, st = timed(lambda: byo.cc(g, opts=o, label=label)[1])
        res[f"cc_{name}_ms"] = round(ms, 3)
        res["cc_rounds"] = st["levels"]
    res["learned_vs_heuristic_bfs"] = round(res["bfs_heuristic_ms"] / res["bfs_learned_ms"], 3)
    res["device_loop_vs_host_loop_bfs"] = round(res["bfs_heuristic_ms"] / res["bfs_heuristic_device_loop_ms"], 3)
    del g
    return res


def bc_workload(byo, g, srcs):
    """Single-source betweenness (forward path counting + backward dependency
    pass) on the benchmark graph: median ms per source over 3 rounds, and
    GTEPS counting each reached undirected edge once per source."""
    import torch
    n = g.n
    delta = torch.empty(n, dtype=torch.float64, device="cuda")
    sigma = torch.empty(n, dtype=torch.float64, device="cuda")
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    run = lambda s: byo.bc(g, int(s), delta=delta, sigma=sigma, depth=depth)[3]  # noqa: E731
    for s in srcs:
        run(s)
    per, edges = [], 0
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        edges = sum(run(s)["edges"] // 2 for s in srcs)
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t) * 1e3 / len(srcs))
    ms = float(np.median(per))
    return {"sources": len(srcs), "ms_per_source": round(ms, 3),
            "gteps": round(edges / len(srcs) / (ms * 1e-3) / 1e9, 2)}


def kcore_workload(byo, g):
    """k-core decomposition of the benchmark graph: median of 3 runs (ms),
    sub-rounds, and the largest coreness."""
    import torch
    core = torch.empty(g.n, dtype=torch.int32, device="cuda")
    byo.kcore(g, core=core)
    ts, st = [], None
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = byo.kcore(g, core=core)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    return {"ms": round(float(np.median(ts)), 3), "sub_rounds": st["levels"], "max_core": int(core.max().item())}


def mis_workload(byo, g):
    """Greedy maximal independent set and greedy colouring of the benchmark
    graph in one seeded random priority order: median of 3 runs (ms), rounds,
    the set's size and the number of colours."""
    import torch
    prio = torch.from_numpy(np.random.default_rng(3).integers(0, 2 ** 63, g.n, dtype=np.uint64).view(np.int64))
    prio = prio.to("cuda")
    out = torch.empty(g.n, dtype=torch.uint8, device="cuda")
    byo.mis(g, prio, in_set=out)
    ts, st = [], None
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = byo.mis(g, prio, in_set=out)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    res = {"ms": round(float(np.median(ts)), 3), "rounds": st["levels"], "size": int(out.sum().item())}
    # greedy colouring in the same order
    color = torch.empty(g.n, dtype=torch.int32, device="cuda")
    byo.coloring(g, prio, color=color)
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = byo.coloring(g, prio, color=color)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1e3)
    res.update({"coloring_ms": round(float(np.median(ts)), 3), "coloring_rounds": st["levels"],
                "colours": int(color.max().item()) + 1})
    return res


def batch_workload(byo, gen, count=64):
    """64 Erdos-Renyi graphs (n log-uniform in [2^10, 2^18], average degree in
    [4, 32]), BFS from the first non-isolated vertex of each: 64 separate
    single-source runs against one batched traversal (one persistent launch,
    the default; the host level loop; hipGraph-replayed device-side levels;
    and autotuned options)."""
    import tempfile
    import torch
    from paper_2405_11671_amd import autotune
    plist = gen.batch_pairs(count, seed=3)
    B = byo.Batch.from_pairs(plist)
    gs = [byo.Graph.from_pairs(p) for p in plist]
    srcs = []
    # first non-isolated vertex of each graph, from the host CSR
    for p in plist:
        off, _ = byo.csr_from_pairs(p.n, p.src, p.dst)
        nz = np.flatnonzero(np.diff(off))
        srcs.append(int(nz[0]) if nz.size else 0)

    def timed(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)), st

    def separate():
        e = 0
        for g, s_ in zip(gs, srcs):
            e += byo.bfs(g, s_)[2]["edges"]
        return {"edges": e}

    res = {"graphs": count, "n": B.n, "m": B.m}
    t_sep, st = timed(separate)
    edges = st["edges"] // 2
    t_pers, pst = timed(lambda: B.bfs(srcs)[2])          # the default: one persistent launch
    t_eager, _ = timed(lambda: B.bfs(srcs, persistent=0)[2])
    t_graph, _ = timed(lambda: B.bfs(srcs, use_graph=1, persistent=0)[2])
    cache = os.path.join(tempfile.gettempdir(), "byo_bench_tune.json")
    opts, rep = autotune.tune_batch(B, srcs, repeats=2, cache=cache, refresh=True)
    t_tuned, _ = timed(lambda: B.bfs(srcs, opts=byo.default_opts(**opts))[2])
    best = min(t_pers, t_eager, t_graph, t_tuned)
    res.update({"separate_ms": round(t_sep * 1e3, 3), "batched_persistent_ms": round(t_pers * 1e3, 3),
                "batched_levels": pst["levels"], "batched_eager_ms": round(t_eager * 1e3, 3),
                "batched_graph_ms": round(t_graph * 1e3, 3), "batched_tuned_ms": round(t_tuned * 1e3, 3),
                "tuned_opts": opts, "separate_gteps": round(edges / t_sep / 1e9, 3),
                "batched_persistent_gteps": round(edges / t_pers / 1e9, 3),
                "batched_best_gteps": round(edges / best / 1e9, 3)})
    res["batched_vs_separate"] = round(t_sep / best, 3)
    return res


PAPER_RMAT_ABCD = (0.5, 0.1, 0.1, 0.3)   # the paper's rMAT generator setting (Section 5)


def api_ablation(byo, gen, args):
    """Container-API ablation (Section 4.2, Table api-components-avg): the same
    CSR container and host-driven level loop, with optional container functions
    left out. BFS (total over the sources), connectivity, PageRank
    (args.pr_iters steps), single-source betweenness and k-core per graph and
    configuration, median of 3 timed runs after one untimed run; slowdown =
    time / time with the full API. Summaries per configuration over every
    (graph, algorithm) case: mean, 95th percentile and maximum, as the table
    reports them."""
    configs = [(k, {"api_omit": v}) for k, v in sorted(byo.API_CONFIGS.items(), key=lambda kv: kv[1])]
    container_study(byo, gen, args, configs, "full", "container API (Table api-components-avg)",
                    "slowdown over full API", extra_algos=True)


def compression_study(byo, gen, args):
    """CSR against the byte-coded CSR (the paper's compressed CSR row of its
    container tables) on the same graphs, algorithms and host-driven level loop;
    slowdown = time / CSR time, and bytes per edge of each container."""
    container_study(byo, gen, args, [("csr", {}), ("byte-coded csr", {"compressed": 1})], "csr",
                    "byte-coded CSR against CSR", "slowdown over CSR")


def container_study(byo, gen, args, configs, base_name, title, unit, extra_algos=False):
    """Times BFS, connectivity and PageRank per graph and configuration (opts
    keyword sets); see api_ablation."""
    import torch
    graphs = [
        (f"rmat-{args.scale} graph500", lambda: gen.rmat_pairs(args.scale, 16, gen.GRAPH500_ABCD, seed=1)),
        (f"rmat-{args.scale - 1} paper abcd", lambda: gen.rmat_pairs(args.scale - 1, 16, PAPER_RMAT_ABCD, seed=3)),
        (f"er n=2^{args.scale - 1} d=50", lambda: gen.er_pairs(1 << (args.scale - 1), 50, seed=4)),
        ("grid 2048x2048 del0.1", lambda: gen.grid_pairs(2048, 2048, 0.1, seed=1)),
    ]
    cases = []
    sizes = {}
    for gname, make in graphs:
        p = make()
        srcs = [int(s) for s in gen.pick_sources(p, 2, seed=5)]
        off, nbr = byo.csr_from_pairs(p.n, p.src, p.dst)
        del p
        g = byo.Graph.from_csr(off, nbr)
        n, m = g.n, g.m
        del off, nbr
        depth = torch.empty(n, dtype=torch.int32, device="cuda")
        parent = torch.empty(n, dtype=torch.int32, device="cuda")
        label = torch.empty(n, dtype=torch.int32, device="cuda")
        rank = torch.empty(n, dtype=torch.float32, device="cuda")
        algos = {
            "bfs": lambda o: [byo.bfs(g, s, opts=o, depth=depth, parent=parent) for s in srcs],
            "cc": lambda o: byo.cc(g, opts=o, label=label),
            "pagerank": lambda o: byo.pagerank(g, 0.85, args.pr_iters, opts=o, rank=rank),
        }
        if extra_algos:
            dl = torch.empty(n, dtype=torch.float64, device="cuda")
            sg = torch.empty(n, dtype=torch.float64, device="cuda")
            algos["bc"] = lambda o: byo.bc(g, srcs[0], opts=o, delta=dl, sigma=sg, depth=depth)
            algos["kcore"] = lambda o: byo.kcore(g, opts=o, core=label)
        if any(kw.get("compressed") for _, kw in configs):
            g.cz_build()
            nbytes = ctypes.c_int64()
            byo._lib.check(byo._lib.load().byo_cz_bytes(g.handle, ctypes.byref(nbytes)))
            sizes[gname] = {"csr_bytes_per_edge": round((8 * (n + 1) + 4 * m) / m, 3),
                            "cz_bytes_per_edge": round((8 * (n + 1) + nbytes.value) / m, 3),
                            "cz_list_bytes_per_edge": round(nbytes.value / m, 3)}
        for cname, kw in configs:
            # the CSR container throughout (the tile layout is a second container)
            o = byo.default_opts(pr_blocked=0, tiled=0, **kw)
            for aname, fn in algos.items():
                fn(o)
                ts = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    fn(o)
                    torch.cuda.synchronize()
                    ts.append((time.perf_counter() - t) * 1e3)
                cases.append({"graph": gname, "n": n, "m": m, "algo": aname, "config": cname,
                              "ms": round(float(np.median(ts)), 4)})
            log(f"[study] {gname} {cname}: " + " ".join(f"{c['algo']}={c['ms']:.2f}ms" for c in cases[-len(algos):]))
        del g, depth, parent, label, rank, algos
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    base = {(c["graph"], c["algo"]): c["ms"] for c in cases if c["config"] == base_name}
    for c in cases:
        c["slowdown"] = round(c["ms"] / base[(c["graph"], c["algo"])], 4)
    summary = {}
    for cname, kw in configs:
        sl = np.array([c["slowdown"] for c in cases if c["config"] == cname])
        summary[cname] = {"opts": kw, "mean": round(float(sl.mean()), 3),
                          "p95": round(float(np.percentile(sl, 95)), 3), "max": round(float(sl.max()), 3)}
    print(json.dumps({"study": title, "unit": unit, "summary": summary, "sizes": sizes or None, "cases": cases}),
          flush=True)


def config_study(byo, gen, args):
    """The other quoted workloads next to the oracle on this host's cores:
    ER n=2^14 (average degree 8), RMAT-20 and the 4096^2 lattice with 10% of
    edges deleted. GPU: BFS from each listed source under the threshold rule
    and the learned selector, connectivity, PageRank; oracle (one thread): the
    same calls on a bounded sample. Rates in GTEPS counting each reached edge
    once for BFS and connectivity and every edge per PageRank step."""
    import torch
    import oracle
    from paper_2405_11671_amd import selector as sel
    params, mu, sd, _ = sel.load_weights(os.path.join(ROOT, "paper_2405_11671_amd", "selector_weights.json"))
    sel.install(params, mu, sd)
    out = {}
    cases = [
        ("er14", gen.er_pairs(1 << 14, 8.0, seed=1), "first", 20, 1, 20, 1),
        ("rmat20", gen.rmat_pairs(20, 16, gen.GRAPH500_ABCD, seed=1, permute=True), 16, 10, 4, 10, 1),
        ("lattice4096", gen.grid_pairs(4096, 4096, 0.1, seed=1), "corner", 0, 1, 0, 1),
    ]
    for name, p, src_spec, pr_iters, cpu_bfs, cpu_pr, cpu_cc in cases:
        log(f"[configs] {name}: n={p.n}")
        g = byo.Graph.from_pairs(p)
        if src_spec == "first" or src_spec == "corner":
            srcs = [0]
        else:
            srcs = [int(x) for x in gen.pick_sources(p, src_spec, seed=2)]
        depth = torch.empty(g.n, dtype=torch.int32, device="cuda")
        parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
        label = torch.empty(g.n, dtype=torch.int32, device="cuda")
        rank = torch.empty(g.n, dtype=torch.float32, device="cuda")

        def gpu(o):
            e, t0 = 0, time.perf_counter()
            for s_ in srcs:
                _, _, st = byo.bfs(g, s_, opts=o, depth=depth, parent=parent)
                e += st["edges"] // 2
            torch.cuda.synchronize()
            return e, time.perf_counter() - t0

        def best(fn, reps=3):
            fn()
            return min(fn() for _ in range(reps))

        plain = byo.default_opts()
        learned = byo.default_opts(selector=byo.SEL_MLP)
        e_bfs, t_plain = best(lambda: gpu(plain))
        _, t_learned = best(lambda: gpu(learned))

        def cc_pr():
            t0 = time.perf_counter()
            byo.cc(g, label=label)
            if pr_iters:
                byo.pagerank(g, 0.85, pr_iters, rank=rank)
            torch.cuda.synchronize()
            return time.perf_counter() - t0
        t_ccpr = best(cc_pr)
        gpu_edges = e_bfs + g.m // 2 + pr_iters * g.m
        row = {"n": g.n, "m": g.m, "bfs_sources": len(srcs), "pr_iters": pr_iters,
               "gpu_bfs_gteps": round(e_bfs / t_plain / 1e9, 3),
               "gpu_bfs_learned_gteps": round(e_bfs / t_learned / 1e9, 3),
               "gpu_all_gteps": round(gpu_edges / (t_plain + t_ccpr) / 1e9, 3),
               "gpu_all_ms": round((t_plain + t_ccpr) * 1e3, 3)}
        og = oracle.Graph.from_pairs(p)
        deg = og.degrees()
        t0 = time.perf_counter()
        e_cpu = 0
        for s_ in srcs[:cpu_bfs]:
            d, _ = og.bfs(s_)
            e_cpu += int(deg[d >= 0].sum()) // 2
        if cpu_cc:
            og.cc()
            e_cpu += og.m // 2
        if cpu_pr:
            og.pagerank(0.85, cpu_pr)
            e_cpu += cpu_pr * og.m
        el = time.perf_counter() - t0
        row.update({"cpu_gteps": round(e_cpu / el / 1e9, 4), "cpu_s": round(el, 2),
                    "cpu_sample": f"BFS from {min(cpu_bfs, len(srcs))} source(s)" + (" + CC" if cpu_cc else "")
                                  + (f" + {cpu_pr} PageRank steps (FP64)" if cpu_pr else ""),
                    "gpu_over_cpu": round((gpu_edges / (t_plain + t_ccpr)) / (e_cpu / el), 1)})
        out[name] = row
        log(f"[configs] {name}: {row}")
        del og, g
    print(json.dumps({"configs": out, "cpu_cores": 1}), flush=True)


def insert_study(byo, gen, args):
    """Batch-insert throughput against batch size (Section 6.6, fig
    inserts_with_sort): on the RMAT graph of the benchmark (the stand-in for
    the paper's billion-edge base graph), a batch of pairs drawn from an RMAT
    generator with (a, b, c, d) = (0.5, 0.1, 0.1, 0.3) is inserted and then
    deleted, three times per batch size; edges per second = batch pairs / time
    of the call (the batch's sort included, as in the paper's measurement).
    The three batch forms are timed on the same batches."""
    import torch
    pairs = gen.rmat_pairs(args.scale, 16, gen.GRAPH500_ABCD, seed=1, permute=True)
    off, nbr = byo.csr_from_pairs(pairs.n, pairs.src, pairs.dst)
    n = pairs.n
    del pairs
    torch.cuda.init()
    g = byo.Graph.from_csr(off, nbr)
    m0 = g.m
    del off, nbr
    sizes = [10 ** e for e in range(1, 9)]
    big = gen.rmat_pairs(args.scale, max(1, sizes[-1] >> args.scale) + 1, (0.5, 0.1, 0.1, 0.3), seed=9)
    src_all = torch.from_numpy(big.src).to("cuda")
    dst_all = torch.from_numpy(big.dst).to("cuda")
    del big
    cases = []
    for k in sizes:
        s_, d_ = src_all[:k].contiguous(), dst_all[:k].contiguous()
        ins, dele, added = [], [], []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            added.append(g.insert_batch(s_, d_))
            torch.cuda.synchronize()
            ins.append(time.perf_counter() - t)
            t = time.perf_counter()
            g.delete_batch(s_, d_)
            torch.cuda.synchronize()
            dele.append(time.perf_counter() - t)
        forms = {}
        for name, form in (("sort", byo.FORM_SORT), ("semisort", byo.FORM_SEMISORT),
                           ("grouped_sort", byo.FORM_GROUPED_SORT)):
            byo.batch_order(s_, d_, n, form)
            ts = []
            for _ in range(3):
                torch.cuda.synchronize()
                t = time.perf_counter()
                byo.batch_order(s_, d_, n, form)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            forms[name] = round(float(np.median(ts)) * 1e3, 4)
        ti, td = float(np.median(ins)), float(np.median(dele))
        cases.append({"batch": k, "insert_ms": round(ti * 1e3, 4), "delete_ms": round(td * 1e3, 4),
                      "insert_edges_per_s": round(k / ti, 1), "delete_edges_per_s": round(k / td, 1),
                      "entries_added": int(np.median(added)), "m_after": g.m, "order_ms": forms})
        log(f"[inserts] batch {k}: insert {ti * 1e3:.3f} ms ({k / ti:.3g} edges/s), delete {td * 1e3:.3f} ms")
    print(json.dumps({"study": "batch inserts (Section 6.6)", "unit": "edges/s",
                      "graph": f"rmat-{args.scale} n={n} m={m0}", "cases": cases}), flush=True)


def probe(g, n, what, ms_srcs, iters=3):
    """Short runs for hardware-counter passes (bytes per dispatch): the tiled
    PageRank (a 1-step call that builds the layout, then an `iters`-step
    call), the tiled 256-source BFS and the tiled connectivity (each once to
    warm up, once more), then a plain 512 MiB elementwise kernel to calibrate
    the counters."""
    import torch
    import paper_2405_11671_amd as byo
    tiled = byo.default_opts(pr_blocked=1, tiled=1)
    if what in ("pr", "all"):
        rank = torch.empty(n, dtype=torch.float32, device="cuda")
        byo.pagerank(g, 0.85, 1, rank=rank, opts=tiled)    # builds the tile layout
        torch.cuda.synchronize()
        byo.pagerank(g, 0.85, iters, rank=rank, opts=tiled)
    if what in ("ms", "all"):
        depth = torch.empty(n * len(ms_srcs), dtype=torch.uint8, device="cuda")
        for _ in range(2):
            byo.msbfs(g, ms_srcs, opts=tiled, depth=depth)
    if what in ("cc", "all"):
        label = torch.empty(n, dtype=torch.int32, device="cuda")
        for _ in range(2):
            byo.cc(g, opts=tiled, label=label)
    # calibration: an elementwise kernel that reads 512 MiB and writes 512 MiB
    a = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"probe": what, "iters": iters, "copy_bytes": 512 << 20}), flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--sources", type=int, default=16)
    ap.add_argument("--pr-iters", type=int, default=20)
    ap.add_argument("--ms-sources", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-sources", type=int, default=6)
    ap.add_argument("--cpu-sample-pr-iters", type=int, default=6)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--probe", choices=["pr", "ms", "cc", "all"], default=None)
    ap.add_argument("--ablation", action="store_true",
                    help="replay the container-API configurations instead of the benchmark step")
    ap.add_argument("--compression", action="store_true",
                    help="compare the byte-coded CSR with the CSR instead of the benchmark step")
    ap.add_argument("--inserts", action="store_true",
                    help="batch-insert throughput against batch size instead of the benchmark step")
    ap.add_argument("--configs", action="store_true",
                    help="ER-14, RMAT-20 and the 4096^2 lattice on the GPU next to the oracle on this host")
    ap.add_argument("--no-grid", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-bc", action="store_true", help="skip the betweenness and k-core detail")
    ap.add_argument("--mis", action="store_true", help="also time greedy MIS and colouring (outside the hot path)")
    ap.add_argument("--grid-side", type=int, default=4096)
    ap.add_argument("--no-tiles", action="store_true",
                    help="PageRank and multi-source BFS over the CSR instead of the tile layout")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only (the library has no multi-GPU path); run with --gpus 1"}))
        sys.exit(2)
    import torch
    import paper_2405_11671_amd as byo
    from paper_2405_11671_amd import gen

    if args.inserts:
        insert_study(byo, gen, args)
        return
    if args.configs:
        torch.cuda.init()
        config_study(byo, gen, args)
        return
    if args.ablation or args.compression:
        torch.cuda.init()
        (api_ablation if args.ablation else compression_study)(byo, gen, args)
        return
    t0 = time.time()
    pairs = gen.rmat_pairs(args.scale, 16, gen.GRAPH500_ABCD, seed=1, permute=True)
    srcs = gen.pick_sources(pairs, args.sources, seed=2)
    off, nbr = byo.csr_from_pairs(pairs.n, pairs.src, pairs.dst)
    n, m = pairs.n, int(off[-1])
    log(f"[bench] rmat-{args.scale}: n={n} m={m} built in {time.time() - t0:.1f}s")
    torch.cuda.init()
    g = byo.Graph.from_csr(off, nbr)
    torch.cuda.synchronize()
    if args.probe:
        probe(g, n, args.probe, gen.pick_sources(pairs, args.ms_sources, seed=2))
        return
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    label = torch.empty(n, dtype=torch.int32, device="cuda")
    rank = torch.empty(n, dtype=torch.float32, device="cuda")
    opts = byo.default_opts()
    tiled = byo.default_opts(pr_blocked=0 if args.no_tiles else 1, tiled=0 if args.no_tiles else 1)
    from paper_2405_11671_amd import selector as sel
    wpath = os.path.join(ROOT, "paper_2405_11671_amd", "selector_weights.json")
    params, mu, sd, _ = sel.load_weights(wpath)
    sel.install(params, mu, sd)
    mlp_opts = byo.default_opts(selector=byo.SEL_MLP)
    mlp_csr_opts = byo.default_opts(selector=byo.SEL_MLP, tiled=0, pr_blocked=0)
    # the whole single-source search in one persistent launch (opt-in)
    pers_opts = byo.default_opts(persistent=2)

    ms_srcs = gen.pick_sources(pairs, args.ms_sources, seed=2)
    ms_depth = torch.empty(n * len(ms_srcs), dtype=torch.uint8, device="cuda")

    def step(record=None):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        _, mst = byo.msbfs(g, ms_srcs, opts=tiled, depth=ms_depth)
        ev[1].record()
        byo.pagerank(g, 0.85, args.pr_iters, opts=tiled, rank=rank)
        ev[2].record()
        _, cst = byo.cc(g, opts=tiled if not args.no_tiles else mlp_csr_opts, label=label)
        ev[3].record()
        ms_edges = mst["edges"] // 2
        if record is not None:
            torch.cuda.synchronize()
            record.append({"ms_ms": ev[0].elapsed_time(ev[1]), "pr_ms": ev[1].elapsed_time(ev[2]),
                           "cc_ms": ev[2].elapsed_time(ev[3]), "ms_edges": ms_edges,
                           "ms_levels": mst["levels"], "cc_rounds": cst["levels"]})
        return ms_edges

    def single_bfs(o, per_source=None):
        torch.cuda.synchronize()
        t = time.perf_counter()
        e = 0
        for s_ in srcs:
            t1 = time.perf_counter()
            _, _, st = byo.bfs(g, int(s_), opts=o, depth=depth, parent=parent)
            e += st["edges"] // 2
            if per_source is not None:  # Graph500 per-source rate (the call returns after its last level sync)
                per_source.append(st["edges"] / 2 / (time.perf_counter() - t1) / 1e9)
        torch.cuda.synchronize()
        return e / (time.perf_counter() - t) / 1e9

    def plain_bfs():
        return single_bfs(opts)

    def learned_bfs():
        return single_bfs(mlp_opts)

    # the degree-ordered tile layout is built once per graph, on first use,
    # and kept with it (like the CSR); its build time is reported, not timed
    torch.cuda.synchronize()
    t = time.perf_counter()
    byo.pagerank(g, 0.85, 1, opts=tiled, rank=rank)
    torch.cuda.synchronize()
    layout_s = time.perf_counter() - t
    for _ in range(args.warmup):
        step()
        plain_bfs()
        learned_bfs()
    torch.cuda.synchronize()
    rec = []
    # HIP events around the roofline kernels (the PageRank step) in the timed
    # region; timing every family would add host time to the level loops
    byo.ktimer_reset()
    byo.ktimer_select(["pr_pull", "pr_chunk"])
    byo.ktimer_enable(True)
    t = time.perf_counter()
    edges_total = 0
    for _ in range(args.steps):
        ms_e = step(rec)
        edges_total += ms_e + args.pr_iters * m + m // 2
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    byo.ktimer_enable(False)
    kt = {f: byo.ktimer_read(f) for f in byo._lib.K_FAMILIES}
    # per-family kernel time from one more step, untimed, with every family recorded
    byo.ktimer_reset()
    byo.ktimer_select(None)
    byo.ktimer_enable(True)
    step()
    torch.cuda.synchronize()
    byo.ktimer_enable(False)
    kt_all = {f: byo.ktimer_read(f) for f in byo._lib.K_FAMILIES}
    ms_per_step = wall * 1e3 / args.steps
    value = edges_total / wall / 1e9
    plain = [plain_bfs() for _ in range(3)]
    learned = [learned_bfs() for _ in range(3)]
    single_bfs(pers_opts)  # the first call sets up the launch's workspace
    persist = [single_bfs(pers_opts) for _ in range(3)]
    per_plain, per_learned = [], []
    single_bfs(opts, per_plain)
    single_bfs(mlp_opts, per_learned)
    hmean = lambda xs: len(xs) / sum(1.0 / x for x in xs)  # noqa: E731
    ms_ms = float(np.median([r["ms_ms"] for r in rec]))
    pr_ms = float(np.median([r["pr_ms"] for r in rec]))
    cc_ms = float(np.median([r["cc_ms"] for r in rec]))
    pr_launches, pr_kms = kt["pr_pull"]
    pr_avg_ms = (pr_kms + kt["pr_chunk"][1]) / max(pr_launches, 1)   # tile kernel + apply kernel per step
    # compulsory bytes of one PageRank step (the hot-path scope's count): the
    # neighbour lists 4m, the offsets 8(n+1), the rank or contribution read
    # 4n, the contribution write and read 8n, the rank write 4n
    pr_bytes = 4 * m + 8 * (n + 1) + 16 * n
    # what the tiled step itself must touch: entry words 4m, relabelled degrees,
    # contributions read and written (no offsets: the layout has none)
    pr_bytes_tiled = 4 * m + 12 * n
    # the other tile passes of the step, per launch, from the untimed step's
    # kernel timers: a dense multi-source level and a tiled connectivity round
    # each stream the entry words once (4m); connectivity also reads each
    # label once (4n). Lower bounds on their bytes.
    fam_bytes = {"msbfs_pull": (4 * m, "4m: one pass over the entry words"),
                 "cc_pull": (4 * m + 4 * n, "4m + 4n: the entry words and each label once")}
    family_roofline = {}
    for fam, (nbytes, model) in fam_bytes.items():
        launches, kms = kt_all.get(fam, (0, 0.0))
        if launches:
            avg = kms / launches
            family_roofline[fam] = {"launches": launches, "avg_launch_ms": round(avg, 4), "bytes_model": model,
                                    "achieved_gbs": round(nbytes / (avg * 1e-3) / 1e9, 1),
                                    "frac": round(nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    bc = None if args.no_bc else bc_workload(byo, g, srcs[:4])
    kcore = None if args.no_bc else kcore_workload(byo, g)
    mis = mis_workload(byo, g) if args.mis else None
    grid = None if args.no_grid else grid_workload(byo, gen, mlp_opts, args.grid_side)
    batch = None if args.no_batch else batch_workload(byo, gen)
    detail = {
        "msbfs_gteps": rec[0]["ms_edges"] / (ms_ms * 1e-3) / 1e9, "msbfs_ms": ms_ms,
        "msbfs_sources": len(ms_srcs), "msbfs_levels": rec[0]["ms_levels"],
        "pr_gteps": args.pr_iters * m / (pr_ms * 1e-3) / 1e9, "pr_ms": pr_ms,
        "cc_ms": cc_ms, "cc_rounds": rec[0]["cc_rounds"],
        "plain_bfs_gteps": float(np.median(plain)),
        "plain_bfs_gteps_hmean": hmean(per_plain), "learned_bfs_gteps_hmean": hmean(per_learned),
        "step_ms_median": float(np.median([r["ms_ms"] + r["pr_ms"] + r["cc_ms"] for r in rec])),
        "step_ms_mean": float(np.mean([r["ms_ms"] + r["pr_ms"] + r["cc_ms"] for r in rec])),
        "learned_bfs_gteps": float(np.median(learned)),
        "learned_vs_plain": float(np.median(learned)) / float(np.median(plain)),
        "persistent_bfs_gteps": float(np.median(persist)),
        "persistent_vs_plain": float(np.median(persist)) / float(np.median(plain)),
        "batched_vs_plain": rec[0]["ms_edges"] / (ms_ms * 1e-3) / 1e9 / float(np.median(plain)),
        "pr_step_avg_ms": pr_avg_ms, "pr_step_alg_gbs": pr_bytes / (pr_avg_ms * 1e-3) / 1e9,
        "pr_step_tiled_bytes": pr_bytes_tiled,
        "pr_step_tiled_frac": pr_bytes_tiled / (pr_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "tile_layout_build_s": layout_s, "tiled": not args.no_tiles,
        "kernel_ms": {f: round(v[1], 3) for f, v in kt_all.items() if v[0]},
        "family_roofline": family_roofline,
        "bc": bc,
        "kcore": kcore,
        "mis": mis,
        "grid": grid,
        "batch64": batch,
    }
    # the committed counters were taken on the RMAT-22 workload with the tile layout
    traffic = counter_traffic(source_tag(PR_SOURCE)) if (not args.no_tiles and args.scale == 22) else None
    achieved = pr_bytes / (pr_avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": pr_kernels(g.n) if not args.no_tiles else "pr_chunk_kernel + pr_pull_kernel<0>",
                "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic / (pr_avg_ms * 1e-3) / 1e9, 2),
                "alg_bytes_per_launch": pr_bytes, "avg_launch_ms": round(pr_avg_ms, 4),
                "launches": pr_launches}
    cpu = None if args.no_cpu_baseline else cpu_baseline(pairs, ms_srcs, args)
    out = {
        "metric": f"GTEPS (batched BFS + PageRank + CC edgeMap traversals) on RMAT-{args.scale}",
        "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32+f32", "data": "synthetic",
        "config": {"workload": f"rmat-{args.scale} ef16 (0.57,0.19,0.19,0.05) symmetrized; "
                               f"msbfs x{len(ms_srcs)} + pagerank {args.pr_iters} it + cc", "n": n, "m": m},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {k: round(v, 4) if isinstance(v, float) else v for k, v in detail.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
