"""ctypes declarations for libbyo.so (the C ABI in include/byo.h).

Argument marshalling only: every step of the traversal runs in the library's
HIP kernels. Importing fails loudly when the built library is missing; there is
no host fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbyo.so")

NUM_VARIANTS = 6
VARIANTS = ("push_thread", "push_wave", "push_bucket", "push_edge", "pull_thread", "pull_wave")
V_PUSH_THREAD, V_PUSH_WAVE, V_PUSH_BUCKET, V_PUSH_EDGE, V_PULL_THREAD, V_PULL_WAVE = range(6)
SEL_HEURISTIC, SEL_MLP, SEL_FIXED = 0, 1, 2
# optional graph-container functions a run may leave out (byo_opts.api_omit)
API_NO_DEGREE, API_NO_NUM_EDGES, API_NO_EARLY_EXIT, API_NO_PAR_MAP, API_NO_PAR_EARLY_EXIT = 1, 2, 4, 8, 16
# the container-API configurations of Table api-components-avg, as api_omit
API_CONFIGS = {
    "min": 31,                       # map_neighbors and num_vertices only
    "min+degree": 30,
    "min_efficient": 28,             # min + degree + num_edges
    "full-num_edges": 2,
    "full-degree": 1,
    "no_early_exit": 20,             # both early-exit maps left out
    "no_parallel_map": 24,           # both parallel maps left out
    "full-parallel_early_exit": 16,
    "full": 0,
}
F_BFS, F_CC_MIN, F_PR_ACC = 0, 1, 2
HOST_INPUT, DEVICE_COPY, DEVICE_BORROW, VALIDATE = 0x1, 0x2, 0x4, 0x8
NOALLOC_MAX_N = 1 << 21  # BYO_NOALLOC_MAX_N
# batch forms (byo_batch_order)
FORM_SORT, FORM_SEMISORT, FORM_GROUPED_SORT = 0, 1, 2

STATUS = {0: "BYO_OK", -1: "BYO_EINVAL", -2: "BYO_ENOMEM", -3: "BYO_EHIP", -4: "BYO_ELIMIT", -5: "BYO_ESTATE"}


class ByoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("selector", ctypes.c_int32), ("fixed_variant", ctypes.c_int32),
                ("dense_divisor", ctypes.c_int32), ("t_wave", ctypes.c_int32),
                ("t_block", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("cc_shortcut", ctypes.c_int32), ("small_frontier", ctypes.c_int32),
                ("pr_blocked", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("tiled", ctypes.c_int32), ("tile_shift", ctypes.c_int32), ("api_omit", ctypes.c_int32),
                ("ms_history", ctypes.c_int32), ("compressed", ctypes.c_int32),
                ("persistent", ctypes.c_int32)]


class RunStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("device_levels", ctypes.c_int32),
                ("variant_count", ctypes.c_int64 * NUM_VARIANTS),
                ("reached", ctypes.c_int64), ("edges", ctypes.c_int64)]

    def as_dict(self):
        return {"levels": self.levels, "device_levels": self.device_levels,
                "variant_count": dict(zip(VARIANTS, list(self.variant_count))),
                "reached": self.reached, "edges": self.edges}


class LevelRecord(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("level", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("dense_in", ctypes.c_int32), ("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("k", ctypes.c_int64), ("degsum", ctypes.c_int64), ("unvisited", ctypes.c_int64),
                ("out_count", ctypes.c_int64), ("out_degsum", ctypes.c_int64), ("max_deg", ctypes.c_int64),
                ("cv", ctypes.c_double), ("ms", ctypes.c_float), ("max_deg_u", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


K_FAMILIES = ("bfs_push", "bfs_pull", "cc_push", "cc_pull", "pr_pull", "pr_chunk", "msbfs_push", "msbfs_pull",
              "compact", "cc_shortcut", "msbfs_finish", "small_loop", "mlp")


class BfsFn(ctypes.Structure):
    _fields_ = [("parent", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("visited", ctypes.c_void_p),
                ("level", ctypes.c_int32)]


class CcFn(ctypes.Structure):
    _fields_ = [("label", ctypes.c_void_p)]


class PrFn(ctypes.Structure):
    _fields_ = [("contrib", ctypes.c_void_p), ("acc", ctypes.c_void_p)]


_lib = None

vp = ctypes.c_void_p
i32 = ctypes.c_int32
fp = ctypes.POINTER(ctypes.c_float)
i64 = ctypes.c_int64
u32 = ctypes.c_uint32
i64p = ctypes.POINTER(ctypes.c_int64)
i32p = ctypes.POINTER(ctypes.c_int32)
dbl = ctypes.c_double
dblp = ctypes.POINTER(ctypes.c_double)
st = ctypes.c_int

# name -> (restype, argtypes)
SIGNATURES = {
    "byo_last_error": (ctypes.c_char_p, []),
    "byo_version": (ctypes.c_char_p, []),
    "byo_opts_default": (None, [ctypes.POINTER(Opts)]),
    "byo_csr_from_pairs": (st, [vp, vp, i64, i64, vp, vp, i64p]),
    "byo_graph_from_csr": (st, [vp, vp, i64, i64, u32, vp, ctypes.POINTER(vp)]),
    "byo_graph_destroy": (None, [vp]),
    "byo_num_vertices": (i64, [vp]),
    "byo_num_edges": (i64, [vp]),
    "byo_degree": (st, [vp, i64, i64p]),
    "byo_get_neighbors": (st, [vp, i64, vp, i64, i64p]),
    "byo_graph_arrays": (st, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]),
    "byo_graph_stats": (st, [vp, i64p, i64p, dblp, dblp]),
    "byo_graph_copy": (st, [vp, vp, vp]),
    "byo_graph_insert_batch": (st, [vp, vp, vp, i64, vp, i64p]),
    "byo_graph_delete_batch": (st, [vp, vp, vp, i64, vp, i64p]),
    "byo_batch_order": (st, [vp, vp, i64, i64, i32, vp, vp, vp]),
    "byo_bc": (st, [vp, i64, vp, vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_kcore": (st, [vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_mis": (st, [vp, vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_coloring": (st, [vp, vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_densest": (st, [vp, dbl, vp, i64p, i64p, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_cz_build": (st, [vp, vp]),
    "byo_cz_bytes": (st, [vp, i64p]),
    "byo_cz_copy": (st, [vp, vp, vp]),
    "byo_cz_decode": (st, [vp, i64, vp, vp]),
    "byo_vset_create": (st, [vp, ctypes.POINTER(vp)]),
    "byo_vset_destroy": (None, [vp]),
    "byo_vset_from_ids": (st, [vp, vp, i64, vp]),
    "byo_vset_from_bitmap": (st, [vp, vp, vp]),
    "byo_vset_fill": (st, [vp, vp]),
    "byo_vset_size": (st, [vp, i64p, vp]),
    "byo_vset_to_ids": (st, [vp, vp, i64, i64p, vp]),
    "byo_vset_to_bitmap": (st, [vp, vp, vp]),
    "byo_edge_map": (st, [vp, vp, i32, vp, vp, i32, ctypes.POINTER(Opts), vp, i32p]),
    "byo_bfs": (st, [vp, i64, vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_bfs_noalloc": (st, [vp, i64, vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_cc": (st, [vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_pagerank": (st, [vp, dbl, i32, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    # batched execution, multi-source BFS, tracing and kernel timers (byo_trace.h), the learned
    # selector (byo_selector.h)
    "byo_selector_features": (st, [ctypes.POINTER(LevelRecord), fp]),
    "byo_heuristic_choice": (i32, [i64, i64, i64, i64, dbl, ctypes.POINTER(Opts), i32, i64]),
    "byo_mlp_forward": (st, [vp, vp, i32, vp, vp]),
    "byo_mlp_loss_grad": (st, [vp, vp, vp, vp, i32, vp, vp, vp]),
    "byo_mlp_adam": (st, [vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]),
    "byo_mlp_train": (st, [vp, vp, vp, vp, i32, i32, ctypes.c_float, vp, vp]),
    "byo_selector_set": (st, [fp, fp, fp]),
    "byo_selector_clear": (st, []),
    "byo_selector_loaded": (st, [i32p]),
    "byo_selector_predict": (st, [fp, i32, fp, i32p]),
    "byo_selector_collect": (st, [vp, i32, i64, i32, vp, ctypes.POINTER(Opts), vp]),
    "byo_batch_create": (st, [i32, vp, vp, vp, vp, ctypes.POINTER(vp)]),
    "byo_batch_destroy": (None, [vp]),
    "byo_batch_info": (st, [vp, i64p, i64p]),
    "byo_batch_vertex_offset": (st, [vp, i32, i64p]),
    "byo_batch_bfs": (st, [vp, vp, vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_batch_cc": (st, [vp, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_msbfs": (st, [vp, vp, i32, vp, ctypes.POINTER(Opts), vp, ctypes.POINTER(RunStats)]),
    "byo_trace_enable": (st, [i32]),
    "byo_trace_read": (st, [ctypes.POINTER(LevelRecord), i64, i64p]),
    "byo_trace_pending": (st, [i64p]),
    "byo_ktimer_enable": (st, [i32]),
    "byo_ktimer_select": (st, [ctypes.c_uint32]),
    "byo_ktimer_reset": (st, []),
    "byo_ktimer_read": (st, [i32, i64p, ctypes.POINTER(dbl)]),
}


def _declare(lib, sigs):
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2405_11671_amd.build.build() "
                              "(the HIP library is required: there is no fallback)")
        # torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
        # Load it first so the library binds to that one runtime: device pointers
        # and streams from torch then belong to the runtime the kernels use.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        _declare(lib, SIGNATURES)
        _lib = lib
    return _lib


def check(status: int):
    if status != 0:
        msg = load().byo_last_error().decode(errors="replace")
        raise ByoError(status, msg)


def default_opts(**kw) -> Opts:
    o = Opts()
    load().byo_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(f"unknown option {k}")
        setattr(o, k, int(v))
    return o
