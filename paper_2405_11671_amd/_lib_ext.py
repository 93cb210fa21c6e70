"""ctypes signatures for the batched and learned-selector entry points."""
import ctypes

from ._lib import LevelRecord, Opts, RunStats, dbl, i32, i32p, i64, i64p, st, vp

fp = ctypes.POINTER(ctypes.c_float)

SIGNATURES = {
    "byo_selector_features": (st, [ctypes.POINTER(LevelRecord), fp]),
    "byo_heuristic_choice": (i32, [i64, i64, i64, i64, dbl, ctypes.POINTER(Opts), i32]),
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
