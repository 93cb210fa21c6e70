"""ctypes signatures for the batched and learned-selector entry points."""
import ctypes

from ._lib import LevelRecord, Opts, RunStats, dbl, i32, i32p, i64, i64p, st, vp

SIGNATURES = {
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
    "byo_ktimer_reset": (st, []),
    "byo_ktimer_read": (st, [i32, i64p, ctypes.POINTER(dbl)]),

}
