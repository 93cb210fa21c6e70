"""ctypes signatures for the batched and learned-selector entry points."""
import ctypes

from ._lib import Opts, RunStats, dbl, i32, i32p, i64, i64p, st, vp

SIGNATURES = {

}
