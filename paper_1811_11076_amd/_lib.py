"""ctypes view of the C-ABI in include/tsknn.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

from .build import lib_path

TSK_OK = 0
TSK_ERR_INVALID_ARG = 1
TSK_ERR_OOM = 2
TSK_ERR_DEVICE = 3
TSK_ERR_UNSUPPORTED = 4
TSK_ERR_IO = 5
TSK_ERR_CANCELLED = 6

TSK_DTW, TSK_DK = 0, 1
TSK_BAND_NONE, TSK_BAND_ABS, TSK_BAND_FRAC = 0, 1, 2
TSK_ORDER_PLAIN, TSK_ORDER_GIVEN, TSK_ORDER_LEARNED = 0, 1, 2
TSK_TUNE_OFF, TSK_TUNE_CACHED = 0, 1

_ERRNAMES = {1: "INVALID_ARG", 2: "OOM", 3: "DEVICE", 4: "UNSUPPORTED", 5: "IO", 6: "CANCELLED"}


class TskError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tsknn error {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Band(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("r", ctypes.c_int32), ("frac", ctypes.c_float)]


class QueryOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int64), ("order", ctypes.c_int32), ("seed_count", ctypes.c_int32),
                ("order_dev", ctypes.c_void_p), ("use_graph", ctypes.c_int32),
                ("dp_kernel", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("walk_pass", ctypes.c_int32), ("task_size", ctypes.c_int32),
                ("tube_rows", ctypes.c_int32), ("lb_qgroup", ctypes.c_int32),
                ("dk_band_slots", ctypes.c_int32), ("surv_order", ctypes.c_int32),
                ("dp_rows", ctypes.c_int32), ("dp_waves_per_cu", ctypes.c_int32),
                ("dk_seed", ctypes.c_int32),
                ("tune", ctypes.c_int32),
                ("model", ctypes.c_void_p),
                ("cancel_flag_host", ctypes.c_void_p),
                ("lb_both", ctypes.c_int32),
                ("raw_keys", ctypes.c_int32),
                ("bound_seed", ctypes.c_int32),
                ("dtw_cascade", ctypes.c_int32), ("dk_box", ctypes.c_int32),
                ("lb_prefix", ctypes.c_int32)]


class IndexOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int64), ("workspace_limit_bytes", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("seed_pairs", ctypes.c_int64),
                ("bound_pruned", ctypes.c_int64), ("dp_started", ctypes.c_int64),
                ("dp_completed", ctypes.c_int64), ("dp_abandoned", ctypes.c_int64),
                ("dp_cells", ctypes.c_int64), ("bound_steps", ctypes.c_int64),
                ("fallback_pairs", ctypes.c_int64), ("dp_valid_cells", ctypes.c_int64),
                ("calls", ctypes.c_int64), ("ms_total", ctypes.c_float),
                ("ms_seed", ctypes.c_float), ("ms_bound", ctypes.c_float),
                ("ms_dp", ctypes.c_float), ("ms_final", ctypes.c_float),
                ("ms_bound_kernel", ctypes.c_float), ("ms_dp_fast", ctypes.c_float),
                ("ms_dp_general", ctypes.c_float), ("dp_valid_cells_general", ctypes.c_int64),
                ("ms_order", ctypes.c_float), ("seed_steps", ctypes.c_int64),
                ("chunks", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TuneOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int64), ("sample_queries", ctypes.c_int32),
                ("reps", ctypes.c_int32)]


class SubseqOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int64), ("chunk_cols", ctypes.c_int32), ("seed", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class MlpShape(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int64), ("dim", ctypes.c_int32), ("points", ctypes.c_int32),
                ("hidden", ctypes.c_int32), ("embed", ctypes.c_int32)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int64), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("seed", ctypes.c_uint64)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32

SIGNATURES = {
    "tsk_version": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "tsk_last_error": (ctypes.c_char_p, []),
    "tsk_index_build": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp, ctypes.POINTER(_vp)]),
    "tsk_index_free": (ctypes.c_int, [_vp]),
    "tsk_validate_values": (ctypes.c_int, [_vp, _i64, ctypes.POINTER(_i64), _vp]),
    "tsk_index_info": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32)]),
    "tsk_knn_query": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, Band, _vp, _vp, _vp, _vp,
                                     _vp]),
    "tsk_knn_query_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, Band, _vp, _vp,
                                             _vp, _vp]),
    "tsk_index_profile": (ctypes.c_int, [_vp, _vp, _i32]),
    "tsk_pair_distances": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, Band, _vp, _vp]),
    "tsk_dk_distances": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "tsk_pair_bounds": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, Band, _vp, _vp, _vp, _vp]),
    "tsk_pair_dk_box": (ctypes.c_int, [_vp, _vp, _vp, _i64, Band, _vp, _vp]),
    "tsk_tune": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, Band, _vp, _vp, _vp, _vp, _vp]),
    # band by pointer: libffi misplaces a float scalar next to a by-value
    # struct with a float member, so this entry point takes neither
    "tsk_range_query": (ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.c_double, _i32, _vp, _vp,
                                       _i64, _vp, _vp, _vp, _vp, _vp]),
    "tsk_subseq_query": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp, _i64, _i32, _vp, _vp, _vp,
                                        _vp, _vp, _vp, _vp]),
    "tsk_model_create": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "tsk_model_free": (ctypes.c_int, [_vp]),
    "tsk_model_info": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_i64)]),
    "tsk_model_get_params": (ctypes.c_int, [_vp, _vp, _i64]),
    "tsk_model_set_params": (ctypes.c_int, [_vp, _vp, _i64]),
    "tsk_model_embed": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "tsk_model_batch_grad": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _vp, _vp,
                                            _vp]),
    "tsk_model_train": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    "tsk_model_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "tsk_model_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_vp)]),
}

_lib = None


def load():
    """Loads libtsknn.so from the package directory; raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"the HIP library {path} is not built; run "
                           "`python -m paper_1811_11076_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != TSK_OK:
        raise TskError(rc, load().tsk_last_error().decode(errors="replace"))


def band_struct(band) -> Band:
    if band is None:
        return Band(TSK_BAND_NONE, 0, 0.0)
    if isinstance(band, float):
        return Band(TSK_BAND_FRAC, 0, band)
    return Band(TSK_BAND_ABS, int(band), 0.0)
