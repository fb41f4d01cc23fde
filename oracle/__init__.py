"""CPU oracle for the exact k-NN scan (arXiv 1811.11076) — TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it and it
never loads the GPU library; the two share no code.

Thin ctypes marshalling over ``oracle.c`` (plain C, built with gcc and
``-ffp-contract=off``).  Every function's citation and reading is in the C
source next to its definition.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import build, lib_path

_lib = None

DTW, DK = 0, 1
BAND_NONE, BAND_ABS, BAND_FRAC = 0, 1, 2

_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        build()
    lib = ctypes.CDLL(path)
    sig = {
        "orc_cost_f32": (ctypes.c_float, [_f32p, _f32p, ctypes.c_int]),
        "orc_cost_f64": (ctypes.c_double, [_f32p, _f32p, ctypes.c_int]),
        "orc_band_ok": (ctypes.c_int, [_i64, _i64, _i64, _i64, _i64]),
        "orc_band_w_frac": (_i64, [ctypes.c_float, _i64, _i64]),
        "orc_dtw_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
        "orc_dtw_f64": (ctypes.c_double, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
        "orc_dk_sq_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
        "orc_dk_unsq_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
        "orc_enumerate_paths": (None, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64, _f64p]),
        "orc_envelope": (None, [_f32p, _i64, _i64, ctypes.c_int, _i64, _f32p, _f32p]),
        "orc_box_term_f32": (ctypes.c_float, [_f32p, _f32p, _f32p, ctypes.c_int]),
        "orc_lb_box_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
        "orc_lb_box_f64": (ctypes.c_double, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
        "orc_lb_box_qenv_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
        "orc_lb_keogh_f64": (ctypes.c_double, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64, ctypes.c_int]),
        "orc_lb_sigmamin_f64": (ctypes.c_double, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
        "orc_gdk_sq_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64,
                                            ctypes.c_float, _i64p]),
        "orc_greedy_sum_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64,
                                                ctypes.c_float, _i64p]),
        "orc_sparse_dk_sq_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64,
                                                  ctypes.c_float, _i64p]),
        "orc_knn_brute": (None, [_f32p, _i64p, _i64, _f32p, _i64p, _i64, ctypes.c_int, _i64,
                                 ctypes.c_int, ctypes.c_int, _i64, ctypes.c_float, _i64p, _f32p]),
        "orc_knn_scan": (None, [_f32p, _i64p, _i64, _f32p, _i64p, _i64, ctypes.c_int, _i64,
                                ctypes.c_int, ctypes.c_int, _i64, ctypes.c_float, _i64p, _f32p,
                                _i64p]),
        "orc_pair_keys": (None, [_f32p, _i64p, _i64, _f32p, _i64p, _i64, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, _i64, ctypes.c_float, _f32p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_f32p)


def _i64a(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_i64p)


def _series(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    if x.ndim == 1:
        x = x[:, None]
    return x


def band_w(band, m: int, n: int) -> int:
    """Band half-width for a pair: None -> -1 (no band), int -> itself,
    float -> floor(frac * max(m, n)) (same rule as the C code)."""
    if band is None:
        return -1
    if isinstance(band, float):
        return int(_load().orc_band_w_frac(ctypes.c_float(band), m, n))
    return int(band)


def _band_args(band):
    if band is None:
        return BAND_NONE, -1, 0.0
    if isinstance(band, float):
        return BAND_FRAC, -1, band
    return BAND_ABS, int(band), 0.0


def cost_f32(s, t) -> float:
    s, sp = _f32(s)
    t, tp = _f32(t)
    return float(_load().orc_cost_f32(sp, tp, s.shape[-1]))


def band_ok(i, j, m, n, w) -> bool:
    return bool(_load().orc_band_ok(i, j, m, n, w))


def _pair_call(name, S, T, w, *extra):
    S = _series(S)
    T = _series(T)
    _, sp = _f32(S)
    _, tp = _f32(T)
    return getattr(_load(), name)(sp, S.shape[0], tp, T.shape[0], S.shape[1], w, *extra)


def dtw_f32(S, T, w=-1) -> float:
    return float(_pair_call("orc_dtw_f32", S, T, w))


def dtw_f64(S, T, w=-1) -> float:
    return float(_pair_call("orc_dtw_f64", S, T, w))


def dk_sq_f32(S, T, w=-1) -> float:
    return float(_pair_call("orc_dk_sq_f32", S, T, w))


def dk_unsq_f32(S, T, w=-1) -> float:
    return float(_pair_call("orc_dk_unsq_f32", S, T, w))


def enumerate_paths(S, T, w=-1):
    """(min fp64 sum, min fp32 path-order sum, min max cost, #paths)."""
    out = np.zeros(4, dtype=np.float64)
    _pair_call("orc_enumerate_paths", S, T, w, out.ctypes.data_as(_f64p))
    return float(out[0]), float(np.float32(out[1])), float(np.float32(out[2])), int(out[3])


def envelope(T, m: int, w=-1):
    T = _series(T)
    _, tp = _f32(T)
    d = T.shape[1]
    lo = np.zeros((m, d), np.float32)
    hi = np.zeros((m, d), np.float32)
    _load().orc_envelope(tp, T.shape[0], m, d, w, lo.ctypes.data_as(_f32p), hi.ctypes.data_as(_f32p))
    return lo, hi


def box_term_f32(x, lo, hi) -> float:
    x, xp = _f32(x)
    lo, lp = _f32(lo)
    hi, hp = _f32(hi)
    return float(_load().orc_box_term_f32(xp, lp, hp, x.shape[-1]))


def lb_box_f32(S, T, w=-1) -> float:
    """LB_Box(S, T) of eq. (1): boxes over T, summed over the rows of S."""
    return float(_pair_call("orc_lb_box_f32", S, T, w))


def lb_box_f64(S, T, w=-1) -> float:
    return float(_pair_call("orc_lb_box_f64", S, T, w))


def lb_box_qenv_f32(S, T, w=-1) -> float:
    """Boxes over the query S, summed over the points of the candidate T."""
    return float(_pair_call("orc_lb_box_qenv_f32", S, T, w))


def lb_keogh_f64(S, T, w=-1, dim=0) -> float:
    return float(_pair_call("orc_lb_keogh_f64", S, T, w, dim))


def lb_sigmamin_f64(S, T, w=-1) -> float:
    return float(_pair_call("orc_lb_sigmamin_f64", S, T, w))


def gdk_sq_f32(S, T, w=-1, eps=float("inf")):
    """(value, steps) of the greedy bound, Alg. 1."""
    st = ctypes.c_int64(0)
    v = _pair_call("orc_gdk_sq_f32", S, T, w, ctypes.c_float(eps), ctypes.byref(st))
    return float(v), int(st.value)


def greedy_sum_f32(S, T, w=-1, eps=float("inf")):
    """(value, steps) of the greedy walk of Alg. 1 summing costs (DTW seed)."""
    st = ctypes.c_int64(0)
    v = _pair_call("orc_greedy_sum_f32", S, T, w, ctypes.c_float(eps), ctypes.byref(st))
    return float(v), int(st.value)


def sparse_dk_sq_f32(S, T, w=-1, eps=float("inf")):
    """(value, visited cells) of the sparse DK, Alg. 3 (whole matching)."""
    cells = ctypes.c_int64(0)
    v = _pair_call("orc_sparse_dk_sq_f32", S, T, w, ctypes.c_float(eps), ctypes.byref(cells))
    return float(v), int(cells.value)


def _knn_common(fn, db, db_off, qs, q_off, k, dist, band, extra_stats=False):
    db, dbp = _f32(db)
    db_off, dop = _i64a(db_off)
    qs, qp = _f32(qs)
    q_off, qop = _i64a(q_off)
    d = db.shape[1]
    assert qs.shape[1] == d
    N = db_off.shape[0] - 1
    nq = q_off.shape[0] - 1
    ids = np.zeros((nq, k), np.int64)
    keys = np.zeros((nq, k), np.float32)
    mode, r, frac = _band_args(band)
    dist_code = DK if dist == "dk" else DTW
    args = [dbp, dop, N, qp, qop, nq, d, k, dist_code, mode, r, ctypes.c_float(frac),
            ids.ctypes.data_as(_i64p), keys.ctypes.data_as(_f32p)]
    stats = None
    if extra_stats:
        stats = np.zeros((nq, 4), np.int64)
        args.append(stats.ctypes.data_as(_i64p))
    fn(*args)
    return ids, keys, stats


def knn_brute(db, db_off, qs, q_off, k, dist="dk", band=None):
    """Plain k-NN: full DP for every pair + (key, id) sort.

    Returns (ids int64 [nq, k], keys float32 [nq, k]); keys are squared for DK
    (take sqrtf for the distance), DTW sums otherwise; (-1, +inf) padding."""
    ids, keys, _ = _knn_common(_load().orc_knn_brute, db, db_off, qs, q_off, k, dist, band)
    return ids, keys


def knn_scan(db, db_off, qs, q_off, k, dist="dk", band=None):
    """The paper's pruned scan (Sec. 4.4 for DK, LB_Box + DTW otherwise).

    Returns (ids, keys, stats[nq, 4] = pruned, DP started, DP finite, cells)."""
    return _knn_common(_load().orc_knn_scan, db, db_off, qs, q_off, k, dist, band, True)


def pair_keys(db, db_off, qs, q_off, dist="dk", band=None):
    """[nq, N] keys of every pair by the full DP."""
    db, dbp = _f32(db)
    db_off, dop = _i64a(db_off)
    qs, qp = _f32(qs)
    q_off, qop = _i64a(q_off)
    N = db_off.shape[0] - 1
    nq = q_off.shape[0] - 1
    out = np.zeros((nq, N), np.float32)
    mode, r, frac = _band_args(band)
    _load().orc_pair_keys(dbp, dop, N, qp, qop, nq, db.shape[1], DK if dist == "dk" else DTW,
                          mode, r, ctypes.c_float(frac), out.ctypes.data_as(_f32p))
    return out


def dk_distance(keys: np.ndarray) -> np.ndarray:
    """Distance from squared DK keys: correctly rounded fp32 square root."""
    return np.sqrt(np.asarray(keys, dtype=np.float32))


def range_brute(db, db_off, qs, q_off, radius, dist="dk", band=None):
    """Plain range query (Sec. 1): for each query, the ids (ascending) of
    every series whose distance is <= radius, and those distances; the
    distance of a pair is its full-DP key (DTW), or the correctly rounded
    fp32 sqrt of the squared key (DK).  Returns a list of (ids, dists)."""
    keys = pair_keys(db, db_off, qs, q_off, dist, band)
    d = dk_distance(keys) if dist == "dk" else keys.astype(np.float32)
    out = []
    for q in range(d.shape[0]):
        ids = np.nonzero(d[q] <= np.float32(radius))[0].astype(np.int64)
        out.append((ids, d[q][ids]))
    return out
