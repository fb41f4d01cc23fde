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
        "orc_lb_dk_box_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
        "orc_lb_dk_box_qenv_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64]),
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
        "orc_knn_verify": (None, [_f32p, _i64p, _i64, _f32p, _i64p, _i64, ctypes.c_int, _i64,
                                  ctypes.c_int, ctypes.c_int, _i64, ctypes.c_float, _i64p, _f32p,
                                  _i64p]),
        "orc_pair_list_keys": (None, [_f32p, _i64p, _f32p, _i64p, ctypes.c_int, _i64, _i64p,
                                      _i64p, ctypes.c_int, ctypes.c_int, _i64, ctypes.c_float,
                                      _f32p]),
        "orc_qenv": (None, [_f32p, _i64, _i64, ctypes.c_int, _i64, _f32p, _f32p]),
        "orc_pair_keys": (None, [_f32p, _i64p, _i64, _f32p, _i64p, _i64, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, _i64, ctypes.c_float, _f32p]),
        "orc_set_threads": (ctypes.c_int, [ctypes.c_int]),
        "orc_subseq_dk_sq_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64p]),
        "orc_subseq_start": (_i64, [_f32p, _i64, _f32p, _i64, ctypes.c_int, ctypes.c_float]),
        "orc_subseq_brute_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int, _i64p,
                                                  _i64p]),
        "orc_sub_gdk_sq_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int,
                                                ctypes.c_float, _i64p]),
        "orc_sparse_dk_sub_sq_f32": (ctypes.c_float, [_f32p, _i64, _f32p, _i64, ctypes.c_int,
                                                      ctypes.c_float, _i64p, _i64p]),
        "orc_subseq_knn": (None, [_f32p, _i64p, _i64, _f32p, _i64p, _i64, ctypes.c_int, _i64,
                                  _i64p, _f32p, _i64p, _i64p]),
        "orc_subseq_scan": (None, [_f32p, _i64p, _i64, _f32p, _i64p, _i64, ctypes.c_int, _i64,
                                   _i64p, _f32p, _i64p, _i64p, _i64p]),
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


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's loops over queries; returns the
    previous setting (n <= 0 only queries it)."""
    return int(_load().orc_set_threads(int(n)))


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


def lb_dk_box_f32(S, T, w=-1) -> float:
    """DK box bound: the largest squared distance of a row of S to its box
    of T (Sec. 3's boxes, the maximum in place of eq. (1)'s sum); <= DK^2."""
    return float(_pair_call("orc_lb_dk_box_f32", S, T, w))


def lb_dk_box_qenv_f32(S, T, w=-1) -> float:
    """The DK box bound with boxes over the query S, the largest over the
    points of the candidate T."""
    return float(_pair_call("orc_lb_dk_box_qenv_f32", S, T, w))


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
    """The paper's pruned scan (Sec. 4.3 for DK, LB_Box + DTW otherwise).

    Returns (ids, keys, stats[nq, 4] = pruned, DP started, DP finite, cells)."""
    return _knn_common(_load().orc_knn_scan, db, db_off, qs, q_off, k, dist, band, True)


def knn_verify(db, db_off, qs, q_off, k, dist="dk", band=None):
    """The pruned scan of knn_scan with each query's envelope kept per
    candidate length (same values, far less work at full size).

    Returns (ids, keys, stats) as knn_scan."""
    return _knn_common(_load().orc_knn_verify, db, db_off, qs, q_off, k, dist, band, True)


def pair_list_keys(db, db_off, qs, q_off, qi, ci, dist="dk", band=None):
    """Full-DP keys of the pairs (qi[p], ci[p]) -> float32 [len(qi)]."""
    db, dbp = _f32(db)
    db_off, dop = _i64a(db_off)
    qs, qp = _f32(qs)
    q_off, qop = _i64a(q_off)
    qi, qip = _i64a(qi)
    ci, cip = _i64a(ci)
    assert qi.shape == ci.shape
    out = np.zeros(qi.shape[0], np.float32)
    mode, r, frac = _band_args(band)
    _load().orc_pair_list_keys(dbp, dop, qp, qop, db.shape[1], qi.shape[0], qip, cip,
                               DK if dist == "dk" else DTW, mode, r, ctypes.c_float(frac),
                               out.ctypes.data_as(_f32p))
    return out


def qenv(S, n: int, w=-1):
    """Envelope of the query S for the columns of a candidate of length n:
    (lo, hi), each float32 [n, d]."""
    S = _series(S)
    m, d = S.shape
    lo = np.zeros((n, d), np.float32)
    hi = np.zeros((n, d), np.float32)
    _, sp = _f32(S)
    _load().orc_qenv(sp, m, n, d, band_w(w, m, n) if isinstance(w, float) else w,
                     lo.ctypes.data_as(_f32p), hi.ctypes.data_as(_f32p))
    return lo, hi


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


# ---------------------------------------------------------------- subsequence search

def _sub_call(name, S, T, *extra):
    S = _series(S)
    T = _series(T)
    assert S.shape[1] == T.shape[1]
    _, sp = _f32(S)
    _, tp = _f32(T)
    return getattr(_load(), name)(sp, S.shape[0], tp, T.shape[0], S.shape[1], *extra)


def subseq_dk(S, T):
    """(squared key, end, start) of the best match of S anywhere in T: the
    plain SUB DP (Alg. 3 with SUB, every cell), the start by definition."""
    e = ctypes.c_int64(-1)
    v = float(_sub_call("orc_subseq_dk_sq_f32", S, T, ctypes.byref(e)))
    if e.value < 0:
        return v, -1, -1
    return v, int(e.value), subseq_start(S, T, int(e.value), v)


def subseq_start(S, T, end, key):
    """Latest a <= end with DK(S, T[a..end]) == key (-1 if none)."""
    S = _series(S)
    T = _series(T)
    _, sp = _f32(S)
    _, tp = _f32(T)
    return int(_load().orc_subseq_start(sp, S.shape[0], tp, end, S.shape[1], ctypes.c_float(key)))


def subseq_brute(S, T):
    """(key, end, start) from the definition: DK(S, T[a..b]) for all a <= b."""
    e, a = ctypes.c_int64(-1), ctypes.c_int64(-1)
    v = float(_sub_call("orc_subseq_brute_f32", S, T, ctypes.byref(e), ctypes.byref(a)))
    return v, int(e.value), int(a.value)


def sub_gdk_sq_f32(S, T, eps=float("inf")):
    """(value, steps) of the greedy bound for subsequence search, Alg. 2."""
    st = ctypes.c_int64(0)
    v = _sub_call("orc_sub_gdk_sq_f32", S, T, ctypes.c_float(eps), ctypes.byref(st))
    return float(v), int(st.value)


def sparse_dk_sub_sq_f32(S, T, eps=float("inf")):
    """(value, end, visited cells) of Alg. 3 with SUB = true."""
    e, cells = ctypes.c_int64(-1), ctypes.c_int64(0)
    v = _sub_call("orc_sparse_dk_sub_sq_f32", S, T, ctypes.c_float(eps), ctypes.byref(e),
                  ctypes.byref(cells))
    return float(v), int(e.value), int(cells.value)


def _subseq_common(fn, ser, s_off, qs, q_off, k, stats):
    ser, sp = _f32(_series(ser))
    s_off, sop = _i64a(s_off)
    qs, qp = _f32(_series(qs))
    q_off, qop = _i64a(q_off)
    d = ser.shape[1]
    assert qs.shape[1] == d
    N = s_off.shape[0] - 1
    nq = q_off.shape[0] - 1
    ids = np.zeros((nq, k), np.int64)
    keys = np.zeros((nq, k), np.float32)
    end = np.zeros((nq, k), np.int64)
    start = np.zeros((nq, k), np.int64)
    args = [sp, sop, N, qp, qop, nq, d, k, ids.ctypes.data_as(_i64p),
            keys.ctypes.data_as(_f32p), end.ctypes.data_as(_i64p), start.ctypes.data_as(_i64p)]
    st = None
    if stats:
        st = np.zeros(nq, np.int64)
        args.append(st.ctypes.data_as(_i64p))
    fn(*args)
    return ids, keys, end, start, st


def subseq_knn(ser, s_off, qs, q_off, k):
    """Plain subsequence k-NN: (ids, squared keys, end, start), each [nq, k];
    series ranked by (key, id); (-1, +inf, -1, -1) padding."""
    return _subseq_common(_load().orc_subseq_knn, ser, s_off, qs, q_off, k, False)[:4]


def subseq_scan(ser, s_off, qs, q_off, k):
    """The paper's pruned subsequence scan (Alg. 2 threshold + Alg. 3 SUB):
    same outputs as subseq_knn plus visited cells per query."""
    return _subseq_common(_load().orc_subseq_scan, ser, s_off, qs, q_off, k, True)
