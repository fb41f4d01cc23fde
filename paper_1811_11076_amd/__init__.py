"""Exact k-NN over multi-dimensional time series on MI355X (gfx950).

Python face of the C-ABI in ``include/tsknn.h``: torch supplies device
memory and the current stream; every step of the scan runs in the HIP
library.  Importing the package does not load the library; the first Index
does, and raises if it has not been built (there is no CPU fallback).

    idx = Index(db_values_cuda_f32[sum_len, d], db_offsets_int64[n+1])
    ids, dist, stats = idx.knn(q_values, q_offsets, k=10, distance="dk",
                               band=0.1, stats=True)
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib

__all__ = ["Index", "Model", "TskError", "subseq_query", "validate_values", "version"]

TskError = _lib.TskError


def version():
    lib = _lib.load()
    a, b = ctypes.c_int(), ctypes.c_int()
    _lib.check(lib.tsk_version(ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def validate_values(values) -> int:
    """Index of the first non-finite value of a CUDA float32 tensor, or -1
    (C: tsk_validate_values)."""
    lib = _lib.load()
    v = values.contiguous()
    if not v.is_cuda or v.dtype != _torch().float32:
        raise TypeError("values must be a CUDA float32 tensor")
    bad = ctypes.c_int64(-1)
    rc = lib.tsk_validate_values(ctypes.c_void_p(v.data_ptr()), int(v.numel()), ctypes.byref(bad),
                                 _stream())
    if rc != _lib.TSK_ERR_INVALID_ARG or bad.value < 0:
        _lib.check(rc)
    return int(bad.value)


def _torch():
    import torch
    return torch


def _offsets(off) -> np.ndarray:
    if hasattr(off, "detach"):
        off = off.detach().cpu().numpy()
    return np.ascontiguousarray(np.asarray(off, dtype=np.int64))


def _values(v, dim=None):
    torch = _torch()
    if not isinstance(v, torch.Tensor) or not v.is_cuda:
        raise TypeError("series values must be a CUDA (HIP) torch tensor")
    if v.dtype != torch.float32:
        raise TypeError("series values must be float32")
    if v.dim() == 1:
        v = v[:, None]
    if dim is not None and v.shape[1] != dim:
        raise ValueError(f"dimension {v.shape[1]} does not match the index ({dim})")
    return v.contiguous()


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


_DIST = {"dtw": _lib.TSK_DTW, "dk": _lib.TSK_DK}


class Index:
    """Read-only device index over database series (C: tsk_index_build)."""

    def __init__(self, values, offsets, workspace_limit_bytes: int = 0):
        """workspace_limit_bytes: bound on a query call's workspace (0 = the
        library default); queries are processed in chunks that fit."""
        self._lib = _lib.load()
        v = _values(values)
        off = _offsets(offsets)
        self.n = int(off.shape[0] - 1)
        self.dim = int(v.shape[1])
        self._h = ctypes.c_void_p()
        io = _lib.IndexOpts(ctypes.sizeof(_lib.IndexOpts), int(workspace_limit_bytes))
        _lib.check(self._lib.tsk_index_build(
            ctypes.c_void_p(v.data_ptr()), off.ctypes.data_as(ctypes.c_void_p), self.n, self.dim,
            ctypes.byref(io), _stream(), ctypes.byref(self._h)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.tsk_index_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def knn(self, queries, q_offsets, k: int, distance: str = "dk", band=None, order=None,
            seed_count: int = 0, stats: bool = False, profile: bool = False,
            walk_pass: int = -1, task_size: int = 0, tube_rows: int = 0, model=None,
            lb_qgroup: int = 0, use_graph: bool = False, tune: bool = False, out=None,
            dk_band_slots: int = 0, surv_order: int = 0, dp_rows: int = 0,
            dp_waves_per_cu: int = 0, dk_seed: int = 0, cancel=None, lb_both: bool = False,
            raw_keys: bool = False, no_alloc: bool = False, bound_seed: int = 0,
            dtw_cascade: int = 0, dk_box: int = 0, lb_prefix: int = 0):
        """Exact k-NN (C: tsk_knn_query).  Returns (ids int64 [nq, k], dist
        float32 [nq, k], stats dict or None); DK distances are unsquared.
        order: None (plain), a CUDA int32 [nq, n] permutation per query, or
        "learned" with model= a Model (candidates by embedding distance).
        use_graph: run as a cached, replayed HIP graph (pass the same `out`
        tensors (ids, dist) to replay); tune: use the index's tuned options
        (see tune()); cancel: a host numpy int32 array whose first entry,
        set non-zero (e.g. by another thread), stops the call before its next
        chunk of queries (TskError with code TSK_ERR_CANCELLED); lb_both:
        DTW on an equal-length index also bounds the survivors with the
        candidate-envelope LB_Box and keeps the larger bound; raw_keys: dist
        receives the ranking keys (DK squared), for exact merges of shards;
        bound_seed: 1 = seed the threshold from each query's candidates of
        smallest corner bound, 2 = from the head of its order, 0 = default
        (1 for the plain order); dtw_cascade: 1 = DTW prunes by the corner
        bound first and computes LB_Box for its survivors only, 2 = LB_Box
        for every pair, 3 = the corner bound alone (no LB_Box), 0 = default
        (1 for the plain order); dk_box: 1 = DK
        on an equal-length index also bounds the corner survivors by the
        DK box bound (see pair_dk_box), 0 / 2 = off; lb_prefix: the corner
        survivors' LB_Box gives up on a pair after this many points when its
        partial sum scaled to all points stays below the threshold (-1 =
        never, 0 = default: 64 before the banded DP, else never);
        no_alloc: the call allocates no device memory (C:
        tsk_knn_query_noalloc, the library's fixed workspace; pass `out`
        to keep the binding from allocating the outputs; no stats)."""
        torch = _torch()
        qv = _values(queries, self.dim)
        qo = _offsets(q_offsets)
        nq = int(qo.shape[0] - 1)
        if out is not None:
            ids, dist = out
            if (ids.dtype != torch.int64 or dist.dtype != torch.float32 or
                    tuple(ids.shape) != (nq, k) or tuple(dist.shape) != (nq, k) or
                    not ids.is_contiguous() or not dist.is_contiguous()):
                raise ValueError("out must be contiguous (int64 [nq, k], float32 [nq, k])")
            if not (ids.is_cuda and dist.is_cuda and ids.device == qv.device and
                    dist.device == qv.device):
                raise ValueError("out tensors must be on the queries' CUDA device")
        else:
            ids = torch.empty((nq, k), dtype=torch.int64, device=qv.device)
            dist = torch.empty((nq, k), dtype=torch.float32, device=qv.device)
        opts = _lib.QueryOpts()
        opts.size = ctypes.sizeof(_lib.QueryOpts)
        opts.seed_count = int(seed_count)
        opts.profile = 1 if profile else 0
        opts.walk_pass = int(walk_pass)
        opts.task_size = int(task_size)
        opts.tube_rows = int(tube_rows)
        opts.lb_qgroup = int(lb_qgroup)
        opts.dk_band_slots = int(dk_band_slots)
        opts.surv_order = int(surv_order)
        opts.dp_rows = int(dp_rows)
        opts.dp_waves_per_cu = int(dp_waves_per_cu)
        opts.dk_seed = int(dk_seed)
        opts.lb_both = 1 if lb_both else 0
        opts.raw_keys = 1 if raw_keys else 0
        opts.bound_seed = int(bound_seed)
        opts.dtw_cascade = int(dtw_cascade)
        opts.dk_box = int(dk_box)
        opts.lb_prefix = int(lb_prefix)
        opts.use_graph = 1 if use_graph else 0
        opts.tune = _lib.TSK_TUNE_CACHED if tune else _lib.TSK_TUNE_OFF
        if cancel is not None:
            if not (isinstance(cancel, np.ndarray) and cancel.dtype == np.int32 and cancel.size >= 1):
                raise TypeError("cancel must be a host numpy int32 array")
            opts.cancel_flag_host = cancel.ctypes.data
        if isinstance(order, str):
            if order != "learned" or model is None:
                raise ValueError('order="learned" needs model=')
            opts.order = _lib.TSK_ORDER_LEARNED
            opts.model = model._h.value
        elif order is not None:
            if order.dtype != torch.int32 or not order.is_cuda or tuple(order.shape) != (nq, self.n):
                raise ValueError("order must be a CUDA int32 tensor [n_queries, n_series]")
            order = order.contiguous()
            opts.order = _lib.TSK_ORDER_GIVEN
            opts.order_dev = order.data_ptr()
        if no_alloc:
            if stats:
                raise ValueError("no_alloc calls report no stats")
            _lib.check(self._lib.tsk_knn_query_noalloc(
                self._h, ctypes.c_void_p(qv.data_ptr()), qo.ctypes.data_as(ctypes.c_void_p), nq,
                int(k), _DIST[distance], _lib.band_struct(band), ctypes.byref(opts),
                ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dist.data_ptr()), _stream()))
            return ids, dist, None
        st = _lib.Stats() if stats else None
        _lib.check(self._lib.tsk_knn_query(
            self._h, ctypes.c_void_p(qv.data_ptr()), qo.ctypes.data_as(ctypes.c_void_p), nq, int(k),
            _DIST[distance], _lib.band_struct(band), ctypes.byref(opts),
            ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
            ctypes.byref(st) if st is not None else None, _stream()))
        return ids, dist, (st.as_dict() if st is not None else None)

    def range(self, queries, q_offsets, radius: float, distance: str = "dk", band=None,
              capacity: int = 0, stats: bool = False):
        """Range query (C: tsk_range_query): every series within `radius` of
        each query.  Returns (offsets int64 [nq+1] numpy, ids int64 CUDA [total],
        dist float32 CUDA [total], stats dict or None); query q's hits are
        ids[offsets[q]:offsets[q+1]] in ascending id order."""
        torch = _torch()
        qv = _values(queries, self.dim)
        qo = _offsets(q_offsets)
        nq = int(qo.shape[0] - 1)
        offs = np.zeros(nq + 1, np.int64)
        cap = int(capacity) if capacity > 0 else 64 * nq
        for attempt in range(2):
            ids = torch.empty(max(cap, 1), dtype=torch.int64, device=qv.device)
            dist = torch.empty(max(cap, 1), dtype=torch.float32, device=qv.device)
            st = _lib.Stats() if stats else None
            rc = self._lib.tsk_range_query(
                self._h, ctypes.c_void_p(qv.data_ptr()), qo.ctypes.data_as(ctypes.c_void_p), nq,
                ctypes.c_double(radius), _DIST[distance], ctypes.byref(_lib.band_struct(band)),
                None, cap,
                ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
                offs.ctypes.data_as(ctypes.c_void_p),
                ctypes.byref(st) if st is not None else None, _stream())
            if rc == _lib.TSK_ERR_INVALID_ARG and offs[nq] > cap and attempt == 0:
                cap = int(offs[nq])  # the first call measured the total
                continue
            _lib.check(rc)
            break
        total = int(offs[nq])
        return offs, ids[:total], dist[:total], (st.as_dict() if st is not None else None)

    def tune(self, queries, q_offsets, k: int, distance: str = "dk", band=None,
             sample_queries: int = 0, reps: int = 0):
        """Autotunes the work-shaping options on a query sample (C: tsk_tune);
        returns (chosen options dict, milliseconds of the sample call).  Later
        knn(..., tune=True) calls with this (distance, band, k) use them."""
        qv = _values(queries, self.dim)
        qo = _offsets(q_offsets)
        nq = int(qo.shape[0] - 1)
        to = _lib.TuneOpts(ctypes.sizeof(_lib.TuneOpts), int(sample_queries), int(reps))
        best = _lib.QueryOpts()
        ms = ctypes.c_float()
        _lib.check(self._lib.tsk_tune(
            self._h, ctypes.c_void_p(qv.data_ptr()), qo.ctypes.data_as(ctypes.c_void_p), nq,
            int(k), _DIST[distance], _lib.band_struct(band), None, ctypes.byref(to),
            ctypes.byref(best), ctypes.byref(ms), _stream()))
        keys = ("seed_count", "tube_rows", "task_size", "walk_pass", "lb_qgroup", "dk_band_slots",
                "surv_order", "dp_rows", "dp_waves_per_cu", "dk_seed")
        return {key: getattr(best, key) for key in keys}, ms.value

    def profile(self, reset: bool = False) -> dict:
        """Counters and stage times accumulated by knn(..., profile=True)
        calls (C: tsk_index_profile); synchronises."""
        st = _lib.Stats()
        _lib.check(self._lib.tsk_index_profile(self._h, ctypes.byref(st), 1 if reset else 0))
        return st.as_dict()

    def pair_distances(self, queries, q_offsets, distance: str = "dk", band=None,
                       dk_sqrt: bool = False):
        """Full-DP key of every (query, series) pair (C: tsk_pair_distances);
        DK keys are squared, or with dk_sqrt the DK distances themselves
        (C: tsk_dk_distances on the keys, in place)."""
        torch = _torch()
        qv = _values(queries, self.dim)
        qo = _offsets(q_offsets)
        nq = int(qo.shape[0] - 1)
        out = torch.empty((nq, self.n), dtype=torch.float32, device=qv.device)
        _lib.check(self._lib.tsk_pair_distances(
            self._h, ctypes.c_void_p(qv.data_ptr()), qo.ctypes.data_as(ctypes.c_void_p), nq,
            _DIST[distance], _lib.band_struct(band), ctypes.c_void_p(out.data_ptr()), _stream()))
        if dk_sqrt and distance == "dk":
            _lib.check(self._lib.tsk_dk_distances(ctypes.c_void_p(out.data_ptr()),
                                                  ctypes.c_void_p(out.data_ptr()), out.numel(),
                                                  _stream()))
        return out

    def pair_bounds(self, queries, q_offsets, distance: str = "dk", band=None):
        """(lb, greedy value, greedy moves) of every pair (C: tsk_pair_bounds)."""
        torch = _torch()
        qv = _values(queries, self.dim)
        qo = _offsets(q_offsets)
        nq = int(qo.shape[0] - 1)
        lb = torch.empty((nq, self.n), dtype=torch.float32, device=qv.device)
        ub = torch.empty((nq, self.n), dtype=torch.float32, device=qv.device)
        steps = torch.empty((nq, self.n), dtype=torch.int32, device=qv.device)
        _lib.check(self._lib.tsk_pair_bounds(
            self._h, ctypes.c_void_p(qv.data_ptr()), qo.ctypes.data_as(ctypes.c_void_p), nq,
            _DIST[distance], _lib.band_struct(band), ctypes.c_void_p(lb.data_ptr()),
            ctypes.c_void_p(ub.data_ptr()), ctypes.c_void_p(steps.data_ptr()), _stream()))
        return lb, ub, steps

    def pair_dk_box(self, queries, q_offsets, band=None):
        """DK box bound of every pair, squared (C: tsk_pair_dk_box); the
        index's series must share one length."""
        torch = _torch()
        qv = _values(queries, self.dim)
        qo = _offsets(q_offsets)
        nq = int(qo.shape[0] - 1)
        out = torch.empty((nq, self.n), dtype=torch.float32, device=qv.device)
        _lib.check(self._lib.tsk_pair_dk_box(
            self._h, ctypes.c_void_p(qv.data_ptr()), qo.ctypes.data_as(ctypes.c_void_p), nq,
            _lib.band_struct(band), ctypes.c_void_p(out.data_ptr()), _stream()))
        return out


def subseq_query(series, s_offsets, queries, q_offsets, k: int = 1, chunk_cols: int = 0,
                 seed: bool = True, waves_per_cu: int = 0, start: bool = True,
                 stats: bool = False):
    """Subsequence k-NN (C: tsk_subseq_query): for each query the k series
    holding the best matches of the query anywhere inside them, by
    subsequence DK.  series: CUDA float32 [sum_len, d] with offsets
    [n+1] (long series; no index); queries likewise (lengths <= 1024).
    Returns (ids int64, dist float32, end int64, start int64 or None), each
    CUDA [nq, k], and the stats dict (or None); a match covers columns
    start..end of its series.  Synchronous."""
    torch = _torch()
    lib = _lib.load()
    sv = _values(series)
    so = _offsets(s_offsets)
    qv = _values(queries, sv.shape[1])
    qo = _offsets(q_offsets)
    n, nq = int(so.shape[0] - 1), int(qo.shape[0] - 1)
    dev = sv.device
    ids = torch.empty((nq, k), dtype=torch.int64, device=dev)
    dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
    end = torch.empty((nq, k), dtype=torch.int64, device=dev)
    st_ = torch.empty((nq, k), dtype=torch.int64, device=dev) if start else None
    o = _lib.SubseqOpts(ctypes.sizeof(_lib.SubseqOpts), int(chunk_cols), 1 if seed else 0,
                        int(waves_per_cu), 0)
    st = _lib.Stats() if stats else None
    _lib.check(lib.tsk_subseq_query(
        ctypes.c_void_p(sv.data_ptr()), so.ctypes.data_as(ctypes.c_void_p), n, int(sv.shape[1]),
        ctypes.c_void_p(qv.data_ptr()), qo.ctypes.data_as(ctypes.c_void_p), nq, int(k),
        ctypes.byref(o), ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dist.data_ptr()),
        ctypes.c_void_p(end.data_ptr()),
        ctypes.c_void_p(st_.data_ptr()) if st_ is not None else None,
        ctypes.byref(st) if st is not None else None, _stream()))
    return ids, dist, end, st_, (st.as_dict() if st is not None else None)


class Model:
    """Encoder for the learned candidate order (C: tsk_model_*).  Predicts
    DK distances as Euclidean distances of embeddings; only reorders the
    scan, never changes its results."""

    def __init__(self, dim: int, points: int = 32, hidden: int = 256, embed: int = 64,
                 seed: int = 0, _handle=None):
        # torch's HIP context first: the encoder's memory lives on torch's
        # current device and later calls run on torch's streams
        _torch().cuda.init()
        self._lib = _lib.load()
        self._h = ctypes.c_void_p()
        if _handle is not None:
            self._h = _handle
        else:
            sh = _lib.MlpShape(ctypes.sizeof(_lib.MlpShape), dim, points, hidden, embed)
            _lib.check(self._lib.tsk_model_create(ctypes.byref(sh), ctypes.c_uint64(seed),
                                                  ctypes.byref(self._h)))
        sh = _lib.MlpShape()
        n = ctypes.c_int64()
        _lib.check(self._lib.tsk_model_info(self._h, ctypes.byref(sh), ctypes.byref(n)))
        self.dim, self.points, self.hidden, self.embed = sh.dim, sh.points, sh.hidden, sh.embed
        self.n_params = n.value

    @classmethod
    def load(cls, path: str) -> "Model":
        _torch().cuda.init()
        h = ctypes.c_void_p()
        _lib.check(_lib.load().tsk_model_load(path.encode(), ctypes.byref(h)))
        return cls(0, _handle=h)

    def save(self, path: str):
        _lib.check(self._lib.tsk_model_save(self._h, path.encode()))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.tsk_model_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _lib.check(self._lib.tsk_model_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                                  self.n_params))
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(np.asarray(flat, dtype=np.float32))
        _lib.check(self._lib.tsk_model_set_params(self._h, flat.ctypes.data_as(ctypes.c_void_p),
                                                  flat.size))

    def embed_series(self, values, offsets):
        """Embeddings [n, embed] (CUDA float32) of the given series."""
        torch = _torch()
        v = _values(values, self.dim)
        off = _offsets(offsets)
        n = int(off.shape[0] - 1)
        out = torch.empty((n, self.embed), dtype=torch.float32, device=v.device)
        _lib.check(self._lib.tsk_model_embed(self._h, ctypes.c_void_p(v.data_ptr()),
                                             off.ctypes.data_as(ctypes.c_void_p), n,
                                             ctypes.c_void_p(out.data_ptr()), _stream()))
        return out

    @staticmethod
    def _pairs(a, b, y):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
        b = np.ascontiguousarray(np.asarray(b, dtype=np.int32))
        y = np.ascontiguousarray(np.asarray(y, dtype=np.float32))
        if not (a.shape == b.shape == y.shape and a.ndim == 1):
            raise ValueError("pair arrays must be 1-D of one length")
        return a, b, y

    def batch_grad(self, values, offsets, a, b, y):
        """(loss, flat gradient [n_params]) of one batch of pairs."""
        v = _values(values, self.dim)
        off = _offsets(offsets)
        a, b, y = self._pairs(a, b, y)
        loss = ctypes.c_float()
        grad = np.empty(self.n_params, np.float32)
        _lib.check(self._lib.tsk_model_batch_grad(
            self._h, ctypes.c_void_p(v.data_ptr()), off.ctypes.data_as(ctypes.c_void_p),
            int(off.shape[0] - 1), a.ctypes.data_as(ctypes.c_void_p),
            b.ctypes.data_as(ctypes.c_void_p), y.ctypes.data_as(ctypes.c_void_p), a.size,
            ctypes.byref(loss), grad.ctypes.data_as(ctypes.c_void_p), _stream()))
        return loss.value, grad

    def train(self, values, offsets, a, b, y, epochs: int = 10, batch: int = 1024,
              lr: float = 1e-3, seed: int = 0):
        """Adam training on pairs (a[i], b[i]) with target distances y[i];
        returns the mean batch loss of every epoch."""
        v = _values(values, self.dim)
        off = _offsets(offsets)
        a, b, y = self._pairs(a, b, y)
        o = _lib.TrainOpts(ctypes.sizeof(_lib.TrainOpts), int(epochs), int(batch), float(lr),
                           0.0, 0.0, 0.0, int(seed))
        losses = np.empty(int(epochs), np.float32)
        _lib.check(self._lib.tsk_model_train(
            self._h, ctypes.c_void_p(v.data_ptr()), off.ctypes.data_as(ctypes.c_void_p),
            int(off.shape[0] - 1), a.ctypes.data_as(ctypes.c_void_p),
            b.ctypes.data_as(ctypes.c_void_p), y.ctypes.data_as(ctypes.c_void_p), a.size,
            ctypes.byref(o), losses.ctypes.data_as(ctypes.c_void_p), _stream()))
        return losses
