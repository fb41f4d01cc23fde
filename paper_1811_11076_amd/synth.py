"""Seeded synthetic inputs: multi-dimensional time series for the k-NN scan.

This module holds no part of the method's arithmetic (no distances, bounds or
DP).  It is the one module that both the oracle-side tests and the GPU path
use to obtain identical inputs.

Two families stand in for the paper's RAM/CBF generators and UCI/ECG data sets
(Sec. 5), which are not available:

* Gaussian random walks: x_0 = e_0, x_t = x_{t-1} + e_t, e_t ~ N(0, I_d).
* Class-warp series: C prototypes (random walks of length L_p).  A member of
  class c is the prototype under a random monotone piecewise-linear time warp
  (8 equal output segments, slopes U[0.8, 1.2] renormalised so that the warp
  maps [0, 1] onto [0, 1], i.e. at most 20 % local stretch), sampled by linear
  interpolation at m points, plus N(0, 0.1^2) noise.  Database member i has
  class i mod C; query classes are uniform.

Every draw comes from numpy's PCG64 seeded by SeedSequence([1811, cfg, stream,
chunk]) with fixed chunks of CHUNK series, so a given (cfg, stream) always
yields the same values however the caller slices it.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 1811
STREAMS = {"proto": 0, "db": 1, "query": 2, "train": 3, "aux": 4}
CHUNK = 2048
N_SEGMENTS = 8
SLOPE_LO, SLOPE_HI = 0.8, 1.2
NOISE_SIGMA = 0.1


def _rng(cfg_id: int, stream: str, index: int) -> np.random.Generator:
    ss = np.random.SeedSequence([BASE_SEED, int(cfg_id), STREAMS[stream], int(index)])
    return np.random.Generator(np.random.PCG64(ss))


def random_walks(n: int, length: int, d: int, cfg_id: int, stream: str,
                 start: int = 0) -> np.ndarray:
    """Series start..start+n-1 of a random-walk stream, float32 [n, length, d]."""
    out = np.empty((n, length, d), dtype=np.float32)
    first_chunk = start // CHUNK
    last_chunk = (start + n - 1) // CHUNK if n > 0 else first_chunk - 1
    for ch in range(first_chunk, last_chunk + 1):
        rng = _rng(cfg_id, stream, ch)
        steps = rng.standard_normal((CHUNK, length, d))
        walks = np.cumsum(steps, axis=1)
        lo = max(start, ch * CHUNK)
        hi = min(start + n, (ch + 1) * CHUNK)
        out[lo - start:hi - start] = walks[lo - ch * CHUNK:hi - ch * CHUNK]
    return out


def _warp_positions(slopes: np.ndarray, m: int, proto_len: int) -> np.ndarray:
    """Sample positions (float64, [cnt, m]) on the prototype axis for each warp."""
    cnt = slopes.shape[0]
    knots_y = np.concatenate([np.zeros((cnt, 1)), np.cumsum(slopes, axis=1)], axis=1)
    knots_y /= knots_y[:, -1:]
    knots_x = np.linspace(0.0, 1.0, N_SEGMENTS + 1)
    u = np.linspace(0.0, 1.0, m) if m > 1 else np.zeros(1)
    seg = np.minimum((u * N_SEGMENTS).astype(np.int64), N_SEGMENTS - 1)
    frac = (u - knots_x[seg]) * N_SEGMENTS
    y0 = np.take_along_axis(knots_y, np.broadcast_to(seg, (cnt, m)), axis=1)
    y1 = np.take_along_axis(knots_y, np.broadcast_to(seg + 1, (cnt, m)), axis=1)
    w = y0 + (y1 - y0) * frac
    return w * (proto_len - 1)


def _interp(protos: np.ndarray, cls: np.ndarray, pos: np.ndarray) -> np.ndarray:
    """Linear interpolation of protos[cls[r]] at positions pos[r, :] -> [cnt, m, d]."""
    proto_len = protos.shape[1]
    p0 = np.clip(np.floor(pos).astype(np.int64), 0, proto_len - 1)
    p1 = np.minimum(p0 + 1, proto_len - 1)
    f = (pos - p0)[..., None]
    flat = protos.reshape(-1, protos.shape[2])
    base = (np.asarray(cls, np.int64) * proto_len)[:, None]
    a = np.take(flat, base + p0, axis=0)
    b = np.take(flat, base + p1, axis=0)
    return a + (b - a) * f


def _workers() -> int:
    import os
    return max(1, min(16, os.cpu_count() or 1))


class ClassWarp:
    """Class-warp generator for one configuration id."""

    def __init__(self, cfg_id: int, n_classes: int, proto_len: int, d: int):
        self.cfg_id = cfg_id
        self.n_classes = n_classes
        self.proto_len = proto_len
        self.d = d
        rng = _rng(cfg_id, "proto", 0)
        steps = rng.standard_normal((n_classes, proto_len, d))
        self.protos = np.cumsum(steps, axis=1)  # float64

    def _chunk_draws(self, ch: int, stream: str, length, class_mode: str):
        """The chunk's draws in their fixed order: lengths, classes, warp
        slopes, then the seed of its noise stream."""
        rng = _rng(self.cfg_id, stream, ch)
        if isinstance(length, tuple):
            lens = rng.integers(length[0], length[1] + 1, size=CHUNK)
        else:
            lens = np.full(CHUNK, int(length))
        if class_mode == "uniform":
            cls = rng.integers(0, self.n_classes, size=CHUNK)
        else:
            cls = np.arange(ch * CHUNK, (ch + 1) * CHUNK) % self.n_classes
        slopes = rng.uniform(SLOPE_LO, SLOPE_HI, size=(CHUNK, N_SEGMENTS))
        noise_seed = rng.integers(0, 2**63 - 1)
        return lens, cls, slopes, noise_seed

    def members(self, n: int, stream: str, start: int = 0,
                length: int | tuple[int, int] = 256, class_mode: str = "mod"):
        """Members start..start+n-1 of a stream.

        length: an int (all equal) or (lo, hi) for lengths uniform in {lo..hi}.
        class_mode: "mod" (class = index mod C) or "uniform" (drawn).
        Returns (values float32 [sum(len), d], offsets int64 [n+1], labels int64 [n]).
        Chunks are generated in worker threads (numpy releases the GIL); every
        value depends only on its chunk's seed, so the result is the same for
        any number of workers.
        """
        from concurrent.futures import ThreadPoolExecutor
        first_chunk = start // CHUNK
        last_chunk = (start + n - 1) // CHUNK if n > 0 else first_chunk - 1
        chunks = list(range(first_chunk, last_chunk + 1))

        def span(ch):
            lo = max(start, ch * CHUNK)
            hi = min(start + n, (ch + 1) * CHUNK)
            return slice(lo - ch * CHUNK, hi - ch * CHUNK), lo - start

        # pass 1: lengths and classes of every member (cheap draws)
        lens_all, labels_all = [], []
        for ch in chunks:
            lens, cls, _, _ = self._chunk_draws(ch, stream, length, class_mode)
            sel, _ = span(ch)
            lens_all.append(lens[sel])
            labels_all.append(cls[sel])
        lens_all = np.concatenate(lens_all) if lens_all else np.zeros(0, np.int64)
        labels = np.concatenate(labels_all) if labels_all else np.zeros(0, np.int64)
        offsets = np.zeros(n + 1, dtype=np.int64)
        offsets[1:] = np.cumsum(lens_all)
        values = np.empty((int(offsets[-1]), self.d), dtype=np.float32)

        # pass 2: each chunk's values, written in place
        def fill(ch):
            lens, cls, slopes, noise_seed = self._chunk_draws(ch, stream, length, class_mode)
            sel, out0 = span(ch)
            nrng = np.random.Generator(np.random.PCG64(noise_seed))
            lens_c, cls_c, slopes_c = lens[sel], cls[sel], slopes[sel]
            # noise for the whole chunk is drawn in one fixed order, then sliced
            total = int(lens.sum())
            noise = nrng.standard_normal((total, self.d)) * NOISE_SIGMA
            noff = np.concatenate([[0], np.cumsum(lens)])
            for ulen in np.unique(lens_c):
                rows = np.nonzero(lens_c == ulen)[0]
                pos = _warp_positions(slopes_c[rows], int(ulen), self.proto_len)
                vals = _interp(self.protos, cls_c[rows], pos)
                r_chunk = rows + sel.start
                gather = noff[r_chunk][:, None] + np.arange(int(ulen))[None, :]
                vals += np.take(noise, gather, axis=0)
                dst = offsets[rows + out0][:, None] + np.arange(int(ulen))[None, :]
                values[dst] = vals

        if len(chunks) > 1:
            with ThreadPoolExecutor(max_workers=min(_workers(), len(chunks))) as ex:
                list(ex.map(fill, chunks))
        else:
            for ch in chunks:
                fill(ch)
        return values, offsets, labels.astype(np.int64)


def flat_equal(arr: np.ndarray):
    """[n, L, d] -> (values [n*L, d], offsets [n+1])."""
    n, length, d = arr.shape
    return (np.ascontiguousarray(arr.reshape(n * length, d)),
            np.arange(n + 1, dtype=np.int64) * length)


# ---------------------------------------------------------------- long series and planted queries
# Subsequence search (Sec. 4.1-4.2 and the long-series experiment of Sec. 5)
# queries short series against long ones; these stand in for the long ECG
# recording.

WALK_PIECE = 1 << 20


def long_walk(length: int, d: int, cfg_id: int, stream: str = "db", index: int = 0) -> np.ndarray:
    """One Gaussian random walk of `length` points, float32 [length, d];
    piece p of 2^20 steps is drawn from its own seed (index * 4096 + p)."""
    out = np.empty((length, d), dtype=np.float32)
    level = np.zeros(d)
    for p in range(0, (length + WALK_PIECE - 1) // WALK_PIECE):
        lo, hi = p * WALK_PIECE, min(length, (p + 1) * WALK_PIECE)
        steps = _rng(cfg_id, stream, int(index) * 4096 + p).standard_normal((hi - lo, d))
        w = np.cumsum(steps, axis=0) + level
        out[lo:hi] = w
        level = w[-1]
    return out


def planted_queries(values: np.ndarray, offsets: np.ndarray, n: int, m: int, cfg_id: int,
                    stream: str = "query"):
    """n queries of m points cut from the given series: query q takes series
    s ~ U{0..N-1}, a window of round(m * U[0.8, 1.2]) points (clipped to the
    series) at a uniform position, resamples it onto m points under a random
    piecewise-linear warp (as the class-warp members) and adds N(0, 0.1^2)
    noise.  Returns (values float32 [n*m, d], offsets int64 [n+1],
    origin int64 [n, 3] = (series, window start, window length))."""
    N = offsets.shape[0] - 1
    d = values.shape[1]
    out = np.empty((n * m, d), dtype=np.float32)
    origin = np.zeros((n, 3), dtype=np.int64)
    for q in range(n):
        rng = _rng(cfg_id, stream, q)
        s = int(rng.integers(0, N))
        L = int(offsets[s + 1] - offsets[s])
        w = int(min(L, max(1, round(m * rng.uniform(SLOPE_LO, SLOPE_HI)))))
        a = int(rng.integers(0, L - w + 1))
        win = values[offsets[s] + a: offsets[s] + a + w].astype(np.float64)
        slopes = rng.uniform(SLOPE_LO, SLOPE_HI, size=(1, N_SEGMENTS))
        pos = _warp_positions(slopes, m, w)
        vals = _interp(win[None], np.zeros(1, np.int64), pos)[0]
        vals += rng.standard_normal((m, d)) * NOISE_SIGMA
        out[q * m:(q + 1) * m] = vals
        origin[q] = (s, a, w)
    return out, np.arange(n + 1, dtype=np.int64) * m, origin


def gaussian_iid(n: int, length: int, d: int, cfg_id: int, stream: str, start: int = 0) -> np.ndarray:
    """Series whose points are independent N(0, I_d) draws (the setting of
    the curse-of-dimensionality theorem for LB_Box), float32 [n, length, d];
    chunked and seeded like random_walks."""
    out = np.empty((n, length, d), dtype=np.float32)
    first_chunk = start // CHUNK
    last_chunk = (start + n - 1) // CHUNK if n > 0 else first_chunk - 1
    for ch in range(first_chunk, last_chunk + 1):
        pts = _rng(cfg_id, stream, ch).standard_normal((CHUNK, length, d))
        lo = max(start, ch * CHUNK)
        hi = min(start + n, (ch + 1) * CHUNK)
        out[lo - start:hi - start] = pts[lo - ch * CHUNK:hi - ch * CHUNK]
    return out
