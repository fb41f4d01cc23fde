"""Pins of the oracle's subsequence search (Sec. 4.1-4.2: Alg. 2 and Alg. 3
with SUB) against what the definitions fix: hand-worked examples
(tests/golden/subseq_examples.json), enumeration of every warping path that
starts in row 0 and ends in the last row, the whole-match DK of every
sub-series, closed forms (one-point query, one-column series, planted exact
copies) and the bound and monotonicity relations."""
import json
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "subseq_examples.json")
INF = float("inf")


def _walk(rng, n, d, scale=1.0):
    return np.cumsum(rng.normal(scale=scale, size=(n, d)), 0).astype(np.float32)


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_hand_examples(ex):
    S = np.array(ex["S"], np.float32)
    T = np.array(ex["T"], np.float32)
    assert O.subseq_dk(S, T) == (ex["key"], ex["end"], ex["start"])
    assert O.subseq_brute(S, T) == (ex["key"], ex["end"], ex["start"])
    assert O.sub_gdk_sq_f32(S, T) == (ex["sub_gdk"], ex["sub_gdk_steps"])
    v, e, _ = O.sparse_dk_sub_sq_f32(S, T, ex["key"])
    assert (v, e) == (ex["key"], ex["end"])


def _paths_min(S, T):
    """Every monotone path with steps (1,0), (0,1), (1,1) that starts at any
    (0, a) and ends at any (m-1, b): min over paths of the max cell cost, the
    first end column reaching it and, for that end, the latest start."""
    m, n = len(S), len(T)
    c = [[O.cost_f32(S[i], T[j]) for j in range(n)] for i in range(m)]
    best = {}  # (start, end) -> min max

    def rec(i, j, a, mx):
        mx = max(mx, c[i][j])
        if i == m - 1:
            key = (a, j)
            if mx < best.get(key, INF):
                best[key] = mx
        if i + 1 < m:
            rec(i + 1, j, a, mx)
        if j + 1 < n:
            rec(i, j + 1, a, mx)
        if i + 1 < m and j + 1 < n:
            rec(i + 1, j + 1, a, mx)

    for a in range(n):
        rec(0, a, a, -INF)
    v = min(best.values())
    e = min(b for (a, b), x in best.items() if x == v)
    s = max(a for (a, b), x in best.items() if x == v and b == e)
    return float(np.float32(v)), e, s


@pytest.mark.parametrize("m,n,d", [(1, 1, 1), (1, 6, 2), (2, 1, 3), (3, 4, 1), (4, 5, 3),
                                   (5, 3, 2), (3, 7, 3)])
def test_sub_dp_equals_path_enumeration(m, n, d):
    rng = np.random.default_rng(100 * m + 10 * n + d)
    for rep in range(4):
        S = _walk(rng, m, d)
        T = _walk(rng, n, d)
        if rep == 3:  # plant a near copy so that ties and short matches occur
            T[: min(m, n)] = S[: min(m, n)] + np.float32(0.25)
        ref = _paths_min(S, T)
        assert O.subseq_dk(S, T) == ref, (rep, ref)
        assert O.subseq_brute(S, T) == ref, (rep, ref)


@pytest.mark.parametrize("m,n,d", [(6, 30, 3), (12, 25, 1), (1, 40, 2), (20, 9, 3)])
def test_sub_dp_equals_every_subseries(m, n, d):
    """The SUB DP equals min over all sub-series of the whole-match DK
    (itself pinned against path enumeration), end and start included."""
    rng = np.random.default_rng(7 + m + n + d)
    for _ in range(3):
        S = _walk(rng, m, d)
        T = _walk(rng, n, d)
        assert O.subseq_dk(S, T) == O.subseq_brute(S, T)


def test_closed_forms():
    rng = np.random.default_rng(5)
    T = _walk(rng, 50, 3)
    # one-point query: the closest point of T, first one on ties
    s = T[17:18] + np.float32(0.5)
    costs = np.array([O.cost_f32(s[0], t) for t in T], np.float32)
    j = int(np.argmin(costs))
    assert O.subseq_dk(s, T) == (float(costs[j]), j, j)
    assert O.sub_gdk_sq_f32(s, T)[0] == float(costs[j])
    # one-column series: every query row against that point
    S = _walk(rng, 9, 3)
    t = T[3:4]
    v = max(O.cost_f32(x, t[0]) for x in S)
    assert O.subseq_dk(S, t) == (float(np.float32(v)), 0, 0)
    assert O.subseq_dk(S, t)[0] == O.dk_sq_f32(S, t)
    # planted exact copy: zero, at the copy (random data has no other zero)
    S = T[20:32].copy()
    assert O.subseq_dk(S, T) == (0.0, 31, 20)
    assert O.sub_gdk_sq_f32(S, T)[0] == 0.0


def test_bounds_and_monotonicity():
    rng = np.random.default_rng(11)
    for rep in range(20):
        m, n = int(rng.integers(1, 15)), int(rng.integers(1, 60))
        S = _walk(rng, m, 3)
        T = _walk(rng, n, 3)
        v, e, a = O.subseq_dk(S, T)
        assert 0 <= a <= e < n
        # the reported match really has that value
        assert O.dk_sq_f32(S, T[a:e + 1]) == v
        # the whole series is one of the candidates
        assert v <= O.dk_sq_f32(S, T)
        # a sub-series has fewer candidates; a prefix of junk changes nothing
        # but the positions
        lo, hi = sorted(rng.integers(0, n, 2))
        assert O.subseq_dk(S, T[lo:hi + 1])[0] >= v
        junk = np.full((5, 3), 1e4, np.float32)
        v2, e2, a2 = O.subseq_dk(S, np.concatenate([junk, T]))
        assert (v2, e2, a2) == (v, e + 5, a + 5)
        # Alg. 2 is an upper bound with at most m - 1 + n - 1 moves
        g, steps = O.sub_gdk_sq_f32(S, T)
        assert g >= v and steps <= m + n - 2
        # an early exit returns a value above eps
        if g > 0:
            ge, _ = O.sub_gdk_sq_f32(S, T, np.float32(g) * np.float32(0.5))
            assert ge > np.float32(g) * np.float32(0.5)


def test_sparse_sub_matches_dense():
    rng = np.random.default_rng(13)
    for rep in range(20):
        m, n = int(rng.integers(1, 12)), int(rng.integers(1, 50))
        S = _walk(rng, m, 2)
        T = _walk(rng, n, 2)
        v, e, _ = O.subseq_dk(S, T)
        for eps in (INF, v, float(np.nextafter(np.float32(v), np.float32(INF))) if v < INF else v):
            got, ge, cells = O.sparse_dk_sub_sq_f32(S, T, eps)
            assert (got, ge) == (v, e)
            assert cells <= m * n
        if v > 0:
            below = float(np.nextafter(np.float32(v), np.float32(0)))
            assert O.sparse_dk_sub_sq_f32(S, T, below)[:2] == (INF, -1)


def test_knn_definition_and_scan_agree():
    """The pruned scan (Alg. 2 threshold + Alg. 3 SUB) returns exactly the
    plain definition's rows; each row's end and start are those of its pair."""
    rng = np.random.default_rng(21)
    d = 3
    lens = rng.integers(20, 120, 30)
    ser = [_walk(rng, int(L), d) for L in lens]
    qs, qo = [], [0]
    for q in range(6):
        src = ser[int(rng.integers(0, len(ser)))]
        m = int(rng.integers(3, 16))
        p = int(rng.integers(0, max(1, len(src) - m)))
        x = src[p:p + m] + rng.normal(scale=0.2, size=(len(src[p:p + m]), d)).astype(np.float32)
        qs.append(x.astype(np.float32))
        qo.append(qo[-1] + len(x))
    off = np.concatenate([[0], np.cumsum(lens)])
    flat = np.concatenate(ser)
    qflat = np.concatenate(qs)
    for k in (1, 4, 40):
        ids, keys, end, start = O.subseq_knn(flat, off, qflat, qo, k)
        sids, skeys, send, sstart, cells = O.subseq_scan(flat, off, qflat, qo, k)
        assert np.array_equal(ids, sids) and np.array_equal(keys.view(np.uint32), skeys.view(np.uint32))
        assert np.array_equal(end, send) and np.array_equal(start, sstart)
        for q in range(len(qo) - 1):
            S = qflat[qo[q]:qo[q + 1]]
            row = [O.subseq_dk(S, ser[c])[0] for c in range(len(ser))]
            order = sorted(range(len(ser)), key=lambda c: (row[c], c))
            for r in range(k):
                if r >= len(ser):
                    assert ids[q, r] == -1 and keys[q, r] == INF and end[q, r] == -1
                    continue
                c = order[r]
                assert ids[q, r] == c and keys[q, r] == np.float32(row[c])
                assert (keys[q, r], end[q, r], start[q, r]) == O.subseq_dk(S, ser[c])
        assert np.all(cells > 0)
