"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test compares the oracle with something other than itself: hand-worked
examples from the definitions (tests/golden), brute-force enumeration of all
warping paths, closed forms, the bound chains and identities stated in the
paper, and invariants (identity, symmetry, triangle inequality).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
INF = float("inf")


def _val(x):
    return INF if x == "inf" else float(x)


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _golden(), ids=lambda e: e["name"])
def test_hand_examples(ex):
    S = np.array(ex["S"], np.float32)
    T = np.array(ex["T"], np.float32)
    w = ex["w"]
    if "dtw" in ex:
        assert O.dtw_f32(S, T, w) == _val(ex["dtw"])
        assert O.dtw_f64(S, T, w) == _val(ex["dtw"])
    if "dk_sq" in ex:
        assert O.dk_sq_f32(S, T, w) == _val(ex["dk_sq"])
    if "gdk_sq" in ex:
        v, steps = O.gdk_sq_f32(S, T, w)
        assert v == ex["gdk_sq"] and steps == ex["gdk_steps"]
    if "greedy_sum" in ex:
        assert O.greedy_sum_f32(S, T, w)[0] == ex["greedy_sum"]
    if "lb_box_paper" in ex:
        assert O.lb_box_f32(S, T, w) == ex["lb_box_paper"]
        assert O.lb_box_f64(S, T, w) == ex["lb_box_paper"]
    if "lb_sigmamin" in ex:
        assert O.lb_sigmamin_f64(S, T, w) == ex["lb_sigmamin"]
    if "envelope_of_T_lo" in ex:
        lo, hi = O.envelope(T, S.shape[0], w)
        assert np.array_equal(lo, np.array(ex["envelope_of_T_lo"], np.float32))
        assert np.array_equal(hi, np.array(ex["envelope_of_T_hi"], np.float32))


# ------------------------------------------------------------------ cost
def test_cost_identity_symmetry_1d(rng):
    for d in (1, 2, 3, 6, 8):
        for _ in range(50):
            s = rng.normal(size=d).astype(np.float32) * 10
            t = rng.normal(size=d).astype(np.float32) * 10
            assert O.cost_f32(s, s) == 0.0
            assert O.cost_f32(s, t) == O.cost_f32(t, s)  # fl(a-b) = -fl(b-a)
            exact = float(np.sum((s.astype(np.float64) - t.astype(np.float64)) ** 2))
            assert abs(O.cost_f32(s, t) - exact) <= 4e-7 * exact + 1e-30
    # d = 1: (s - t)^2 rounded once after the rounded difference
    for _ in range(200):
        s, t = rng.normal(size=2).astype(np.float32) * 100
        e = np.float32(s - t)
        assert O.cost_f32([s], [t]) == float(np.float32(e * e))


# ------------------------------------------------------------------ brute force paths
def _small_pairs(rng, count=60):
    for _ in range(count):
        m = int(rng.integers(1, 8))
        n = int(rng.integers(1, 8))
        d = int(rng.integers(1, 4))
        S = rng.normal(size=(m, d)).astype(np.float32)
        T = rng.normal(size=(n, d)).astype(np.float32)
        yield S, T


@pytest.mark.parametrize("band", [None, 0, 1, 2, 0.3])
def test_dp_equals_path_enumeration(rng, band):
    """The DP equals the minimum over every warping path (Sec. 2.1)."""
    for S, T in _small_pairs(rng):
        w = O.band_w(band, S.shape[0], T.shape[0])
        s64, s32, mx, count = O.enumerate_paths(S, T, w)
        if count == 0:
            assert O.dtw_f32(S, T, w) == INF and O.dk_sq_f32(S, T, w) == INF
            continue
        assert O.dtw_f64(S, T, w) == pytest.approx(s64, rel=1e-12)
        assert O.dtw_f32(S, T, w) == s32  # same rounding chain, bit for bit
        assert O.dk_sq_f32(S, T, w) == mx  # max/min only select: exact


def test_path_count_is_delannoy():
    # unbanded m x n grid: central Delannoy numbers on the diagonal
    S = np.zeros((8, 1), np.float32)
    assert O.enumerate_paths(S, S)[3] == 48639   # D(7)
    assert O.enumerate_paths(S[:7], S[:7])[3] == 8989
    assert O.enumerate_paths(S[:3], S[:3])[3] == 13


# ------------------------------------------------------------------ closed forms
def test_zero_band_is_euclidean(rng):
    """w = 0 and m = n leave only the diagonal path: DTW is the squared
    Euclidean distance of the stacked series, DK the largest point cost."""
    for _ in range(30):
        L = int(rng.integers(1, 40))
        d = int(rng.integers(1, 5))
        S = rng.normal(size=(L, d)).astype(np.float32)
        T = rng.normal(size=(L, d)).astype(np.float32)
        sq = np.sum((S.astype(np.float64) - T.astype(np.float64)) ** 2, axis=1)
        assert O.dtw_f64(S, T, 0) == pytest.approx(float(sq.sum()), rel=1e-12)
        assert O.dk_sq_f32(S, T, 0) == pytest.approx(float(sq.max()), rel=1e-6)
        assert O.dtw_f32(S, T, 0) == pytest.approx(float(sq.sum()), rel=1e-5)


def test_single_point_query(rng):
    """m = 1: the only path visits every point of T."""
    for _ in range(30):
        n = int(rng.integers(1, 30))
        d = int(rng.integers(1, 4))
        S = rng.normal(size=(1, d)).astype(np.float32)
        T = rng.normal(size=(n, d)).astype(np.float32)
        sq = np.sum((S.astype(np.float64) - T.astype(np.float64)) ** 2, axis=1)
        assert O.dtw_f64(S, T) == pytest.approx(float(sq.sum()), rel=1e-12)
        assert O.dk_sq_f32(S, T) == pytest.approx(float(sq.max()), rel=1e-6)
        assert O.dtw_f64(T, S) == pytest.approx(float(sq.sum()), rel=1e-12)


def test_identity_and_symmetry(rng):
    for _ in range(40):
        m = int(rng.integers(1, 30))
        n = int(rng.integers(1, 30))
        d = int(rng.integers(1, 4))
        S = rng.normal(size=(m, d)).astype(np.float32)
        T = rng.normal(size=(n, d)).astype(np.float32)
        for band in (None, 2, 0.2):
            w = O.band_w(band, m, n)
            assert O.dtw_f32(S, S, O.band_w(band, m, m)) == 0.0
            assert O.dk_sq_f32(S, S, O.band_w(band, m, m)) == 0.0
            # transposed DP takes the min of the same three values
            assert O.dtw_f32(S, T, w) == O.dtw_f32(T, S, w)
            assert O.dk_sq_f32(S, T, w) == O.dk_sq_f32(T, S, w)


def test_band_monotone_and_full(rng):
    for _ in range(20):
        L = int(rng.integers(2, 30))
        S = rng.normal(size=(L, 3)).astype(np.float32)
        T = rng.normal(size=(L, 3)).astype(np.float32)
        prev_t, prev_k = INF, INF
        for w in range(0, L + 1):
            t, k = O.dtw_f64(S, T, w), O.dk_sq_f32(S, T, w)
            assert t <= prev_t and k <= prev_k
            prev_t, prev_k = t, k
        assert O.dtw_f32(S, T, L - 1) == O.dtw_f32(S, T, -1)
        assert O.dk_sq_f32(S, T, L - 1) == O.dk_sq_f32(S, T, -1)


def test_band_rule():
    # equal lengths: |i - j| <= w exactly
    for L in (2, 5, 17):
        for w in range(0, L):
            for i, j in itertools.product(range(L), range(L)):
                assert O.band_ok(i, j, L, L, w) == (abs(i - j) <= w)
    # length-1 series: everything allowed
    assert all(O.band_ok(0, j, 1, 9, 0) for j in range(9))
    # fractional width uses floor(frac * L)
    assert O.band_w(0.1, 256, 256) == 25 and O.band_w(0.1, 512, 512) == 51
    assert O.band_w(0.1, 64, 1024) == 102


def test_slanted_band_feasible_for_uneven_lengths(rng):
    """Every length pair of the uneven-length workload has a path in band."""
    for _ in range(40):
        m = int(rng.integers(64, 1025))
        n = int(rng.integers(64, 1025))
        w = O.band_w(0.1, m, n)
        S = np.zeros((m, 1), np.float32)
        T = np.zeros((n, 1), np.float32)
        assert O.dk_sq_f32(S, T, w) == 0.0


# ------------------------------------------------------------------ DK extras
def test_dk_sqrt_domain(rng):
    """sqrt is monotone: the DP on sqrt'ed costs ends in sqrtf(DK^2)."""
    for S, T in _small_pairs(rng, 100):
        assert O.dk_unsq_f32(S, T) == float(np.sqrt(np.float32(O.dk_sq_f32(S, T))))


def test_dk_triangle_inequality(rng):
    """DK is a metric (Sec. 6), up to fp32 rounding of the costs."""
    for _ in range(200):
        d = int(rng.integers(1, 4))
        A, B, C = (rng.normal(size=(int(rng.integers(1, 12)), d)).astype(np.float32) for _ in range(3))
        ab = math.sqrt(O.dk_sq_f32(A, B))
        bc = math.sqrt(O.dk_sq_f32(B, C))
        ac = math.sqrt(O.dk_sq_f32(A, C))
        assert ac <= (ab + bc) * (1 + 1e-6) + 1e-12


def test_dk_corner_bound(rng):
    for S, T in _small_pairs(rng, 100):
        dk = O.dk_sq_f32(S, T)
        assert dk >= O.cost_f32(S[0], T[0]) and dk >= O.cost_f32(S[-1], T[-1])


# ------------------------------------------------------------------ bounds
@pytest.mark.parametrize("band", [None, 0, 1, 3, 0.25])
def test_lb_chain(rng, band):
    """LB_Box <= LB_Sigma-min <= DTW (Sec. 3), and the fp32 LB_Box summed in
    series order never exceeds the fp32 DTW, in either orientation."""
    for _ in range(60):
        m = int(rng.integers(1, 25))
        n = m if band is not None and not isinstance(band, float) else int(rng.integers(1, 25))
        d = int(rng.integers(1, 5))
        S = rng.normal(size=(m, d)).astype(np.float32)
        T = rng.normal(size=(n, d)).astype(np.float32)
        w = O.band_w(band, m, n)
        dtw64 = O.dtw_f64(S, T, w)
        if dtw64 == INF:
            continue
        lb64 = O.lb_box_f64(S, T, w)
        smin = O.lb_sigmamin_f64(S, T, w)
        assert lb64 <= smin * (1 + 1e-12) + 1e-12
        assert smin <= dtw64 * (1 + 1e-12) + 1e-12
        dtw32 = O.dtw_f32(S, T, w)
        assert O.lb_box_f32(S, T, w) <= dtw32
        assert O.lb_box_qenv_f32(S, T, w) <= dtw32
        # exchanging the roles of the two series is the same bound as the
        # query-envelope orientation
        assert O.lb_box_qenv_f32(S, T, w) == O.lb_box_f32(T, S, w)


def test_lb_box_is_sum_of_keogh(rng):
    """eq. (1): LB_Box = sum over dimensions of LB_Keogh; d = 1 identical."""
    for _ in range(40):
        L = int(rng.integers(1, 30))
        d = int(rng.integers(1, 6))
        w = int(rng.integers(0, 6))
        S = rng.normal(size=(L, d)).astype(np.float32)
        T = rng.normal(size=(L, d)).astype(np.float32)
        total = sum(O.lb_keogh_f64(S, T, w, k) for k in range(d))
        assert O.lb_box_f64(S, T, w) == pytest.approx(total, rel=1e-12, abs=1e-12)
        if d == 1:
            assert O.lb_box_f64(S, T, w) == O.lb_keogh_f64(S, T, w, 0)


def test_lb_box_zero_band_equals_dtw(rng):
    """w = 0: each box is the point itself, LB_Box = DTW bit for bit."""
    for _ in range(40):
        L = int(rng.integers(1, 40))
        d = int(rng.integers(1, 5))
        S = rng.normal(size=(L, d)).astype(np.float32)
        T = rng.normal(size=(L, d)).astype(np.float32)
        assert O.lb_box_f32(S, T, 0) == O.dtw_f32(S, T, 0)


def test_envelope_bruteforce(rng):
    for _ in range(20):
        n = int(rng.integers(1, 30))
        m = int(rng.integers(1, 30))
        w = int(rng.integers(0, 5))
        T = rng.normal(size=(n, 2)).astype(np.float32)
        lo, hi = O.envelope(T, m, w)
        for i in range(m):
            cols = [j for j in range(n) if O.band_ok(i, j, m, n, w)]
            if cols:
                assert np.array_equal(lo[i], T[cols].min(0)) and np.array_equal(hi[i], T[cols].max(0))


def test_wider_window_lowers_lb_box(rng):
    """A superset window can only widen each box, so LB_Box over a wider
    band is never larger (the bound stays valid when a kernel uses a
    superset of the exact window), and every band's LB_Box stays below its
    own DTW."""
    for _ in range(40):
        m = int(rng.integers(1, 30))
        n = int(rng.integers(1, 30))
        d = int(rng.integers(1, 4))
        S = rng.normal(size=(m, d)).astype(np.float32)
        T = rng.normal(size=(n, d)).astype(np.float32)
        prev = None
        for w in (0, 1, 3, 7, 30, -1):
            lb = O.lb_box_f64(S, T, w)
            if prev is not None:
                assert lb <= prev * (1 + 1e-12) + 1e-12
            dtw = O.dtw_f64(S, T, w)
            assert lb <= dtw * (1 + 1e-12) + 1e-12
            prev = lb


def test_dk_box_bound_below_dk(rng):
    """The DK box bound (Sec. 3's boxes, the largest box distance) never
    exceeds the fp32 DK^2 of the same band, in either orientation; it is
    never below the box distance of any single row; exchanging the series
    exchanges the orientations."""
    for band in (None, 0, 1, 3, 0.25):
        for _ in range(50):
            m = int(rng.integers(1, 25))
            n = m if band is not None and not isinstance(band, float) else int(rng.integers(1, 25))
            d = int(rng.integers(1, 5))
            S = rng.normal(size=(m, d)).astype(np.float32)
            T = rng.normal(size=(n, d)).astype(np.float32)
            w = O.band_w(band, m, n)
            dk = O.dk_sq_f32(S, T, w)
            lb = O.lb_dk_box_f32(S, T, w)
            lbq = O.lb_dk_box_qenv_f32(S, T, w)
            assert lb <= dk and lbq <= dk, (band, m, n, lb, lbq, dk)
            assert lbq == O.lb_dk_box_f32(T, S, w)
            lo, hi = O.envelope(T, m, w)
            i = int(rng.integers(0, m))
            assert lb >= O.box_term_f32(S[i], lo[i], hi[i])


def test_dk_box_bound_closed_forms(rng):
    """Closed forms, bit for bit: with w = 0 and m = n every box is one
    point and only the diagonal path remains, so both orientations equal
    DK^2 (the largest diagonal cost); with m = 1 every column's query box is
    the one query point and the only path visits all of T, so the
    query-box orientation equals DK^2 (and with n = 1 the other one)."""
    for _ in range(40):
        L = int(rng.integers(1, 40))
        d = int(rng.integers(1, 5))
        S = rng.normal(size=(L, d)).astype(np.float32)
        T = rng.normal(size=(L, d)).astype(np.float32)
        dk = O.dk_sq_f32(S, T, 0)
        assert O.lb_dk_box_f32(S, T, 0) == dk
        assert O.lb_dk_box_qenv_f32(S, T, 0) == dk
        assert dk == max(O.cost_f32(S[i], T[i]) for i in range(L))
        n = int(rng.integers(1, 30))
        P = rng.normal(size=(1, d)).astype(np.float32)
        U = rng.normal(size=(n, d)).astype(np.float32)
        assert O.lb_dk_box_qenv_f32(P, U) == O.dk_sq_f32(P, U)
        assert O.lb_dk_box_f32(U, P) == O.dk_sq_f32(U, P)
        # a point inside every box contributes nothing: a series against
        # itself, unbanded, has bound 0 = DK^2
        assert O.lb_dk_box_f32(S, S) == 0.0 == O.dk_sq_f32(S, S)


def test_dk_box_bound_wider_window_lower(rng):
    """A superset window widens each box: the bound over a wider band is
    never larger, and each band's bound stays below that band's DK^2."""
    for _ in range(40):
        m = int(rng.integers(1, 30))
        n = int(rng.integers(1, 30))
        d = int(rng.integers(1, 4))
        S = rng.normal(size=(m, d)).astype(np.float32)
        T = rng.normal(size=(n, d)).astype(np.float32)
        prev = prevq = None
        for w in (0, 1, 3, 7, 30, -1):
            lb, lbq = O.lb_dk_box_f32(S, T, w), O.lb_dk_box_qenv_f32(S, T, w)
            if prev is not None:
                assert lb <= prev and lbq <= prevq
            dk = O.dk_sq_f32(S, T, w)
            assert lb <= dk and lbq <= dk
            prev, prevq = lb, lbq


# ------------------------------------------------------------------ greedy bounds
def test_greedy_upper_bounds(rng):
    """Alg. 1 returns an upper bound of DK (Sec. 4.1) in at most m+n-2 moves;
    the summing walk is an upper bound of DTW."""
    for band in (None, 2, 0.3):
        for _ in range(80):
            m = int(rng.integers(1, 30))
            n = int(rng.integers(1, 30))
            d = int(rng.integers(1, 4))
            S = rng.normal(size=(m, d)).astype(np.float32)
            T = rng.normal(size=(n, d)).astype(np.float32)
            w = O.band_w(band, m, n)
            g, steps = O.gdk_sq_f32(S, T, w)
            assert g >= O.dk_sq_f32(S, T, w)
            assert steps <= m + n - 2
            gs, _ = O.greedy_sum_f32(S, T, w)
            assert gs >= O.dtw_f32(S, T, w)
            if m == 1 or n == 1 or w == 0 and m == n:
                assert g == O.dk_sq_f32(S, T, w)
                assert gs == O.dtw_f32(S, T, w)


def test_greedy_early_return(rng):
    for _ in range(100):
        S = rng.normal(size=(20, 3)).astype(np.float32)
        T = rng.normal(size=(25, 3)).astype(np.float32)
        full, _ = O.gdk_sq_f32(S, T)
        eps = float(rng.uniform(0, full * 1.2))
        v, _ = O.gdk_sq_f32(S, T, eps=eps)
        if full > eps:
            assert v > eps
        else:
            assert v == full


# ------------------------------------------------------------------ sparse DK (Alg. 3)
def test_sparse_dk_equals_dense(rng):
    """Alg. 3 returns DK when DK <= eps and +inf otherwise (Sec. 4.2)."""
    for band in (None, 3):
        for _ in range(150):
            m = int(rng.integers(1, 30))
            n = int(rng.integers(1, 30))
            S = rng.normal(size=(m, 3)).astype(np.float32)
            T = rng.normal(size=(n, 3)).astype(np.float32)
            w = O.band_w(band, m, n)
            dk = O.dk_sq_f32(S, T, w)
            assert O.sparse_dk_sq_f32(S, T, w)[0] == dk
            for eps in (dk, dk * 0.999, dk * 1.5, float(rng.uniform(0, 10))):
                v, cells = O.sparse_dk_sq_f32(S, T, w, eps)
                assert v == (dk if dk <= eps else INF)
                assert cells <= m * n


def test_sparse_dk_visits_few_cells_on_similar_series(rng):
    # a tight threshold keeps the visited set close to the warping path
    base = np.cumsum(rng.normal(size=(200, 3)), axis=0).astype(np.float32)
    other = (base + rng.normal(scale=0.05, size=base.shape)).astype(np.float32)
    dk = O.dk_sq_f32(base, other)
    v, cells = O.sparse_dk_sq_f32(base, other, eps=dk)
    assert v == dk and cells < 0.05 * 200 * 200


# ------------------------------------------------------------------ k-NN
def _db(rng, N, lens, d):
    L = rng.integers(lens[0], lens[1] + 1, size=N)
    off = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    vals = np.cumsum(rng.normal(size=(int(off[-1]), d)), axis=0).astype(np.float32)
    return vals, off


@pytest.mark.parametrize("dist,band", [("dk", None), ("dtw", None), ("dtw", 3), ("dtw", 0.15),
                                       ("dk", 0.2)])
def test_knn_scan_equals_brute(rng, dist, band):
    """The paper's pruned scan (Sec. 4.3 / LB_Box + DTW) equals the plain
    definition: full DP for every pair and a (distance, id) sort."""
    db, dbo = _db(rng, 300, (5, 40), 3)
    qs, qo = _db(rng, 7, (5, 40), 3)
    for k in (1, 5, 17):
        ids_b, keys_b = O.knn_brute(db, dbo, qs, qo, k, dist, band)
        ids_s, keys_s, st = O.knn_scan(db, dbo, qs, qo, k, dist, band)
        assert np.array_equal(ids_b, ids_s)
        assert np.array_equal(keys_b, keys_s)
        if dist == "dtw" and band is not None:
            assert st[:, 0].sum() > 0  # LB_Box prunes something


@pytest.mark.parametrize("dist,band", [("dk", None), ("dtw", None), ("dtw", 3), ("dtw", 0.15),
                                       ("dk", 0.2)])
def test_knn_verify_equals_brute(rng, dist, band):
    """The full-size check (the pruned scan with each query's envelope kept
    per candidate length) equals the plain definition, on uneven lengths
    (many envelope lengths) and equal lengths (one)."""
    for lens in ((5, 40), (24, 24)):
        db, dbo = _db(rng, 300, lens, 3)
        qs, qo = _db(rng, 7, lens, 3)
        for k in (1, 5, 17):
            ids_b, keys_b = O.knn_brute(db, dbo, qs, qo, k, dist, band)
            ids_v, keys_v, _ = O.knn_verify(db, dbo, qs, qo, k, dist, band)
            assert np.array_equal(ids_b, ids_v)
            assert np.array_equal(keys_b, keys_v)


def test_query_envelope_bruteforce(rng):
    """orc_qenv: for column j of a candidate of length n, the per-dimension
    min / max of the query rows the band lets j align with."""
    for _ in range(20):
        n = int(rng.integers(1, 30))
        m = int(rng.integers(1, 30))
        w = int(rng.integers(-1, 5))
        S = rng.normal(size=(m, 2)).astype(np.float32)
        lo, hi = O.qenv(S, n, w)
        for j in range(n):
            rows = [i for i in range(m) if O.band_ok(i, j, m, n, w)]
            if rows:
                assert np.array_equal(lo[j], S[rows].min(0)) and np.array_equal(hi[j], S[rows].max(0))
            else:
                assert np.all(lo[j] == INF) and np.all(hi[j] == -INF)


def test_pair_list_keys_equal_all_pairs(rng):
    db, dbo = _db(rng, 40, (3, 30), 2)
    qs, qo = _db(rng, 5, (3, 30), 2)
    for dist, band in (("dk", None), ("dtw", 0.2), ("dtw", 2)):
        allk = O.pair_keys(db, dbo, qs, qo, dist, band)
        qi = rng.integers(0, 5, size=64)
        ci = rng.integers(0, 40, size=64)
        got = O.pair_list_keys(db, dbo, qs, qo, qi, ci, dist, band)
        assert np.array_equal(got, allk[qi, ci])


def test_knn_ties_and_padding():
    # identical candidates: ties resolved by id; k > N padded with (-1, inf)
    T = np.ones((4, 2), np.float32)
    db = np.concatenate([T, T, T + 1, T]).astype(np.float32)
    dbo = np.array([0, 4, 8, 12, 16], np.int64)
    qs = T.copy()
    qo = np.array([0, 4], np.int64)
    for dist in ("dk", "dtw"):
        ids, keys = O.knn_brute(db, dbo, qs, qo, 6, dist)
        assert ids.tolist() == [[0, 1, 3, 2, -1, -1]]
        assert keys[0, 4] == INF and keys[0, 0] == 0.0
        ids2, keys2, _ = O.knn_scan(db, dbo, qs, qo, 6, dist)
        assert np.array_equal(ids, ids2) and np.array_equal(keys, keys2)


def test_knn_permutation_invariance(rng):
    db, dbo = _db(rng, 120, (8, 20), 2)
    qs, qo = _db(rng, 3, (8, 20), 2)
    perm = rng.permutation(120)
    lens = np.diff(dbo)
    series = [db[dbo[i]:dbo[i + 1]] for i in range(120)]
    db2 = np.concatenate([series[p] for p in perm]).astype(np.float32)
    dbo2 = np.concatenate([[0], np.cumsum(lens[perm])]).astype(np.int64)
    for dist in ("dk", "dtw"):
        ids, keys = O.knn_brute(db, dbo, qs, qo, 4, dist)
        ids2, keys2 = O.knn_brute(db2, dbo2, qs, qo, 4, dist)
        assert np.array_equal(keys, keys2)
        # ids agree wherever the key is unique among the candidates
        assert np.array_equal(perm[ids2], ids)


def _merge_shards(parts, k):
    """Per-query top-k of the shards' top-k lists, ordered by (key, id)."""
    ids = np.concatenate([p[0] for p in parts], axis=1)
    keys = np.concatenate([p[1] for p in parts], axis=1)
    out_i = np.full((ids.shape[0], k), -1, np.int64)
    out_k = np.full((ids.shape[0], k), INF, np.float32)
    for q in range(ids.shape[0]):
        cand = sorted((float(keys[q, t]), int(ids[q, t])) for t in range(ids.shape[1])
                      if ids[q, t] >= 0)[:k]
        for r, (kk, ii) in enumerate(cand):
            out_i[q, r], out_k[q, r] = ii, kk
    return out_i, out_k


@pytest.mark.parametrize("shards", [2, 3, 5])
def test_knn_shard_and_merge(rng, shards):
    """The k-NN definition splits over database shards: each shard's top-k
    (ids offset by the shard's first series), merged by (key, id), equals
    the top-k of the whole database, padding included when k exceeds a
    shard."""
    db, dbo = _db(rng, 61, (5, 30), 3)
    qs, qo = _db(rng, 4, (5, 30), 3)
    cuts = np.linspace(0, 61, shards + 1).astype(int)
    for dist, band in (("dk", None), ("dtw", 0.2), ("dtw", None)):
        for k in (1, 6, 15):
            full = O.knn_brute(db, dbo, qs, qo, k, dist, band)
            parts = []
            for a, b in zip(cuts[:-1], cuts[1:]):
                sdb = db[dbo[a]:dbo[b]]
                sdo = (dbo[a:b + 1] - dbo[a]).astype(np.int64)
                ids, keys = O.knn_brute(sdb, sdo, qs, qo, k, dist, band)
                parts.append((np.where(ids >= 0, ids + a, -1), keys))
            mi, mk = _merge_shards(parts, k)
            assert np.array_equal(mi, full[0]) and np.array_equal(mk, full[1])


def test_fp32_dtw_close_to_fp64():
    """fp32 accumulation stays within 1e-5 relative of fp64 at length 1024."""
    r = np.random.default_rng(7)
    worst = 0.0
    for _ in range(4):
        base = np.cumsum(r.normal(size=(1024, 3)), axis=0)
        S = (base + r.normal(scale=0.1, size=base.shape)).astype(np.float32)
        T = (base + r.normal(scale=0.1, size=base.shape)).astype(np.float32)
        for w in (102, -1):
            a, b = O.dtw_f32(S, T, w), O.dtw_f64(S, T, w)
            worst = max(worst, abs(a - b) / b)
    assert worst < 1e-5


def test_range_brute_against_knn_definitions():
    """The range query's definition checked against the k-NN one: radius +inf
    returns every series; radius = the k-th nearest distance returns the k
    nearest (and only series at or below it); just below the nearest
    distance returns nothing."""
    r = np.random.default_rng(41)
    N, d = 40, 3
    L = r.integers(5, 14, size=N)
    dbo = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    db = np.cumsum(r.normal(size=(int(dbo[-1]), d)), axis=0).astype(np.float32)
    qs = np.cumsum(r.normal(size=(20, d)), axis=0).astype(np.float32)
    qo = np.array([0, 9, 20], np.int64)
    for dist, band in (("dk", None), ("dtw", 2), ("dtw", None)):
        k = 6
        ids, keys = O.knn_brute(db, dbo, qs, qo, k, dist, band)
        dk_ = O.dk_distance(keys) if dist == "dk" else keys
        allr = O.range_brute(db, dbo, qs, qo, np.inf, dist, band)
        for q in range(2):
            finite = np.isfinite(O.pair_keys(db, dbo, qs, qo, dist, band)[q])
            assert np.array_equal(allr[q][0], np.nonzero(finite)[0])
            rk = O.range_brute(db, dbo, qs, qo, dk_[q, k - 1], dist, band)[q]
            assert set(ids[q].tolist()) <= set(rk[0].tolist())
            assert np.all(rk[1] <= dk_[q, k - 1]) and np.all(np.diff(rk[0]) > 0)
            below = np.nextafter(np.float32(dk_[q, 0]), np.float32(-1))
            assert O.range_brute(db, dbo, qs, qo, below, dist, band)[q][0].size == 0
