"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Bit-exact: k-NN ids, squared DK keys, DK distances (fp32 sqrt), fp32 DTW
keys (the oracle's fp32 mirror arithmetic), LB_Box, greedy bounds and move
counts.  DTW also within 1e-5 relative of the fp64 oracle."""
import numpy as np
import pytest

import oracle as O
from gpu_cases import assert_same_knn, classwarp, ragged_walks, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"\n[gpu] {torch.cuda.get_device_name(0)}", flush=True)


def _index(vals, off):
    from paper_1811_11076_amd import Index
    return Index(to_dev(vals), off)


PAIR_CASES = [
    # (name, seed, Q, N, lens, d)
    ("ragged_small", 1, 3, 70, (1, 40), 3),
    ("multistrip", 2, 2, 20, (250, 600), 2),
    ("d1", 3, 2, 30, (10, 80), 1),
    ("d6", 4, 2, 30, (10, 80), 6),
    ("d8", 5, 2, 30, (10, 80), 8),
    ("equal64", 6, 3, 100, (64, 64), 3),
    # ~100 series per length: length buckets split into several tiles
    ("buckets", 7, 3, 400, (20, 23), 3),
]
BANDS = [None, 3, 0.2]


@pytest.mark.parametrize("case", PAIR_CASES, ids=lambda c: c[0])
@pytest.mark.parametrize("band", BANDS, ids=lambda b: f"band{b}")
def test_pair_distances(case, band):
    name, seed, Q, N, lens, d = case
    print(f"[case] pair_distances {name} band={band}", flush=True)
    db, dbo = ragged_walks(seed, N, lens, d)
    qs, qo = ragged_walks(seed + 100, Q, lens, d)
    idx = _index(db, dbo)
    for dist in ("dk", "dtw"):
        got = idx.pair_distances(to_dev(qs), qo, dist, band).cpu().numpy()
        ref = O.pair_keys(db, dbo, qs, qo, dist, band)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (dist, np.argwhere(got != ref)[:5])
        if dist == "dtw":
            for q in range(Q):
                for c in range(0, N, max(1, N // 10)):
                    w = O.band_w(band, qo[q + 1] - qo[q], dbo[c + 1] - dbo[c])
                    ref64 = O.dtw_f64(qs[qo[q]:qo[q + 1]], db[dbo[c]:dbo[c + 1]], w)
                    if np.isfinite(ref64) and ref64 > 0:
                        assert abs(got[q, c] - ref64) <= 1e-5 * ref64
                    else:
                        assert got[q, c] == ref64
    idx.close()


@pytest.mark.parametrize("case", PAIR_CASES[:2] + PAIR_CASES[5:], ids=lambda c: c[0])
@pytest.mark.parametrize("band", BANDS, ids=lambda b: f"band{b}")
def test_pair_bounds(case, band):
    name, seed, Q, N, lens, d = case
    print(f"[case] pair_bounds {name} band={band}", flush=True)
    db, dbo = ragged_walks(seed, N, lens, d)
    qs, qo = ragged_walks(seed + 100, Q, lens, d)
    idx = _index(db, dbo)
    for dist in ("dk", "dtw"):
        lb, ub, steps = (t.cpu().numpy() for t in idx.pair_bounds(to_dev(qs), qo, dist, band))
        for q in range(Q):
            S = qs[qo[q]:qo[q + 1]]
            for c in range(N):
                T = db[dbo[c]:dbo[c + 1]]
                w = O.band_w(band, S.shape[0], T.shape[0])
                if dist == "dk":
                    corner = max(O.cost_f32(S[0], T[0]), O.cost_f32(S[-1], T[-1]))
                    assert lb[q, c] == np.float32(corner)
                    v, st = O.gdk_sq_f32(S, T, w)
                else:
                    assert lb[q, c] == np.float32(O.lb_box_qenv_f32(S, T, w)), (q, c)
                    v, st = O.greedy_sum_f32(S, T, w)
                assert ub[q, c] == np.float32(v) and steps[q, c] == st, (dist, q, c, ub[q, c], v)
    idx.close()


@pytest.mark.parametrize("d,lens", [(5, (40, 300)), (6, (10, 80)), (8, (100, 400))])
@pytest.mark.parametrize("band", BANDS, ids=lambda b: f"band{b}")
def test_pair_bounds_high_dim(d, lens, band):
    """The greedy walks for d >= 5 (points padded to 8 floats: the walk's
    candidate ring refills every 4 moves instead of 8): values and move
    counts bit-exact against Alg. 1 in the oracle, for both distances, over
    walks long enough for many refills."""
    print(f"[case] pair_bounds d={d} lens={lens} band={band}", flush=True)
    db, dbo = ragged_walks(40 + d, 24, lens, d)
    qs, qo = ragged_walks(140 + d, 2, lens, d)
    idx = _index(db, dbo)
    for dist in ("dk", "dtw"):
        _, ub, steps = (t.cpu().numpy() for t in idx.pair_bounds(to_dev(qs), qo, dist, band))
        for q in range(len(qo) - 1):
            S = qs[qo[q]:qo[q + 1]]
            for c in range(len(dbo) - 1):
                T = db[dbo[c]:dbo[c + 1]]
                w = O.band_w(band, S.shape[0], T.shape[0])
                v, st = O.gdk_sq_f32(S, T, w) if dist == "dk" else O.greedy_sum_f32(S, T, w)
                assert ub[q, c] == np.float32(v) and steps[q, c] == st, (dist, q, c, ub[q, c], v)
    idx.close()


@pytest.mark.parametrize("band", [0.1, 3, None], ids=lambda b: f"band{b}")
def test_knn_dtw_lb_both_orientations(band):
    """DTW with LB_Box in both orientations (option lb_both: the survivors of
    the query-envelope bound also get the candidate-envelope bound, eq. (1)
    in the paper's own orientation, and keep the larger): rows equal the
    oracle's on random walks and class-warp data; queries of another length
    than the (equal-length) series keep their one bound; a graph replay
    gives the same rows."""
    print(f"[case] knn dtw lb_both band={band}", flush=True)
    from paper_1811_11076_amd import synth
    rw_db, rw_dbo = synth.flat_equal(synth.random_walks(600, 64, 3, 61, "db"))
    rw_qs, rw_qo = synth.flat_equal(synth.random_walks(6, 64, 3, 61, "query"))
    cases = [(rw_db, rw_dbo, rw_qs, rw_qo), classwarp(2, 10, 128, 3, 1200, 5)]
    # equal-length index, queries of mixed lengths (64 and others)
    mq, mqo = ragged_walks(62, 4, (40, 90), 3)
    qs_mix = np.concatenate([rw_qs, mq])
    qo_mix = np.concatenate([rw_qo, rw_qo[-1] + mqo[1:]])
    cases.append((rw_db, rw_dbo, qs_mix, qo_mix))
    for db, dbo, qs, qo in cases:
        idx = _index(db, dbo)
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, "dtw", band)
        ids, dst, st = idx.knn(to_dev(qs), qo, 10, "dtw", band, stats=True, lb_both=True)
        assert_same_knn(ids, dst, ref_ids, ref_keys, "dtw")
        _, _, st0 = idx.knn(to_dev(qs), qo, 10, "dtw", band, stats=True)
        print(f"  pruned {st['bound_pruned']} vs {st0['bound_pruned']}, DPs started "
              f"{st['dp_started']} vs {st0['dp_started']}", flush=True)
        import torch
        out = (torch.empty_like(ids), torch.empty_like(dst))
        for _ in range(2):
            idx.knn(to_dev(qs), qo, 10, "dtw", band, use_graph=True, out=out, lb_both=True)
            torch.cuda.synchronize()
            assert_same_knn(out[0], out[1], ref_ids, ref_keys, "dtw")
        idx.close()


KNN_CASES = [
    # (name, seed, Q, N, lens, d, k)
    ("tiny_k_gt_n", 10, 2, 5, (3, 12), 2, 8),
    ("ragged", 11, 5, 300, (5, 60), 3, 7),
    ("multistrip", 12, 2, 40, (200, 520), 3, 3),
    ("equal", 13, 4, 500, (50, 50), 3, 10),
    ("d6", 14, 3, 200, (20, 40), 6, 5),
]


@pytest.mark.parametrize("case", KNN_CASES, ids=lambda c: c[0])
@pytest.mark.parametrize("band", BANDS, ids=lambda b: f"band{b}")
def test_knn_small(case, band):
    name, seed, Q, N, lens, d, k = case
    print(f"[case] knn {name} band={band}", flush=True)
    db, dbo = ragged_walks(seed, N, lens, d)
    qs, qo = ragged_walks(seed + 100, Q, lens, d)
    idx = _index(db, dbo)
    for dist in ("dk", "dtw"):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, k, dist, band)
        ids, dst, st = idx.knn(to_dev(qs), qo, k, dist, band, stats=True)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
        assert st["pairs"] == Q * N
        # every pair is counted once: discarded by a bound, or a DP began
        assert st["bound_pruned"] + st["dp_started"] == st["pairs"], st
    idx.close()


def test_knn_cfg1_full():
    """Random walks, 1 query x 1000 series, length 64, d = 3, k = 1, unbanded."""
    from paper_1811_11076_amd import synth
    print("[case] knn cfg1", flush=True)
    db, dbo = synth.flat_equal(synth.random_walks(1000, 64, 3, 1, "db"))
    qs, qo = synth.flat_equal(synth.random_walks(1, 64, 3, 1, "query"))
    idx = _index(db, dbo)
    for dist in ("dk", "dtw"):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 1, dist, None)
        ids, dst, _ = idx.knn(to_dev(qs), qo, 1, dist, None)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
    idx.close()


def test_knn_ties_and_order():
    """Duplicated series tie; ties go to the lower id; a given candidate
    order changes nothing."""
    import torch
    print("[case] knn ties/order", flush=True)
    db, dbo = ragged_walks(21, 50, (10, 30), 3)
    series = [db[dbo[i]:dbo[i + 1]] for i in range(50)]
    series += series[:20]  # ids 50..69 duplicate 0..19
    dbo2 = np.concatenate([[0], np.cumsum([len(s) for s in series])]).astype(np.int64)
    db2 = np.concatenate(series).astype(np.float32)
    qs = np.concatenate([series[3], series[7]]).astype(np.float32)
    qo = np.array([0, len(series[3]), len(series[3]) + len(series[7])], np.int64)
    idx = _index(db2, dbo2)
    perm = torch.stack([torch.randperm(70, generator=torch.Generator().manual_seed(s)) for s in (1, 2)])
    perm = perm.to(torch.int32).cuda()
    for dist in ("dk", "dtw"):
        ref_ids, ref_keys = O.knn_brute(db2, dbo2, qs, qo, 6, dist, 4)
        assert ref_ids[0, 0] == 3 and ref_ids[0, 1] == 53
        ids, dst, _ = idx.knn(to_dev(qs), qo, 6, dist, 4)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
        ids, dst, _ = idx.knn(to_dev(qs), qo, 6, dist, 4, order=perm, seed_count=9)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
    idx.close()


def test_knn_classwarp_reduced():
    """Class-warp series (10 classes, length 256, d = 3), 12 queries x 3000."""
    print("[case] knn classwarp reduced", flush=True)
    db, dbo, qs, qo = classwarp(2, 10, 256, 3, 3000, 12)
    idx = _index(db, dbo)
    for dist, band in (("dk", None), ("dtw", 0.1)):
        ref_ids, ref_keys, _ = O.knn_scan(db, dbo, qs, qo, 10, dist, band)
        ids, dst, st = idx.knn(to_dev(qs), qo, 10, dist, band, stats=True)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
        print(f"  {dist}: {st}", flush=True)
    idx.close()


def test_knn_classwarp_uneven_reduced():
    """The uneven-length class-warp generator (50 classes, prototypes of
    length 1024, members of length U{64..1024}, d = 3), 6 queries x 1500:
    slanted 10 % band for DTW (length-bucket LB_Box), unbanded DK."""
    print("[case] knn classwarp uneven reduced", flush=True)
    db, dbo, qs, qo = classwarp(3, 50, (64, 1024), 3, 1500, 6, proto_len=1024)
    idx = _index(db, dbo)
    for dist, band in (("dk", None), ("dtw", 0.1)):
        ref_ids, ref_keys, _ = O.knn_scan(db, dbo, qs, qo, 10, dist, band)
        ids, dst, st = idx.knn(to_dev(qs), qo, 10, dist, band, stats=True)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
        print(f"  {dist}: {st}", flush=True)
    idx.close()


@pytest.mark.parametrize("w", [3, 12, 20, 23, 24, 25, 27, 30, 45, 60])
def test_knn_band_kernel_widths(w):
    """Equal lengths, band widths covering every lane-per-pair window size
    (2w+1 of 7, 25, 41, 47, 49, 51, 55, 61, 91, 121 in windows of 16, 32, 52,
    52, 52 (tight mask), 52 (tight mask), 56, 64, 104, 128 slots), both
    distances, against the oracle."""
    print(f"[case] knn band widths w={w}", flush=True)
    db, dbo = ragged_walks(40 + w, 150, (128, 128), 3)
    qs, qo = ragged_walks(140 + w, 3, (128, 128), 3)
    idx = _index(db, dbo)
    for dist in ("dk", "dtw"):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 6, dist, w)
        ids, dst, st = idx.knn(to_dev(qs), qo, 6, dist, w, stats=True)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
        assert st["fallback_pairs"] == 0
    idx.close()


@pytest.mark.parametrize("w", [12, 45, 60])
def test_knn_band_dead_groups(w):
    """The band kernel skips groups of slots whose predecessors all exceed
    the threshold.  Series that put the live cells far from the diagonal
    (copies of a query shifted by up to most of the band, forwards and
    back) and long zero-cost runs (a constant stretch shared by query and
    copy: live cells climb a whole column through the upward chain) must
    still give the oracle's rows, for both distances and for k from 1 to
    beyond the planted copies."""
    print(f"[case] knn band dead groups w={w}", flush=True)
    L, d = 160, 3
    db, dbo = ragged_walks(700 + w, 300, (L, L), d)
    qs, qo = ragged_walks(710 + w, 3, (L, L), d)
    q0 = qs[qo[0]:qo[1]].copy()
    q0[50:90] = q0[50]  # a constant stretch
    qs[qo[0]:qo[1]] = q0
    for i, sh in enumerate((w * 3 // 4, -(w * 3 // 4), w // 3, -1, 0)):
        c = 20 + 7 * i
        src = np.roll(q0, sh, axis=0)
        src[:max(sh, 0)] = q0[0]
        if sh < 0:
            src[sh:] = q0[-1]
        db[dbo[c]:dbo[c + 1]] = src + np.float32(0.01 * i)
    idx = _index(db, dbo)
    for dist in ("dk", "dtw"):
        for k in (1, 4, 9):
            ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, k, dist, w)
            ids, dst, st = idx.knn(to_dev(qs), qo, k, dist, w, stats=True)
            assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
            assert st["bound_pruned"] + st["dp_started"] == st["pairs"], st
    idx.close()


@pytest.mark.parametrize("rows", [8, 16, 32])
def test_knn_tube_overflow_goes_to_general_dp(rows):
    """k = N keeps every DK cell alive, so every tube outgrows its window and
    the pair is finished by the general DP; results stay exact."""
    print(f"[case] knn tube overflow rows={rows}", flush=True)
    db, dbo = ragged_walks(51, 40, (60, 90), 2)
    qs, qo = ragged_walks(52, 2, (60, 90), 2)
    idx = _index(db, dbo)
    ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 40, "dk", None)
    ids, dst, st = idx.knn(to_dev(qs), qo, 40, "dk", None, stats=True, tube_rows=rows)
    assert_same_knn(ids, dst, ref_ids, ref_keys, "dk")
    assert st["fallback_pairs"] > 0
    # a handed-over pair counts once, in the general DP
    assert st["bound_pruned"] + st["dp_started"] == st["pairs"], st
    assert st["dp_completed"] + st["dp_abandoned"] == st["dp_started"], st
    # queries no taller than the window never overflow it
    db2, dbo2 = ragged_walks(53, 40, (5, 40), 2)
    qs2, qo2 = ragged_walks(54, 2, (5, rows), 2)
    idx2 = _index(db2, dbo2)
    ref_ids, ref_keys = O.knn_brute(db2, dbo2, qs2, qo2, 40, "dk", None)
    ids, dst, st = idx2.knn(to_dev(qs2), qo2, 40, "dk", None, stats=True, tube_rows=rows)
    assert_same_knn(ids, dst, ref_ids, ref_keys, "dk")
    assert st["fallback_pairs"] == 0
    idx.close()
    idx2.close()


@pytest.mark.parametrize("equal", [False, True], ids=["uneven", "equal"])
@pytest.mark.parametrize("rows", [8, 16, 32])
def test_knn_tube_end_row_above_window(rows, equal):
    """A pair whose only path within tau runs along row 0 and then climbs
    the whole last column (query 0, 1.5, 1.5, ...; candidate 0, ..., 0, e):
    the window stays at rows 0 .. rows-1 and the end row (39) lies above it
    while the window's top slot is live, so the pair must go to the general
    DP; rows equal the oracle's (DK^2 = 0.5625 for e = 0.75).  With every
    series as long as the query the tube runs its equal-length column
    count, otherwise the other one."""
    import numpy as np
    print(f"[case] knn tube end row above window rows={rows} equal={equal}", flush=True)
    rng = np.random.default_rng(70 + rows)
    m = 40
    q = np.full((m, 1), 1.5, np.float32)
    q[0] = 0.0
    series = []
    near = ((0.75, 40), (0.7, 40), (0.8, 40), (0.65, 40)) if equal else \
        ((0.75, 40), (0.7, 40), (0.8, 33), (0.75, 55))
    for e, n in near:
        t = np.zeros((n, 1), np.float32)
        t[-1] = e
        series.append(t)
    for _ in range(40):  # far from the query: pruned by their corner bounds
        n = m if equal else int(rng.integers(20, 60))
        series.append((20.0 + np.cumsum(rng.standard_normal((n, 1)), 0)).astype(np.float32))
    perm = rng.permutation(len(series))
    series = [series[i] for i in perm]
    db = np.concatenate(series)
    dbo = np.concatenate([[0], np.cumsum([len(x) for x in series])]).astype(np.int64)
    qo = np.array([0, m], np.int64)
    idx = _index(db, dbo)
    for k in (1, 3):
        ref_ids, ref_keys = O.knn_brute(db, dbo, q, qo, k, "dk", None)
        ids, dst, st = idx.knn(to_dev(q), qo, k, "dk", None, stats=True, tube_rows=rows)
        assert_same_knn(ids, dst, ref_ids, ref_keys, "dk")
        assert st["bound_pruned"] + st["dp_started"] == st["pairs"], st
        # the pair with e = 0.8 (DK^2 = 0.49 <= every tau of the scan)
        # reaches its last column with its end row above the window
        assert st["fallback_pairs"] >= 1, st
        print(f"  k={k} fallback {st['fallback_pairs']}", flush=True)
    idx.close()


@pytest.mark.parametrize("walk,task,seed", [(1, 128, 64), (0, 32, 0), (1, 256, 3000)])
def test_knn_dk_pipeline_options(walk, task, seed):
    """The DK bound-stage options (greedy pass over survivors, task size,
    seed size) change work, never results."""
    print(f"[case] knn dk options walk={walk} task={task} seed={seed}", flush=True)
    db, dbo, qs, qo = classwarp(2, 10, 256, 3, 2000, 5)
    idx = _index(db, dbo)
    ref_ids, ref_keys, _ = O.knn_scan(db, dbo, qs, qo, 10, "dk", None)
    ids, dst, _ = idx.knn(to_dev(qs), qo, 10, "dk", None, walk_pass=walk, task_size=task,
                          seed_count=seed)
    assert_same_knn(ids, dst, ref_ids, ref_keys, "dk")
    idx.close()


@pytest.mark.parametrize("slots", [32, 56, 104, 128])
def test_knn_dk_virtual_band(slots):
    """Unbanded DK through the lockstep banded kernel in a virtual band:
    pairs whose live cells reach the band's edge go to the general DP; rows
    equal the oracle's (class-warp pairs mostly fit, random walks often
    overflow)."""
    print(f"[case] knn dk virtual band slots={slots}", flush=True)
    db, dbo, qs, qo = classwarp(2, 10, 256, 3, 1500, 5)
    rdb, rdbo = ragged_walks(70 + slots, 300, (90, 90), 3)
    rqs, rqo = ragged_walks(170 + slots, 3, (90, 90), 3)
    for (d, do, q, qo_) in ((db, dbo, qs, qo), (rdb, rdbo, rqs, rqo)):
        idx = _index(d, do)
        ref_ids, ref_keys = O.knn_brute(d, do, q, qo_, 10, "dk", None)
        ids, dst, st = idx.knn(to_dev(q), qo_, 10, "dk", None, stats=True, dk_band_slots=slots)
        assert_same_knn(ids, dst, ref_ids, ref_keys, "dk")
        print(f"  fallback {st['fallback_pairs']} of {st['dp_started']}", flush=True)
        idx.close()


@pytest.mark.parametrize("so", [1, 2])
@pytest.mark.parametrize("kind", ["classwarp", "uneven", "ragged"])
def test_knn_survivor_orders(kind, so):
    """Survivors taken in ascending-bound order (surv_order = 1) or in
    candidate order (2): same rows as the oracle for both distances."""
    print(f"[case] knn survivor order {so} {kind}", flush=True)
    if kind == "classwarp":
        db, dbo, qs, qo = classwarp(2, 10, 256, 3, 2000, 6)
    elif kind == "uneven":
        db, dbo, qs, qo = classwarp(3, 50, (64, 512), 3, 800, 4, proto_len=512)
    else:
        db, dbo = ragged_walks(23, 300, (5, 60), 3)
        qs, qo = ragged_walks(123, 5, (5, 60), 3)
    idx = _index(db, dbo)
    for dist, band in (("dk", None), ("dtw", 0.1)):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, dist, band)
        ids, dst, _ = idx.knn(to_dev(qs), qo, 10, dist, band, surv_order=so)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
    idx.close()


@pytest.mark.parametrize("rows", [1, 2, 4])
def test_knn_general_dp_tile_rows(rows):
    """The general DP's strip shape (1, 2 or 4 rows per lane) on uneven
    lengths, where every DTW survivor and every DK tube overflow runs in it:
    rows equal the oracle's."""
    print(f"[case] knn general DP rows={rows}", flush=True)
    db, dbo = ragged_walks(31 + rows, 200, (30, 400), 3)
    qs, qo = ragged_walks(131 + rows, 4, (30, 400), 3)
    idx = _index(db, dbo)
    for dist, band in (("dk", None), ("dtw", 0.1), ("dtw", None), ("dk", 7)):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 8, dist, band)
        ids, dst, _ = idx.knn(to_dev(qs), qo, 8, dist, band, dp_rows=rows)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
    idx.close()


@pytest.mark.parametrize("seed", [64, 1024])
def test_knn_dk_diagonal_seed(seed):
    """DK seeded by the diagonal path's largest cost (equal lengths; ragged
    data falls back to the greedy walks): rows equal the oracle's."""
    print(f"[case] knn dk diagonal seed S={seed}", flush=True)
    cases = [classwarp(2, 10, 256, 3, 2000, 5),
             ragged_walks(51, 300, (20, 60), 3) + ragged_walks(151, 4, (20, 60), 3)]
    for db, dbo, qs, qo in cases:
        idx = _index(db, dbo)
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, "dk", None)
        ids, dst, _ = idx.knn(to_dev(qs), qo, 10, "dk", None, dk_seed=1, seed_count=seed)
        assert_same_knn(ids, dst, ref_ids, ref_keys, "dk")
        idx.close()


def test_knn_general_dp_forced_equals_fast():
    """dp_kernel = 1 (general DP only) and the default give identical rows."""
    import ctypes
    from paper_1811_11076_amd import _lib
    print("[case] knn general vs fast", flush=True)
    db, dbo, qs, qo = classwarp(2, 10, 256, 3, 2000, 6)
    idx = _index(db, dbo)
    for dist, band in (("dk", None), ("dtw", 0.1)):
        a_ids, a_d, _ = idx.knn(to_dev(qs), qo, 10, dist, band)
        lib = _lib.load()
        opts = _lib.QueryOpts()
        opts.size = ctypes.sizeof(_lib.QueryOpts)
        opts.dp_kernel = 1
        import torch
        ids = torch.empty((6, 10), dtype=torch.int64, device="cuda")
        dd = torch.empty((6, 10), dtype=torch.float32, device="cuda")
        qv = to_dev(qs)
        _lib.check(lib.tsk_knn_query(idx._h, ctypes.c_void_p(qv.data_ptr()),
                                     qo.ctypes.data_as(ctypes.c_void_p), 6, 10,
                                     _lib.TSK_DK if dist == "dk" else _lib.TSK_DTW,
                                     _lib.band_struct(band), ctypes.byref(opts),
                                     ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(dd.data_ptr()),
                                     None, None))
        torch.cuda.synchronize()
        assert torch.equal(ids, a_ids) and torch.equal(dd.view(torch.int32), a_d.view(torch.int32))
    idx.close()


@pytest.mark.parametrize("lbq", [1, 16])
@pytest.mark.parametrize("w", [0, 3, 25, 60, None])
@pytest.mark.parametrize("d,L", [(1, 33), (3, 128), (6, 300), (8, 17)])
def test_knn_dtw_lb_per_pair_abandoning(d, L, w, lbq):
    """DTW with the per-pair early-abandoning LB_Box kernel (lb_qgroup = 1)
    and with 16 queries per candidate load (lb_qgroup = 16): rows equal the
    oracle's for lengths that are and are not multiples of a step (ragged
    last step), unbanded and banded, 5 queries (a partial group), and equal
    the default kernel's rows; the class-warp data has ties at the
    threshold's scale."""
    print(f"[case] dtw lb kernel {lbq} d={d} L={L} w={w}", flush=True)
    db, dbo = ragged_walks(700 + d + L, 600, (L, L), d)
    qs, qo = ragged_walks(800 + d + L, 5, (L, L), d)
    db[dbo[17]:dbo[18]] = qs[qo[1]:qo[2]]  # an exact copy: DTW 0, LB 0
    idx = _index(db, dbo)
    ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 7, "dtw", w)
    ids, dst, st = idx.knn(to_dev(qs), qo, 7, "dtw", w, stats=True, lb_qgroup=lbq)
    assert_same_knn(ids, dst, ref_ids, ref_keys, "dtw")
    ids0, dst0, st0 = idx.knn(to_dev(qs), qo, 7, "dtw", w, stats=True)
    assert torch_equal(ids, ids0) and torch_equal(dst, dst0)
    assert st["pairs"] == st0["pairs"] == 5 * 600
    print(f"  LB terms {st['bound_steps']} vs {st0['bound_steps']}", flush=True)
    idx.close()
    db, dbo, qs, qo = classwarp(2, 10, 256, 3, 3000, 6)
    idx = _index(db, dbo)
    ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, "dtw", 0.1)
    ids, dst, _ = idx.knn(to_dev(qs), qo, 10, "dtw", 0.1, lb_qgroup=lbq)
    assert_same_knn(ids, dst, ref_ids, ref_keys, "dtw")
    idx.close()


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


@pytest.mark.parametrize("rows", [8, 16, 32])
def test_knn_dk_tube_rows_classwarp(rows):
    """Class-warp DK (the live region follows the warped diagonal) with every
    tube window: rows equal the oracle's."""
    print(f"[case] knn dk tube rows={rows} classwarp", flush=True)
    db, dbo, qs, qo = classwarp(2, 10, 256, 3, 3000, 6)
    idx = _index(db, dbo)
    ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, "dk", None)
    ids, dst, st = idx.knn(to_dev(qs), qo, 10, "dk", None, stats=True, tube_rows=rows)
    assert_same_knn(ids, dst, ref_ids, ref_keys, "dk")
    print(f"  fallback {st['fallback_pairs']} cells {st['dp_valid_cells']}", flush=True)
    idx.close()


def test_knn_cancel_flag():
    """A set host flag stops a k-NN call (eager or graph) before any device
    work (TSK_ERR_CANCELLED, outputs untouched); a clear flag changes
    nothing."""
    import numpy as np
    import torch
    from paper_1811_11076_amd import TskError, _lib
    print("[case] cancel flag", flush=True)
    db, dbo = ragged_walks(61, 200, (40, 40), 3)
    qs, qo = ragged_walks(62, 4, (40, 40), 3)
    idx = _index(db, dbo)
    flag = np.zeros(1, np.int32)
    ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 5, "dtw", 4)
    ids, dst, _ = idx.knn(to_dev(qs), qo, 5, "dtw", 4, cancel=flag)
    assert_same_knn(ids, dst, ref_ids, ref_keys, "dtw")
    flag[0] = 1
    out = (torch.full((4, 5), -7, dtype=torch.int64, device="cuda"),
           torch.full((4, 5), -7.0, dtype=torch.float32, device="cuda"))
    for kw in ({}, {"use_graph": True}):
        with pytest.raises(TskError) as ei:
            idx.knn(to_dev(qs), qo, 5, "dk", None, out=out, cancel=flag, **kw)
        assert ei.value.code == _lib.TSK_ERR_CANCELLED
        torch.cuda.synchronize()
        assert bool((out[0] == -7).all()) and bool((out[1] == -7.0).all())
    idx.close()


@pytest.mark.parametrize("limit", [1, 300_000, 2_000_000])
def test_knn_workspace_limit_chunks(limit):
    """An index with a small workspace bound splits calls into chunks (down
    to one query each); rows equal the oracle's for both distances and the
    range query."""
    from paper_1811_11076_amd import Index
    print(f"[case] workspace limit {limit}", flush=True)
    db, dbo = ragged_walks(71, 500, (30, 90), 3)
    qs, qo = ragged_walks(72, 9, (30, 90), 3)
    idx = Index(to_dev(db), dbo, workspace_limit_bytes=limit)
    for dist, band in (("dk", None), ("dtw", 0.1)):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 6, dist, band)
        ids, dst, st = idx.knn(to_dev(qs), qo, 6, dist, band, stats=True)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
        assert st["pairs"] == 9 * 500
    offs, rids, _, _ = idx.range(to_dev(qs), qo, 4.0, "dk", None)
    ref = O.range_brute(db, dbo, qs, qo, 4.0, "dk", None)
    for q in range(9):
        assert np.array_equal(rids[offs[q]:offs[q + 1]].cpu().numpy(), ref[q][0])
    idx.close()


def test_validate_values_finds_first_nonfinite():
    import torch
    from paper_1811_11076_amd import validate_values
    v = torch.randn(1_000_003, device="cuda")
    assert validate_values(v) == -1
    v[777_777] = float("inf")
    v[900_001] = float("nan")
    assert validate_values(v) == 777_777
    v[5] = float("-inf")
    assert validate_values(v) == 5
