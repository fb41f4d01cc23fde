"""GPU parity above 8 dimensions (d = 9 .. 27, the range of Table 1's data
sets): the library stores and scans the series padded with zero coordinates
to 12, 16, 24 or 32, which leaves every point cost, bound and DP value equal
bit for bit to the unpadded arithmetic of the oracle.  Pair distances,
greedy bounds with their move counts and k-NN rows (DK and DTW, bands,
ragged and equal lengths, the corner cascade, graphs, the allocation-free
entry) all against the oracle on the unpadded inputs."""
import numpy as np
import pytest

import oracle as O
from gpu_cases import assert_same_knn, classwarp, ragged_walks, to_dev

pytestmark = pytest.mark.gpu

DIMS = [9, 13, 22, 27]
BANDS = [None, 3, 0.2]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _index(vals, off):
    from paper_1811_11076_amd import Index
    return Index(to_dev(vals), off)


@pytest.mark.parametrize("d", DIMS)
@pytest.mark.parametrize("band", BANDS, ids=lambda b: f"band{b}")
def test_pair_distances_and_bounds_high_dim(d, band):
    print(f"[case] highdim pairs d={d} band={band}", flush=True)
    db, dbo = ragged_walks(500 + d, 20, (5, 90), d)
    qs, qo = ragged_walks(600 + d, 3, (5, 90), d)
    idx = _index(db, dbo)
    assert idx.dim == d
    for dist in ("dk", "dtw"):
        got = idx.pair_distances(to_dev(qs), qo, dist, band).cpu().numpy()
        ref = O.pair_keys(db, dbo, qs, qo, dist, band)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (dist, np.argwhere(got != ref)[:5])
        lb, ub, steps = (t.cpu().numpy() for t in idx.pair_bounds(to_dev(qs), qo, dist, band))
        for q in range(len(qo) - 1):
            S = qs[qo[q]:qo[q + 1]]
            for c in range(len(dbo) - 1):
                T = db[dbo[c]:dbo[c + 1]]
                w = O.band_w(band, S.shape[0], T.shape[0])
                v, st = O.gdk_sq_f32(S, T, w) if dist == "dk" else O.greedy_sum_f32(S, T, w)
                assert ub[q, c] == np.float32(v) and steps[q, c] == st, (dist, q, c, ub[q, c], v)
                if dist == "dtw":
                    assert lb[q, c] <= got[q, c]
    idx.close()


@pytest.mark.parametrize("d", DIMS)
@pytest.mark.parametrize("band", BANDS, ids=lambda b: f"band{b}")
def test_knn_ragged_high_dim(d, band):
    print(f"[case] highdim knn ragged d={d} band={band}", flush=True)
    db, dbo = ragged_walks(700 + d, 250, (8, 70), d)
    qs, qo = ragged_walks(800 + d, 4, (8, 70), d)
    idx = _index(db, dbo)
    for dist in ("dk", "dtw"):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 7, dist, band)
        ids, dst, st = idx.knn(to_dev(qs), qo, 7, dist, band, stats=True)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
        assert st["pairs"] == 4 * 250
    idx.close()


@pytest.mark.parametrize("d", DIMS)
def test_knn_equal_length_cascade_high_dim(d):
    """Equal lengths (the corner cascade, the diagonal and greedy seeds,
    LB_Box of the survivors) on class-warp data: rows equal the oracle's
    for every cascade setting, and a graph replay gives the same rows."""
    print(f"[case] highdim knn classwarp d={d}", flush=True)
    import torch
    db, dbo, qs, qo = classwarp(5, 8, 96, d, 1500, 6)
    idx = _index(db, dbo)
    for dist, band in (("dk", None), ("dtw", 0.1), ("dtw", None)):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, dist, band)
        for bs, dc in ((0, 0), (2, 2), (1, 1)):
            ids, dst, st = idx.knn(to_dev(qs), qo, 10, dist, band, bound_seed=bs, dtw_cascade=dc,
                                   stats=True)
            assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
            assert st["bound_pruned"] + st["dp_started"] == st["pairs"], (bs, dc, st)
        out = (torch.empty_like(ids), torch.empty_like(dst))
        for _ in range(2):
            idx.knn(to_dev(qs), qo, 10, dist, band, use_graph=True, out=out)
            torch.cuda.synchronize()
            assert_same_knn(out[0], out[1], ref_ids, ref_keys, dist)
    idx.close()


@pytest.mark.parametrize("d", [13, 27])
def test_knn_no_alloc_high_dim(d):
    """The allocation-free entry pads the queries inside its fixed workspace:
    two calls in a row, the second smaller, equal the allocating entry."""
    print(f"[case] highdim knn no_alloc d={d}", flush=True)
    import torch
    db, dbo = ragged_walks(900 + d, 400, (20, 60), d)
    qs, qo = ragged_walks(950 + d, 5, (20, 60), d)
    idx = _index(db, dbo)
    for nq in (5, 2):
        sub_q = qs[:qo[nq]]
        sub_o = qo[:nq + 1]
        for dist, band in (("dk", None), ("dtw", 4)):
            ids, dst, _ = idx.knn(to_dev(sub_q), sub_o, 6, dist, band)
            out = (torch.empty_like(ids), torch.empty_like(dst))
            idx.knn(to_dev(sub_q), sub_o, 6, dist, band, no_alloc=True, out=out)
            torch.cuda.synchronize()
            assert torch.equal(out[0], ids) and torch.equal(out[1].view(torch.int32), dst.view(torch.int32))
    idx.close()


def test_knn_uneven_lengths_high_dim():
    """Uneven lengths at d = 22: DTW by length-bucket LB_Box, slanted band."""
    print("[case] highdim knn uneven d=22", flush=True)
    db, dbo, qs, qo = classwarp(6, 10, (32, 200), 22, 600, 4, proto_len=200)
    idx = _index(db, dbo)
    for dist, band in (("dk", None), ("dtw", 0.1)):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 5, dist, band)
        ids, dst, _ = idx.knn(to_dev(qs), qo, 5, dist, band)
        assert_same_knn(ids, dst, ref_ids, ref_keys, dist)
    idx.close()
