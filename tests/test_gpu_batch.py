"""Batched scan over uneven lengths: one call for many queries equals one
call per query; a captured, replayed HIP graph equals the eager call on
every replay; the autotuner's choices leave the rows unchanged."""
import numpy as np
import pytest

import oracle as O
from gpu_cases import assert_same_knn, classwarp, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _uneven(n_db, n_q):
    # the 50-class, prototype-length-1024 generator at reduced size
    return classwarp(3, 50, (64, 1024), 3, n_db, n_q, proto_len=1024)


def test_batched_equals_per_query_uneven():
    print("[case] batched vs per-query (uneven lengths)", flush=True)
    from paper_1811_11076_amd import Index
    db, dbo, qs, qo = _uneven(1200, 6)
    idx = Index(to_dev(db), dbo)
    dq = to_dev(qs)
    for dist, band in (("dk", None), ("dtw", 0.1)):
        ids, dst, _ = idx.knn(dq, qo, 10, dist, band)
        for q in range(len(qo) - 1):
            sub = to_dev(qs[qo[q]:qo[q + 1]])
            i1, d1, _ = idx.knn(sub, np.array([0, qo[q + 1] - qo[q]]), 10, dist, band)
            assert np.array_equal(i1.cpu().numpy()[0], ids.cpu().numpy()[q]), (dist, q)
            assert np.array_equal(d1.cpu().numpy()[0].view(np.uint32),
                                  dst.cpu().numpy()[q].view(np.uint32)), (dist, q)
    ref_ids, ref_keys, _ = O.knn_scan(db, dbo, qs, qo, 10, "dtw", 0.1)
    ids, dst, _ = idx.knn(dq, qo, 10, "dtw", 0.1)
    assert_same_knn(ids, dst, ref_ids, ref_keys, "dtw")
    idx.close()


@pytest.mark.parametrize("kind", ["equal", "uneven"])
def test_graph_replays_match_eager(kind):
    """Each replay runs after other eager work on the same index and a
    synchronisation, and must reproduce the eager rows exactly."""
    print(f"[case] graph replay {kind}", flush=True)
    import torch
    from paper_1811_11076_amd import Index
    if kind == "equal":
        db, dbo, qs, qo = classwarp(2, 10, 256, 3, 2000, 8)
    else:
        db, dbo, qs, qo = _uneven(1000, 5)
    _, _, qs2, qo2 = classwarp(2, 10, 256, 3, 10, 3) if kind == "equal" else _uneven(10, 3)
    idx = Index(to_dev(db), dbo)
    dq, dq2 = to_dev(qs), to_dev(qs2)
    nq = len(qo) - 1
    for dist, band in (("dk", None), ("dtw", 0.1)):
        e_ids, e_d, _ = idx.knn(dq, qo, 10, dist, band)
        out = (torch.full((nq, 10), -7, dtype=torch.int64, device="cuda"),
               torch.full((nq, 10), -7.0, dtype=torch.float32, device="cuda"))
        for rep in range(4):
            out[0].fill_(-7)
            out[1].fill_(-7.0)
            ids, dst, st = idx.knn(dq, qo, 10, dist, band, use_graph=True, out=out,
                                   stats=(rep == 3))
            torch.cuda.synchronize()
            assert torch.equal(ids, e_ids) and torch.equal(dst, e_d), (dist, rep)
            # eager work on the same workspace between replays
            idx.knn(dq2, qo2, 10, dist, band)
            torch.cuda.synchronize()
        print(f"  {dist}: graph call {st['ms_total']:.3f} ms", flush=True)
    idx.close()


def test_tuner_keeps_rows_and_caches():
    print("[case] tuner", flush=True)
    from paper_1811_11076_amd import Index
    db, dbo, qs, qo = _uneven(1500, 8)
    idx = Index(to_dev(db), dbo)
    dq = to_dev(qs)
    for dist, band in (("dk", None), ("dtw", 0.1)):
        base_ids, base_d, _ = idx.knn(dq, qo, 10, dist, band)
        best, ms = idx.tune(dq, qo, 10, dist, band, sample_queries=4, reps=1)
        print(f"  {dist}: {best} {ms:.3f} ms", flush=True)
        assert ms > 0
        ids, dst, _ = idx.knn(dq, qo, 10, dist, band, tune=True)
        assert np.array_equal(ids.cpu().numpy(), base_ids.cpu().numpy())
        assert np.array_equal(dst.cpu().numpy(), base_d.cpu().numpy())
    idx.close()


def test_profile_counters_start_at_zero():
    """A new index's profile starts from zero even where its buffer reuses
    the memory of an earlier index's profile: the pair count of two profiled
    calls is exactly twice the queries x series, for both distances."""
    import torch
    from paper_1811_11076_amd import Index
    db, dbo, qs, qo = classwarp(2, 10, 128, 3, 3000, 8)
    dq = to_dev(qs)
    for rep in range(3):
        idx = Index(to_dev(db), dbo)
        idx.profile(reset=True)
        for distance, band in (("dk", None), ("dtw", 0.1)):
            for _ in range(2):
                idx.knn(dq, qo, 10, distance, band, profile=True)
            p = idx.profile(reset=True)
            assert p["calls"] == 2 and p["chunks"] == 2
            assert p["pairs"] == 2 * 8 * 3000, (rep, distance, p["pairs"])
            assert p["dp_started"] <= p["pairs"] and p["fallback_pairs"] <= p["dp_started"]
        idx.close()
        torch.cuda.synchronize()
