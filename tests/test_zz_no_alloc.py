"""The fixed-workspace k-NN call (C: tsk_knn_query_noalloc) against the
allocating one (tsk_knn_query): identical ids and distance bits, on two
calls in a row of which the second is smaller, for both distances, equal
and uneven lengths, and a database large enough that the fixed workspace
splits the queries into several chunks.  A database too large for one
query's workspace is refused before any device work."""
import numpy as np
import pytest

from gpu_cases import classwarp, ragged_walks, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _index(vals, off):
    from paper_1811_11076_amd import Index
    return Index(to_dev(vals), off)


def _pair(idx, dq, qo, k, distance, band):
    """(reference rows from the allocating call, rows from the fixed one)."""
    import torch
    nq = len(qo) - 1
    ref = idx.knn(dq, qo, k, distance, band)
    out = (torch.full((nq, k), -7, dtype=torch.int64, device="cuda"),
           torch.full((nq, k), -7.0, dtype=torch.float32, device="cuda"))
    idx.knn(dq, qo, k, distance, band, no_alloc=True, out=out)
    torch.cuda.synchronize()
    return ref, out


def _same(ref, got):
    assert np.array_equal(ref[0].cpu().numpy(), got[0].cpu().numpy())
    assert np.array_equal(ref[1].cpu().numpy().view(np.uint32), got[1].cpu().numpy().view(np.uint32))


CASES = [
    # (name, distance, band)
    ("dk_unbanded", "dk", None),
    ("dtw_band10", "dtw", 0.1),
    ("dk_band10", "dk", 0.1),
]


@pytest.mark.parametrize("name,distance,band", CASES)
def test_noalloc_equal_lengths(name, distance, band):
    print(f"\n[case] no-alloc equal lengths {name}", flush=True)
    db, dbo, qs, qo = classwarp(2, 10, 256, 3, 3000, 24)
    idx = _index(db, dbo)
    dq = to_dev(qs)
    _same(*_pair(idx, dq, qo, 10, distance, band))
    # second call, smaller: 5 queries
    _same(*_pair(idx, dq[:int(qo[5])], qo[:6], 10, distance, band))
    idx.close()


@pytest.mark.parametrize("distance,band", [("dk", None), ("dtw", 0.1), ("dtw", 7)])
def test_noalloc_uneven_lengths(distance, band):
    print(f"\n[case] no-alloc uneven lengths {distance} {band}", flush=True)
    db, dbo = ragged_walks(11, 700, (20, 300), 3)
    qs, qo = ragged_walks(12, 9, (30, 280), 3)
    idx = _index(db, dbo)
    dq = to_dev(qs)
    _same(*_pair(idx, dq, qo, 5, distance, band))
    _same(*_pair(idx, dq[:int(qo[3])], qo[:4], 5, distance, band))
    idx.close()


def test_noalloc_several_chunks():
    """200 000 series: about 4 MB of workspace per query, so the 40
    queries take several chunks of the fixed workspace."""
    print("\n[case] no-alloc several chunks: 40 x 200000", flush=True)
    from paper_1811_11076_amd import synth
    db, dbo = synth.flat_equal(synth.random_walks(200_000, 32, 3, 5, "db"))
    qs, qo = synth.flat_equal(synth.random_walks(40, 32, 3, 5, "query"))
    idx = _index(db, dbo)
    dq = to_dev(qs)
    for distance, band in (("dtw", 3), ("dk", None)):
        _same(*_pair(idx, dq, qo, 10, distance, band))
        _same(*_pair(idx, dq[:int(qo[7])], qo[:8], 10, distance, band))
    idx.close()


def test_noalloc_refuses_oversized_database():
    """One query's workspace above the fixed size: INVALID_ARG, outputs
    untouched."""
    import torch
    from paper_1811_11076_amd import _lib
    n = 5_000_000  # 16 bytes per series and more: above 64 MiB
    vals = np.random.default_rng(3).normal(size=(n, 1)).astype(np.float32)
    off = np.arange(n + 1, dtype=np.int64)
    idx = _index(vals, off)
    q = to_dev(vals[:4])
    out = (torch.full((4, 1), -7, dtype=torch.int64, device="cuda"),
           torch.full((4, 1), -7.0, dtype=torch.float32, device="cuda"))
    with pytest.raises(_lib.TskError) as e:
        idx.knn(q, np.arange(5, dtype=np.int64), 1, "dtw", None, no_alloc=True, out=out)
    assert e.value.code == _lib.TSK_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((out[0] == -7).all()) and bool((out[1] == -7.0).all())
    idx.close()


def test_noalloc_excluded_options():
    from paper_1811_11076_amd import _lib
    db, dbo = ragged_walks(13, 50, (16, 16), 2)
    idx = _index(db, dbo)
    dq = to_dev(db[:32])
    qo = np.array([0, 16, 32], np.int64)
    for kw in ({"use_graph": True}, {"profile": True}, {"lb_both": True}):
        with pytest.raises(_lib.TskError) as e:
            idx.knn(dq, qo, 3, "dtw", 2, no_alloc=True, **kw)
        assert e.value.code == _lib.TSK_ERR_UNSUPPORTED
    idx.close()
