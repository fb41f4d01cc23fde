"""Full-size parity of the uneven-length batching workload: 1024 queries
against 100 000 class-warp series of lengths uniform in {64..1024}, d = 3,
k = 10, DK unbanded and DTW in the slanted 10 % band.

The GPU answers all 1024 queries in one call per distance, through the
C-ABI, in its default and its graph-replayed configurations.  The oracle
checks:
  * the first queries against every series (its pruned scan, equal to the
    plain definition: ids and distance bits);
  * every (id, distance) returned for every query, recomputed by its full DP;
  * each row ascending by (distance, id).
"""
import numpy as np
import pytest

import oracle as O
from gpu_cases import classwarp, to_dev

pytestmark = pytest.mark.gpu

Q, N, LENS, D, K, BAND = 1024, 100_000, (64, 1024), 3, 10, 0.1
CHECK_QUERIES = {"dk": 16, "dtw": 8}


@pytest.fixture(scope="module")
def workload():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[case] full-size uneven workload: generating 1024 x 100000 series", flush=True)
    db, dbo, qs, qo = classwarp(3, 50, LENS, D, N, Q, proto_len=1024)
    from paper_1811_11076_amd import Index
    idx = Index(to_dev(db), dbo)
    yield db, dbo, qs, qo, idx
    idx.close()


def _check(db, dbo, qs, qo, ids, dist, distance, band):
    ids = ids.cpu().numpy()
    dist = dist.cpu().numpy()
    sel = CHECK_QUERIES[distance]
    rids, rkeys, _ = O.knn_verify(db, dbo, qs[:qo[sel]], qo[:sel + 1], K, distance, band)
    exp = np.sqrt(rkeys.astype(np.float32)) if distance == "dk" else rkeys.astype(np.float32)
    assert np.array_equal(ids[:sel], rids), (ids[:sel], rids)
    assert np.array_equal(dist[:sel].view(np.uint32), exp.view(np.uint32))
    qi, ri = np.nonzero(ids >= 0)
    assert qi.size == Q * K  # every query has k finite neighbours here
    keys = O.pair_list_keys(db, dbo, qs, qo, qi, ids[qi, ri], distance, band)
    want = np.sqrt(keys) if distance == "dk" else keys
    assert np.array_equal(dist[qi, ri].view(np.uint32), want.astype(np.float32).view(np.uint32))
    for q in range(Q):
        row = list(zip(dist[q].tolist(), ids[q].tolist()))
        assert row == sorted(row) and len(set(ids[q].tolist())) == K


def _same_or_report(db, dbo, qs, qo, runs, distance, band):
    """Rows of two runs equal; if not, the differing rows are checked
    against the oracle so that the failure names the wrong side."""
    (na, (ia, da)), (nb, (ib, dbb)) = runs.items()
    ia, da, ib, dbb = (t.cpu().numpy() for t in (ia, da, ib, dbb))
    rows = np.nonzero((ia != ib).any(1) | (da.view(np.uint32) != dbb.view(np.uint32)).any(1))[0]
    if rows.size == 0:
        return
    report = [f"{rows.size} rows differ: {rows[:16].tolist()}"]
    for q in rows[:4]:
        one = qs[qo[q]:qo[q + 1]]
        rids, rkeys, _ = O.knn_verify(db, dbo, one, np.array([0, len(one)], np.int64), K,
                                      distance, band)
        exp = np.sqrt(rkeys.astype(np.float32)) if distance == "dk" else rkeys.astype(np.float32)
        for name, ids, dist in ((na, ia, da), (nb, ib, dbb)):
            ok = np.array_equal(ids[q], rids[0]) and \
                np.array_equal(dist[q].view(np.uint32), exp[0].view(np.uint32))
            report.append(f"query {q} {name} {'equals' if ok else 'differs from'} the oracle: "
                          f"{ids[q].tolist()} {dist[q].tolist()} vs {rids[0].tolist()} "
                          f"{exp[0].tolist()}")
    raise AssertionError("\n".join(report))


@pytest.mark.parametrize("distance,band", [("dk", None), ("dtw", BAND)])
def test_uneven_full_size(workload, distance, band):
    db, dbo, qs, qo, idx = workload
    print(f"[case] full-size uneven {distance}: 1024 queries in one call", flush=True)
    ids, dist, st = idx.knn(to_dev(qs), qo, K, distance, band, stats=True)
    print(f"[case] full-size uneven {distance}: GPU {st['ms_total']:.1f} ms, checking", flush=True)
    _check(db, dbo, qs, qo, ids, dist, distance, band)


def test_uneven_full_size_graph_replay(workload):
    """The same rows from the call captured as one HIP graph and replayed,
    with other eager work on the index between replays."""
    import torch
    db, dbo, qs, qo, idx = workload
    dq = to_dev(qs)
    ref = {dist: idx.knn(dq, qo, K, dist, band) for dist, band in (("dk", None), ("dtw", BAND))}
    out = {dist: (torch.empty((Q, K), dtype=torch.int64, device="cuda"),
                  torch.empty((Q, K), dtype=torch.float32, device="cuda")) for dist in ref}
    for rep in range(3):
        for dist, band in (("dk", None), ("dtw", BAND)):
            print(f"[case] full-size uneven graph replay {rep} {dist}", flush=True)
            idx.knn(dq, qo, K, dist, band, use_graph=True, out=out[dist])
            torch.cuda.synchronize()
            _same_or_report(db, dbo, qs, qo, {"eager": ref[dist][:2], "graph": out[dist]},
                            dist, band)
            # eager work between replays
            idx.knn(dq[:int(qo[4])], qo[:5], K, "dtw", BAND)
            torch.cuda.synchronize()
