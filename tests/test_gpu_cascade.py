"""The corner-bound cascade and the bound-ordered threshold seed, through
the C-ABI, against the oracle's plain k-NN definition.

Every warping path contains the first and the last cell, so the corner
bound (DK: the larger of their costs, DTW: their sum) never exceeds the
distance; seeding the threshold from the candidates of smallest corner
bound and computing LB_Box (eq. (1)) only for the corner survivors change
which pairs are pruned, never the rows: ids and distance bits equal the
oracle's, the other settings' rows, and graph replays of the call."""
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


def _index(vals, off):
    from paper_1811_11076_amd import Index
    return Index(to_dev(vals), off)


SETTINGS = [
    # (bound_seed, dtw_cascade); dtw_cascade 3 = the corner bound alone
    (0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (2, 1), (0, 3), (2, 3),
]


@pytest.mark.parametrize("d", [1, 3, 6, 8])
@pytest.mark.parametrize("band", [None, 0, 4, 0.1])
def test_cascade_random_walks(d, band):
    """Random walks of one length (L = 97: ragged steps), an exact copy of a
    query (distance 0 at both corners) and a copy with its end point moved
    (same first cell, a larger corner bound), k = 7 of 500."""
    print(f"[case] cascade walks d={d} band={band}", flush=True)
    db, dbo = ragged_walks(900 + d, 500, (97, 97), d)
    qs, qo = ragged_walks(901 + d, 6, (97, 97), d)
    db[dbo[40]:dbo[41]] = qs[qo[2]:qo[3]]
    db[dbo[41]:dbo[42]] = qs[qo[2]:qo[3]]
    db[dbo[42] - 1] += 0.5
    idx = _index(db, dbo)
    dq = to_dev(qs)
    for distance in ("dk", "dtw"):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 7, distance, band)
        for bs, cas in SETTINGS:
            ids, dst, st = idx.knn(dq, qo, 7, distance, band, stats=True, bound_seed=bs,
                                   dtw_cascade=cas)
            assert_same_knn(ids, dst, ref_ids, ref_keys, distance)
            assert st["pairs"] == 6 * 500
            # every pair is either discarded by a bound or reaches a DP
            assert st["bound_pruned"] + st["dp_started"] == st["pairs"], (bs, cas, st)
    idx.close()


@pytest.mark.parametrize("seed_count", [1, 10, 512, 3000])
def test_cascade_classwarp(seed_count):
    """Class-warp series (10 classes, L = 256, d = 3), k = 10: DK unbanded
    and DTW in the 10 % band, seed sets from one candidate to all of them,
    every setting of the seed and the cascade."""
    print(f"[case] cascade classwarp seed_count={seed_count}", flush=True)
    db, dbo, qs, qo = classwarp(2, 10, 256, 3, 3000, 12)
    idx = _index(db, dbo)
    dq = to_dev(qs)
    for distance, band in (("dk", None), ("dtw", 0.1)):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, distance, band)
        st = {}
        for bs, cas in SETTINGS:
            ids, dst, st[(bs, cas)] = idx.knn(dq, qo, 10, distance, band, stats=True,
                                              seed_count=seed_count, bound_seed=bs,
                                              dtw_cascade=cas)
            assert_same_knn(ids, dst, ref_ids, ref_keys, distance)
            s_ = st[(bs, cas)]
            assert s_["bound_pruned"] + s_["dp_started"] == s_["pairs"], (bs, cas, s_)
        print(f"  {distance}: completed DPs bound-ordered {st[(1, 0)]['dp_completed']} "
              f"head {st[(2, 0)]['dp_completed']}; seed+bound steps cascade "
              f"{st[(0, 1)]['bound_steps']} all-pairs LB_Box {st[(0, 0)]['bound_steps']}",
              flush=True)
    idx.close()


def test_cascade_graph_replay_and_chunks_cascade_on():
    _graph_and_chunks(dict(dtw_cascade=1))


def test_cascade_graph_replay_and_chunks():
    _graph_and_chunks({})


def _graph_and_chunks(kw):
    """The cascade inside a captured graph (three replays, eager work and a
    synchronisation between them) and over several query chunks (a small
    workspace bound: six chunks, eager and as one graph) gives the oracle's
    rows."""
    import torch
    from paper_1811_11076_amd import Index
    db, dbo, qs, qo = classwarp(2, 10, 128, 3, 2000, 16)
    dq = to_dev(qs)
    idx = _index(db, dbo)
    small = Index(to_dev(db), dbo, workspace_limit_bytes=2000 * 20 * 3 + 128 * 64 * 3)
    for distance, band in (("dk", None), ("dtw", 0.1)):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, distance, band)
        ids, dst, _ = small.knn(dq, qo, 10, distance, band, **kw)
        assert_same_knn(ids, dst, ref_ids, ref_keys, distance)
        out = (torch.empty((16, 10), dtype=torch.int64, device="cuda"),
               torch.empty((16, 10), dtype=torch.float32, device="cuda"))
        for rep in range(3):
            idx.knn(dq, qo, 10, distance, band, use_graph=True, out=out, **kw)
            torch.cuda.synchronize()
            assert_same_knn(out[0], out[1], ref_ids, ref_keys, distance)
            idx.knn(dq[:int(qo[3])], qo[:4], 10, "dtw", 3)
            torch.cuda.synchronize()
            # all six chunks of the small-workspace index in one graph
            small.knn(dq, qo, 10, distance, band, use_graph=True, out=out, **kw)
            torch.cuda.synchronize()
            assert_same_knn(out[0], out[1], ref_ids, ref_keys, distance)
            small.knn(dq[:int(qo[5])], qo[:6], 10, distance, band)
            torch.cuda.synchronize()
    small.close()
    idx.close()


@pytest.mark.parametrize("N", [70001, 65536 + 4096 * 3])
def test_compaction_long_lists(N):
    """Candidate lists of 64 Ki and more are compacted by many waves per
    query (segments of 4096 candidates): rows equal the oracle's for both
    distances and both survivor orders, also when the threshold is still
    +inf at compaction (one seed candidate for k = 10: every candidate
    survives), with lists whose length is not a multiple of 4 (unaligned
    rows of the bound matrix) or of the segment length."""
    print(f"[case] long-list compaction N={N}", flush=True)
    import torch
    db, dbo = ragged_walks(960, N, (16, 16), 2)
    qs, qo = ragged_walks(961, 5, (16, 16), 2)
    idx = _index(db, dbo)
    dq = to_dev(qs)
    # a given candidate order per query (the unsorted compaction gathers
    # the bounds through it)
    rng = np.random.default_rng(962)
    perm = torch.from_numpy(np.stack([rng.permutation(N) for _ in range(5)]).astype(np.int32)).cuda()
    for distance, band in (("dk", None), ("dtw", 3)):
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, distance, band)
        for kw in ({}, {"seed_count": 1}, {"surv_order": 1}, {"surv_order": 2},
                   {"dtw_cascade": 3}, {"bound_seed": 2, "dtw_cascade": 2},
                   {"order": perm}, {"order": perm, "surv_order": 2, "seed_count": 1}):
            ids, dst, st = idx.knn(dq, qo, 10, distance, band, stats=True, **kw)
            assert_same_knn(ids, dst, ref_ids, ref_keys, distance)
            assert st["bound_pruned"] + st["dp_started"] == st["pairs"], (kw, st)
    idx.close()


@pytest.mark.parametrize("prefix", [-1, 64, 128, 256])
def test_lb_prefix_give_up(prefix):
    """The corner survivors' LB_Box may stop after a prefix of the candidate
    and keep the partial sum (a lower bound too): rows equal the oracle's
    whatever the prefix, on class-warp series (LB_Box prunes the other
    classes) and random walks, and each pair is counted once."""
    print(f"[case] lb_prefix={prefix}", flush=True)
    cw = classwarp(2, 10, 300, 3, 2000, 6)
    rw_db, rw_dbo = ragged_walks(970, 700, (300, 300), 4)
    rw_qs, rw_qo = ragged_walks(971, 4, (300, 300), 4)
    for db, dbo, qs, qo in (cw, (rw_db, rw_dbo, rw_qs, rw_qo)):
        idx = _index(db, dbo)
        for band in (0.1, 4):
            ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, "dtw", band)
            ids, dst, st = idx.knn(to_dev(qs), qo, 10, "dtw", band, stats=True,
                                   lb_prefix=prefix, dtw_cascade=1)
            assert_same_knn(ids, dst, ref_ids, ref_keys, "dtw")
            assert st["bound_pruned"] + st["dp_started"] == st["pairs"], st
        idx.close()
