"""One GPU standing in for a sharded database: the series split into S
contiguous shards, one index per shard queried in turn (ids offset by the
shard's first series) for its ranking keys (DK: squared), the per-shard
top-k merged on the host by (key, id).  The merged rows equal the unsharded
index's and the oracle's plain definition bit for bit: the merge is the
only step a run over several GPUs would add to the single-GPU path."""
import numpy as np
import pytest

import oracle as O
from gpu_cases import classwarp, ragged_walks, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _merge(parts, k):
    """Per query, the k smallest (key, id) over the shards' rows."""
    ids = np.concatenate([p[0] for p in parts], axis=1)
    keys = np.concatenate([p[1] for p in parts], axis=1)
    out_i = np.full((ids.shape[0], k), -1, np.int64)
    out_k = np.full((ids.shape[0], k), np.inf, np.float32)
    for q in range(ids.shape[0]):
        cand = sorted((float(keys[q, t]), int(ids[q, t])) for t in range(ids.shape[1])
                      if ids[q, t] >= 0)[:k]
        for r, (kk, ii) in enumerate(cand):
            out_i[q, r], out_k[q, r] = ii, kk
    return out_i, out_k


def _check_keys(mi, mk, ref_ids, ref_keys):
    """Merged (id, key) rows equal the oracle's bit for bit."""
    assert np.array_equal(mi, ref_ids), (mi, ref_ids)
    assert np.array_equal(mk.view(np.uint32), ref_keys.astype(np.float32).view(np.uint32))


def _check(ids, dist, ref_ids, ref_keys, dist_name):
    """Rows of one call: ids exact, distances bit-exact (DK: the correctly
    rounded sqrt of the oracle's squared key)."""
    exp = np.sqrt(ref_keys.astype(np.float32)) if dist_name == "dk" else ref_keys.astype(np.float32)
    assert np.array_equal(ids, ref_ids), (ids, ref_ids)
    assert np.array_equal(dist.view(np.uint32), exp.view(np.uint32)), (dist, exp)


def _run_shards(db, dbo, qs, qo, k, dist, band, shards):
    from paper_1811_11076_amd import Index
    n = len(dbo) - 1
    cuts = np.linspace(0, n, shards + 1).astype(int)
    dq = to_dev(qs)
    parts = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        sdo = (dbo[a:b + 1] - dbo[a]).astype(np.int64)
        idx = Index(to_dev(db[dbo[a]:dbo[b]]), sdo)
        ids, key, _ = idx.knn(dq, qo, k, dist, band, raw_keys=True)
        ids = ids.cpu().numpy()
        parts.append((np.where(ids >= 0, ids + a, -1), key.cpu().numpy()))
        idx.close()
    return _merge(parts, k)


@pytest.mark.parametrize("shards", [2, 3, 7])
@pytest.mark.parametrize("dist,band", [("dtw", 0.1), ("dk", None)])
def test_equal_length_shards(shards, dist, band):
    print(f"[case] shards={shards} {dist} equal lengths", flush=True)
    db, dbo, qs, qo = classwarp(2, 10, 128, 3, 1400, 6)
    ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, dist, band)
    mi, mk = _run_shards(db, dbo, qs, qo, 10, dist, band, shards)
    _check_keys(mi, mk, ref_ids, ref_keys)
    from paper_1811_11076_amd import Index
    idx = Index(to_dev(db), dbo)
    ids, d, _ = idx.knn(to_dev(qs), qo, 10, dist, band)
    idx.close()
    _check(ids.cpu().numpy(), d.cpu().numpy(), ref_ids, ref_keys, dist)


@pytest.mark.parametrize("dist,band", [("dtw", 0.1), ("dk", None), ("dtw", None)])
def test_uneven_shards_and_padding(dist, band):
    """Uneven lengths, a shard smaller than k (its padding must not leak
    into the merge), k = 12."""
    print(f"[case] shards uneven {dist} band={band}", flush=True)
    db, dbo = ragged_walks(71, 205, (20, 160), 3)
    qs, qo = ragged_walks(171, 5, (20, 160), 3)
    ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 12, dist, band)
    # shards of 102, 102 and 1 series: the last holds fewer than k
    from paper_1811_11076_amd import Index
    dq = to_dev(qs)
    parts = []
    for a, b in ((0, 102), (102, 204), (204, 205)):
        sdo = (dbo[a:b + 1] - dbo[a]).astype(np.int64)
        idx = Index(to_dev(db[dbo[a]:dbo[b]]), sdo)
        ids, key, _ = idx.knn(dq, qo, 12, dist, band, raw_keys=True)
        ids = ids.cpu().numpy()
        if b - a < 12:
            assert (ids[:, b - a:] == -1).all() and np.isinf(key.cpu().numpy()[:, b - a:]).all()
        parts.append((np.where(ids >= 0, ids + a, -1), key.cpu().numpy()))
        idx.close()
    mi, mk = _merge(parts, 12)
    _check_keys(mi, mk, ref_ids, ref_keys)
