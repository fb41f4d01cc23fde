"""Shared helpers for the GPU parity tests: seeded inputs and comparisons.

Inputs come from the seeded generators only; expected values come from the
oracle only."""
import numpy as np

from paper_1811_11076_amd import synth


def ragged_walks(seed, n, lens, d):
    """n random walks with lengths uniform in [lens[0], lens[1]]."""
    r = np.random.default_rng(seed)
    L = r.integers(lens[0], lens[1] + 1, size=n)
    off = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    vals = np.empty((int(off[-1]), d), np.float32)
    for i in range(n):
        vals[off[i]:off[i + 1]] = np.cumsum(r.normal(size=(L[i], d)), axis=0)
    return vals, off


def classwarp(cfg_id, n_classes, length, d, n_db, n_q, proto_len=None):
    g = synth.ClassWarp(cfg_id, n_classes, proto_len or (length if isinstance(length, int) else length[1]), d)
    db, dbo, dbl = g.members(n_db, "db", length=length)
    qs, qo, ql = g.members(n_q, "query", length=length, class_mode="uniform")
    return db, dbo, qs, qo


def to_dev(vals):
    import torch
    return torch.from_numpy(np.ascontiguousarray(vals)).cuda()


def assert_same_knn(ids, dist, ref_ids, ref_keys, distance):
    """ids bit-exact; DK distances = fp32 sqrt of the oracle's squared keys,
    DTW distances = the oracle's fp32 keys, both bit-exact."""
    ids = ids.cpu().numpy()
    dist = dist.cpu().numpy()
    assert np.array_equal(ids, ref_ids), (ids, ref_ids)
    exp = np.sqrt(ref_keys.astype(np.float32)) if distance == "dk" else ref_keys.astype(np.float32)
    assert np.array_equal(dist.view(np.uint32), exp.view(np.uint32)), (dist, exp)
