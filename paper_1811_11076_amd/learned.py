"""Training data for the learned candidate order: DK distances that the scan's
own DP computes on generated pairs.

Pairs are half same-class and half random: every anchor series is paired
with `per_class` pool members of its class and `per_class` pool members
drawn uniformly, and each pair's target is its DK distance from the library's
full DP (tsk_pair_distances).  Series come from a seeded class-warp stream
kept apart from the evaluation data.
"""
from __future__ import annotations

import numpy as np

from . import synth


def dk_training_set(gen: "synth.ClassWarp", n_pool: int, n_anchor: int, per_class: int,
                    length, stream: str = "train", seed: int = 0):
    """Returns (values float32 [sum_len, d], offsets int64 [n+1], a, b, y):
    series 0..n_pool-1 are the pool, n_pool.. the anchors; (a[i], b[i]) index
    that set and y[i] is their DK distance."""
    import torch

    from . import Index
    pv, po, pl = gen.members(n_pool, stream, start=0, length=length)
    av, ao, al = gen.members(n_anchor, stream, start=n_pool, length=length)
    idx = Index(torch.from_numpy(pv).cuda(), po)
    dist = idx.pair_distances(torch.from_numpy(av).cuda(), ao, "dk", None,
                              dk_sqrt=True).cpu().numpy()
    idx.close()
    rng = np.random.default_rng([int(seed), n_pool, n_anchor])
    a, b, y = [], [], []
    for i in range(n_anchor):
        same = np.nonzero(pl == al[i])[0]
        pick_same = rng.choice(same, size=min(per_class, same.size), replace=False)
        pick_any = rng.choice(n_pool, size=per_class, replace=False)
        for j in np.concatenate([pick_same, pick_any]):
            a.append(n_pool + i)
            b.append(int(j))
            y.append(dist[i, j])
    values = np.concatenate([pv, av])
    offsets = np.concatenate([po, po[-1] + ao[1:]])
    return (values, offsets, np.asarray(a, np.int32), np.asarray(b, np.int32),
            np.asarray(y, np.float32))
