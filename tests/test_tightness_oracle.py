"""Thm. 3.3 (curse of dimensionality of LB_Box) on the oracle: with i.i.d.
series points (the theorem's assumption) and a Sakoe-Chiba band of a fixed
fraction of the length, the tightness E[LB_Box] / E[DTW] falls as the
dimension grows and as the length grows (towards 0).  Seeded, so the check
is deterministic; the margins between neighbouring grid points are wide."""
import numpy as np

import oracle as O


def _tightness(rng, d, n, reps=40, frac=0.1):
    w = int(frac * n)
    lb = dtw = 0.0
    for _ in range(reps):
        S = rng.normal(size=(n, d)).astype(np.float32)
        T = rng.normal(size=(n, d)).astype(np.float32)
        lb += O.lb_box_f64(S, T, w)
        dtw += O.dtw_f64(S, T, w)
    return lb / dtw


def test_tightness_falls_with_dimension_and_length():
    rng = np.random.default_rng(33)
    dims, lens = (1, 3, 9, 27), (16, 64, 256)
    t = np.array([[_tightness(rng, d, n) for n in lens] for d in dims])
    print(t)
    assert np.all(t > 0) and np.all(t < 1)
    assert np.all(np.diff(t, axis=0) < 0), "falls with the dimension at every length"
    assert np.all(np.diff(t, axis=1) < 0), "falls with the length at every dimension"
    assert t[-1, -1] < 0.05 * t[0, 0]
