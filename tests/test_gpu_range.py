"""GPU parity of the range query (through the C-ABI) against the oracle's
plain definition: every series within the radius, ids ascending, distances
bit-exact."""
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


def _check(idx, qs, qo, radius, dist, band, ref):
    offs, ids, dst, st = idx.range(to_dev(qs), qo, radius, dist, band, stats=True)
    ids = ids.cpu().numpy()
    dst = dst.cpu().numpy()
    for q, (rid, rd) in enumerate(ref):
        a, b = offs[q], offs[q + 1]
        assert np.array_equal(ids[a:b], rid), (dist, q, ids[a:b], rid)
        assert np.array_equal(dst[a:b].view(np.uint32), rd.astype(np.float32).view(np.uint32))
    return st


CASES = [("ragged", None), ("classwarp", None), ("uneven", None)]


@pytest.mark.parametrize("kind", ["ragged", "classwarp", "uneven"])
def test_range_matches_oracle(kind):
    print(f"[case] range {kind}", flush=True)
    from paper_1811_11076_amd import Index
    if kind == "ragged":
        db, dbo = ragged_walks(61, 300, (5, 60), 3)
        qs, qo = ragged_walks(161, 5, (5, 60), 3)
    elif kind == "classwarp":
        db, dbo, qs, qo = classwarp(2, 10, 256, 3, 1500, 4)
    else:
        db, dbo, qs, qo = classwarp(3, 50, (64, 512), 3, 600, 3, proto_len=512)
    idx = Index(to_dev(db), dbo)
    for dist, band in (("dk", None), ("dtw", 0.1), ("dtw", None)):
        keys = O.pair_keys(db, dbo, qs, qo, dist, band)
        dd = O.dk_distance(keys) if dist == "dk" else keys
        # radii around the 2 % and 10 % quantiles of the finite distances
        fin = dd[np.isfinite(dd)]
        for qt in (0.02, 0.10):
            radius = float(np.quantile(fin, qt))
            ref = O.range_brute(db, dbo, qs, qo, radius, dist, band)
            st = _check(idx, qs, qo, radius, dist, band, ref)
            print(f"  {dist} band={band} r={radius:.3g}: hits {sum(len(r[0]) for r in ref)} "
                  f"pruned {st['bound_pruned']} of {st['pairs']}", flush=True)
    idx.close()


def test_range_edges_and_capacity():
    print("[case] range edges", flush=True)
    import ctypes
    import torch
    from paper_1811_11076_amd import Index, _lib
    db, dbo = ragged_walks(71, 200, (10, 40), 3)
    # query 1 is a copy of series 5: its DK and DTW to it are exactly 0
    qs = np.concatenate([ragged_walks(171, 1, (10, 40), 3)[0], db[dbo[5]:dbo[6]]])
    qo = np.array([0, qs.shape[0] - (dbo[6] - dbo[5]), qs.shape[0]], np.int64)
    idx = Index(to_dev(db), dbo)
    for dist in ("dk", "dtw"):
        # radius 0: exactly the duplicates
        _check(idx, qs, qo, 0.0, dist, None, O.range_brute(db, dbo, qs, qo, 0.0, dist, None))
        # radius +inf: every series
        _check(idx, qs, qo, float("inf"), dist, None,
               O.range_brute(db, dbo, qs, qo, np.inf, dist, None))
    # a capacity below the hit count: offsets filled, INVALID_ARG
    lib = _lib.load()
    offs = np.zeros(3, np.int64)
    out_i = torch.empty(4, dtype=torch.int64, device="cuda")
    out_d = torch.empty(4, dtype=torch.float32, device="cuda")
    dq = to_dev(qs)
    rc = lib.tsk_range_query(idx._h, ctypes.c_void_p(dq.data_ptr()),
                             qo.ctypes.data_as(ctypes.c_void_p), 2, ctypes.c_double(float("inf")),
                             _lib.TSK_DTW, None, None, 4,
                             ctypes.c_void_p(out_i.data_ptr()), ctypes.c_void_p(out_d.data_ptr()),
                             offs.ctypes.data_as(ctypes.c_void_p), None, None)
    assert rc == _lib.TSK_ERR_INVALID_ARG and offs[2] == 400 and offs[1] == 200
    # a negative radius is rejected before any work
    rc = lib.tsk_range_query(idx._h, ctypes.c_void_p(dq.data_ptr()),
                             qo.ctypes.data_as(ctypes.c_void_p), 2, ctypes.c_double(-1.0),
                             _lib.TSK_DK, None, None, 4,
                             ctypes.c_void_p(out_i.data_ptr()), ctypes.c_void_p(out_d.data_ptr()),
                             offs.ctypes.data_as(ctypes.c_void_p), None, None)
    assert rc == _lib.TSK_ERR_INVALID_ARG
    idx.close()
