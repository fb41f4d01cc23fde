"""The DK box bound (Sec. 3's boxes with the largest box distance in place of
eq. (1)'s sum; a lower bound of the squared DK, Sec. 2.1) through the C-ABI:
the bound of every pair bit-exact against the oracle, never above the
library's own squared DK, and k-NN rows with the bound in the DK cascade
equal to the oracle's plain k-NN definition."""
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


@pytest.mark.parametrize("d", [1, 3, 6, 8, 13])
@pytest.mark.parametrize("band", [None, 0, 3, 0.2], ids=lambda b: f"band{b}")
def test_pair_dk_box(d, band):
    """Equal-length series (L = 70: a partial last chunk of 64 points), and
    queries of that length and of others (shorter, longer, one point)."""
    print(f"[case] pair_dk_box d={d} band={band}", flush=True)
    db, dbo = ragged_walks(300 + d, 40, (70, 70), d)
    qa, qao = ragged_walks(310 + d, 3, (70, 70), d)
    qb, qbo = ragged_walks(320 + d, 3, (1, 130), d)
    qs = np.concatenate([qa, qb, qa[:1]])
    qo = np.concatenate([qao, qao[-1] + qbo[1:], [qao[-1] + qbo[-1] + 1]])
    idx = _index(db, dbo)
    got = idx.pair_dk_box(to_dev(qs), qo, band).cpu().numpy()
    dk = idx.pair_distances(to_dev(qs), qo, "dk", band).cpu().numpy()
    for q in range(len(qo) - 1):
        S = qs[qo[q]:qo[q + 1]]
        for c in range(len(dbo) - 1):
            T = db[dbo[c]:dbo[c + 1]]
            w = O.band_w(band, S.shape[0], T.shape[0])
            ref = np.float32(O.lb_dk_box_qenv_f32(S, T, w))
            assert got[q, c].view(np.uint32) == ref.view(np.uint32), (q, c, got[q, c], ref)
            assert got[q, c] <= dk[q, c]
    idx.close()


def test_pair_dk_box_needs_equal_lengths():
    from paper_1811_11076_amd import TskError
    db, dbo = ragged_walks(330, 10, (20, 40), 3)
    qs, qo = ragged_walks(331, 2, (20, 40), 3)
    idx = _index(db, dbo)
    with pytest.raises(TskError, match="one length"):
        idx.pair_dk_box(to_dev(qs), qo, None)
    idx.close()


@pytest.mark.parametrize("band", [None, 0.1, 4], ids=lambda b: f"band{b}")
def test_knn_dk_box(band):
    """k-NN DK with the box bound over the corner survivors: rows equal the
    oracle's (class-warp and random walks, an exact copy of a query
    planted), each pair counted once, graph replays equal."""
    print(f"[case] knn dk_box band={band}", flush=True)
    import torch
    cw = classwarp(2, 10, 128, 3, 2500, 8)
    rw_db, rw_dbo = ragged_walks(340, 800, (97, 97), 6)
    rw_qs, rw_qo = ragged_walks(341, 5, (97, 97), 6)
    rw_db[rw_dbo[17]:rw_dbo[18]] = rw_qs[rw_qo[1]:rw_qo[2]]
    for db, dbo, qs, qo in (cw, (rw_db, rw_dbo, rw_qs, rw_qo)):
        idx = _index(db, dbo)
        dq = to_dev(qs)
        ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, "dk", band)
        for bs in (0, 1):
            ids, dst, st = idx.knn(dq, qo, 10, "dk", band, stats=True, dk_box=1, bound_seed=bs)
            assert_same_knn(ids, dst, ref_ids, ref_keys, "dk")
            assert st["bound_pruned"] + st["dp_started"] == st["pairs"], st
        _, _, st0 = idx.knn(dq, qo, 10, "dk", band, stats=True)
        print(f"  DPs started: box {st['dp_started']} corner only {st0['dp_started']}", flush=True)
        out = (torch.empty_like(ids), torch.empty_like(dst))
        for _ in range(2):
            idx.knn(dq, qo, 10, "dk", band, use_graph=True, out=out, dk_box=1)
            torch.cuda.synchronize()
            assert_same_knn(out[0], out[1], ref_ids, ref_keys, "dk")
        idx.close()
