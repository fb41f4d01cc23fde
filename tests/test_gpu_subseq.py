"""GPU parity of the subsequence search (C: tsk_subseq_query) against the
oracle's plain definition (SUB DP for every pair, (key, id) sort, match end
and start): ids, end and start columns bit-exact, distances the correctly
rounded sqrt of the oracle's squared keys, bit-exact."""
import numpy as np
import pytest

import oracle as O
from gpu_cases import ragged_walks, to_dev
from paper_1811_11076_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(ser, soff, qs, qoff, k, **kw):
    from paper_1811_11076_amd import subseq_query
    ids, dist, end, start, st = subseq_query(to_dev(ser), soff, to_dev(qs), qoff, k, stats=True, **kw)
    return ids.cpu().numpy(), dist.cpu().numpy(), end.cpu().numpy(), start.cpu().numpy(), st


def _check(got, ref):
    ids, dist, end, start, _ = got
    rids, rkeys, rend, rstart = ref
    assert np.array_equal(ids, rids), (ids, rids)
    exp = np.sqrt(rkeys.astype(np.float32))
    assert np.array_equal(dist.view(np.uint32), exp.view(np.uint32)), (dist, exp)
    assert np.array_equal(end, rend), (end, rend)
    assert np.array_equal(start, rstart), (start, rstart)


@pytest.mark.parametrize("m", [1, 7, 64, 65, 130, 300])
def test_one_long_series(m):
    """Planted warped copies in one long random walk, several query lengths
    (rows per lane 1 .. 8), default chunking."""
    print(f"[case] one long series m={m}", flush=True)
    ser = synth.long_walk(60000, 3, 31)
    soff = np.array([0, len(ser)], np.int64)
    qs, qo, _ = synth.planted_queries(ser, soff, 5, m, 31)
    ref = O.subseq_knn(ser, soff, qs, qo, 1)
    got = _run(ser, soff, qs, qo, 1)
    _check(got, ref)
    print("  stats", {k: got[4][k] for k in ("dp_started", "bound_pruned", "dp_cells")}, flush=True)


@pytest.mark.parametrize("chunk", [1, 64, 100, 5000, 1 << 16])
def test_chunking_and_no_seed(chunk):
    """Matches crossing chunk boundaries: any chunk width gives the same
    rows, with and without the greedy seed."""
    print(f"[case] chunk={chunk}", flush=True)
    ser = synth.long_walk(8000, 2, 32)
    soff = np.array([0, len(ser)], np.int64)
    qs, qo, _ = synth.planted_queries(ser, soff, 3, 90, 32)
    ref = O.subseq_knn(ser, soff, qs, qo, 1)
    for seed in (True, False):
        _check(_run(ser, soff, qs, qo, 1, chunk_cols=chunk, seed=seed), ref)


@pytest.mark.parametrize("d,k", [(1, 1), (3, 5), (6, 10), (8, 64)])
def test_database_of_uneven_series(d, k):
    """k-NN over series of uneven lengths (some shorter than the query),
    k above the number of series included (padding)."""
    print(f"[case] database d={d} k={k}", flush=True)
    ser, soff = ragged_walks(500 + d, 40, (1, 2500), d)
    qs, qo, _ = synth.planted_queries(ser, soff, 4, 48, 33 + d)
    qs2, qo2 = ragged_walks(600 + d, 3, (1, 120), d)  # unrelated queries, uneven lengths
    qs = np.concatenate([qs, qs2])
    qo = np.concatenate([qo, qo[-1] + qo2[1:]])
    ref = O.subseq_knn(ser, soff, qs, qo, k)
    _check(_run(ser, soff, qs, qo, k), ref)
    _check(_run(ser, soff, qs, qo, k, chunk_cols=128), ref)


def test_ties_and_constant_runs():
    """Exact copies planted twice (the first end wins) and constant runs
    (the latest start of equal matches), one-point series and queries."""
    print("[case] ties", flush=True)
    r = np.random.default_rng(3)
    base = np.cumsum(r.normal(size=(3000, 3)), 0).astype(np.float32)
    q = base[500:540].copy()
    ser = base.copy()
    ser[2000:2040] = q                      # second exact copy, later end
    ser[1200:1210] = base[700]              # a constant run
    ser[1210] = base[701]
    series = [ser, base[:1], base[10:11], np.repeat(base[700:701], 50, 0)]
    soff = np.concatenate([[0], np.cumsum([len(x) for x in series])]).astype(np.int64)
    flat = np.concatenate(series)
    queries = [q, base[700:702], base[5:6], base[700:701]]
    qo = np.concatenate([[0], np.cumsum([len(x) for x in queries])]).astype(np.int64)
    qflat = np.concatenate(queries)
    ref = O.subseq_knn(flat, soff, qflat, qo, 4)
    assert ref[1][0, 0] == 0 and ref[2][0, 0] == 539 and ref[3][0, 0] == 500
    _check(_run(flat, soff, qflat, qo, 4), ref)
    _check(_run(flat, soff, qflat, qo, 4, chunk_cols=7), ref)


def test_without_start_pass():
    from paper_1811_11076_amd import subseq_query
    ser = synth.long_walk(5000, 3, 34)
    soff = np.array([0, len(ser)], np.int64)
    qs, qo, _ = synth.planted_queries(ser, soff, 2, 40, 34)
    ids, dist, end, start, st = subseq_query(to_dev(ser), soff, to_dev(qs), qo, 1, start=False)
    assert start is None and st is None
    rids, rkeys, rend, _ = O.subseq_knn(ser, soff, qs, qo, 1)
    assert np.array_equal(ids.cpu().numpy(), rids) and np.array_equal(end.cpu().numpy(), rend)


def test_longest_query_and_long_series():
    """m = 1024 (16 rows per lane) and a series of 2^21 points spanning
    several walk pieces; the oracle runs the full SUB DP."""
    print("[case] m=1024 and n=2^21", flush=True)
    ser = synth.long_walk(1 << 21, 3, 35)
    soff = np.array([0, len(ser)], np.int64)
    qs, qo, org = synth.planted_queries(ser, soff, 2, 1024, 35)
    qs2, qo2, _ = synth.planted_queries(ser, soff, 2, 200, 36)
    ref = O.subseq_knn(ser, soff, qs, qo, 1)
    got = _run(ser, soff, qs, qo, 1)
    _check(got, ref)
    print("  stats", got[4], flush=True)
    ref2 = O.subseq_knn(ser, soff, qs2, qo2, 1)
    _check(_run(ser, soff, qs2, qo2, 1), ref2)
