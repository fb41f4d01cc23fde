"""GPU parity of the learned-ordering encoder (through the C-ABI) against the
fp64 oracle at the same bfloat16 rounding points, and what the trained
encoder gains: exact k-NN results unchanged, fewer DPs."""
import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from gpu_cases import assert_same_knn, classwarp, ragged_walks, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _split(flat, d_in, h, e):
    out, o = [], 0
    for s in M.param_shapes(d_in, h, e):
        n = int(np.prod(s))
        out.append(flat[o:o + n].astype(np.float64).reshape(s))
        o += n
    return out


def _test_params(d, seed, hidden=256, embed=64):
    """Flat float32 parameters drawn by the test (seeded numpy): weights
    U(+-sqrt(6 / fan_in)), biases U(+-0.1) so that every block is exercised."""
    r = np.random.default_rng([seed, d, hidden, embed])
    blocks = []
    for s in M.param_shapes(32 * d, hidden, embed):
        lim = np.sqrt(6.0 / s[1]) if len(s) == 2 else 0.1
        blocks.append(r.uniform(-lim, lim, int(np.prod(s))))
    return np.concatenate(blocks).astype(np.float32)


def _model(d, seed, hidden=256, embed=64):
    from paper_1811_11076_amd import Model
    m = Model(d, hidden=hidden, embed=embed, seed=seed)
    p = _test_params(d, seed, hidden, embed)
    m.set_params(p)
    return m, _split(p, 32 * d, hidden, embed)


@pytest.mark.parametrize("d,lens", [(3, (256, 256)), (3, (20, 700)), (6, (40, 90)), (1, (5, 50))])
def test_embed_matches_oracle(d, lens):
    print(f"[case] embed d={d} lens={lens}", flush=True)
    vals, off = ragged_walks(300 + d, 150, lens, d)
    m, params = _model(d, 11 + d)
    got = m.embed_series(to_dev(vals), off).cpu().numpy().astype(np.float64)
    ref, _ = M.forward(params, M.resample(vals, off), rounding=True)
    assert got.shape == ref.shape
    # element-wise: the GPU rounds its fp32 layer inputs to bfloat16 where
    # the oracle rounds fp64 ones; an input whose two values fall on
    # opposite sides of a rounding midpoint moves by one bfloat16 step
    # (2^-8 of itself), so every embedding entry stays within 2^-8 of its
    # row's largest entry (measured: at most 1.1e-3 of it, d = 6)
    err = np.abs(got - ref)
    bound = 2.0 ** -8 * np.abs(ref).max(axis=1, keepdims=True)
    assert np.all(err <= bound), (err / bound).max()
    m.close()


@pytest.mark.parametrize("n_pairs", [1, 37, 300, 1024])
def test_batch_grad_matches_oracle(n_pairs):
    print(f"[case] batch grad n_pairs={n_pairs}", flush=True)
    d = 3
    vals, off = ragged_walks(77, 120, (30, 300), d)
    m, params = _model(d, 5)
    r = np.random.default_rng(n_pairs)
    a = r.integers(0, 120, n_pairs).astype(np.int32)
    b = r.integers(0, 120, n_pairs).astype(np.int32)
    y = r.uniform(0.5, 20.0, n_pairs).astype(np.float32)
    loss, grad = m.batch_grad(to_dev(vals), off, a, b, y)
    X = M.resample(vals, off)
    ref_loss, ref_grads = M.batch_grads(params, X[a], X[b], y.astype(np.float64), rounding=True)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss, (loss, ref_loss)
    got = _split(grad, 32 * d, 256, 64)
    for i, (g, rg) in enumerate(zip(got, ref_grads)):
        if i == 5:
            # the output bias cancels in e_a - e_b: zero up to rounding
            assert np.abs(g).max() <= 1e-4 * max(np.abs(got[4]).max(), 1e-30)
            continue
        # element-wise within 2^-10 of the block's largest entry: a bfloat16
        # rounding flip (2^-8 of one operand) reaches a gradient entry through
        # a sum of many terms (measured: at most 1.2e-4 of the block maximum
        # at 300 pairs, 1e-7 at one pair)
        err = np.abs(g - rg)
        bound = 2.0 ** -10 * np.abs(rg).max()
        assert np.all(err <= bound), (i, err.max() / np.abs(rg).max())
    m.close()


def test_train_lowers_loss_and_save_load(tmp_path):
    print("[case] train + save/load", flush=True)
    from paper_1811_11076_amd import Model
    d = 3
    vals, off = ragged_walks(91, 200, (64, 128), d)
    r = np.random.default_rng(3)
    a = r.integers(0, 200, 4000).astype(np.int32)
    b = r.integers(0, 200, 4000).astype(np.int32)
    # a learnable target: the distance between series means
    mu = np.stack([vals[off[i]:off[i + 1]].mean(0) for i in range(200)])
    y = np.linalg.norm(mu[a] - mu[b], axis=1).astype(np.float32)
    m = Model(d, seed=1)
    losses = m.train(to_dev(vals), off, a, b, y, epochs=8, batch=256, lr=1e-3, seed=9)
    print("  losses", losses, flush=True)
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    path = str(tmp_path / "enc.bin")
    m.save(path)
    m2 = Model.load(path)
    assert np.array_equal(m2.get_params(), m.get_params())
    e1 = m.embed_series(to_dev(vals), off).cpu().numpy()
    e2 = m2.embed_series(to_dev(vals), off).cpu().numpy()
    assert np.array_equal(e1, e2)
    m.close()
    m2.close()


def test_learned_order_exact_and_gain():
    """The class-warp workload at reduced size (10 classes, L = 256, d = 3):
    an encoder trained on DK distances from the train stream orders each
    query's candidates; the k-NN rows equal the oracle's and the plain
    scan's, and fewer DPs run to completion than with the plain order.  The
    threshold seeded by Alg. 1 over every candidate (the paper's first
    pass) gives the same rows in either order.  An
    untrained (random-weight) encoder is reported beside it: random ReLU
    features already preserve much of the resampled series' geometry on
    this data, so no margin over it is asserted."""
    print("[case] learned order gain", flush=True)
    import torch
    from paper_1811_11076_amd import Index, Model, synth
    from paper_1811_11076_amd.learned import dk_training_set
    gen = synth.ClassWarp(2, 10, 256, 3)
    tv, to, ta, tb, ty = dk_training_set(gen, 1000, 200, 100, 256, seed=1)
    assert ta.size == 200 * 200
    trained = Model(3, seed=4)
    losses = trained.train(to_dev(tv), to, ta, tb, ty, epochs=15, batch=1024, lr=1e-3, seed=2)
    print("  losses", losses[0], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]
    untrained = Model(3, seed=4)
    db, dbo, qs, qo = classwarp(2, 10, 256, 3, 3000, 24)
    idx = Index(to_dev(db), dbo)
    ref_ids, ref_keys, _ = O.knn_scan(db, dbo, qs, qo, 10, "dk", None)
    res = {}
    full = dict(seed_count=len(dbo) - 1)   # Alg. 1 over every candidate
    # "plain": the first candidates of the plain order seed the threshold;
    # "plain_bound_seed": the library default for the plain order, the
    # candidates of smallest corner bound
    for name, kw in (("plain", dict(bound_seed=2)), ("plain_bound_seed", {}),
                     ("untrained", dict(order="learned", model=untrained)),
                     ("trained", dict(order="learned", model=trained)),
                     ("plain_full_seed", dict(bound_seed=2, **full)),
                     ("trained_full_seed", dict(order="learned", model=trained, **full))):
        ids, dst, st = idx.knn(to_dev(qs), qo, 10, "dk", None, stats=True, **kw)
        assert_same_knn(ids, dst, ref_ids, ref_keys, "dk")
        res[name] = st
        print(f"  {name}: started {st['dp_started']} completed {st['dp_completed']} "
              f"cells {st['dp_valid_cells']} ms_order {st['ms_order']:.3f}", flush=True)
    # the corner bound leaves the same survivors whatever the order; the
    # order decides how early the threshold falls while they are evaluated:
    # DPs run to completion and cells evaluated drop against the plain order
    assert res["trained"]["dp_completed"] < 0.7 * res["plain"]["dp_completed"]
    assert res["trained"]["dp_valid_cells"] < res["plain"]["dp_valid_cells"]
    idx.close()
    trained.close()
    untrained.close()


def test_adam_steps_match_oracle():
    """Two training steps (forward, backward, Adam) on one batch, from
    parameters the test draws, against the oracle's gradient and Adam step
    (oracle.mlp.adam_step) in fp64.  At step 1 Adam moves every parameter
    by lr * g / (|g| + eps), i.e. by lr in the gradient's sign wherever
    |g| >> eps, so the two sides agree to fp32 rounding wherever the
    gradient's sign is certain; at step 2 the move depends on the ratio of
    the two steps' gradients (bounded through the gradients' own error).
    Elements whose gradient is within rounding noise of zero (the output
    bias, which cancels in e_a - e_b) are checked only for the bound every
    Adam move obeys at step 1: |move| <= lr."""
    print("[case] adam steps", flush=True)
    d, hidden, embed, lr = 3, 64, 32, 1e-3
    vals, off = ragged_walks(131, 60, (30, 200), d)
    m, params = _model(d, 41, hidden, embed)
    r = np.random.default_rng(7)
    n = 96
    a = r.integers(0, 60, n).astype(np.int32)
    b = (a + 1 + r.integers(0, 59, n).astype(np.int32)) % 60
    y = r.uniform(0.5, 20.0, n).astype(np.float32)
    X = M.resample(vals, off)
    dv = to_dev(vals)
    ref = [p.copy() for p in params]
    mom = [np.zeros_like(p) for p in params]
    vel = [np.zeros_like(p) for p in params]
    prev = np.concatenate([p.ravel() for p in params])
    for t in (1, 2):
        _, g_ref = M.batch_grads(ref, X[a], X[b], y.astype(np.float64), rounding=True)
        ref, mom, vel = M.adam_step(ref, g_ref, mom, vel, t, lr=lr)
        m.train(dv, off, a, b, y, epochs=1, batch=n, lr=lr, seed=t)
        got = m.get_params().astype(np.float64)
        want = np.concatenate([p.ravel() for p in ref])
        g = np.concatenate([x.ravel() for x in g_ref])
        scale = np.concatenate([np.full(x.size, np.abs(x).max()) for x in g_ref])
        # sign certain, and |g| >> eps so that eps moves the step by < 1e-4 of it
        sure = (np.abs(g) >= 1e-2 * scale) & (np.abs(g) >= 1e-4)
        sure[-embed:] = False  # the output bias: zero gradient up to rounding
        err = np.abs(got - want)
        # fp32 storage of the result (half an ulp) + the move's own error:
        # fp32 rounding at step 1, the gradients' relative error (< 1e-2 on
        # the sure elements) carried through m / sqrt(v) at step 2
        tol = np.abs(want) * 2.0 ** -23 + (1e-8 if t == 1 else 4e-2 * lr)
        bad = np.nonzero(sure & (err > tol))[0]
        print(f"  step {t}: {sure.sum()} sure elements, max err {err[sure].max():.3e}, "
              f"{bad.size} outside", flush=True)
        assert bad.size == 0, (t, bad[:10], got[bad[:10]], want[bad[:10]])
        if t == 1:
            assert np.all(np.abs(got - prev) <= lr * (1 + 1e-6) + np.abs(prev) * 2.0 ** -23)
        prev = got
    m.close()


def test_dk_distances_correctly_rounded():
    """tsk_dk_distances: the correctly rounded fp32 square root (numpy's
    float32 sqrt is IEEE, correctly rounded) of every key, in place and
    out of place; 0 and +inf map to themselves."""
    import ctypes
    import torch
    from paper_1811_11076_amd import _lib
    lib = _lib.load()
    r = np.random.default_rng(5)
    keys = np.concatenate([
        r.uniform(0, 1e4, 200_000), np.exp(r.uniform(-80, 80, 50_000)),
        [0.0, np.inf, 1.0, 4.0, 2.0, 3.4e38]]).astype(np.float32)
    dk = torch.from_numpy(keys).cuda()
    out = torch.empty_like(dk)
    _lib.check(lib.tsk_dk_distances(ctypes.c_void_p(dk.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    keys.size, None))
    want = np.sqrt(keys)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want.view(np.uint32))
    _lib.check(lib.tsk_dk_distances(ctypes.c_void_p(dk.data_ptr()), ctypes.c_void_p(dk.data_ptr()),
                                    keys.size, None))
    assert np.array_equal(dk.cpu().numpy().view(np.uint32), want.view(np.uint32))


def test_learned_order_graph_replays():
    """The learned candidate order inside a captured graph: the embedding,
    scoring and ordering kernels run in the graph, the candidates'
    embeddings are recomputed outside it when the encoder changes; rows
    equal the oracle's on every replay, also after more training and over
    several query chunks."""
    print("[case] learned order graph", flush=True)
    import torch
    from paper_1811_11076_amd import Index, Model
    db, dbo, qs, qo = classwarp(2, 10, 128, 3, 2000, 12)
    dq = to_dev(qs)
    ref_ids, ref_keys = O.knn_brute(db, dbo, qs, qo, 10, "dk", None)
    m, _ = _model(3, 8)
    vals, off = ragged_walks(95, 100, (64, 128), 3)
    r = np.random.default_rng(1)
    a = r.integers(0, 100, 500).astype(np.int32)
    b = r.integers(0, 100, 500).astype(np.int32)
    y = r.uniform(1.0, 10.0, 500).astype(np.float32)
    for ws in (0, 2000 * 24 * 4 + 128 * 64 * 4):   # one chunk; three chunks
        idx = Index(to_dev(db), dbo, workspace_limit_bytes=ws)
        out = (torch.empty((12, 10), dtype=torch.int64, device="cuda"),
               torch.empty((12, 10), dtype=torch.float32, device="cuda"))
        for rep in range(3):
            idx.knn(dq, qo, 10, "dk", None, order="learned", model=m, use_graph=True, out=out)
            torch.cuda.synchronize()
            assert_same_knn(out[0], out[1], ref_ids, ref_keys, "dk")
            if rep == 1:
                m.train(to_dev(vals), off, a, b, y, epochs=1, batch=100, lr=1e-3, seed=rep)
            idx.knn(dq[:int(qo[2])], qo[:3], 10, "dtw", 0.1)
            torch.cuda.synchronize()
        idx.close()
    m.close()
