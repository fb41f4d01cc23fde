"""Pins of the learned-ordering oracle (oracle/mlp.py): rounding, resampling,
gradients and the optimiser checked against values fixed by their
definitions, not against the oracle itself."""
import numpy as np
import pytest

from oracle import mlp as M


def _bf16_bits_rne(x32):
    """Independent bfloat16 rounding of float32 values: round the 32-bit
    pattern at bit 16, ties to even, on the integer representation."""
    u = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_known_values():
    one = 1.0
    assert M.bf16_round(one) == 1.0
    # spacing at 1 is 2^-7: the midpoint 1 + 2^-8 ties to the even neighbour 1
    assert M.bf16_round(1 + 2 ** -8) == 1.0
    # 1 + 3 2^-8 lies midway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert M.bf16_round(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    assert M.bf16_round(-(1 + 3 * 2 ** -8)) == -(1 + 2 ** -6)
    assert M.bf16_round(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7
    assert M.bf16_round(0.0) == 0.0
    assert M.bf16_round(1.0 / 3.0) == 0.333984375  # 0x3EAB
    # 8 significant bits: 255 is exact; 257 and 259 are midpoints of spacing 2
    assert M.bf16_round(255.0) == 255.0
    assert M.bf16_round(257.0) == 256.0 and M.bf16_round(259.0) == 260.0


def test_bf16_matches_integer_rounding():
    r = np.random.default_rng(7)
    x = (r.standard_normal(20000) * np.exp(r.uniform(-20, 20, 20000))).astype(np.float32)
    assert np.array_equal(M.bf16_round(x.astype(np.float64)), _bf16_bits_rne(x))


def test_resample_identity_and_closed_forms():
    r = np.random.default_rng(1)
    s = r.standard_normal((32, 3))
    off = np.array([0, 32])
    assert np.array_equal(M.resample(s, off), s.reshape(1, -1))
    # L = 63: t_k = 2k hits sample points exactly
    s63 = r.standard_normal((63, 2))
    assert np.array_equal(M.resample(s63, np.array([0, 63])), s63[::2].reshape(1, -1))
    # L = 1: every point is the single sample
    s1 = np.array([[1.5, -2.0]])
    assert np.array_equal(M.resample(s1, np.array([0, 1])), np.tile(s1, (1, 32)))
    # a linear ramp resamples to the ramp at t_k = k (L - 1) / 31
    L = 100
    ramp = (0.25 + 0.5 * np.arange(L))[:, None]
    got = M.resample(ramp, np.array([0, L]))[0]
    t = np.arange(32) * (L - 1) / 31
    assert np.allclose(got, 0.25 + 0.5 * t, rtol=0, atol=1e-12)


def test_forward_hand_example():
    """Weights and inputs exact in bfloat16; every value by hand."""
    W1 = np.array([[1.0, -1.0], [0.5, 2.0]])
    b1 = np.array([0.0, -1.0])
    W2 = np.array([[1.0, 1.0], [-1.0, 0.25]])
    b2 = np.array([0.5, 0.0])
    W3 = np.array([[2.0, -0.5]])
    b3 = np.array([1.0])
    x = np.array([[3.0, 1.0]])
    # z1 = (3 - 1, 1.5 + 2 - 1) = (2, 2.5); h1 = (2, 2.5)
    # z2 = (2 + 2.5 + 0.5, -2 + 0.625) = (5, -1.375); h2 = (5, 0)
    # e = 2 * 5 - 0.5 * 0 + 1 = 11
    for rounding in (True, False):
        e, _ = M.forward([W1, b1, W2, b2, W3, b3], x, rounding)
        assert e.shape == (1, 1) and e[0, 0] == 11.0


def _tiny(seed, d_in=6, h=8, d_out=5):
    r = np.random.default_rng(seed)
    params = [r.standard_normal(s) * (0.6 if len(s) == 2 else 0.2)
              for s in M.param_shapes(d_in, h, d_out)]
    return params, r


def test_gradients_match_central_differences():
    params, r = _tiny(3)
    n = 7
    xa = r.standard_normal((n, 6))
    xb = r.standard_normal((n, 6))
    y = np.abs(r.standard_normal(n)) * 2
    _, grads = M.batch_grads(params, xa, xb, y, rounding=False)
    h = 1e-6
    for pi, p in enumerate(params):
        num = np.zeros_like(p)
        for idx in np.ndindex(p.shape):
            old = p[idx]
            p[idx] = old + h
            lp, _ = M.batch_grads(params, xa, xb, y, rounding=False)
            p[idx] = old - h
            lm, _ = M.batch_grads(params, xa, xb, y, rounding=False)
            p[idx] = old
            num[idx] = (lp - lm) / (2 * h)
        scale = max(np.abs(num).max(), 1.0)
        assert np.abs(num - grads[pi]).max() <= 1e-6 * scale, (pi, num, grads[pi])
    # the output bias cancels in e_a - e_b: its gradient vanishes
    assert np.abs(grads[5]).max() < 1e-12


def test_pair_loss_value_and_zero_distance():
    ea = np.array([[3.0, 4.0], [1.0, 1.0]])
    eb = np.array([[0.0, 0.0], [1.0, 1.0]])
    y = np.array([4.0, 2.0])
    loss, pred, dea, deb = M.pair_loss(ea, eb, y)
    assert np.array_equal(pred, [5.0, 0.0])
    assert loss == ((5 - 4) ** 2 + (0 - 2) ** 2) / 2
    # d/d ea of (|ea - eb| - y)^2 / n = 2 (pred - y) / n * (ea - eb) / pred
    assert np.allclose(dea[0], 2 * 1 / 2 * np.array([3.0, 4.0]) / 5)
    assert np.array_equal(dea[1], [0.0, 0.0]) and np.array_equal(deb, -dea)


def test_adam_first_steps_closed_form():
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 0.0])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    p1, m1, v1 = M.adam_step(p, g, m, v, 1, lr=0.1)
    # bias-corrected first step: m^ = g, v^ = g^2, so the move is lr g / (|g| + eps)
    assert np.allclose(p1[0], p[0] - 0.1 * g[0] / (np.abs(g[0]) + 1e-8), rtol=0, atol=1e-15)
    # a second step with the same gradient moves by the same amount
    p2, _, _ = M.adam_step(p1, g, m1, v1, 2, lr=0.1)
    assert np.allclose(p2[0] - p1[0], p1[0] - p[0], rtol=0, atol=1e-12)


def test_rounded_network_close_to_smooth_one():
    """bfloat16 rounding perturbs outputs by about 2^-8 relative per layer."""
    params, r = _tiny(5, d_in=96, h=64, d_out=16)
    x = r.standard_normal((20, 96))
    e1, _ = M.forward(params, x, True)
    e0, _ = M.forward(params, x, False)
    rel = np.abs(e1 - e0).max() / np.abs(e0).max()
    assert 0 < rel < 0.05
