"""Pins of the MLP oracle (CPU only): finite differences, library routines, closed forms."""
import math

import numpy as np
import pytest

from oracle import mlp


def small_params(rng, layers=(10, 12, 9, 6)):
    ps = []
    for fi, fo in zip(layers[:-1], layers[1:]):
        ps.append((rng.normal(0, 0.7, (fo, fi)), rng.normal(0, 0.3, fo)))
    return ps


def test_gelu_is_x_times_normal_cdf():
    from scipy.stats import norm
    x = np.linspace(-6, 6, 1001)
    np.testing.assert_allclose(mlp.gelu(x), x * norm.cdf(x), rtol=1e-13, atol=1e-15)
    assert mlp.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-14)


@pytest.mark.parametrize("f,g", [(mlp.gelu, mlp.gelu_grad), (mlp.gelu_tanh, mlp.gelu_tanh_grad)])
def test_gelu_derivatives_by_finite_differences(f, g):
    x = np.linspace(-5, 5, 401)
    d = 1e-6
    np.testing.assert_allclose(g(x), (f(x + d) - f(x - d)) / (2 * d), rtol=1e-7, atol=1e-8)


def test_tanh_form_is_close_to_exact_gelu():
    """The published tanh approximation stays within 1e-3 of x Phi(x)."""
    x = np.linspace(-10, 10, 20001)
    assert np.max(np.abs(mlp.gelu_tanh(x) - mlp.gelu(x))) < 1e-3


def test_bf16_rounding_matches_torch_and_ties_to_even():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 10000), rng.normal(0, 1e6, 1000), [0.0, -0.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert mlp.bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    ps = small_params(rng)
    x = rng.uniform(0, 1, (7, 10))
    t = rng.uniform(-1, 1, (7, 6))
    y, cache = mlp.forward(ps, x)
    grads = mlp.backward(ps, cache, y, t)
    d = 1e-7
    for l, (W, b) in enumerate(ps):
        for (i, j) in [(0, 0), (W.shape[0] - 1, W.shape[1] - 1), (1, 2)]:
            Wp = W.copy(); Wp[i, j] += d
            Wm = W.copy(); Wm[i, j] -= d
            lp = mlp.l1_loss(mlp.forward([*ps[:l], (Wp, b), *ps[l + 1:]], x)[0], t)
            lm = mlp.l1_loss(mlp.forward([*ps[:l], (Wm, b), *ps[l + 1:]], x)[0], t)
            assert grads[l][0][i, j] == pytest.approx((lp - lm) / (2 * d), rel=1e-5, abs=1e-10)
        bp = b.copy(); bp[0] += d
        bm = b.copy(); bm[0] -= d
        lp = mlp.l1_loss(mlp.forward([*ps[:l], (W, bp), *ps[l + 1:]], x)[0], t)
        lm = mlp.l1_loss(mlp.forward([*ps[:l], (W, bm), *ps[l + 1:]], x)[0], t)
        assert grads[l][1][0] == pytest.approx((lp - lm) / (2 * d), rel=1e-5, abs=1e-10)


def test_bf16_forward_tracks_float64_forward():
    rng = np.random.default_rng(2)
    ps = mlp.init_params(rng)
    x = rng.uniform(0, 1, (256, 10))
    y64, _ = mlp.forward(ps, x)
    y16, _ = mlp.forward_bf16(ps, x)
    assert np.max(np.abs(y16 - y64)) < 0.02 * np.max(np.abs(y64)) + 1e-3


def test_bf16_backward_tracks_float64_backward():
    rng = np.random.default_rng(3)
    ps = mlp.init_params(rng)
    x = rng.uniform(0, 1, (512, 10))
    t = rng.uniform(0, 1, (512, 6))
    y, c = mlp.forward(ps, x)
    g64 = mlp.backward(ps, c, y, t)
    y2, c2 = mlp.forward_bf16(ps, x)
    g16 = mlp.backward_bf16(ps, c2, y2, t)
    for (a, _), (b, _) in zip(g64, g16):
        assert np.linalg.norm(a - b) <= 0.05 * np.linalg.norm(a)


def test_output_transform_round_trip():
    rng = np.random.default_rng(4)
    Y = np.column_stack([rng.uniform(10, 1200, 50), rng.uniform(-9e6, 2e6, 50), rng.uniform(900, 9000, 50),
                         rng.uniform(200, 1500, 50), rng.uniform(1e-5, 2e-4, 50), rng.uniform(0.02, 0.3, 50)])
    X = rng.uniform(0, 1, (50, 10))
    ilo, ihi, olo, ohi = mlp.fit_scalers(X, Y)
    S = mlp.transform_outputs(Y, olo, ohi)
    assert S.min() >= 0 and S.max() <= 1 + 1e-15
    np.testing.assert_allclose(mlp.untransform_outputs(S, olo, ohi), Y, rtol=1e-12)
    assert np.all(mlp.scale_inputs(X, ilo, ihi) >= 0)


# ------------------------------------------------------------------ training: optimizer, schedule, sample order

def test_constant_target_scales_to_zero_and_maps_back():
    """A target constant over the training data (empty range) scales to 0, as a constant
    input feature does, and 0 maps back to that constant; the other targets are unaffected."""
    rng = np.random.default_rng(3)
    Y = np.exp(rng.uniform(-1.0, 1.0, (5, 6)))
    Y[:, 2] = 4.25
    flags = mlp.log_flags(0x35)
    lo, hi = mlp.fit_scalers(np.zeros((5, 10)), Y, flags)[2:]
    assert lo[2] == hi[2]
    S = mlp.transform_outputs(Y, lo, hi, flags)
    assert np.all(np.isfinite(S)) and np.all(S[:, 2] == 0.0)
    assert np.allclose(mlp.untransform_outputs(S, lo, hi, flags), Y, rtol=1e-14, atol=0)


def test_splitmix64_reproduces_the_published_outputs():
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "textbook_values.json")))
    state, got = 0, []
    for _ in range(3):
        state, out = mlp.splitmix64(state)
        got.append(f"{out:016x}")
    assert got == gold["splitmix64_seed0"]["outputs_hex"]


@pytest.mark.parametrize("n", [1, 2, 7, 256, 4096, 65536, 95536, 1_000_003])
def test_epoch_permutation_is_a_bijection(n):
    for seed, epoch in ((0, 0), (3, 1), (12345, 17)):
        p = mlp.epoch_permutation(seed, epoch, n)
        assert p.shape == (n,) and p.min() >= 0 and p.max() < n
        assert np.unique(p).size == n


def test_epoch_permutations_differ_between_epochs_and_seeds():
    n = 65536 + 30000
    a, b, c = (mlp.epoch_permutation(s, e, n) for s, e in ((3, 0), (3, 1), (4, 0)))
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    # the first batch of 65536 samples is a different subset in each
    assert np.setdiff1d(a[:65536], b[:65536]).size > 1000


def test_cosine_schedule_closed_forms():
    lr, lo, E = 1e-3, 1e-5, 12
    assert mlp.cosine_lr(lr, lo, 0, E) == lr
    assert mlp.cosine_lr(lr, lo, E // 2, E) == pytest.approx(0.5 * (lr + lo), rel=1e-15)
    assert mlp.cosine_lr(lr, lo, E // 3, E) == pytest.approx(lo + 0.75 * (lr - lo), rel=1e-14)   # cos(pi/3) = 1/2
    assert mlp.cosine_lr(lr, lo, E, E) == pytest.approx(lo, rel=1e-14)
    assert mlp.cosine_lr(lr, lo, 3 * E, E) == pytest.approx(lo, rel=1e-14)   # capped
    seq = [mlp.cosine_lr(lr, lo, e, E) for e in range(E + 1)]
    assert all(x > y for x, y in zip(seq, seq[1:]))


def test_adam_first_step_and_constant_gradient():
    """With bias correction, m_hat = g and v_hat = g^2 whenever every gradient so far is the
    same g, so each step moves w by lr g / (|g| + eps): about lr, whatever the gradient's
    scale.  (Without the correction the first step would be 0.1 / sqrt(0.001) = 3.16 lr.)"""
    g = np.array([3.0, -2e-4, 1e-12, 0.0, -7.5e3])
    w, m, v = np.zeros(5), np.zeros(5), np.zeros(5)
    for t in range(1, 6):
        w_new, m, v = mlp.adam_step(w, g, m, v, t, lr=1e-3)
        np.testing.assert_allclose(w - w_new, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        w = w_new


def test_adam_minimises_a_quadratic():
    c = np.array([1.0, 10.0, 0.01])
    w, m, v = np.array([1.0, -2.0, 3.0]), np.zeros(3), np.zeros(3)
    for t in range(1, 4001):
        w, m, v = mlp.adam_step(w, c * w, m, v, t, lr=1e-2)
    assert np.all(np.abs(w) < 0.05)


def test_full_batch_step_does_not_depend_on_the_sample_order():
    """With one batch per epoch the gradient is a sum over the same samples whatever their
    order: the trained parameters agree to rounding for two different seeds."""
    rng = np.random.default_rng(5)
    n = 512
    X = np.column_stack([rng.uniform(0, 1, (n, 2)), rng.dirichlet(np.ones(8), n)])
    Y = np.column_stack([np.exp(X[:, 0]), X[:, 1] - X[:, 2], 1 + X[:, 3], 3 * X[:, 4], np.exp(-X[:, 5]), 0.1 + X[:, 6]])
    box = mlp.fit_scalers(X, Y)
    ps = mlp.init_params(np.random.default_rng(6))
    a = mlp.train_bf16(ps, X, Y, box, mlp.LOG_OUTPUTS, 2, n, 1e-3, 1e-4, 2, seed=1)
    b = mlp.train_bf16(ps, X, Y, box, mlp.LOG_OUTPUTS, 2, n, 1e-3, 1e-4, 2, seed=2)
    for (Wa, ba), (Wb, bb) in zip(a[0], b[0]):
        np.testing.assert_allclose(Wa, Wb, rtol=0, atol=1e-12)
        np.testing.assert_allclose(ba, bb, rtol=0, atol=1e-12)
    assert a[2][1] < a[2][0]


def test_training_lowers_the_l1_loss():
    rng = np.random.default_rng(7)
    n = 2048
    X = np.column_stack([rng.uniform(0, 1, (n, 2)), rng.dirichlet(np.ones(8), n)])
    Y = np.column_stack([np.exp(X[:, 0]), X[:, 1] - X[:, 2], 1 + X[:, 3], 3 * X[:, 4], np.exp(-X[:, 5]), 0.1 + X[:, 6]])
    box = mlp.fit_scalers(X, Y)
    ps = mlp.init_params(np.random.default_rng(8))
    _, state, losses, recs = mlp.train_bf16(ps, X, Y, box, mlp.LOG_OUTPUTS, 6, 512, 2e-3, 1e-4, 6, seed=3)
    assert state["step"] == 24 and state["epoch"] == 6 and len(recs) == 24
    assert losses[-1] < 0.5 * losses[0]
