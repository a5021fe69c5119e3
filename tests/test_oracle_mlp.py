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
