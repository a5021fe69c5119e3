"""CPU oracle of the MLP surrogate — TEST INFRASTRUCTURE ONLY.

The paper's surrogate (Section 4.1) is a multilayer perceptron with GELU activations,
trained with an L1 loss (Section 4.3) on scaled inputs and outputs, with a Box-Cox
transform of density (Section 4.2).  This module states that network plainly in numpy:

* ``forward`` / ``backward`` in float64: z_l = h_{l-1} W_l^T + b_l, h_l = GELU(z_l) for the
  hidden layers, a linear output layer, and the exact gradient of the mean absolute error.
  GELU is the exact form x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.
* ``forward_bf16`` / ``backward_bf16``: the same network evaluated the way a BF16 matrix
  engine with FP32 accumulation does it: weights, activations and back-propagated
  gradients rounded to bfloat16 (round to nearest even) where a BF16 kernel stores them,
  products summed exactly (float64 here), GELU in the tanh form of Hendrycks & Gimpel
  (2016), 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))).
* Input and output scaling: min-max to [0, 1]; outputs flagged ``log`` are log-transformed
  first (the Box-Cox transform with lambda = 0).

Nothing here is shared with the GPU library.
"""
import math

import numpy as np
from scipy.special import erf

LAYERS = (10, 256, 256, 256, 256, 6)
LOG_OUTPUTS = (True, False, True, False, True, True)   # rho, h, cp, c, mu, lambda
SQ2PI = math.sqrt(2.0 / math.pi)


# ------------------------------------------------------------------ activations
def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def gelu_tanh(x):
    return 0.5 * x * (1.0 + np.tanh(SQ2PI * (x + 0.044715 * x ** 3)))


def gelu_tanh_grad(x):
    u = SQ2PI * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * SQ2PI * (1.0 + 3 * 0.044715 * x * x)


# ------------------------------------------------------------------ bfloat16
def bf16(x):
    """Round float32 values to bfloat16 (nearest even) and return them as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    rnd = ((b >> 16) & 1) + 0x7FFF
    r = ((b + rnd) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


# ------------------------------------------------------------------ scaling
def scale_inputs(X, lo, hi):
    """X: [n, 10] raw (P, T, Y_1..8); min-max to [0, 1] in float64.  A feature with an
    empty range (constant in the training data) carries no information and scales to 0."""
    rng = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    safe = np.where(rng > 0, rng, 1.0)
    return np.where(rng > 0, (X - lo) / safe, 0.0)


def log_flags(mask):
    """Per-output log flags from a bit mask (bit j: output j is log-transformed)."""
    return tuple(bool(mask >> j & 1) for j in range(len(LOG_OUTPUTS)))


def transform_outputs(Y, lo, hi, log_outputs=LOG_OUTPUTS):
    """Raw outputs [n, 6] -> targets in [0, 1] (log first for the flagged outputs)."""
    T = np.array(Y, dtype=np.float64, copy=True)
    for j, lg in enumerate(log_outputs):
        if lg:
            T[:, j] = np.log(T[:, j])
    return (T - lo) / (hi - lo)


def untransform_outputs(S, lo, hi, log_outputs=LOG_OUTPUTS):
    T = lo + S * (hi - lo)
    for j, lg in enumerate(log_outputs):
        if lg:
            T[:, j] = np.exp(T[:, j])
    return T


def fit_scalers(X, Y, log_outputs=LOG_OUTPUTS):
    """Min-max box of the inputs and of the (log-)transformed outputs."""
    T = np.array(Y, dtype=np.float64, copy=True)
    for j, lg in enumerate(log_outputs):
        if lg:
            T[:, j] = np.log(T[:, j])
    return X.min(0), X.max(0), T.min(0), T.max(0)


# ------------------------------------------------------------------ float64 network
def forward(params, xs):
    """params: list of (W [out, in], b [out]); xs: scaled inputs [n, 10]."""
    h = np.asarray(xs, dtype=np.float64)
    cache = [h]
    for l, (W, b) in enumerate(params):
        z = h @ W.T + b
        if l < len(params) - 1:
            cache.append(z)
            h = gelu(z)
            cache.append(h)
        else:
            cache.append(z)
    return z, cache


def l1_loss(y, t):
    return float(np.mean(np.abs(y - t)))


def backward(params, cache, y, t):
    """Gradient of mean |y - t| over all n x 6 entries (subgradient 0 at 0)."""
    n = y.shape[0]
    dz = np.sign(y - t) / (n * y.shape[1])
    grads = [None] * len(params)
    L = len(params)
    for l in range(L - 1, -1, -1):
        h_prev = cache[2 * l]
        W, _ = params[l]
        grads[l] = (dz.T @ h_prev, dz.sum(0))
        if l > 0:
            dh = dz @ W
            z_prev = cache[2 * l - 1]
            dz = dh * gelu_grad(z_prev)
    return grads


# ------------------------------------------------------------------ bf16-emulating network
def forward_bf16(params, xs):
    """BF16 weights/activations, exact products, tanh-form GELU; returns the float32-rounded
    output layer and the cache of pre-activations (float64) and bf16 activations."""
    h = bf16(np.asarray(xs, dtype=np.float32))
    cache = [h]
    L = len(params)
    for l, (W, b) in enumerate(params):
        z = h @ bf16(W).T + np.asarray(b, dtype=np.float32).astype(np.float64)
        z = z.astype(np.float32).astype(np.float64)
        cache.append(z)
        if l < L - 1:
            h = bf16(gelu_tanh(z))
            cache.append(h)
    return z, cache


def backward_bf16(params, cache, y, t, n_total=None):
    """Gradients with the back-propagated signal rounded to bf16 where a BF16 GEMM
    consumes it; products exact, sums in float64."""
    n = y.shape[0] if n_total is None else n_total
    dz = bf16(np.sign(y - t) / (n * y.shape[1]))
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        h_prev = cache[2 * l]
        W, _ = params[l]
        grads[l] = (dz.T @ h_prev, dz.sum(0))
        if l > 0:
            dh = dz @ bf16(W)
            z_prev = cache[2 * l - 1]
            dz = bf16(dh * gelu_tanh_grad(z_prev))
    return grads


def init_params(rng):
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (PyTorch Linear style)."""
    params = []
    for fi, fo in zip(LAYERS[:-1], LAYERS[1:]):
        k = 1.0 / math.sqrt(fi)
        params.append((rng.uniform(-k, k, (fo, fi)), rng.uniform(-k, k, fo)))
    return params
