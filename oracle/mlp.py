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
* Training (``train_bf16``): per epoch a permutation of the samples (``epoch_permutation``),
  mini-batches, the bf16-emulating forward and backward, and Adam (``adam_step``) with a
  cosine learning-rate decay over epochs (``cosine_lr``).

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
    return 0.5 * x * (1.0 + np.tanh(SQ2PI * (x + 0.044715 * x * x * x)))


def gelu_tanh_grad(x):
    u = SQ2PI * (x + 0.044715 * x * x * x)
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
    """Raw outputs [n, 6] -> targets in [0, 1] (log first for the flagged outputs).  A target
    with an empty range (constant in the training data) scales to 0, like a constant input
    feature: the network then learns 0, which maps back to that constant."""
    T = np.array(Y, dtype=np.float64, copy=True)
    for j, lg in enumerate(log_outputs):
        if lg:
            T[:, j] = np.log(T[:, j])
    rng = np.asarray(hi, dtype=np.float64) - np.asarray(lo, dtype=np.float64)
    safe = np.where(rng > 0, rng, 1.0)
    return np.where(rng > 0, (T - lo) / safe, 0.0)


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


def backward_bf16(params, cache, y, t, n_total=None, magnitudes=False):
    """Gradients with the back-propagated signal rounded to bf16 where a BF16 GEMM
    consumes it, and the GELU derivative taken at the bf16-rounded pre-activation (the
    precision in which a BF16 engine keeps it between the passes); products exact, sums in
    float64.  With magnitudes=True also returns, per
    layer, for each gradient element the sum of the magnitudes of its terms (|dz|^T |h| and
    sum |dz|), the scale against which the rounding of a finite-precision sum is measured,
    and the sum of the squares of its terms ((dz^2)^T h^2 and sum dz^2), the scale of a sum
    of independent one-term perturbations: (S_W, S_b, Q_W, Q_b)."""
    n = y.shape[0] if n_total is None else n_total
    dz = bf16(np.sign(y - t) / (n * y.shape[1]))
    grads = [None] * len(params)
    mags = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        h_prev = cache[2 * l]
        W, _ = params[l]
        grads[l] = (dz.T @ h_prev, dz.sum(0))
        if magnitudes:
            adz, ah = np.abs(dz), np.abs(h_prev)
            mags[l] = (adz.T @ ah, adz.sum(0), (adz * adz).T @ (ah * ah), (adz * adz).sum(0))
        if l > 0:
            dh = dz @ bf16(W)
            z_prev = bf16(cache[2 * l - 1])      # pre-activations kept in bf16 for the backward
            dz = bf16(dh * gelu_tanh_grad(z_prev))
    return (grads, mags) if magnitudes else grads


def init_params(rng, layers=LAYERS):
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (PyTorch Linear style) for the
    layer widths `layers` (inputs, hidden..., outputs)."""
    params = []
    for fi, fo in zip(layers[:-1], layers[1:]):
        k = 1.0 / math.sqrt(fi)
        params.append((rng.uniform(-k, k, (fo, fi)), rng.uniform(-k, k, fo)))
    return params


# ------------------------------------------------------------------ training (Section 4.3)
# The paper trains each network with an L1 loss for up to 1000 epochs and states neither
# the optimizer nor the batch order; the readings here are Adam (Kingma & Ba 2015,
# Algorithm 1), a cosine learning-rate decay per epoch (Loshchilov & Hutter 2017, without
# restarts), and a fresh permutation of the samples each epoch, i -> (a i + c) mod n with
# a, c drawn from SplitMix64 (Steele, Lea & Flood 2014).

MASK64 = (1 << 64) - 1


def splitmix64(state):
    """One SplitMix64 step: the state advances by the 64-bit golden-ratio increment and the
    output is the state passed through the generator's two xor-shift-multiply rounds.
    Returns (new state, output); Python integers modulo 2^64."""
    state = (state + 0x9E3779B97F4A7C15) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def epoch_permutation(seed, epoch, n):
    """Sample order of one epoch: position i takes sample (a i + c) mod n.  The stream
    starts from the first SplitMix64 output of state `seed`, xor-ed with
    epoch * 0xD1B54A32D192ED03 (mod 2^64); a = (next % n) | 1, redrawn until gcd(a, n) = 1
    (so that the map is a bijection), then c = next % n.  n = 1 gives the identity."""
    n = int(n)
    if n == 1:
        return np.zeros(1, dtype=np.int64)
    _, hashed = splitmix64(int(seed) & MASK64)
    state = hashed ^ ((int(epoch) * 0xD1B54A32D192ED03) & MASK64)
    while True:
        state, r = splitmix64(state)
        a = (r % n) | 1
        if math.gcd(a, n) == 1:
            break
    state, r = splitmix64(state)
    c = r % n
    i = np.arange(n, dtype=np.int64)
    return (a * i + c) % n          # a, c < n <= 2^31: no overflow in int64


def cosine_lr(lr, lr_min, epoch, total_epochs):
    """Learning rate of an epoch: lr_min + (lr - lr_min)(1 + cos(pi e / E)) / 2, with the
    progress e / E capped at 1."""
    prog = min(1.0, epoch / total_epochs)
    return lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * prog))


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam update t (1-based) of parameters w with gradient g: biased moment estimates
    m <- beta1 m + (1 - beta1) g, v <- beta2 v + (1 - beta2) g^2, their bias-corrected
    values m / (1 - beta1^t), v / (1 - beta2^t), and w <- w - lr m_hat / (sqrt(v_hat) + eps).
    Returns (w, m, v) as new arrays."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def train_bf16(params, X, Y, box, log_outputs, epochs, batch, lr, lr_min, total_epochs, seed,
               state=None, beta1=0.9, beta2=0.999, eps=1e-8):
    """Mini-batch training as a BF16 matrix engine runs it: each epoch permutes the samples,
    cuts them into batches of `batch` rows (the last one ragged), and per batch evaluates
    forward_bf16 / backward_bf16 on the scaled inputs and (log-)scaled targets (targets
    rounded to float32, the precision the loss is taken in), then takes one Adam step with
    the epoch's cosine learning rate.

    params: list of (W, b) float64; X [n, 10], Y [n, 6] raw; box = (in_lo, in_hi, out_lo,
    out_hi).  state: {"step", "epoch", "m", "v"} to continue a run (None: fresh).
    Returns (params, state, loss per epoch, per-step records), where a record holds the
    batch's sample indices, the gradient, the learning rate and the parameters after it."""
    in_lo, in_hi, out_lo, out_hi = box
    n = X.shape[0]
    xs = scale_inputs(X, in_lo, in_hi)
    ts = transform_outputs(Y, out_lo, out_hi, log_outputs).astype(np.float32).astype(np.float64)
    params = [(W.copy(), b.copy()) for W, b in params]
    if state is None:
        state = {"step": 0, "epoch": 0,
                 "m": [(np.zeros_like(W), np.zeros_like(b)) for W, b in params],
                 "v": [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]}
    losses, records = [], []
    for _ in range(epochs):
        perm = epoch_permutation(seed, state["epoch"], n)
        rate = cosine_lr(lr, lr_min, state["epoch"], total_epochs)
        total = 0.0
        for row0 in range(0, n, batch):
            rows = perm[row0:row0 + batch]
            y, cache = forward_bf16(params, xs[rows])
            total += float(np.abs(y - ts[rows]).sum())
            grads = backward_bf16(params, cache, y, ts[rows])
            state["step"] += 1
            new, ms, vs = [], [], []
            for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, state["m"], state["v"]):
                W2, mW2, vW2 = adam_step(W, gW, mW, vW, state["step"], rate, beta1, beta2, eps)
                b2, mb2, vb2 = adam_step(b, gb, mb, vb, state["step"], rate, beta1, beta2, eps)
                new.append((W2, b2))
                ms.append((mW2, mb2))
                vs.append((vW2, vb2))
            params, state["m"], state["v"] = new, ms, vs
            records.append({"rows": rows, "grads": grads, "lr": rate, "params": params})
        losses.append(total / (n * Y.shape[1]))
        state["epoch"] += 1
    return params, state, losses, records
