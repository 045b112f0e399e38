"""Plain float64 reference of the learned part (TEST INFRASTRUCTURE ONLY).

The learned sample budget and finite-source predictor is not in the paper;
it is the multilayer perceptron 8 -> 128 -> 128 -> 128 -> 2 with erf-GELU
activations x * Phi(x) between the layers, taking the eight per-epoch
features of the point-source probe (standardised by a stored mean and
standard deviation) and returning

  out[:, 0]  log2 of the limb-sample count the contour integration needs,
  out[:, 1]  the logit of "the point-source magnification is off by more
             than the tolerance".

Loss: mean Huber (delta) on out[:, 0] plus mean binary cross-entropy on the
logit out[:, 1].  Optimiser: Adam with bias correction.

Everything here is written out in numpy float64 with no blocking or
fusion, so that each line can be checked against the textbook definition.
Only the test suite imports this module.  The optional bf16 emulation
rounds each layer's input and weight matrix to bfloat16 (round to nearest
even, through float32) before the product, which is where the device
kernels round; the products and sums themselves stay in float64.
"""
import numpy as np
from scipy.special import erf

DIMS = (8, 128, 128, 128, 2)
NLAYER = len(DIMS) - 1


def n_params():
    """Length of the flat parameter vector: feature mean and std (8 + 8),
    then per layer W (in x out, row-major) and b (out)."""
    n = 2 * DIMS[0]
    for l in range(NLAYER):
        n += DIMS[l] * DIMS[l + 1] + DIMS[l + 1]
    return n


def unflatten(flat):
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == n_params()
    p = {"mean": flat[0:8].copy(), "std": flat[8:16].copy()}
    o = 16
    for l in range(NLAYER):
        a, b = DIMS[l], DIMS[l + 1]
        p[f"W{l}"] = flat[o:o + a * b].reshape(a, b).copy()
        o += a * b
        p[f"b{l}"] = flat[o:o + b].copy()
        o += b
    return p


def flatten(p):
    parts = [p["mean"], p["std"]]
    for l in range(NLAYER):
        parts += [p[f"W{l}"].ravel(), p[f"b{l}"]]
    return np.concatenate(parts)


def init(seed, mean=None, std=None):
    """Seeded He-normal weights, zero biases (used by tests only)."""
    rng = np.random.default_rng(seed)
    p = {"mean": np.zeros(8) if mean is None else np.asarray(mean, float),
         "std": np.ones(8) if std is None else np.asarray(std, float)}
    for l in range(NLAYER):
        a, b = DIMS[l], DIMS[l + 1]
        p[f"W{l}"] = rng.normal(0.0, np.sqrt(2.0 / a), size=(a, b))
        p[f"b{l}"] = rng.normal(0.0, 0.1, size=b)
    return p


def gelu(x):
    """x Phi(x), Phi the standard normal distribution function."""
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through float32; finite values only."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, X, emulate_bf16=False):
    """Returns (out [n, 2], cache).  cache holds each layer's input a_l and
    pre-activation z_l for the backward pass."""
    x = (np.asarray(X, dtype=np.float64) - p["mean"]) / p["std"]
    cache = []
    for l in range(NLAYER):
        W = p[f"W{l}"]
        a = x
        if emulate_bf16:
            a = bf16(a)
            W = bf16(W)
        z = a @ W + p[f"b{l}"]
        cache.append((a, z))
        x = gelu(z) if l < NLAYER - 1 else z
    return x, cache


def huber(r, delta):
    ar = np.abs(r)
    return np.where(ar <= delta, 0.5 * r * r, delta * (ar - 0.5 * delta))


def bce_logits(o, y):
    """-[y log sigma(o) + (1-y) log(1 - sigma(o))], written stably."""
    return np.maximum(o, 0.0) - o * y + np.log1p(np.exp(-np.abs(o)))


def loss(out, y_budget, y_fs, delta=1.0):
    return float(np.mean(huber(out[:, 0] - y_budget, delta)) + np.mean(bce_logits(out[:, 1], y_fs)))


def loss_and_grad(p, X, y_budget, y_fs, delta=1.0, emulate_bf16=False):
    """Loss and the gradient of every weight and bias (a dict like p,
    without mean/std), by the chain rule through the layers."""
    out, cache = forward(p, X, emulate_bf16)
    n = out.shape[0]
    r = out[:, 0] - y_budget
    d_out = np.empty_like(out)
    d_out[:, 0] = np.clip(r, -delta, delta) / n
    d_out[:, 1] = (1.0 / (1.0 + np.exp(-out[:, 1])) - y_fs) / n
    g = {}
    dz = d_out
    for l in range(NLAYER - 1, -1, -1):
        a, z = cache[l]
        g[f"W{l}"] = a.T @ dz
        g[f"b{l}"] = dz.sum(axis=0)
        if l > 0:
            W = bf16(p[f"W{l}"]) if emulate_bf16 else p[f"W{l}"]
            da = dz @ W.T
            dz = da * gelu_grad(cache[l - 1][1])
    return loss(out, y_budget, y_fs, delta), g


def adam_step(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with bias correction, in place on p; state holds
    t and the first and second moments."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k, gk in g.items():
        m = state.setdefault("m_" + k, np.zeros_like(gk))
        v = state.setdefault("v_" + k, np.zeros_like(gk))
        m[...] = beta1 * m + (1.0 - beta1) * gk
        v[...] = beta2 * v + (1.0 - beta2) * gk * gk
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        p[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return p
