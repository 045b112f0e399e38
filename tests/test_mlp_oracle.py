"""Pins of the learned-part oracle (MLP, loss, Adam) and of the per-epoch
features, against closed forms, finite differences, hand-built networks and
independent lens-equation solutions."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as M
from tests import pins


# ---------------------------------------------------------------- GELU ----
def test_gelu_closed_forms():
    # Phi(1) = 0.841344746068542948... (standard normal table)
    assert M.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    x = np.linspace(-6, 6, 101)
    # x Phi(x) - (-x) Phi(-x) = x Phi(x) + x (1 - Phi(x)) = x
    np.testing.assert_allclose(M.gelu(x) - M.gelu(-x), x, rtol=0, atol=1e-14)
    assert M.gelu(np.array([40.0]))[0] == 40.0


def test_gelu_grad_by_differences():
    x = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(x), fd, rtol=0, atol=1e-8)
    # phi(0) = 1/sqrt(2 pi), so the slope at 0 is Phi(0) = 1/2
    assert M.gelu_grad(np.array([0.0]))[0] == 0.5


# ---------------------------------------------------------------- bf16 ----
def test_bf16_rounding_cases():
    one = 1.0
    ulp = 2.0 ** -7
    assert M.bf16(one) == one
    assert M.bf16(one + ulp / 2) == one                  # tie to even (down)
    assert M.bf16(one + 3 * ulp / 2) == one + 2 * ulp     # tie to even (up)
    assert M.bf16(one + 0.51 * ulp) == one + ulp
    assert M.bf16(3.14159) == 3.140625
    assert M.bf16(-2.0 ** -130) == -2.0 ** -130           # subnormal, exact


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).normal(size=4096) * np.exp(np.random.default_rng(1).normal(size=4096) * 5)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)


# ---------------------------------------------------------- losses --------
def test_loss_closed_forms():
    assert M.huber(np.array([0.5]), 1.0)[0] == 0.125
    assert M.huber(np.array([-3.0]), 1.0)[0] == 2.5
    assert M.huber(np.array([1.0]), 1.0)[0] == 0.5          # both branches meet
    assert M.bce_logits(np.array([0.0]), np.array([1.0]))[0] == pytest.approx(math.log(2), rel=1e-15)
    o = np.array([-3.0, -0.5, 0.7, 4.0])
    sig = 1 / (1 + np.exp(-o))
    np.testing.assert_allclose(M.bce_logits(o, np.ones(4)), -np.log(sig), rtol=1e-14)
    np.testing.assert_allclose(M.bce_logits(o, np.zeros(4)), -np.log(1 - sig), rtol=1e-14)


# ------------------------------------------------------- forward ----------
def _routing_net():
    """Hand-built net: feature 0 -> hidden unit 3 -> unit 7 -> unit 11 ->
    (out0 = k + 0.5, out1 = -2 k + 1).  Any transposed weight or wrong
    index sends the signal elsewhere."""
    p = M.init(0)
    for l in range(M.NLAYER):
        p[f"W{l}"][:] = 0.0
        p[f"b{l}"][:] = 0.0
    p["W0"][0, 3] = 1.0
    p["W1"][3, 7] = 1.0
    p["W2"][7, 11] = 1.0
    p["W3"][11, 0] = 1.0
    p["W3"][11, 1] = -2.0
    p["b3"][:] = [0.5, 1.0]
    p["mean"][:] = np.arange(8) * 0.1
    p["std"][:] = 2.0
    return p


def test_forward_hand_built_network():
    p = _routing_net()
    X = np.random.default_rng(3).normal(size=(16, 8))
    out, _ = M.forward(p, X)
    phi = lambda t: 0.5 * (1 + math.erf(t / math.sqrt(2)))
    for i in range(16):
        x0 = (X[i, 0] - 0.0) / 2.0
        g = x0
        for _ in range(3):
            g = g * phi(g)
        assert out[i, 0] == pytest.approx(g + 0.5, rel=1e-14, abs=1e-15)
        assert out[i, 1] == pytest.approx(-2 * g + 1.0, rel=1e-14, abs=1e-15)


def test_bf16_emulation_exact_on_representable_values():
    p = M.init(5)
    for l in range(M.NLAYER):
        p[f"W{l}"] = M.bf16(p[f"W{l}"])
    X = M.bf16(np.random.default_rng(6).normal(size=(32, 8)))
    a, _ = M.forward(p, X)
    # only the hidden activations are rounded now; the first layer is exact
    _, ca = M.forward(p, X, emulate_bf16=True)
    _, cb = M.forward(p, X)
    np.testing.assert_array_equal(ca[0][1], cb[0][1])
    b, _ = M.forward(p, X, emulate_bf16=True)
    assert np.max(np.abs(a - b)) < 0.05 * (1 + np.max(np.abs(a)))


# ------------------------------------------------------ gradient ----------
@pytest.mark.parametrize("delta", [1.0, 0.25])
def test_gradient_by_central_differences(delta):
    rng = np.random.default_rng(11)
    p = M.init(7)
    X = rng.normal(size=(24, 8))
    yb = rng.normal(loc=7.0, scale=1.5, size=24)
    yf = (rng.random(24) < 0.4).astype(float)
    _, g = M.loss_and_grad(p, X, yb, yf, delta)
    h = 1e-6
    for k in [f"W{l}" for l in range(M.NLAYER)] + [f"b{l}" for l in range(M.NLAYER)]:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = M.loss(M.forward(p, X)[0], yb, yf, delta)
            flat[idx] = old - h
            lm = M.loss(M.forward(p, X)[0], yb, yf, delta)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (k, idx)


def test_flatten_roundtrip_and_size():
    assert M.n_params() == 16 + 8 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 2 + 2
    p = M.init(2)
    q = M.unflatten(M.flatten(p))
    for k in p:
        np.testing.assert_array_equal(p[k], q[k])


# ---------------------------------------------------------- Adam ----------
def test_adam_first_steps_closed_form():
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g1 = np.array([0.3, -1e-3, 4.0])
    st = {}
    M.adam_step(p, {"w": g1}, st, lr=0.01, eps=1e-8)
    # step 1: mhat = g, vhat = g^2
    np.testing.assert_allclose(p["w"], np.array([1.0, -2.0, 0.5]) - 0.01 * g1 / (np.abs(g1) + 1e-8),
                               rtol=1e-15)
    w1 = p["w"].copy()
    g2 = np.array([-0.1, 2e-3, 4.0])
    M.adam_step(p, {"w": g2}, st, lr=0.01, eps=1e-8)
    m = 0.9 * 0.1 * g1 + 0.1 * g2
    v = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    mhat = m / (1 - 0.81)
    vhat = v / (1 - 0.999 ** 2)
    np.testing.assert_allclose(p["w"], w1 - 0.01 * mhat / (np.sqrt(vhat) + 1e-8), rtol=1e-14)


# ------------------------------------------------------- features ---------
def _mu_newton(s, q, zeta):
    z = pins.real_images_newton(s, q, zeta)
    return float(np.sum(1.0 / np.abs(pins.jacobian(s, q, z)))), len(z)


@pytest.mark.parametrize("case", [
    (1.0, 1e-3, 0.6 + 0.0j, 1e-3),      # far from caustics, 3 images
    (1.0, 1e-3, 0.02 + 0.01j, 1e-2),    # central caustic region
    (0.8, 0.1, 0.05 - 0.02j, 3e-3),
    (1.2, 0.3, -0.3 + 0.25j, 2e-3),
])
def test_features_against_independent_solutions(oracle, case):
    s, q, zeta, rho = case
    f, mu, ok = oracle.features(s, q, zeta, rho, 1e-4)
    assert f[0] == np.float32(s)
    assert f[1] == np.float32(math.log10(q))
    assert f[2] == np.float32(zeta.real) and f[3] == np.float32(zeta.imag)
    assert f[4] == np.float32(math.log10(rho))
    mu0, n0 = _mu_newton(s, q, zeta)
    assert mu == pytest.approx(mu0, rel=1e-9)
    assert f[5] == pytest.approx(math.log10(mu0), rel=1e-6, abs=1e-6)
    # caustic-proximity sign follows the independent image count
    assert (f[6] > 0) == (n0 == 3)
    # relative gradient over the probe radius, by the same central differences
    # of independently solved magnifications
    mx = [_mu_newton(s, q, zeta + d)[0] for d in (rho, 1j * rho, -rho, -1j * rho)]
    g = 0.5 * math.hypot(mx[0] - mx[2], mx[1] - mx[3]) / mu0
    assert f[7] == pytest.approx(math.log10(max(g, 1e-30)), rel=1e-5, abs=1e-5)


def test_features_proximity_grows_with_distance(oracle):
    # along the symmetry axis away from the central caustic of a planetary
    # lens the ghost statistic (an estimate of the distance to the fold)
    # grows, so the proximity feature increases monotonically
    s, q, rho = 1.0, 1e-3, 1e-3
    xs = [0.05, 0.1, 0.2, 0.4, 0.8]
    vals = [oracle.features(s, q, complex(x, 0.01), rho, 1e-4)[0][6] for x in xs]
    assert all(b > a for a, b in zip(vals, vals[1:])), vals
