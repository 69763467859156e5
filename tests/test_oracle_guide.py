"""Pins for the oracle of the learned proposal (numpy, FP64).

- Backward pass (decode + loss + MLP) equals central finite differences of
  the directly evaluated loss.
- vMF lobes integrate to one; E[mu.w] = coth(kappa) - 1/kappa and the CDF
  of mu.w under the sampler match the closed forms.
- The first Adam step is -lr g / (|g| + eps).
- Encoding and BF16 rounding fixed points.
- Training on samples of a known vMF recovers its mean direction and
  concentration (maximum likelihood).
"""
import math

import numpy as np
import pytest

import scenegen as g
from oracle import guide as G


def test_bf16_rounding():
    assert G.to_bf16(1.0) == 1.0
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins (1.0)
    assert G.to_bf16(1.0 + 2 ** -8) == 1.0
    assert G.to_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert G.to_bf16(-2.5) == -2.5
    x = np.random.default_rng(0).normal(size=1000)
    r = G.to_bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8 + 1e-40)


def test_encoding_fixed_points():
    X = G.encode([[0.0, 0.0, 0.0]], [[0.0, 1.0, 0.0]], [0, 0, 0], [1, 1, 1])[0]
    assert X.shape == (32,)
    assert np.allclose(X[0:24:2], 0.0) and np.allclose(X[1:24:2], 1.0)
    # straight up: theta = 0; azimuth of (0, 1, 0) is atan2(+0, -0) = pi, i.e. 1/2
    assert np.allclose(X[24:], [0, 1, 0, 1, 0, -1, 0, 1])
    X = G.encode([[0.5, 1.0, 0.25]], [[1.0, 0.0, 0.0]], [0, 0, 0], [1, 1, 1])[0]
    assert np.isclose(X[0], 1.0) and np.isclose(X[1], 0.0)          # sin, cos of pi/2
    assert np.isclose(X[24], 1.0) and np.isclose(X[25], 0.0)        # theta = pi/2
    # phi = atan2(1, -0) = pi/2, i.e. 1/4: sin/cos of pi/2 then of pi
    assert np.allclose(X[28:], [1.0, 0.0, 0.0, -1.0])


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    X = G.encode(rng.uniform(-1, 1, (n, 3)), rng.normal(size=(n, 3)) / 1.7, [-1, -1, -1], [2, 2, 2])
    w = rng.normal(size=(n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    wt = rng.uniform(0.1, 2.0, n)
    return X, w, wt


def test_backward_matches_finite_differences():
    theta = g.guide_init(3).astype(np.float64) * 0.7
    X, w, wt = _batch(16, 1)
    out, cache = G.forward(theta, X, bf16=False)
    grad = G.backward(theta, cache, G.loss_grad(out, w, wt), bf16=False)
    rng = np.random.default_rng(2)
    idx = rng.choice(G.NPARAM, 200, replace=False)
    idx[:8] = [0, 2047, 2048, 2111, 6271, 10431, 12991, 13031]  # layer edges and biases
    h = 1e-6
    fd = np.empty(idx.shape[0])
    for j, i in enumerate(idx):
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd[j] = (G.loss(G.forward(tp, X, False)[0], w, wt) - G.loss(G.forward(tm, X, False)[0], w, wt)) / (2 * h)
    err = np.abs(fd - grad[idx])
    assert np.all(err <= 1e-6 * np.maximum(1.0, np.abs(fd)) + 1e-8), (idx[np.argmax(err)], err.max())


def test_output_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    out = rng.normal(size=(6, 40)) * 1.5
    _, w, wt = _batch(6, 6)
    d = G.loss_grad(out, w, wt)
    h = 1e-6
    for r in range(6):
        for c in range(40):
            op = out.copy(); op[r, c] += h
            om = out.copy(); om[r, c] -= h
            fd = (G.loss(op, w, wt) - G.loss(om, w, wt)) / (2 * h)
            assert abs(fd - d[r, c]) <= 1e-6 * max(1.0, abs(fd)), (r, c, fd, d[r, c])


@pytest.mark.parametrize("kappa", [0.01, 1.0, 10.0, 100.0, 1000.0])
def test_vmf_normalised(kappa):
    from scipy.integrate import quad
    mu = np.array([0.3, -0.5, 0.81])
    mu /= np.linalg.norm(mu)
    # integrate over the angle to mu: 2 pi int f(cos) sin dtheta
    f = lambda t: 2 * math.pi * math.sin(t) * math.exp(
        float(G.vmf_log_pdf(mu, np.array(kappa), np.cos(t) * mu + np.sin(t) * np.array([0.0, 0.85, 0.525]) * 0)))
    val, _ = quad(lambda c: 2 * math.pi * math.exp(math.log(kappa) - math.log(2 * math.pi * -math.expm1(-2 * kappa))
                                                   + kappa * (c - 1.0)), -1, 1, points=[1 - 10 / kappa] if kappa > 10 else None)
    assert abs(val - 1.0) < 1e-9
    # the oracle's log pdf agrees with the formula along a great circle
    for t in (0.0, 0.3, 1.2, 3.0):
        w = math.cos(t) * mu + math.sin(t) * G.onb(mu)[0]
        want = math.log(kappa / (2 * math.pi * (1 - math.exp(-2 * kappa)))) + kappa * (math.cos(t) - 1)
        assert abs(float(G.vmf_log_pdf(mu, np.array(kappa), w)) - want) < 1e-9
    del f


@pytest.mark.parametrize("kappa", [0.5, 5.0, 50.0])
def test_vmf_sampler_closed_forms(kappa):
    rng = np.random.default_rng(int(kappa * 10))
    N = 200_000
    mu = np.tile(np.array([[0.0, 0.6, -0.8]]), (N, 1))
    k = np.full(N, kappa)
    w = G.vmf_sample(mu, k, rng.uniform(size=N), rng.uniform(size=N))
    assert np.allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-12)
    c = w @ np.array([0.0, 0.6, -0.8])
    mean = 1.0 / math.tanh(kappa) - 1.0 / kappa
    assert abs(c.mean() - mean) < 4 * c.std() / math.sqrt(N)
    for t in (-0.5, 0.0, 0.5, 0.9, 0.99):
        cdf = (math.exp(kappa * (t - 1)) - math.exp(-2 * kappa)) / (1 - math.exp(-2 * kappa))
        p = np.mean(c <= t)
        assert abs(p - cdf) < 4 * math.sqrt(cdf * (1 - cdf) / N) + 1e-4


def test_mixture_sampler_matches_pdf():
    rng = np.random.default_rng(9)
    out = rng.normal(size=(1, 40)) * 2.0
    pi, mu, kappa, _ = G.decode(out)
    N = 200_000
    P = np.repeat(pi, N, 0)
    M = np.repeat(mu, N, 0)
    K = np.repeat(kappa, N, 0)
    w, _ = G.mixture_sample(P, M, K, rng.uniform(size=N), rng.uniform(size=N), rng.uniform(size=N))
    # E[1 / q(w)] over the sampler = area of the sphere
    q = G.mixture_pdf(P, M, K, w)
    est = 1.0 / q
    assert abs(est.mean() - 4 * math.pi) < 5 * est.std() / math.sqrt(N)


def test_adam_first_step():
    rng = np.random.default_rng(4)
    th = rng.normal(size=100)
    gr = rng.normal(size=100) * 1e-3
    t2, m, v = G.adam(th, gr, np.zeros(100), np.zeros(100), 1, lr=1e-3)
    assert np.allclose(t2 - th, -1e-3 * gr / (np.abs(gr) + 1e-8), rtol=1e-12, atol=1e-18)


def test_training_recovers_a_vmf():
    """Maximum likelihood on samples of one vMF lobe at a fixed input."""
    rng = np.random.default_rng(12)
    mu_t = np.array([0.36, 0.48, 0.8])
    mu_t /= np.linalg.norm(mu_t)
    k_t = 20.0
    theta = g.guide_init(11).astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    X = np.tile(G.encode([[0.2, 0.3, 0.4]], [[0.0, 1.0, 0.0]], [0, 0, 0], [1, 1, 1]), (512, 1))
    for t in range(1, 301):
        w = G.vmf_sample(np.tile(mu_t, (512, 1)), np.full(512, k_t), rng.uniform(size=512), rng.uniform(size=512))
        theta, m, v, _, _ = G.train_step(theta, m, v, t, X, w, np.ones(512), lr=1e-2, bf16=False)
    out, _ = G.forward(theta, X[:1], bf16=False)
    pi, mu, kappa, _ = G.decode(out)
    # the fitted mixture's mean resultant vector matches the target's
    N = 100_000
    ws, _ = G.mixture_sample(np.repeat(pi, N, 0), np.repeat(mu, N, 0), np.repeat(kappa, N, 0),
                             rng.uniform(size=N), rng.uniform(size=N), rng.uniform(size=N))
    r = ws.mean(0)
    ang = math.degrees(math.acos(np.clip(r @ mu_t / np.linalg.norm(r), -1, 1)))
    want_len = 1 / math.tanh(k_t) - 1 / k_t
    assert ang < 2.0, ang
    assert abs(np.linalg.norm(r) - want_len) / want_len < 0.1
