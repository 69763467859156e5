"""Oracle for the learned proposal -- test infrastructure only (numpy, FP64).

A small network maps an encoded hit position and outgoing direction to an
8-lobe von Mises-Fisher mixture over incident directions; it is trained
online by maximum likelihood of radiance-weighted sample directions with
Adam, and mixed with BSDF sampling under MIS so the estimator stays
consistent. None of this is in the paper (whose path tracer it extends);
every definition below is stated in the design notes.

Precision: the workload fixes BF16 weights and activations with FP32
accumulation. The oracle computes in FP64 on BF16-rounded weights and
inputs and, with `bf16` set, rounds each hidden activation and each
backpropagated gradient to BF16 (round to nearest even) where the GPU path
feeds them to its matrix units -- so the two differ only by FP32-vs-FP64
accumulation.
"""
from __future__ import annotations

import math

import numpy as np

SIZES = (32, 64, 64, 64, 40)
LOBES = 8
KAPPA_MIN, KAPPA_MAX = 1e-3, 1e4


# ------------------------------------------------------------------ BF16

def to_bf16(x) -> np.ndarray:
    """Round to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def bf16_bits(x) -> np.ndarray:
    return (to_bf16(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


# -------------------------------------------------------------- params

def unpack(theta):
    """Flat parameter vector -> [(W_l (in x out), b_l)]."""
    theta = np.asarray(theta, np.float64)
    out, o = [], 0
    for fi, fo in zip(SIZES[:-1], SIZES[1:]):
        W = theta[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        b = theta[o:o + fo]
        o += fo
        out.append((W, b))
    assert o == theta.shape[0]
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


NPARAM = sum(fi * fo + fo for fi, fo in zip(SIZES[:-1], SIZES[1:]))


# ------------------------------------------------------------- encoding

def encode(x, wo, bbox_min, bbox_ext):
    """32 features: sin/cos of 2^o pi x_hat per axis and octave o = 0..3
    (axis-major, octave, then sin before cos), then sin/cos of pi th, 2 pi th,
    2 pi ph, 4 pi ph for the outgoing direction's normalised polar angle th
    (from +y) and azimuth ph = atan2(x, -z) / 2 pi in [0, 1)."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    wo = np.atleast_2d(np.asarray(wo, np.float64))
    xh = (x - np.asarray(bbox_min, np.float64)) / np.asarray(bbox_ext, np.float64)
    feats = []
    for a in range(3):
        for o in range(4):
            ang = (2.0 ** o) * math.pi * xh[:, a]
            feats += [np.sin(ang), np.cos(ang)]
    th = np.arccos(np.clip(wo[:, 1], -1.0, 1.0)) / math.pi
    ph = np.arctan2(wo[:, 0], -wo[:, 2])
    ph = np.where(ph < 0, ph + 2 * math.pi, ph) / (2 * math.pi)
    for ang in (math.pi * th, 2 * math.pi * th, 2 * math.pi * ph, 4 * math.pi * ph):
        feats += [np.sin(ang), np.cos(ang)]
    return np.stack(feats, axis=1)


# ------------------------------------------------------------------ MLP

def forward(theta, X, bf16=True):
    """Returns (outputs (n x 40), cache). bf16: weights, inputs and hidden
    activations rounded to BF16 (the GPU's rounding points)."""
    layers = unpack(theta)
    rnd = to_bf16 if bf16 else (lambda a: np.asarray(a, np.float64))
    a = rnd(X)
    acts, pre = [a], []
    for li, (W, b) in enumerate(layers):
        Wr = rnd(W)
        z = a @ Wr + rnd(b) if bf16 else a @ Wr + b
        pre.append(z)
        if li < len(layers) - 1:
            a = rnd(np.maximum(z, 0.0))
            acts.append(a)
        else:
            a = z
    return a, (acts, pre, layers)


def backward(theta, cache, dout, bf16=True):
    """Gradient of sum(dout * outputs) w.r.t. the flat parameters. With bf16
    the pre-activation gradient enters every gradient product rounded to BF16
    (the GPU's MFMA operands): the weight gradient, the bias gradient (a sum
    over rows, i.e. a product with a column of ones) and the data gradient;
    the sums themselves are exact here and FP32 on the GPU."""
    acts, pre, layers = cache
    rnd = to_bf16 if bf16 else (lambda a: np.asarray(a, np.float64))
    grads = [None] * len(layers)
    g = np.asarray(dout, np.float64)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        gb = rnd(g)
        grads[li] = (acts[li].T @ gb, gb.sum(0))
        if li > 0:
            g = (gb @ rnd(W).T) * (pre[li - 1] > 0)
    return pack(grads)


# ------------------------------------------------------------------ vMF

def softplus(r):
    return np.where(r > 30, r, np.log1p(np.exp(np.minimum(r, 30))))


def sigmoid(r):
    return 1.0 / (1.0 + np.exp(-r))


def decode(out):
    """out (n x 40) -> pi (n x 8), mu (n x 8 x 3, unit), kappa (n x 8), and
    the raw pieces for the gradient. Lobe k uses outputs 5k..5k+4:
    logit, mu_raw xyz, kappa_raw."""
    o = np.asarray(out, np.float64).reshape(-1, LOBES, 5)
    s = o[:, :, 0]
    s = s - s.max(1, keepdims=True)
    e = np.exp(s)
    pi = e / e.sum(1, keepdims=True)
    m = o[:, :, 1:4]
    mn = np.maximum(np.linalg.norm(m, axis=2, keepdims=True), 1e-12)
    mu = m / mn
    k = softplus(o[:, :, 4]) + KAPPA_MIN
    kappa = np.minimum(k, KAPPA_MAX)
    return pi, mu, kappa, dict(mn=mn[..., 0], raw_k=o[:, :, 4], clamped=k >= KAPPA_MAX)


def vmf_log_pdf(mu, kappa, w):
    """log vMF on the sphere: log(kappa / (2 pi (1 - e^-2kappa))) + kappa (mu.w - 1)."""
    cosw = np.einsum("...c,...c->...", mu, w)
    return np.log(kappa) - np.log(2 * math.pi * -np.expm1(-2 * kappa)) + kappa * (cosw - 1.0)


def mixture_pdf(pi, mu, kappa, w):
    """q(w) for n directions w (n x 3) under n mixtures."""
    w = np.asarray(w, np.float64)[:, None, :]
    return np.sum(pi * np.exp(vmf_log_pdf(mu, kappa, w)), axis=1)


def onb(n):
    """Orthonormal basis around unit n (Duff et al. 2017)."""
    s = np.copysign(1.0, n[..., 2])
    a = -1.0 / (s + n[..., 2])
    b = n[..., 0] * n[..., 1] * a
    t1 = np.stack([1 + s * n[..., 0] ** 2 * a, s * b, -s * n[..., 0]], -1)
    t2 = np.stack([b, s + n[..., 1] ** 2 * a, -n[..., 1]], -1)
    return t1, t2


def vmf_sample(mu, kappa, u1, u2):
    """Stable vMF sampling (Jakob 2012): w = 1 + log(u1 + (1 - u1) e^-2kappa) / kappa."""
    w = 1.0 + np.log(u1 + (1.0 - u1) * np.exp(-2.0 * kappa)) / kappa
    w = np.clip(w, -1.0, 1.0)
    ph = 2 * math.pi * u2
    t1, t2 = onb(mu)
    r = np.sqrt(np.maximum(0.0, 1.0 - w * w))
    return (w[..., None] * mu + (r * np.cos(ph))[..., None] * t1 + (r * np.sin(ph))[..., None] * t2)


def mixture_sample(pi, mu, kappa, u_lobe, u1, u2):
    """Lobe by the cumulative weights (first k with u < cdf_k), then vMF sampling."""
    cdf = np.cumsum(pi, axis=1)
    k = np.minimum((u_lobe[:, None] >= cdf).sum(1), LOBES - 1)
    idx = np.arange(pi.shape[0])
    return vmf_sample(mu[idx, k], kappa[idx, k], u1, u2), k


# ---------------------------------------------------------------- loss

def loss(out, w_dirs, weights):
    """-sum_b w_b log q(w_b) / sum_b w_b."""
    pi, mu, kappa, _ = decode(out)
    q = mixture_pdf(pi, mu, kappa, w_dirs)
    return -np.sum(weights * np.log(q)) / np.sum(weights)


def loss_grad(out, w_dirs, weights):
    """d loss / d outputs through the decode, written with the lobe
    responsibilities g_k = pi_k f_k / q:
      d/dlogit_k  = -w (g_k - pi_k)
      d/dmu_raw_k = -w g_k kappa_k (w - (mu_k.w) mu_k) / |mu_raw_k|
      d/dkraw_k   = -w g_k (1/kappa_k - 2/expm1(2 kappa_k) + mu_k.w - 1) sigmoid(kraw_k)
    (zero where kappa is clamped), all divided by sum_b w_b."""
    pi, mu, kappa, aux = decode(out)
    wd = np.asarray(w_dirs, np.float64)
    lf = vmf_log_pdf(mu, kappa, wd[:, None, :]) + np.log(pi)
    lmax = lf.max(1, keepdims=True)
    g = np.exp(lf - lmax)
    g = g / g.sum(1, keepdims=True)
    wgt = (np.asarray(weights, np.float64) / np.sum(weights))[:, None]
    cosw = np.einsum("nkc,nc->nk", mu, wd)
    d = np.zeros((out.shape[0], LOBES, 5))
    d[:, :, 0] = -wgt * (g - pi)
    perp = wd[:, None, :] - cosw[..., None] * mu
    d[:, :, 1:4] = (-wgt * g * kappa / aux["mn"])[..., None] * perp
    dk = 1.0 / kappa - 2.0 / np.expm1(np.minimum(2.0 * kappa, 700.0)) + cosw - 1.0
    d[:, :, 4] = np.where(aux["clamped"], 0.0, -wgt * g * dk * sigmoid(aux["raw_k"]))
    return d.reshape(out.shape[0], 40)


# ----------------------------------------------------------------- Adam

def adam(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (t counts from 1); returns new theta, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train_step(theta, m, v, t, X, w_dirs, weights, lr=1e-3, bf16=True):
    """Forward, loss gradient, backward and one Adam step on a batch."""
    out, cache = forward(theta, X, bf16)
    d = loss_grad(out, w_dirs, weights)
    g = backward(theta, cache, d, bf16)
    theta, m, v = adam(theta, g, m, v, t, lr)
    return theta, m, v, g, out
