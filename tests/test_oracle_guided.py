"""Pins for the oracle's guided branch (the learned proposal mixed one-sided
with BSDF sampling under MIS, an extension of Sec. 2.1-2.2) and for its
training records, against what the mathematics and the readings fix:

- BF16 / FP16 rounding: hand-picked ties, carries and subnormals;
- the record hash: the published first output of SplitMix64 (seed 0) and
  uniformity of its thresholded subset;
- features and network outputs against the numpy oracle (pinned on its own
  by fixed points and finite differences), an independent implementation;
- the stored mixture: numpy's float16 rounding of the numpy decode,
  renormalised; weights sum to 1, unit means;
- mixture density integrates to 1 (quadrature); single-lobe samples have
  the closed-form mean cosine coth(kappa) - 1/kappa; sample histogram
  follows the density (chi-square);
- alpha = 0 leaves the oracle's plain estimator bit for bit;
- a white furnace rendered with the guide mixed in keeps the closed-form
  mean E (1 - rho^D) / (1 - rho) (BSDF-only and MIS), as any proposal must;
  a planted wrong density (q doubled) breaks it;
- record weights in the furnace with BSDF sampling only and no roulette are
  exactly rho E (1 - rho^(D - v)) / (1 - rho) at vertex v, and the records'
  vertices, directions and densities are those of the path;
- guided and plain images of the Cornell box agree within 3 standard errors
  per 8 x 8 block (unbiasedness with a non-trivial proposal).
"""
import math

import numpy as np
import pytest

import scenegen as g
from oracle import guide as G


def _mean_and_se(s, s2, c):
    c = c.astype(np.float64)[:, None]
    m = s / c
    var = np.maximum(s2 / c - m * m, 0.0) / c
    return m.mean(0), np.sqrt(var.sum(0)) / m.shape[0]


def test_round_bf16_fp16(orc):
    b, h = orc.round_bf16, orc.round_fp16
    # ties to even at 1 + half an ulp, and at an odd last bit
    assert b(1.0 + 2 ** -8) == 1.0
    assert b(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert b(1.0 + 2 ** -8 + 2 ** -30) == 1.0 + 2 ** -7
    # carry into the exponent
    assert b(2.0 - 2 ** -9) == 2.0
    assert b(-(2.0 - 2 ** -9)) == -2.0
    assert h(1.0 + 2 ** -11) == 1.0
    assert h(1.0 + 3 * 2 ** -11) == 1.0 + 2 ** -9
    assert h(2048.0 + 1.0) == 2048.0 and h(2048.0 + 3.0) == 2052.0
    assert h(65504.0) == 65504.0 and h(1e4) == 10000.0
    # FP16 subnormals: steps of 2^-24, ties to even
    assert h(2 ** -25) == 0.0 and h(3 * 2 ** -25) == 2 ** -23 and h(2 ** -24) == 2 ** -24
    # against numpy's float16 conversion on random values
    rng = np.random.default_rng(3)
    x = rng.normal(size=2000) * 10.0 ** rng.uniform(-6, 4, 2000)
    want = x.astype(np.float16).astype(np.float64)
    got = np.array([h(v) for v in x])
    assert np.array_equal(got, want)


def test_rec_hash(orc):
    # z = 1 * golden gamma is SplitMix64's first state for seed 0, whose
    # published first output is 0xE220A8397B1DCDAF
    assert orc.rec_hash(1, 0) == 0xE220A839
    rng = np.random.default_rng(5)
    idx = rng.integers(0, 2 ** 63, 20000, dtype=np.uint64)
    thr = 0x40000000
    frac = np.mean([orc.rec_hash(int(i), 3) < thr for i in idx])
    assert abs(frac - 0.25) < 4 * math.sqrt(0.25 * 0.75 / idx.shape[0])
    # vertices of one path are decorrelated
    a = np.array([orc.rec_hash(int(i), 1) < thr for i in idx[:5000]])
    c = np.array([orc.rec_hash(int(i), 2) < thr for i in idx[:5000]])
    assert abs(np.mean(a & c) - 0.0625) < 0.02


@pytest.fixture(scope="module")
def frozen(orc):
    sc = g.cornell(width=32, height=32)
    S = orc.Scene(sc)
    theta = g.guide_frozen(5)
    S.guide_set(theta, alpha=0.7)
    return sc, S, theta


def _vertices(sc, n, seed):
    rng = np.random.default_rng(seed)
    pos = sc.positions.astype(np.float64)
    lo, hi = pos.min(0), pos.max(0)
    x = lo + rng.uniform(0, 1, (n, 3)) * (hi - lo)
    wo = rng.normal(size=(n, 3))
    wo /= np.linalg.norm(wo, axis=1, keepdims=True)
    return x, wo, lo, np.maximum(hi - lo, 1e-6)


def test_features_and_forward_match_numpy(frozen):
    sc, S, theta = frozen
    x, wo, lo, ext = _vertices(sc, 500, 1)
    f, out = S.guide_forward(x, wo)
    want_f = G.encode(x, wo, lo, ext)
    assert np.allclose(f, want_f, rtol=0, atol=1e-12)
    want_o, _ = G.forward(theta.astype(np.float64), want_f, bf16=True)
    assert np.allclose(out, want_o, rtol=1e-12, atol=1e-12)


def test_stored_mixture(frozen):
    sc, S, theta = frozen
    x, wo, lo, ext = _vertices(sc, 500, 2)
    w, mu, kappa = S.guide_mix(x, wo)
    out, _ = G.forward(theta.astype(np.float64), G.encode(x, wo, lo, ext), bf16=True)
    pi, m, k, _ = G.decode(out)
    h16 = lambda a: np.asarray(a).astype(np.float16).astype(np.float64)
    mh = h16(m)
    mh /= np.linalg.norm(mh, axis=2, keepdims=True)
    ph = h16(pi)
    ph /= ph.sum(1, keepdims=True)
    assert np.allclose(w, ph, rtol=1e-13, atol=1e-15)
    assert np.allclose(mu, mh, rtol=0, atol=1e-13)
    assert np.array_equal(kappa, h16(k))
    assert np.allclose(w.sum(1), 1.0, atol=1e-14)
    assert np.allclose(np.linalg.norm(mu, axis=2), 1.0, atol=1e-14)


def _sphere_grid(n_th=400, n_ph=800):
    th = (np.arange(n_th) + 0.5) * math.pi / n_th
    ph = (np.arange(n_ph) + 0.5) * 2 * math.pi / n_ph
    T, P = np.meshgrid(th, ph, indexing="ij")
    d = np.stack([np.sin(T) * np.sin(P), np.cos(T), -np.sin(T) * np.cos(P)], -1).reshape(-1, 3)
    dA = (np.sin(T) * (math.pi / n_th) * (2 * math.pi / n_ph)).reshape(-1)
    return d, dA


def test_mixture_density_integrates_to_one(frozen, orc):
    sc, S, _ = frozen
    x, wo, _, _ = _vertices(sc, 3, 3)
    w, mu, kappa = S.guide_mix(x, wo)
    d, dA = _sphere_grid()
    for r in range(3):
        n = d.shape[0]
        pdf, _ = orc.guide_mix_eval(np.repeat(w[r:r + 1], n, 0), np.repeat(mu[r:r + 1], n, 0),
                                    np.repeat(kappa[r:r + 1], n, 0), dirs=d)
        assert abs(np.sum(pdf * dA) - 1.0) < 2e-4


@pytest.mark.parametrize("kappa", [0.05, 1.0, 8.0, 200.0])
def test_single_lobe_mean_cosine(orc, kappa):
    n = 40000
    rng = np.random.default_rng(7)
    m = rng.normal(size=3)
    m /= np.linalg.norm(m)
    w = np.zeros((n, 8))
    w[:, 3] = 1.0
    mu = np.tile(rng.normal(size=(8, 3)), (n, 1, 1))
    mu /= np.linalg.norm(mu, axis=2, keepdims=True)
    mu[:, 3] = m
    kap = np.full((n, 8), 1.0)
    kap[:, 3] = kappa
    # u_lobe in [3/8, 1) still picks lobe 3 (the weights of lobes 0..2 are 0)
    u = np.stack([rng.uniform(0, 1, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)], 1)
    _, smp = orc.guide_mix_eval(w, mu, kap, u=u)
    assert np.allclose(np.linalg.norm(smp, axis=1), 1.0, atol=1e-12)
    c = smp @ m
    want = 1.0 / math.tanh(kappa) - 1.0 / kappa
    se = np.std(c) / math.sqrt(n)
    assert abs(c.mean() - want) < 4 * se + 1e-12


def test_mixture_sampler_matches_density(frozen, orc):
    sc, S, _ = frozen
    x, wo, _, _ = _vertices(sc, 1, 9)
    w, mu, kappa = S.guide_mix(x, wo)
    n = 200000
    rng = np.random.default_rng(11)
    u = rng.uniform(0, 1, (n, 3))
    rep = lambda a: np.repeat(a, n, 0)
    _, smp = orc.guide_mix_eval(rep(w), rep(mu), rep(kappa), u=u)
    # histogram over 12 x 24 cells of (cos theta, phi) against the density's cell mass
    nt, nph = 12, 24
    ct = np.clip(smp[:, 1], -1, 1)
    ph = np.mod(np.arctan2(smp[:, 0], -smp[:, 2]), 2 * math.pi)
    it = np.minimum(((1 - ct) / 2 * nt).astype(int), nt - 1)
    ip = np.minimum((ph / (2 * math.pi) * nph).astype(int), nph - 1)
    hist = np.bincount(it * nph + ip, minlength=nt * nph).astype(np.float64)
    d, dA = _sphere_grid(240, 480)
    m = d.shape[0]
    pdf, _ = orc.guide_mix_eval(np.repeat(w, m, 0), np.repeat(mu, m, 0), np.repeat(kappa, m, 0), dirs=d)
    jt = np.minimum(((1 - d[:, 1]) / 2 * nt).astype(int), nt - 1)
    jp = np.minimum((np.mod(np.arctan2(d[:, 0], -d[:, 2]), 2 * math.pi) / (2 * math.pi) * nph).astype(int), nph - 1)
    mass = np.bincount(jt * nph + jp, weights=pdf * dA, minlength=nt * nph)
    exp = mass / mass.sum() * n
    keep = exp > 20
    chi2 = np.sum((hist[keep] - exp[keep]) ** 2 / exp[keep])
    dof = keep.sum() - 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof), (chi2, dof)


def test_alpha_zero_is_plain(orc):
    sc = g.cornell(width=24, height=20, max_depth=6)
    S = orc.Scene(sc)
    S.guide_set(g.guide_frozen(5), alpha=0.0)
    a = S.render(npasses=8)
    b = S.render(npasses=8, guide=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("mode,rr", [(1, False), (0, False), (0, True)])
def test_guided_furnace_mean(orc, mode, rr):
    E, rho, D = 1.0, 0.5, 6
    sc = g.furnace(E, rho, width=16, height=16, max_depth=D)
    S = orc.Scene(sc)
    S.guide_set(g.guide_frozen(5), alpha=0.7)
    s, s2, c, _ = S.render(npasses=128, rr=rr, mode=mode, guide=True)
    m, se = _mean_and_se(s, s2, c)
    want = E * (1 - rho ** D) / (1 - rho)
    assert np.all(se > 1e-4), "the guided estimator must not be the constant BSDF-only one"
    assert np.all(np.abs(m - want) < 4 * se), (m, se, want)


def test_guided_furnace_catches_a_wrong_density(orc):
    """A proposal whose density is misreported (a planted factor 2 on q) is
    biased: the furnace mean moves far outside the error bars."""
    E, rho, D = 1.0, 0.5, 6
    sc = g.furnace(E, rho, width=16, height=16, max_depth=D)
    S = orc.Scene(sc)
    S.guide_set(g.guide_frozen(5), alpha=0.7)
    orc.plant(1)
    try:
        s, s2, c, _ = S.render(npasses=128, rr=False, mode=1, guide=True)
    finally:
        orc.plant(0)
    m, se = _mean_and_se(s, s2, c)
    want = E * (1 - rho ** D) / (1 - rho)
    assert np.all(np.abs(m - want) > 6 * se), (m, se, want)


def test_furnace_record_weights_closed_form(orc):
    E, rho, D = 1.0, 0.5, 6
    sc = g.furnace(E, rho, width=8, height=8, max_depth=D)
    S = orc.Scene(sc)
    S.guide_set(g.guide_frozen(5), alpha=0.0)
    s, cnt, rec = S.records(npasses=4, rr=False, mode=1)
    npath = sc.width * sc.height * 4
    # every path scatters at vertices 1..D-1 and continues: one record each
    assert rec["weight"].shape[0] == npath * (D - 1)
    v = rec["vertex"]
    want = rho * E * (1 - rho ** (D - v)) / (1 - rho)
    assert np.allclose(rec["weight"], want, rtol=1e-12)
    # Lambert cosine sampling: the recorded density is cos(wi) / pi about the
    # inward normal, and every record belongs to a distinct (pixel, pass, vertex)
    ident = rec["pixel"] * 1000 + rec["pass_"] * 10 + v
    assert np.unique(ident).shape[0] == ident.shape[0]
    assert np.all(rec["pdf"] > 0)
    assert np.allclose(np.linalg.norm(rec["wi"], axis=1), 1.0, atol=1e-12)
    assert np.allclose(np.linalg.norm(rec["wo"], axis=1), 1.0, atol=1e-12)
    # the positions lie on the cube's faces
    assert np.allclose(np.abs(rec["x"]).max(1), 1.0, atol=1e-9)
    # a planted mistake (weights not divided by the throughput) fails the closed form
    orc.plant(2)
    try:
        _, _, bad = S.records(npasses=1, rr=False, mode=1)
    finally:
        orc.plant(0)
    vb = bad["vertex"]
    assert not np.allclose(bad["weight"], rho * E * (1 - rho ** (D - vb)) / (1 - rho), rtol=1e-3)


def test_furnace_record_weights_with_nee_mean(orc):
    """With next-event estimation and MIS the weight leaves out the vertex's
    own NEE; weight + NEE term is the sample's whole estimate of the light
    scattered at the vertex, whose mean in the furnace is the closed form
    rho E (1 - rho^(D - v)) / (1 - rho) (Lambert sampling without roulette
    continues every path, so the records see every vertex; a guided vertex
    whose sample falls below the surface ends its path without a record, which
    conditions the mean). A planted weight that keeps the NEE term overshoots
    by that term's mean."""
    E, rho, D = 1.0, 0.5, 5
    sc = g.furnace(E, rho, width=16, height=16, max_depth=D)
    S = orc.Scene(sc)
    S.guide_set(g.guide_frozen(5), alpha=0.0)
    _, _, rec = S.records(npasses=64, rr=False, mode=0)
    assert np.all(np.isfinite(rec["weight"])) and np.all(rec["weight"] >= 0)
    for planted in (False, True):
        if planted:
            orc.plant(3)
            try:
                _, _, rec = S.records(npasses=64, rr=False, mode=0)
            finally:
                orc.plant(0)
        ok = True
        for v in range(1, D):
            tot = (rec["weight"] + rec["nee"])[rec["vertex"] == v]
            want = rho * E * (1 - rho ** (D - v)) / (1 - rho)
            se = tot.std() / np.sqrt(tot.shape[0])
            if planted:
                ok &= abs(tot.mean() - want) < 6 * se
            else:
                assert abs(tot.mean() - want) < 4 * se, (v, tot.mean(), want, se)
                assert np.mean(rec["nee"][rec["vertex"] == v] > 0) > 0.5
        if planted:
            assert not ok


@pytest.mark.parametrize("mode", [0, 1])
def test_guided_cornell_unbiased_per_block(orc, mode):
    sc = g.cornell(width=32, height=32, max_depth=6)
    S = orc.Scene(sc)
    S.guide_set(g.guide_frozen(5), alpha=0.7)
    n = 256
    s_p, s2_p, c_p, _ = S.render(npasses=n, pass0=0, mode=mode)
    s_g, s2_g, c_g, _ = S.render(npasses=n, pass0=1 << 20, guide=True, mode=mode)

    def blocks(s, s2, c):
        c = c.astype(np.float64)[:, None]
        m = s / c
        v = np.maximum(s2 / c - m * m, 0.0) / c     # per pixel and channel
        return m.reshape(4, 8, 4, 8, 3).mean((1, 3)), v.reshape(4, 8, 4, 8, 3).sum((1, 3)) / 64 ** 2

    mp, vp = blocks(s_p, s2_p, c_p)
    mg, vg = blocks(s_g, s2_g, c_g)
    z = (mg - mp) / np.sqrt(vp + vg + 1e-30)
    # 48 (block, channel) pairs at 3 sigma (the sample variance overstates the
    # QMC error, so this is conservative)
    assert np.sum(np.abs(z) > 3) <= 1, z
    assert np.abs(z).max() < 4.5, z
