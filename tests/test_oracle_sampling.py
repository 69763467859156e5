"""Pins for the oracle's light tables, environment tables and BSDFs.

Fixed by mathematics, not by the oracle's code: the alias table must
reconstruct its input distribution, the realised light pmf must sum to the
triangle share, a constant environment must give pdf 1/(4 pi), Lambert has
closed forms, GGX's D is normalised, the layered BSDF is reciprocal, keeps
energy <= 1, and its sampler draws from the pdf it reports.
"""
import math

import numpy as np
import pytest

import scenegen as g


def test_alias_reconstructs_distribution(orc):
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 7, 100, 1000):
        w = rng.lognormal(0.0, 1.5, n)
        prob, alias = orc.alias_build(w)
        mass = np.zeros(n)
        for c in range(n):
            mass[c] += prob[c] / n
            mass[alias[c]] += (1.0 - prob[c]) / n
        assert np.allclose(mass, w / w.sum(), rtol=1e-12, atol=1e-15)
        assert np.all((prob >= 0) & (prob <= 1))


def test_light_tables_grid_scene(orc):
    sc = g.grid_scene(grid=2)
    S = orc.Scene(sc)
    L = S.lights()
    assert L["tri"].shape[0] == 256
    # realised pmf of the integer selection rule sums to one and tracks the flux
    assert abs(L["pmf"].sum() - 1.0) < 1e-12
    ref = L["flux"] / L["flux"].sum()
    assert np.allclose(L["pmf"], ref, rtol=256 * 2.0 ** -31, atol=0)


def test_untextured_flux_is_pi_area_luminance(orc):
    sc = g.workload("cornell")
    S = orc.Scene(sc)
    L = S.lights()
    area = 0.25 * 0.25 / 2
    assert np.allclose(L["flux"], math.pi * area * 15.0, rtol=1e-12)
    assert np.allclose(L["pmf"], 0.5)


def test_constant_env_pdf(orc):
    sc = g.convex_under_env()
    S = orc.Scene(sc)
    rq, cq, pdf = S.env_tables()
    assert np.allclose(pdf, 1.0 / (4 * math.pi), rtol=1e-6)
    eh, ew = pdf.shape
    th = np.pi * np.arange(eh + 1) / eh
    om = (2 * np.pi / ew) * (np.cos(th[:-1]) - np.cos(th[1:]))
    assert abs(np.sum(pdf * om[:, None]) - 1.0) < 1e-12
    rng = np.random.default_rng(1)
    for _ in range(50):
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        rgb, p = S.env_lookup(w)
        assert np.allclose(rgb, 2.0) and abs(p - 1 / (4 * math.pi)) < 1e-8


def _material_scene():
    b = g._Builder()
    b.material((0.3, 0.6, 0.9))                               # 0: Lambert
    for a in (0.05, 0.2, 0.5, 0.8):
        b.material((1.0, 1.0, 1.0), roughness=a, flags=g.MAT_GGX)   # 1..4: rho = 1
    b.material((0.4, 0.5, 0.2), roughness=0.3, flags=g.MAT_GGX)     # 5
    b.quad((0, 0, 0), (0, 0, 1), (1, 0, 1), (1, 0, 0), 0)
    cam = g.Camera((0, 1, -1), (0, 0, 0), (0, 1, 0), 40.0)
    return b.scene("materials", cam, 4, 4, 1, 2)


@pytest.fixture(scope="module")
def mats(orc):
    return orc.Scene(_material_scene())


def _hemi_grid(nt=500, nphi=1000):
    th = (np.arange(nt) + 0.5) * (0.5 * np.pi / nt)
    ph = (np.arange(nphi) + 0.5) * (2 * np.pi / nphi)
    T, P = np.meshgrid(th, ph, indexing="ij")
    w = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    dom = (np.sin(T) * (0.5 * np.pi / nt) * (2 * np.pi / nphi)).reshape(-1)
    return w, dom


def test_lambert_closed_form(mats):
    n = np.array([0, 0, 1.0])
    rng = np.random.default_rng(2)
    for _ in range(20):
        wo = rng.normal(size=3); wo[2] = abs(wo[2]); wo /= np.linalg.norm(wo)
        wi = rng.normal(size=3); wi[2] = abs(wi[2]); wi /= np.linalg.norm(wi)
        f, pdf = mats.bsdf(0, n, wo, wi)
        assert np.allclose(f, np.array([0.3, 0.6, 0.9]) / math.pi, rtol=1e-6)
        assert abs(pdf - wi[2] / math.pi) < 1e-15
        f, pdf = mats.bsdf(0, n, wo, -wi)   # below the surface: nothing
        assert np.all(f == 0) and pdf == 0


@pytest.mark.parametrize("alpha", [0.05, 0.2, 0.5, 0.8])
def test_ggx_D_normalised(orc, alpha):
    from scipy.integrate import quad
    val, _ = quad(lambda t: orc.ggx_D(math.cos(t), alpha) * math.cos(t) * math.sin(t) * 2 * math.pi,
                  0, math.pi / 2, limit=400, points=[alpha * 0.5, alpha, 2 * alpha])
    assert abs(val - 1.0) < 1e-6


def test_layered_reciprocity(mats):
    n = np.array([0.3, -0.2, 0.9]); n /= np.linalg.norm(n)
    rng = np.random.default_rng(4)
    for m in (1, 2, 3, 4, 5):
        for _ in range(30):
            a = rng.normal(size=3); a /= np.linalg.norm(a)
            b = rng.normal(size=3); b /= np.linalg.norm(b)
            if a @ n < 0: a = -a
            if b @ n < 0: b = -b
            f1, _ = mats.bsdf(m, n, a, b)
            f2, _ = mats.bsdf(m, n, b, a)
            assert np.allclose(f1, f2, rtol=1e-12, atol=0)


@pytest.mark.parametrize("m", [2, 3, 4, 5])
def test_layered_pdf_normalised_and_energy(mats, m):
    n = np.array([0, 0, 1.0])
    w, dom = _hemi_grid()
    rng = np.random.default_rng(m)
    for th in (0.1, 0.7, 1.2):
        wo = np.array([math.sin(th), 0.0, math.cos(th)])
        f, pdf = mats.bsdf_batch(m, n, wo, w)
        # the pdf's mass plus the sampler's below-horizon failures is one
        ok, _ = mats.bsdf_sample_batch(m, n, wo, rng.uniform(0, 1, (100_000, 3)))
        fail = 1.0 - ok.mean()
        se = math.sqrt(max(fail, 1e-5) / 100_000)
        assert abs(np.sum(pdf * dom) + fail - 1.0) < 2e-3 + 4 * se, (m, th, np.sum(pdf * dom), fail)
        albedo = np.sum(f * w[:, 2:3] * dom[:, None], axis=0)
        assert np.all(albedo <= 1.0 + 2e-3), albedo


@pytest.mark.parametrize("m", [0, 1, 3, 5])
def test_sampler_matches_pdf(mats, m):
    """Mean of f cos / pdf over the sampler's directions equals the quadrature of f cos."""
    n = np.array([0, 0, 1.0])
    wo = np.array([math.sin(0.6), 0.0, math.cos(0.6)])
    rng = np.random.default_rng(8)
    N = 200_000
    u = rng.uniform(0, 1, (N, 3))
    ok, wi = mats.bsdf_sample_batch(m, n, wo, u)
    f, pdf = mats.bsdf_batch(m, n, wo, wi)
    est = np.where(ok[:, None] & (pdf[:, None] > 0), f * wi[:, 2:3] / np.where(pdf > 0, pdf, 1)[:, None], 0)
    w, dom = _hemi_grid(1000, 2000) if m == 1 else _hemi_grid()
    fq, _ = mats.bsdf_batch(m, n, wo, w)
    ref = np.sum(fq * w[:, 2:3] * dom[:, None], axis=0)
    mean = est.mean(0)
    se = est.std(0) / math.sqrt(N)
    assert np.all(np.abs(mean - ref) < 4 * se + 2e-3 * ref), (mean, ref, se)
    # the sampled directions' distribution: P(cos theta > 0.9) from samples vs pdf quadrature
    _, pq = mats.bsdf_batch(m, n, wo, w)
    p_ref = np.sum(pq[w[:, 2] > 0.9] * dom[w[:, 2] > 0.9])
    p_smp = np.mean(ok & (wi[:, 2] > 0.9))
    assert abs(p_smp - p_ref) < 4 * math.sqrt(p_ref * (1 - p_ref) / N) + 2e-3
