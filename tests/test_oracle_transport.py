"""Pins for the oracle's whole estimator against closed forms (Sec. 2, Sec. 3.2.2).

- White furnace: a closed enclosure whose walls all emit E and reflect rho.
  With BSDF sampling only and no roulette, every path carries exactly
  E (1 - rho^D) / (1 - rho); with NEE, MIS and roulette the mean does.
- A convex Lambert object under a constant sky E: every BSDF-sampled path
  that hits the object returns exactly rho E.
- A one-sided quad light over a Lambert plane: radiance rho/pi times the
  irradiance from Lambert's polygon formula.
- NEE-only, BSDF-only and MIS estimate the same image.
- Passes may be split into any ranges: the FP64 sums are bit-identical.
"""
import math

import numpy as np
import pytest

import scenegen as g


def _mean_and_se(s, s2, c):
    """Image-mean of the per-pixel means and its standard error."""
    c = c.astype(np.float64)[:, None]
    m = s / c
    var = np.maximum(s2 / c - m * m, 0.0) / c
    return m.mean(0), np.sqrt(var.sum(0)) / m.shape[0]


@pytest.mark.parametrize("D", [1, 2, 8])
def test_furnace_bsdf_only_every_path_exact(orc, D):
    E, rho = 1.0, 0.5
    sc = g.furnace(E, rho, max_depth=D)
    S = orc.Scene(sc)
    s, s2, c, _ = S.render(npasses=16, rr=False, mode=1)
    want = E * (1 - rho ** D) / (1 - rho)
    assert np.allclose(s / c[:, None], want, rtol=1e-12)
    assert np.allclose(s2 / c[:, None], want * want, rtol=1e-12)


@pytest.mark.parametrize("mode,rr", [(0, False), (0, True), (2, False)])
def test_furnace_mean(orc, mode, rr):
    E, rho, D = 1.0, 0.5, 6
    sc = g.furnace(E, rho, width=16, height=16, max_depth=D)
    S = orc.Scene(sc)
    s, s2, c, _ = S.render(npasses=64, rr=rr, mode=mode)
    m, se = _mean_and_se(s, s2, c)
    want = E * (1 - rho ** D) / (1 - rho)
    assert np.all(np.abs(m - want) < 4 * se + 1e-12), (m, se, want)


def test_furnace_infinite_depth_with_roulette(orc):
    E, rho = 1.0, 0.5
    sc = g.furnace(E, rho, width=16, height=16, max_depth=64)
    S = orc.Scene(sc)
    s, s2, c, _ = S.render(npasses=64, rr=True, mode=0)
    m, se = _mean_and_se(s, s2, c)
    want = E / (1 - rho)
    assert np.all(np.abs(m - want) < 4 * se + 1e-9), (m, se)


def test_convex_under_constant_env(orc):
    rho, E = 0.6, 2.0
    sc = g.convex_under_env(rho, E, width=8, height=8, max_depth=4)
    rho = float(np.float32(rho))  # the scene stores FP32 albedo
    S = orc.Scene(sc)
    s, s2, c, _ = S.render(npasses=32, rr=False, mode=1)
    m = s / c[:, None]
    # every pixel mean is a mix of object (rho E) and sky (E) samples
    frac = (E - m) / (E - rho * E)
    assert np.all(frac > -1e-12) and np.all(frac < 1 + 1e-12)
    full = np.all(np.abs(frac - 1.0) < 1e-12, axis=1)
    assert 8 < full.sum() < 56  # the centre sees only the object, the border some sky
    assert np.allclose(s2[full] / c[full, None], (rho * E) ** 2, rtol=1e-12)
    # with NEE of the sky and MIS the mean over those pixels is still rho E
    s, s2, c, _ = S.render(npasses=64, rr=False, mode=0)
    m, se = _mean_and_se(s[full], s2[full], c[full])
    assert np.all(np.abs(m - rho * E) < 4 * se + 1e-12), (m, se)


def _polygon_irradiance(x, n, verts, Le):
    """Lambert's formula: E = Le/2 * sum_i angle_i * (n . unit(a_i x a_{i+1}))."""
    a = [np.asarray(v, float) - x for v in verts]
    a = [v / np.linalg.norm(v) for v in a]
    tot = 0.0
    for i in range(len(a)):
        p, q = a[i], a[(i + 1) % len(a)]
        cr = np.cross(p, q)
        tot += math.acos(np.clip(p @ q, -1, 1)) * (n @ (cr / np.linalg.norm(cr)))
    return abs(0.5 * Le * tot)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_quad_light_over_plane(orc, mode):
    rho, Le = 0.7, 4.0
    sc = g.quad_over_plane(rho, Le)
    S = orc.Scene(sc)
    npass = 4096 if mode != 1 else 65536
    s, s2, c, _ = S.render(npasses=npass, rr=False, mode=mode)
    m, se = _mean_and_se(s, s2, c)
    want = rho / math.pi * _polygon_irradiance(np.array(sc.extra["target"]), np.array([0, 1.0, 0]),
                                               sc.extra["light_quad"], Le)
    assert np.all(np.abs(m - want) < 4 * se + 1e-6 * want), (m, se, want)


@pytest.mark.parametrize("D", [3, 8])
def test_estimators_agree_cornell(orc, D):
    sc = g.cornell(width=32, height=32)
    S = orc.Scene(sc)
    res = []
    for mode in (0, 1, 2):
        s, s2, c, _ = S.render(npasses=256, max_depth=D, rr=True, mode=mode)
        res.append(_mean_and_se(s, s2, c))
    (m0, e0), (m1, e1), (m2, e2) = res
    assert np.all(np.abs(m0 - m1) < 4 * np.hypot(e0, e1)), (m0, m1, e0, e1)
    assert np.all(np.abs(m0 - m2) < 4 * np.hypot(e0, e2)), (m0, m2, e0, e2)


def test_pass_ranges_are_bit_identical(orc):
    sc = g.cornell(width=16, height=16)
    S = orc.Scene(sc)
    a, a2, ac, _ = S.render(npasses=8)
    b = np.zeros_like(a)
    b2 = np.zeros_like(a2)
    bc = np.zeros_like(ac)
    lib = orc.lib()
    for p0, n in ((0, 3), (3, 5)):
        s, s2, c, _ = S.render(pass0=p0, npasses=n)
        # the same additions in the same order as one call: sum over passes in order
        b, b2, bc = b + s, b2 + s2, bc + c
    assert np.array_equal(ac, bc)
    assert np.allclose(a, b, rtol=1e-14, atol=0)
    del lib
