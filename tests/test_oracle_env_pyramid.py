"""Pins for the oracle's environment pyramid (Sec. 2.1.2): hierarchical
importance sampling of the lat-long map, with the top levels weighted per
discretised surface normal.

- Exactness: the final integer intervals of all texels tile [0, 2^32)^2, so
  their probabilities sum to exactly 1 for every normal bin; a sampled
  descent and the descent steered to the texel it found end on the same
  intervals (the probability the MIS weight at an environment hit uses).
- Without the normal weighting the pyramid selects texels by intensity times
  solid angle (as the 2D CDF does) up to 24-bit rounding; a constant map
  gives the uniform density 1/(4 pi).
- With it, every texel that some normal of the bin can see (a direction
  above the normal's horizon) keeps a non-zero probability, texels far below
  every normal of the bin get none, and the mass above the horizon rises.
- Transport: a convex Lambert box under a constant sky returns rho E with
  NEE only and with MIS, for both pyramid modes; a sky-lit scene renders the
  same image (within its noise) with the 2D CDF and the oriented pyramid; an
  environment hit's MIS probability equals, bit for bit, the descent's from
  the previous vertex.
"""
import math

import numpy as np
import pytest

import scenegen as g

TWO64 = 1 << 64


def _sky_scene(width=16, height=12, env=(64, 32)):
    return g.instanced_env_scene(width=width, height=height, target_tris=3000, env_size=env, max_depth=4)


def _omega(r, W, H):
    return (2 * math.pi / W) * (math.cos(math.pi * r / H) - math.cos(math.pi * (r + 1) / H))


def _all_texel_probs(S, bin_, W, H):
    rows, cols = np.divmod(np.arange(W * H), W)
    r, c, iv = S.env_descend(np.full(W * H, bin_), rows=rows, cols=cols)
    assert np.array_equal(r, rows) and np.array_equal(c, cols)
    return [int(a) * int(b) for a, b in zip(iv[:, 0], iv[:, 2])]


@pytest.mark.parametrize("bin_", [-1, 0, 37, 136, 255])
def test_intervals_tile_exactly(orc, bin_):
    sc = _sky_scene()
    S = orc.Scene(sc, build_bvh=False)
    H, W = sc.env.shape[:2]
    assert S.env_pyramid()["m"] == 5
    probs = _all_texel_probs(S, bin_, W, H)
    assert sum(probs) == TWO64


def test_sampled_and_steered_descents_agree(orc):
    sc = _sky_scene()
    S = orc.Scene(sc, build_bvh=False)
    rng = np.random.default_rng(1)
    n = 20000
    bins = rng.integers(-1, 256, n).astype(np.int32)
    u = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    v = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    u[:2], v[:2] = [0, 0xFFFFFFFF], [0, 0xFFFFFFFF]
    r, c, iv = S.env_descend(bins, u=u, v=v)
    assert np.all(iv[:, 1] < iv[:, 0]) and np.all(iv[:, 3] < iv[:, 2])  # remainders inside their intervals
    r2, c2, iv2 = S.env_descend(bins, rows=r, cols=c)
    assert np.array_equal(iv[:, 0], iv2[:, 0]) and np.array_equal(iv[:, 2], iv2[:, 2])


def test_unoriented_pyramid_selects_by_power(orc):
    sc = _sky_scene()
    S = orc.Scene(sc, build_bvh=False)
    H, W = sc.env.shape[:2]
    env = sc.env.astype(np.float64)
    w = (env @ np.array([0.2126, 0.7152, 0.0722])) * np.array([_omega(r, W, H) for r in range(H)])[:, None]
    want = (w / w.sum()).reshape(-1)
    got = np.array(_all_texel_probs(S, -1, W, H), dtype=np.float64) / 2.0 ** 64
    big = want > 1e-6
    assert np.max(np.abs(got[big] / want[big] - 1)) < 2e-4
    assert np.all(got[~big] <= 1e-5)


def test_constant_map_is_uniform(orc):
    sc = g.convex_under_env()
    S = orc.Scene(sc, build_bvh=False)
    H, W = sc.env.shape[:2]
    got = np.array(_all_texel_probs(S, -1, W, H), dtype=np.float64) / 2.0 ** 64
    pdf = got / np.array([_omega(r, W, H) for r in range(H)]).repeat(W)
    assert np.allclose(pdf, 1 / (4 * math.pi), rtol=1e-6)


def _texel_dirs(W, H, fy, fx):
    rows, cols = np.divmod(np.arange(W * H), W)
    th = math.pi * (rows + fy) / H
    ph = 2 * math.pi * (cols + fx) / W
    return np.stack([np.sin(th) * np.sin(ph), np.cos(th), -np.sin(th) * np.cos(ph)], 1)


def test_oriented_levels_cover_the_hemisphere(orc):
    sc = _sky_scene()
    S = orc.Scene(sc, build_bvh=False)
    H, W = sc.env.shape[:2]
    rng = np.random.default_rng(2)
    corners = [_texel_dirs(W, H, a, b) for a in (0.0, 1.0) for b in (0.0, 1.0)]
    centre = _texel_dirs(W, H, 0.5, 0.5)
    flat = np.array(_all_texel_probs(S, -1, W, H), dtype=np.float64) / 2.0 ** 64
    for _ in range(24):
        n = rng.normal(size=3)
        n = (n / np.linalg.norm(n)).astype(np.float32)
        b = orc.env_bin(n)
        p = np.array(_all_texel_probs(S, b, W, H), dtype=np.float64) / 2.0 ** 64
        nn = n.astype(np.float64)
        visible = np.max([c @ nn for c in corners + [centre]], axis=0) > 1e-3
        assert np.all(p[visible & (flat > 0)] > 0)          # nothing this normal sees is left out
        below = np.max([c @ nn for c in corners], axis=0) < -0.5
        assert np.all(p[below] == 0)                         # far below every normal of the bin
        up = centre @ nn > 0
        assert p[up].sum() > max(0.85, flat[up].sum())


def _mean_and_se(s, s2, c):
    c = c.astype(np.float64)[:, None]
    m = s / c
    var = np.maximum(s2 / c - m * m, 0.0) / c
    return m.mean(0), np.sqrt(var.sum(0)) / m.shape[0]


@pytest.mark.parametrize("mode,env_sampling", [(2, 1), (2, 2), (0, 2)])
def test_convex_under_constant_sky(orc, mode, env_sampling):
    rho, E = 0.6, 2.0
    sc = g.convex_under_env(rho, E)
    rho = float(np.float32(rho))  # the scene stores FP32 albedo
    S = orc.Scene(sc)
    # pixels whose every sample lands on the box: BSDF sampling returns rho E on each path there
    s, _, c, _ = S.render(npasses=32, mode=1, rr=False, max_depth=2)
    full = np.all(np.abs(s / c[:, None] - rho * E) < 1e-12, axis=1)
    assert full.sum() > 8
    s, s2, c, _ = S.render(npasses=2048, mode=mode, rr=False, max_depth=2, env_sampling=env_sampling)
    m, se = _mean_and_se(s[full], s2[full], c[full])
    assert np.all(np.abs(m - rho * E) < 4 * se + 1e-9), (m, se)


def test_oriented_pyramid_and_cdf_agree(orc):
    sc = _sky_scene(width=24, height=16)
    S = orc.Scene(sc)
    res = []
    for es in (0, 2):
        s, s2, c, _ = S.render(npasses=256, env_sampling=es)
        m = s / c[:, None]
        res.append((m, np.maximum(s2 / c[:, None] - m * m, 0.0) / c[:, None]))
    (ma, va), (mb, vb) = res
    blk = lambda a: a.reshape(4, 4, 6, 4, 3).sum(axis=(1, 3))
    z = np.abs(blk(ma) - blk(mb)) / np.sqrt(np.maximum(blk(va) + blk(vb), 1e-30))
    assert np.mean(z < 4) > 0.97 and z.max() < 6, z.max()


def test_env_hit_pdf_is_the_sampling_pdf(orc):
    """A floor under the sky, seen at one point: the logged pdf of every
    environment hit equals the oriented pyramid's from the floor's normal."""
    b = g._Builder()
    m = b.material((0.7, 0.7, 0.7))
    b.quad((-50, 0, -50), (-50, 0, 50), (50, 0, 50), (50, 0, -50), m)
    cam = g.Camera((0.0, 2.0, -3.0), (0.3, 0.0, 0.2), (0.0, 1.0, 0.0), 0.002)
    sc = b.scene("floor_sky", cam, 1, 1, 1, 2, env=g.sky_env(64, 32))
    S = orc.Scene(sc)
    H, W = sc.env.shape[:2]
    bin_up = orc.env_bin(np.array([0, 1, 0], np.float32))
    hits = 0
    for j in range(1500):
        _, log = S.debug_path(0, 0, j, max_depth=2, rr=False, mode=0, env_sampling=2)
        for rec in log:
            if rec[0] == 5:
                r, c = int(rec[2]), int(rec[3])
                _, _, iv = S.env_descend(np.array([bin_up]), rows=[r], cols=[c])
                want = float(int(iv[0, 0]) * int(iv[0, 2])) * 2.0 ** -64 / _omega(r, W, H)
                assert rec[4] == want, (j, rec, want)
                hits += 1
    assert hits > 300
