"""Pins for the pixel filter (Appendix A.1): box film samples, or filter
importance sampling of a Gaussian of standard deviation 1/2 pixel around the
pixel centre (its 3 sigma range spans 3 x 3 pixels), untruncated.

- A straight edge of a large emitter across the view, vertical or
  horizontal: with the box filter a pixel returns Le times the part of the
  pixel beyond the edge; with the Gaussian, Le times the normal CDF of the
  centre's distance to the edge over sigma (up to the QMC error of the film
  samples).
- An emitter filling the view returns Le on every path with either filter.
"""
import math

import numpy as np
import pytest

import scenegen as g


def _edge_scene(width, height, x_edge, Le=2.0, fov=40.0, y_edge=None):
    """Camera at the origin looking down -z; an emitting quad at z = -5 covers
    x > x_edge (or, with y_edge, y > y_edge), its front facing the camera."""
    b = g._Builder()
    m = b.material((0, 0, 0), emission=(Le, Le, Le))
    z = -5.0
    if y_edge is None:
        b.quad((x_edge, -100, z), (100, -100, z), (100, 100, z), (x_edge, 100, z), m)
    else:
        b.quad((-100, y_edge, z), (100, y_edge, z), (100, 100, z), (-100, 100, z), m)
    cam = g.Camera((0.0, 0.0, 0.0), (0.0, 0.0, -1.0), (0.0, 1.0, 0.0), fov)
    return b.scene("edge", cam, width, height, 1, 1)


def _edge_film_x(sc, x_edge, z=5.0):
    # film x of the edge: the ray through film x hits the plane at X = z * sx,
    # with sx = (2 fx / W - 1) tan(fov/2) aspect
    th = math.tan(math.radians(sc.camera.vfov_deg) / 2)
    aspect = sc.width / sc.height
    return sc.width / 2 * (1 + x_edge / (z * th * aspect))


def _edge_film_y(sc, y_edge, z=5.0):
    # film y grows downwards: sy = (1 - 2 fy / H) tan(fov/2); the plane is hit above y_edge
    th = math.tan(math.radians(sc.camera.vfov_deg) / 2)
    return sc.height / 2 * (1 - y_edge / (z * th))


def _phi(x):
    return 0.5 * (1 + math.erf(x / math.sqrt(2)))


@pytest.mark.parametrize("gauss", [False, True])
def test_edge_closed_form(orc, gauss):
    W, H, Le = 12, 4, 2.0
    x_edge = 0.3137
    sc = _edge_scene(W, H, x_edge, Le)
    S = orc.Scene(sc)
    s, _, c, _ = S.render(npasses=16384, rr=False, gauss=gauss)
    img = (s[:, 0] / c).reshape(H, W)
    e = _edge_film_x(sc, x_edge)
    for px in range(W):
        if gauss:
            want = Le * _phi((px + 0.5 - e) / 0.5)
        else:
            want = Le * min(1.0, max(0.0, px + 1 - e))
        assert np.allclose(img[:, px], want, atol=2e-3 * Le), (px, img[:, px], want)


@pytest.mark.parametrize("gauss", [False, True])
def test_horizontal_edge_closed_form(orc, gauss):
    W, H, Le = 4, 12, 2.0
    y_edge = -0.2719
    sc = _edge_scene(W, H, 0.0, Le, y_edge=y_edge)
    S = orc.Scene(sc)
    s, _, c, _ = S.render(npasses=16384, rr=False, gauss=gauss)
    img = (s[:, 0] / c).reshape(H, W)
    e = _edge_film_y(sc, y_edge)
    for py in range(H):
        if gauss:
            want = Le * _phi((e - (py + 0.5)) / 0.5)
        else:
            want = Le * min(1.0, max(0.0, e - py))
        assert np.allclose(img[py, :], want, atol=2e-3 * Le), (py, img[py, :], want)


@pytest.mark.parametrize("gauss", [False, True])
def test_filled_view_is_exact(orc, gauss):
    Le = 3.0
    sc = _edge_scene(8, 6, -1000.0, Le)
    S = orc.Scene(sc)
    s, s2, c, _ = S.render(npasses=64, rr=False, gauss=gauss)
    assert np.all(s == Le * c[:, None]) and np.all(s2 == Le * Le * c[:, None])
