"""Pins for the oracle's light tree (the many-light hierarchy of Sec. 2.1.1).

- Structure: every emitter in exactly one leaf of at most 8; the two children
  of a node split its emitter range; bounding spheres hold their triangles;
  a region's flux lies between the flux of the triangles facing into the
  region and the node's total flux; leaf weights rise from 0 below 2^24.
- The integer descent partitions [0, 2^63) exactly: interval sizes of all
  emitters sum to 2^63 at any shading point, and a sample falls in the
  interval (laid out in leaf order) of the emitter it returns, whose size is
  the pdf the estimator divides by.
- Closed forms: up to 8 emitters the tree is one leaf and selects by flux
  (to 2^-24); a cluster facing the shading point against one facing away
  gets the clamp 15/16 (1/16 mirrored); two equal clusters along the normal
  at distances d1 and d2 split by the inverse square law.
- The probability behind the MIS weight at an emitter hit is, bit for bit,
  the one the tree samples with from the previous vertex.
- Unbiasedness: with the subdivided quad light over a plane, tree NEE and
  tree MIS reach Lambert's polygon formula; in a field of 2000 lights the
  tree's image agrees with the flux alias table's, with and without an
  environment; at single floor points its direct-light variance is well
  below the alias table's.
"""
import math

import numpy as np
import pytest

import scenegen as g

R63 = 1 << 63


def _clusters(away: bool, d1=4.0, d2=4.0, lateral=3.0, s=0.02, width=4, height=4, fov=30.0):
    """Shading point at the origin, normal +y. Eight small lights at height
    d1 over x = -lateral facing down and eight at height d2 over x = +lateral,
    facing up when `away`."""
    b = g._Builder()
    floor = b.material((0.5, 0.5, 0.5))
    b.quad((-9, 0, -9), (-9, 0, 9), (9, 0, 9), (9, 0, -9), floor)
    lm = b.material((0, 0, 0), emission=(3.0, 3.0, 3.0))
    for side, h, up in ((-1, d1, False), (1, d2, away)):
        for k in range(8):
            cx, cz = side * lateral + 2.5 * s * (k % 4 - 1.5), 2.5 * s * (k // 4 - 0.5)
            tri = [(cx - s, h, cz - s), (cx + s, h, cz - s), (cx, h, cz + s)]
            if up:
                tri = tri[::-1]  # as listed the corners face down (counter-clockwise from below)
            b.mesh(np.array(tri), np.array([[0, 1, 2]]), lm)
    cam = g.Camera((0.0, 1.0, -3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), fov)
    return b.scene("clusters", cam, width, height, 1, 2)


def test_tree_structure(orc):
    sc = g.light_field(n_lights=700)
    S = orc.Scene(sc, build_bvh=False)
    t = S.light_tree()
    lt = S.lights()
    ne = lt["tri"].shape[0]
    nn = t["left"].shape[0]
    assert np.array_equal(np.sort(t["emit"]), np.arange(ne, dtype=np.uint32))
    assert t["first"][0] == 0 and t["count"][0] == ne
    pos = sc.positions.astype(np.float64)
    nrm_all = []
    for e in range(ne):
        a, b_, c = pos[sc.indices[lt["tri"][e]]]
        n = np.cross(b_ - a, c - a)
        nrm_all.append(n / np.linalg.norm(n))
    nrm_all = np.array(nrm_all)
    parents = np.zeros(nn, int)
    tc = math.acos(1 / math.sqrt(3))
    for k in range(nn):
        f, c, l = int(t["first"][k]), int(t["count"][k]), int(t["left"][k])
        es = t["emit"][f:f + c]
        # bounding sphere holds every corner
        cen, rad = t["center"][k, :3].astype(np.float64), float(t["center"][k, 3])
        corners = pos[sc.indices[lt["tri"][es]]].reshape(-1, 3)
        assert np.all(np.linalg.norm(corners - cen, axis=1) <= rad * (1 + 1e-5) + 1e-6)
        # region fluxes: at least the flux of triangles whose normal lies in
        # the region's cone, at most the total
        tot = lt["flux"][es].sum()
        fl = t["flux"][k].astype(np.float64)
        assert np.all(fl <= tot * (1 + 1e-5))
        for r in range(6):
            axis = np.zeros(3)
            axis[r // 2] = -1.0 if r & 1 else 1.0
            inside = np.arccos(np.clip(nrm_all[es] @ axis, -1, 1)) <= tc
            assert fl[r] >= lt["flux"][es][inside].sum() * (1 - 1e-5)
        if l < 0:
            assert 1 <= c <= 8
            w = t["w"][f:f + c].astype(np.int64)
            assert w[0] == 0 and np.all(np.diff(w) >= 0) and w[-1] < (1 << 24)
        else:
            assert c > 8
            parents[l] += 1
            parents[l + 1] += 1
            assert t["first"][l] == f and t["first"][l + 1] == f + t["count"][l]
            assert t["count"][l] + t["count"][l + 1] == c and abs(int(t["count"][l]) - int(t["count"][l + 1])) <= 1
    assert parents[0] == 0 and np.all(parents[1:] == 1)


@pytest.mark.parametrize("env", [False, True])
def test_descent_partitions_exactly(orc, env):
    sc = g.light_field(n_lights=300, env=env)
    S = orc.Scene(sc, build_bvh=False)
    t = S.light_tree()
    rng = np.random.default_rng(3)
    for q in range(12):
        x = rng.uniform([-15, 0, -15], [15, 6, 15]).astype(np.float32)
        n = rng.normal(size=3)
        n = (n / np.linalg.norm(n)).astype(np.float32)
        sizes = S.light_tree_sizes(x, n)
        assert sum(int(v) for v in sizes) == R63  # exact, in integers
        # intervals in leaf order; random samples land in the returned one
        starts = np.zeros(sizes.shape[0], object)
        acc = 0
        for e in t["emit"]:
            starts[e] = acc
            acc += int(sizes[e])
        Ss = rng.integers(0, R63, 400, dtype=np.uint64, endpoint=False)
        Ss[:3] = [0, R63 - 1, int(starts[t["emit"][5]])]
        es, sz = S.light_tree_sample(Ss, np.tile(x, (Ss.shape[0], 1)), np.tile(n, (Ss.shape[0], 1)))
        for Sv, e, z in zip(Ss, es, sz):
            assert int(z) == int(sizes[e]) > 0
            assert starts[e] <= int(Sv) < starts[e] + int(z)


def test_single_leaf_selects_by_flux(orc):
    sc = g.light_field(n_lights=7)
    S = orc.Scene(sc, build_bvh=False)
    t = S.light_tree()
    assert t["left"].shape[0] == 1 and t["left"][0] == -1
    flux = S.lights()["flux"]
    p = S.light_tree_sizes(np.zeros(3, np.float32), np.array([0, 1, 0], np.float32)).astype(np.float64) / R63
    assert np.all(np.abs(p - flux / flux.sum()) <= 2.0 ** -23)


@pytest.mark.parametrize("mirror", [False, True])
def test_cluster_facing_away_gets_the_clamp(orc, mirror):
    sc = _clusters(away=True)
    S = orc.Scene(sc, build_bvh=False)
    t = S.light_tree()
    assert t["left"][0] == 1 and t["count"][1] == 8
    left_is_minus_x = t["center"][1, 0] < 0
    x = np.array([0.0, 0.0, 0.0], np.float32)
    n = np.array([0.0, 1.0, 0.0], np.float32)
    q = S.light_tree_left_q(0, x, n)
    # the cluster at -x faces the point, the one at +x faces away
    assert q == (0xF00000 if left_is_minus_x else 0x100000)
    if mirror:
        # seen from above both clusters, the downward cluster emits away and
        # the upward one towards the point
        x2 = np.array([0.0, 8.0, 0.0], np.float32)
        n2 = np.array([0.0, -1.0, 0.0], np.float32)
        q2 = S.light_tree_left_q(0, x2, n2)
        assert q2 == (0x100000 if left_is_minus_x else 0xF00000)


def test_inverse_square_split(orc):
    d1, d2 = 3.0, 6.0
    sc = _clusters(away=False, d1=d1, d2=d2, lateral=0.0)
    S = orc.Scene(sc, build_bvh=False)
    t = S.light_tree()
    # the two clusters sit one above the other: the split is along y
    lower = 1 if t["center"][1, 1] < t["center"][2, 1] else 2
    x = np.array([0.0, 0.0, 0.0], np.float32)
    n = np.array([0.0, 1.0, 0.0], np.float32)
    p_left = S.light_tree_left_q(0, x, n) / 2.0 ** 24
    p_lower = p_left if lower == 1 else 1.0 - p_left
    want = (1 / d1 ** 2) / (1 / d1 ** 2 + 1 / d2 ** 2)
    assert abs(p_lower - want) < 0.01, (p_lower, want)


@pytest.mark.parametrize("scene", ["quad", "field"])
def test_emitter_hit_pdf_is_the_sampling_pdf(orc, scene):
    """MIS at an emitter hit divides by the probability with which the tree
    would have chosen that emitter from the previous vertex: the logged
    selection probability equals the interval size computed from that
    vertex's ray origin and normal (here the floor's, +y), bit for bit."""
    if scene == "quad":
        sc = g.quad_over_plane(subdiv=12)
    else:
        sc = g.light_field(n_lights=2000, width=1, height=1, max_depth=2)
        sc.camera = g.Camera((6.1, 9.0, -18.9), (6.1, 0.0, -12.9), (0.0, 1.0, 0.0), 0.002)
    S = orc.Scene(sc)
    emit_of = {int(t): e for e, t in enumerate(S.lights()["tri"])}
    n_floor = np.array([0.0, 1.0, 0.0], np.float32)
    hits = 0
    for j in range(3000):
        _, log = S.debug_path(0, 0, j, max_depth=2, rr=False, mode=0, light_tree=True)
        origin, on_floor = None, False
        for rec in log:
            if rec[0] == 1 and rec[1] == 1:
                on_floor = abs(rec[5]) < 1e-12  # the first vertex lies on the floor y = 0
            elif rec[0] == 2:
                origin = rec[1:4]
            elif rec[0] == 4 and rec[1] == 2 and on_floor:
                e = emit_of[int(rec[2])]
                size = S.light_tree_sizes(origin.astype(np.float32), n_floor)[e]
                assert rec[3] == float(size) * 2.0 ** -63, (j, rec)
                hits += 1
    assert hits > 30


def _mean_and_se(s, s2, c):
    c = c.astype(np.float64)[:, None]
    m = s / c
    var = np.maximum(s2 / c - m * m, 0.0) / c
    return m.mean(0), np.sqrt(var.sum(0)) / m.shape[0]


def _polygon_irradiance(x, n, quad, Le):
    a = [np.array(p, np.float64) - x for p in quad]
    a = [v / np.linalg.norm(v) for v in a]
    tot = 0.0
    for i in range(len(a)):
        p, q = a[i], a[(i + 1) % len(a)]
        cr = np.cross(p, q)
        tot += math.acos(np.clip(p @ q, -1, 1)) * (n @ (cr / np.linalg.norm(cr)))
    return abs(0.5 * Le * tot)


@pytest.mark.parametrize("mode", [0, 2])
def test_subdivided_quad_light_closed_form(orc, mode):
    rho, Le = 0.7, 4.0
    sc = g.quad_over_plane(rho, Le, subdiv=12)  # 288 emitters, tree of depth 6
    S = orc.Scene(sc)
    s, s2, c, _ = S.render(npasses=8192, rr=False, mode=mode, light_tree=True)
    m, se = _mean_and_se(s, s2, c)
    want = rho / math.pi * _polygon_irradiance(np.array(sc.extra["target"]), np.array([0, 1.0, 0]),
                                               sc.extra["light_quad"], Le)
    assert np.all(np.abs(m - want) < 4 * se + 1e-6 * want), (m, se, want)


@pytest.mark.parametrize("env", [False, True])
def test_tree_and_alias_agree_light_field(orc, env):
    sc = g.light_field(n_lights=2000, width=24, height=18, env=env, max_depth=4)
    S = orc.Scene(sc)
    res = {}
    for tree in (False, True):
        s, s2, c, _ = S.render(npasses=192, light_tree=tree)
        m = s / c[:, None]
        var = np.maximum(s2 / c[:, None] - m * m, 0.0) / c[:, None]
        res[tree] = (m, var)
    (ma, va), (mt, vt) = res[False], res[True]
    # 4x4-pixel blocks: means agree within 4 standard errors
    blk = lambda a: a.reshape(18 // 3, 3, 24 // 4, 4, 3).sum(axis=(1, 3))
    za = np.abs(blk(ma) - blk(mt)) / np.sqrt(np.maximum(blk(va) + blk(vt), 1e-30))
    assert np.mean(za < 4) > 0.97 and za.max() < 6, za.max()


@pytest.mark.parametrize("target", [(-0.6, 0.0, -8.4), (6.1, 0.0, -12.9), (-11.4, 0.0, -4.2)])
def test_tree_lowers_nee_variance(orc, target):
    """Direct light at one floor point of the light field (a one-pixel camera
    of tiny field of view): the tree's estimate agrees with the alias table's
    and its sample variance is well below it."""
    sc = g.light_field(n_lights=2000, width=1, height=1, max_depth=2)
    sc.camera = g.Camera((target[0], 9.0, target[2] - 6.0), target, (0.0, 1.0, 0.0), 0.002)
    S = orc.Scene(sc)
    res = []
    for tree in (False, True):
        s, s2, c, _ = S.render(npasses=16384, mode=2, light_tree=tree)
        m = s[0] / c[0]
        res.append((m, s2[0] / c[0] - m * m, c[0]))
    (ma, va, n), (mt, vt, _) = res
    assert np.all(np.abs(ma - mt) < 4 * np.sqrt((va + vt) / n)), (ma, mt)
    assert np.all(vt < 0.6 * va), (vt, va)
