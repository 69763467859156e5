"""Bit-exact closest hits on the full-size workloads (Sec. 2.3: watertight
traversal and intersection), through the C-ABI:

- the 0.97M-triangle grid and the 16M-triangle city: closest hit (triangle
  id, t, barycentrics) and occlusion through the BVH equal the GPU's brute
  force over every triangle, bit for bit, on a few thousand rays each:
  camera rays of the workload's camera, random rays aimed at vertices and
  edges, and (city) street-level rays along the blocks; the deepest
  traversal stack of each ray is reported;
- a subset of the same rays against the oracle's FP32 brute force (C, run
  on host threads), bit for bit;
- a comb of 120,000 sliver triangles whose boxes all contain one line while
  the triangles miss it: rays along the line open every node, so their
  stacks outgrow the 15 entries kept in LDS and spill to the workspace (the
  test requires it), and BVH equals brute force bit for bit there too.
"""
import math
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import scenegen as g

pytestmark = pytest.mark.gpu
# traversal stack entries per ray kept in LDS (deeper entries spill to the workspace)
SHORT_STACK = 15
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Renderer():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01263_amd import Renderer as R
    return R


def _camera_rays(sc, n, rng):
    cam = sc.camera
    eye = np.asarray(cam.eye, np.float64)
    fwd = np.asarray(cam.look, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(cam.up, np.float64))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(0.5 * math.radians(cam.vfov_deg))
    asp = sc.width / sc.height
    sx = (2 * rng.uniform(0, 1, n) - 1) * th * asp
    sy = (1 - 2 * rng.uniform(0, 1, n)) * th
    d = fwd + sx[:, None] * right + sy[:, None] * up
    return np.repeat(eye[None], n, 0), d


def _aimed_rays(sc, n, rng):
    lo = sc.positions.min(0).astype(np.float64)
    hi = sc.positions.max(0).astype(np.float64)
    o = lo + rng.uniform(0, 1, (n, 3)) * (hi - lo)
    tri = rng.integers(0, sc.num_triangles, n)
    w = rng.choice([0.0, 0.5, 1.0], (n, 2))
    p = sc.positions[sc.indices[tri]].astype(np.float64)
    tgt = p[:, 0] + w[:, :1] * (p[:, 1] - p[:, 0]) + w[:, 1:] * 0.5 * (p[:, 2] - p[:, 0])
    return o, tgt - o


def _street_rays(sc, n, rng):
    lo = sc.positions.min(0).astype(np.float64)
    hi = sc.positions.max(0).astype(np.float64)
    o = np.stack([rng.uniform(lo[0], hi[0], n), rng.uniform(0.5, 6.0, n), rng.uniform(lo[2], hi[2], n)], 1)
    ang = rng.choice([0.0, 0.5, 1.0, 1.5], n) * math.pi + rng.normal(0, 0.02, n)
    d = np.stack([np.cos(ang), rng.normal(0, 0.01, n), np.sin(ang)], 1)
    return o, d


def _pack(o, d):
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((o.shape[0], 8), np.float32)
    rays[:, 0:3] = o
    rays[:, 3] = np.inf
    rays[:, 4:7] = d
    return rays


def _trace(r, rays, any_hit, brute):
    n = rays.shape[0]
    dr = torch.from_numpy(rays).to("cuda")
    t = torch.empty(n, dtype=torch.float32, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    b = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    depth = torch.zeros(n, dtype=torch.int32, device="cuda")
    if any_hit:
        r.ctx.debug_trace(dr, n, 1, brute, None, tri, None, None if brute else depth)
    else:
        r.ctx.debug_trace(dr, n, 0, brute, t, tri, b, None if brute else depth)
    torch.cuda.synchronize()
    return t.cpu().numpy(), tri.cpu().numpy().view(np.uint32), b.cpu().numpy(), depth.cpu().numpy()


def _oracle_f32(orc, sc, rays, threads=16):
    chunks = np.array_split(np.arange(rays.shape[0]), threads)
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda ix: orc.trace_f32(sc, rays[ix]), chunks))
    return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
            np.concatenate([p[2] for p in parts]))


@pytest.mark.parametrize("which", ["grid_1m", "city_16m"])
def test_fullsize_hits_bitexact(Renderer, orc, which):
    sc = g.workload(which)
    rng = np.random.default_rng(17)
    parts = [_camera_rays(sc, 3000, rng), _aimed_rays(sc, 2000, rng)]
    if which == "city_16m":
        parts.append(_street_rays(sc, 3000, rng))
    rays = np.concatenate([_pack(o, d) for o, d in parts])
    n = rays.shape[0]
    _say(f"[full-size hits] {which}: {sc.num_triangles} triangles, {n} rays")
    r = Renderer(sc, pool_paths=1 << 16)
    t, tri, b, depth = _trace(r, rays, False, 0)
    t_b, tri_b, b_b, _ = _trace(r, rays, False, 1)
    hit = tri != 0xFFFFFFFF
    _say(f"    hits {hit.sum()}, deepest stack {depth.max()}, rays past the LDS stack (> {SHORT_STACK}): {(depth > SHORT_STACK).sum()}")
    assert np.array_equal(tri, tri_b)
    assert np.array_equal(t[hit], t_b[hit]) and np.array_equal(b[hit], b_b[hit])
    # rays whose stack spilled past the LDS entries (the comb test below makes
    # sure some do) are part of the comparison above
    _, occ, _, _ = _trace(r, rays, True, 0)
    _, occ_b, _, _ = _trace(r, rays, True, 1)
    assert np.array_equal(occ, occ_b)
    assert np.array_equal(occ.astype(bool), hit)
    del r
    torch.cuda.empty_cache()
    # a subset against the oracle's FP32 brute force; rays that spill first
    m = 256 if which == "city_16m" else 1024
    order = np.argsort(-depth, kind="stable")
    sub = np.sort(np.concatenate([order[:m // 4], rng.choice(n, m - m // 4, replace=False)]))
    sub = np.unique(sub)
    t_o, tri_o, b_o = _oracle_f32(orc, sc, rays[sub])
    _say(f"    oracle subset {sub.shape[0]} rays, of them past the LDS stack: {(depth[sub] > SHORT_STACK).sum()}")
    assert np.array_equal(tri[sub], tri_o)
    h = tri_o != 0xFFFFFFFF
    assert np.array_equal(t[sub][h], t_o[h]) and np.array_equal(b[sub][h], b_o[h])


def _comb(n=120_000):
    """Sliver triangles in the planes x = 0.001 k, each spanning y, z in
    [-0.01, 0.01] x [-0.005, 0.01] (a box around the x axis) while the
    triangle lies above the line from (-0.01, 0.01) to (0.01, -0.005) in
    (y, z) and so misses the axis; a wall at x = n / 1000 + 1 ends it."""
    b = g._Builder()
    m = b.material((0.5, 0.5, 0.5))
    x = 0.001 * np.arange(n, dtype=np.float64)
    v = np.zeros((n, 3, 3))
    v[:, :, 0] = x[:, None]
    v[:, 0, 1:] = (-0.01, 0.01)
    v[:, 1, 1:] = (0.01, 0.01)
    v[:, 2, 1:] = (0.01, -0.005)
    b.mesh(v.reshape(-1, 3), np.arange(3 * n).reshape(-1, 3), m)
    xe = 0.001 * n + 1.0
    b.quad((xe, -1, -1), (xe, -1, 1), (xe, 1, 1), (xe, 1, -1), m)
    cam = g.Camera((-1.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 10.0)
    return b.scene("comb", cam, 16, 16, 1, 4)


def test_stack_spill_comb(Renderer, orc):
    sc = _comb()
    rng = np.random.default_rng(5)
    n = 256
    # along the axis (inside every box), with small offsets that keep them inside
    o = np.stack([np.full(n, -1.0), rng.uniform(-0.004, 0.004, n), rng.uniform(-0.004, 0.0, n)], 1)
    d = np.stack([np.ones(n), rng.normal(0, 1e-6, n), rng.normal(0, 1e-6, n)], 1)
    rays = _pack(o, d)
    _say(f"[stack spill] comb: {sc.num_triangles} triangles, {n} rays along the axis")
    r = Renderer(sc, pool_paths=1 << 16)
    t, tri, b, depth = _trace(r, rays, False, 0)
    t_b, tri_b, b_b, _ = _trace(r, rays, False, 1)
    hit = tri != 0xFFFFFFFF
    spill = int((depth > SHORT_STACK).sum())
    _say(f"    hits {hit.sum()}, deepest stack {depth.max()}, rays past the LDS stack (> {SHORT_STACK}): {spill}")
    assert spill >= n // 2, "rays along the comb should spill the LDS stack"
    assert np.array_equal(tri, tri_b)
    assert np.array_equal(t[hit], t_b[hit]) and np.array_equal(b[hit], b_b[hit])
    _, occ, _, _ = _trace(r, rays, True, 0)
    _, occ_b, _, _ = _trace(r, rays, True, 1)
    assert np.array_equal(occ, occ_b) and np.array_equal(occ.astype(bool), hit)
    # the rays that hit end on the wall; against the oracle's FP32 brute force
    t_o, tri_o, b_o = _oracle_f32(orc, sc, rays[:32], threads=8)
    assert np.array_equal(tri[:32], tri_o)
    h = tri_o != 0xFFFFFFFF
    assert np.array_equal(t[:32][h], t_o[h]) and np.array_equal(b[:32][h], b_o[h])
