"""Seeded synthetic scenes for the progressive QMC path tracer.

This module holds input data only: triangle meshes, material parameters,
environment-map texels and camera placements, drawn from a self-written
splitmix64 generator so the bytes do not depend on the numpy version. It
contains none of the renderer's arithmetic (no sampling, no intersection,
no shading) and is the one module that both the CPU oracle and the GPU
library read their inputs from.

The scenes stand in for the paper's proprietary production scenes (Sec. 3.2,
Table 1): 0.02-8 MP frames, many small textured emitters, an environment sky
with a sun, and million-triangle instanced geometry.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# material flag bits (input convention shared by both consumers)
MAT_GGX = 1            # GGX specular layer over the Lambert base
MAT_EMIT_TEXTURE = 2   # emission modulated by the analytic stripe texture

_M64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64 (Steele, Lea, Flood 2014), vectorised over numpy uint64."""

    def __init__(self, seed: int):
        self.state = np.uint64(seed & _M64)

    def next_u64(self, n: int) -> np.ndarray:
        with np.errstate(over="ignore"):
            inc = np.uint64(0x9E3779B97F4A7C15)
            base = self.state
            k = np.arange(1, n + 1, dtype=np.uint64)
            z = base + inc * k
            self.state = base + inc * np.uint64(n)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        return z

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = (self.next_u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
        return lo + (hi - lo) * u

    def normal(self, n: int) -> np.ndarray:
        u1 = self.uniform(n)
        u2 = self.uniform(n)
        return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


@dataclass
class Camera:
    eye: tuple
    look: tuple
    up: tuple
    vfov_deg: float


@dataclass
class Scene:
    name: str
    positions: np.ndarray          # (nv, 3) float32
    indices: np.ndarray            # (nt, 3) uint32
    tri_material: np.ndarray       # (nt,) uint32
    albedo: np.ndarray             # (nm, 3) float32, Lambert base reflectance
    roughness: np.ndarray          # (nm,) float32, GGX alpha (used when MAT_GGX)
    emission: np.ndarray           # (nm, 3) float32, front-face radiance scale
    mat_flags: np.ndarray          # (nm,) uint32
    camera: Camera
    width: int
    height: int
    spp: int
    max_depth: int
    env: Optional[np.ndarray] = None   # (eh, ew, 3) float32 lat-long radiance
    extra: dict = field(default_factory=dict)

    @property
    def num_triangles(self) -> int:
        return int(self.indices.shape[0])

    def validate(self) -> None:
        assert self.positions.dtype == np.float32 and self.positions.ndim == 2
        assert self.indices.dtype == np.uint32 and self.indices.shape[1] == 3
        assert self.tri_material.dtype == np.uint32
        assert self.tri_material.shape[0] == self.indices.shape[0]
        assert int(self.indices.max()) < self.positions.shape[0]
        assert int(self.tri_material.max()) < self.albedo.shape[0]
        for a in (self.albedo, self.roughness, self.emission):
            assert a.dtype == np.float32
        assert self.mat_flags.dtype == np.uint32
        if self.env is not None:
            assert self.env.dtype == np.float32 and self.env.ndim == 3


class _Builder:
    """Accumulates triangles and materials into flat arrays."""

    def __init__(self):
        self.pos = []
        self.idx = []
        self.mat = []
        self.nv = 0
        self.albedo = []
        self.rough = []
        self.emis = []
        self.flags = []

    def material(self, albedo, roughness=0.0, emission=(0.0, 0.0, 0.0), flags=0) -> int:
        self.albedo.append(np.asarray(albedo, np.float64))
        self.rough.append(float(roughness))
        self.emis.append(np.asarray(emission, np.float64))
        self.flags.append(int(flags))
        return len(self.albedo) - 1

    def mesh(self, verts: np.ndarray, tris: np.ndarray, mat) -> None:
        verts = np.asarray(verts, np.float64).reshape(-1, 3)
        tris = np.asarray(tris, np.int64).reshape(-1, 3)
        self.pos.append(verts)
        self.idx.append(tris + self.nv)
        m = np.asarray(mat, np.int64)
        self.mat.append(np.broadcast_to(m, (tris.shape[0],)).copy())
        self.nv += verts.shape[0]

    def quad(self, p0, p1, p2, p3, mat) -> None:
        """Quad p0,p1,p2,p3 counter-clockwise seen from its front side."""
        self.mesh(np.array([p0, p1, p2, p3]), np.array([[0, 1, 2], [0, 2, 3]]), mat)

    def scene(self, name, camera, width, height, spp, max_depth, env=None) -> Scene:
        s = Scene(
            name=name,
            positions=np.concatenate(self.pos).astype(np.float32),
            indices=np.concatenate(self.idx).astype(np.uint32),
            tri_material=np.concatenate(self.mat).astype(np.uint32),
            albedo=np.array(self.albedo, np.float32).reshape(-1, 3),
            roughness=np.array(self.rough, np.float32),
            emission=np.array(self.emis, np.float32).reshape(-1, 3),
            mat_flags=np.array(self.flags, np.uint32),
            camera=camera, width=width, height=height, spp=spp,
            max_depth=max_depth, env=env)
        s.validate()
        return s


# ----------------------------------------------------------------- meshes

def _yaw(deg: float) -> np.ndarray:
    a = math.radians(deg)
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def box_mesh(center, size, yaw_deg=0.0, subdiv=1, inward=False):
    """Axis-aligned box (then yawed), each face split into subdiv x subdiv quads."""
    n = subdiv
    g = np.linspace(-0.5, 0.5, n + 1)
    # each face: (fixed axis, sign); build a grid in the two other axes
    verts = []
    tris = []
    base = 0
    for axis in range(3):
        for sign in (-1.0, 1.0):
            a1, a2 = (axis + 1) % 3, (axis + 2) % 3
            uu, vv = np.meshgrid(g, g, indexing="ij")
            p = np.zeros((n + 1, n + 1, 3))
            p[..., axis] = 0.5 * sign
            p[..., a1] = uu
            p[..., a2] = vv
            verts.append(p.reshape(-1, 3))
            i = np.arange(n)[:, None] * (n + 1) + np.arange(n)[None, :]
            q0, q1, q2, q3 = i, i + (n + 1), i + (n + 2), i + 1
            # (a1 x a2) = axis direction: CCW order q0,q1,q2 faces +axis
            t = np.stack([np.stack([q0, q1, q2], -1), np.stack([q0, q2, q3], -1)], -2).reshape(-1, 3)
            if (sign < 0) != inward:
                t = t[:, [0, 2, 1]]
            tris.append(t + base)
            base += (n + 1) * (n + 1)
    v = np.concatenate(verts) * np.asarray(size, np.float64)
    v = v @ _yaw(yaw_deg).T + np.asarray(center, np.float64)
    return v, np.concatenate(tris)


def uv_sphere_mesh(center, radius, nu=50, nv=26):
    """UV sphere: nu slices, nv stacks, fans at the poles (nu*(2*nv-2) triangles)."""
    th = np.linspace(0.0, math.pi, nv + 1)[1:-1]
    ph = np.linspace(0.0, 2 * math.pi, nu, endpoint=False)
    T, P = np.meshgrid(th, ph, indexing="ij")
    ring = np.stack([np.sin(T) * np.cos(P), np.cos(T), np.sin(T) * np.sin(P)], -1).reshape(-1, 3)
    v = np.concatenate([[[0.0, 1.0, 0.0]], ring, [[0.0, -1.0, 0.0]]])
    top, bot = 0, v.shape[0] - 1
    r0 = lambda k: 1 + k * nu  # first vertex of ring k
    tris = []
    j = np.arange(nu)
    jn = (j + 1) % nu
    tris.append(np.stack([np.full(nu, top), r0(0) + jn, r0(0) + j], -1))
    for k in range(nv - 2):
        a, b = r0(k) + j, r0(k) + jn
        c, d = r0(k + 1) + j, r0(k + 1) + jn
        tris.append(np.stack([a, b, d], -1))
        tris.append(np.stack([a, d, c], -1))
    tris.append(np.stack([np.full(nu, bot), r0(nv - 2) + j, r0(nv - 2) + jn], -1))
    return v * radius + np.asarray(center, np.float64), np.concatenate(tris)


def torus_mesh(R, r, nu, nv):
    u = np.linspace(0, 2 * math.pi, nu, endpoint=False)
    w = np.linspace(0, 2 * math.pi, nv, endpoint=False)
    U, W = np.meshgrid(u, w, indexing="ij")
    v = np.stack([(R + r * np.cos(W)) * np.cos(U), r * np.sin(W),
                  (R + r * np.cos(W)) * np.sin(U)], -1).reshape(-1, 3)
    i = np.arange(nu)[:, None]
    k = np.arange(nv)[None, :]
    a = i * nv + k
    b = ((i + 1) % nu) * nv + k
    c = ((i + 1) % nu) * nv + (k + 1) % nv
    d = i * nv + (k + 1) % nv
    t = np.concatenate([np.stack([a, d, c], -1).reshape(-1, 3), np.stack([a, c, b], -1).reshape(-1, 3)])
    return v, t


def blob_mesh(rng: SplitMix64, nu, nv):
    v, t = uv_sphere_mesh((0, 0, 0), 1.0, nu, nv)
    amp = rng.uniform(6, 0.03, 0.12)
    fr = rng.uniform(6, 1.0, 4.0)
    ph = rng.uniform(6, 0.0, 2 * math.pi)
    d = (amp[0] * np.sin(fr[0] * v[:, 0] + ph[0]) + amp[1] * np.sin(fr[1] * v[:, 1] + ph[1])
         + amp[2] * np.sin(fr[2] * v[:, 2] + ph[2]) + amp[3] * np.sin(fr[3] * (v[:, 0] + v[:, 2]) + ph[3]))
    return v * (1.0 + d)[:, None], t


# --------------------------------------------------------------- env map

def sky_env(width=2048, height=1024, sun_elev_deg=35.0, sun_azim_deg=40.0,
            sun_peak=5.0e4, sun_width_deg=0.5) -> np.ndarray:
    """Analytic sun plus sky gradient, evaluated at lat-long texel centres.

    Texel (ix, iy) has polar angle theta = pi*(iy+0.5)/H measured from +y and
    azimuth phi = 2*pi*(ix+0.5)/W, with direction
    (sin theta sin phi, cos theta, -sin theta cos phi).
    """
    th = math.pi * (np.arange(height) + 0.5) / height
    ph = 2 * math.pi * (np.arange(width) + 0.5) / width
    T, P = np.meshgrid(th, ph, indexing="ij")
    wx, wy, wz = np.sin(T) * np.sin(P), np.cos(T), -np.sin(T) * np.cos(P)
    e, a = math.radians(sun_elev_deg), math.radians(sun_azim_deg)
    sd = (math.cos(e) * math.sin(a), math.sin(e), -math.cos(e) * math.cos(a))
    cosg = np.clip(wx * sd[0] + wy * sd[1] + wz * sd[2], -1.0, 1.0)
    gam = np.degrees(np.arccos(cosg))
    sun = sun_peak * np.exp(-(gam / sun_width_deg) ** 2)
    up = wy >= 0
    sky = np.stack([0.3, 0.5, 1.0])[None, None, :] * (0.5 + 0.5 * wy)[..., None] \
        + 0.2 * ((1.0 - wy) ** 4)[..., None]
    ground = np.broadcast_to(np.array([0.10, 0.09, 0.08]), sky.shape)
    env = np.where(up[..., None], sky, ground) + sun[..., None] * np.array([1.0, 0.95, 0.9])
    return env.astype(np.float32)


def constant_env(value, width=16, height=8) -> np.ndarray:
    return np.broadcast_to(np.asarray(value, np.float32), (height, width, 3)).copy()


# ------------------------------------------------------------ the scenes

def cornell(seed: int = 1, width=128, height=128, spp=16, max_depth=8) -> Scene:
    """Cornell-style room: unit cube open at z=0, two yawed boxes, one ceiling quad light."""
    rng = SplitMix64(seed)
    b = _Builder()
    alb = rng.uniform(21, 0.2, 0.8).reshape(7, 3)
    m = [b.material(alb[k]) for k in range(7)]
    light = b.material((0, 0, 0), emission=(15.0, 15.0, 15.0))
    # walls face the interior
    b.quad((0, 0, 0), (0, 0, 1), (1, 0, 1), (1, 0, 0), m[0])   # floor, +y
    b.quad((0, 1, 0), (1, 1, 0), (1, 1, 1), (0, 1, 1), m[1])   # ceiling, -y
    b.quad((0, 0, 1), (0, 1, 1), (1, 1, 1), (1, 0, 1), m[2])   # back, -z
    b.quad((0, 0, 0), (0, 1, 0), (0, 1, 1), (0, 0, 1), m[3])   # left, +x
    b.quad((1, 0, 0), (1, 0, 1), (1, 1, 1), (1, 1, 0), m[4])   # right, -x
    v, t = box_mesh((0.32, 0.15, 0.40), (0.3, 0.3, 0.3), -17.0)
    b.mesh(v, t, m[5])
    v, t = box_mesh((0.67, 0.30, 0.67), (0.3, 0.6, 0.3), 17.0)
    b.mesh(v, t, m[6])
    h = 0.125
    y = 0.999
    b.quad((0.5 - h, y, 0.5 - h), (0.5 + h, y, 0.5 - h), (0.5 + h, y, 0.5 + h), (0.5 - h, y, 0.5 + h), light)
    cam = Camera((0.5, 0.5, -1.0), (0.5, 0.5, 0.0), (0.0, 1.0, 0.0), 45.0)
    return b.scene("cornell", cam, width, height, spp, max_depth)


def _random_surface_material(b: _Builder, rng: SplitMix64) -> int:
    alpha = float(rng.uniform(1, 0.05, 0.8)[0])
    rho = rng.uniform(3, 0.2, 0.8)
    return b.material(rho, roughness=alpha, flags=MAT_GGX)


def cornell_indirect(seed: int = 1, width=128, height=128, spp=64, max_depth=8) -> Scene:
    """The Cornell room with its light turned to face the ceiling 0.07 below
    it: every visible surface is lit only indirectly, through the bright spot
    the light throws on the ceiling."""
    sc = cornell(seed, width, height, spp, max_depth)
    em = np.nonzero(sc.emission.max(axis=1) > 0)[0]
    lt = np.isin(sc.tri_material, em)
    vids = np.unique(sc.indices[lt])
    sc.positions = sc.positions.copy()
    sc.positions[vids, 1] = np.float32(0.93)
    sc.indices = sc.indices.copy()
    sc.indices[lt] = sc.indices[lt][:, [0, 2, 1]]
    sc.name = "cornell_indirect"
    sc.validate()
    return sc


def grid_scene(seed: int = 2, width=1920, height=1080, spp=64, max_depth=12,
               grid=20, spacing=2.2) -> Scene:
    """Seeded grid of tessellated spheres and boxes on a ground plane, 256 textured emitters."""
    rng = SplitMix64(seed)
    b = _Builder()
    ground = b.material((0.5, 0.5, 0.5))
    L = 25.0
    b.quad((-L, 0, -L), (-L, 0, L), (L, 0, L), (L, 0, -L), ground)
    off = -0.5 * (grid - 1) * spacing
    for gx in range(grid):
        for gz in range(grid):
            jit = rng.uniform(2, -0.3, 0.3)
            kind = rng.uniform(1)[0]
            r = float(rng.uniform(1, 0.1, 1.0)[0])
            yaw = float(rng.uniform(1, 0.0, 90.0)[0])
            c = (off + gx * spacing + jit[0], r, off + gz * spacing + jit[1])
            mat = _random_surface_material(b, rng)
            if kind < 0.5:
                v, t = uv_sphere_mesh(c, r, 50, 26)
            else:
                v, t = box_mesh(c, (2 * r, 2 * r, 2 * r), yaw, subdiv=14)
            b.mesh(v, t, mat)
    h = 0.25
    for ex in range(16):
        for ez in range(8):
            jit = rng.uniform(2, -0.5, 0.5)
            E = 20.0 * rng.uniform(3, 0.5, 1.0)
            mat = b.material((0, 0, 0), emission=E, flags=MAT_EMIT_TEXTURE)
            cx = -22.0 + (ex + 0.5) * 44.0 / 16 + jit[0]
            cz = -22.0 + (ez + 0.5) * 44.0 / 8 + jit[1]
            y = 6.0
            b.quad((cx - h, y, cz - h), (cx + h, y, cz - h), (cx + h, y, cz + h), (cx - h, y, cz + h), mat)
    cam = Camera((0.0, 8.0, -30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 40.0)
    return b.scene("grid_1m", cam, width, height, spp, max_depth)


def _base_meshes(rng: SplitMix64):
    """Eight unit-scale meshes of roughly 40k-80k triangles, resting on y=0."""
    out = []
    specs = [("sphere", 160, 130), ("torus", 200, 120), ("box", 60, 0), ("blob", 180, 150),
             ("sphere", 200, 100), ("torus", 260, 150), ("box", 80, 0), ("blob", 220, 180)]
    for kind, a, c in specs:
        if kind == "sphere":
            v, t = uv_sphere_mesh((0, 0, 0), 1.0, a, c)
        elif kind == "torus":
            v, t = torus_mesh(0.8, 0.3, a, c)
        elif kind == "box":
            v, t = box_mesh((0, 0, 0), (1.6, 1.0, 1.2), 0.0, subdiv=a)
        else:
            v, t = blob_mesh(rng, a, c)
        v = v - np.array([0.0, v[:, 1].min(), 0.0])
        out.append((v, t))
    return out


def instanced_env_scene(seed: int = 3, width=1920, height=1080, spp=256, max_depth=16,
                        target_tris=4_000_000, env_size=(2048, 1024)) -> Scene:
    """Random instances of eight tessellated meshes (flattened) under a sun-and-sky map."""
    rng = SplitMix64(seed)
    b = _Builder()
    ground = b.material((0.5, 0.5, 0.5))
    L = 40.0
    b.quad((-L, 0, -L), (-L, 0, L), (L, 0, L), (L, 0, -L), ground)
    meshes = _base_meshes(rng)
    total = 2
    while total < target_tris:
        k = int(rng.uniform(1, 0, 8)[0])
        v, t = meshes[min(k, 7)]
        s = float(rng.uniform(1, 0.2, 1.5)[0])
        yaw = float(rng.uniform(1, 0.0, 360.0)[0])
        p = rng.uniform(2, -30.0, 30.0)
        w = (v * s) @ _yaw(yaw).T + np.array([p[0], 0.0, p[1]])
        b.mesh(w, t, _random_surface_material(b, rng))
        total += t.shape[0]
    cam = Camera((0.0, 8.0, -30.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 40.0)
    env = sky_env(*env_size)
    s = b.scene("instanced_env_4m", cam, width, height, spp, max_depth, env=env)
    return s


def slit_scene(seed: int = 3, width=1920, height=1080, spp=64, max_depth=16,
               target_tris=4_000_000, env_size=(2048, 1024)) -> Scene:
    """The instanced scene inside an enclosure whose roof leaves a 0.1-wide slit.

    Sunlight through the slit lands on a thin strip near x = -11; the camera
    stands at x = -5 and looks towards +x, at the half of the enclosure the
    strip does not reach, so every pixel it sees is lit indirectly."""
    s = instanced_env_scene(seed, width, height, spp, max_depth, target_tris, env_size)
    b = _Builder()
    b.pos = [s.positions.astype(np.float64)]
    b.idx = [s.indices.astype(np.int64)]
    b.mat = [s.tri_material.astype(np.int64)]
    b.nv = s.positions.shape[0]
    b.albedo = list(s.albedo.astype(np.float64))
    b.rough = list(s.roughness.astype(np.float64))
    b.emis = list(s.emission.astype(np.float64))
    b.flags = list(s.mat_flags.astype(np.int64))
    wall = b.material((0.5, 0.5, 0.5))
    X, Y, Z = 32.0, 12.0, 32.0
    # inward-facing walls
    b.quad((-X, 0, Z), (-X, Y, Z), (X, Y, Z), (X, 0, Z), wall)        # z=+Z, normal -z
    b.quad((-X, 0, -Z), (X, 0, -Z), (X, Y, -Z), (-X, Y, -Z), wall)    # z=-Z, normal +z
    b.quad((-X, 0, -Z), (-X, Y, -Z), (-X, Y, Z), (-X, 0, Z), wall)    # x=-X, normal +x
    b.quad((X, 0, -Z), (X, 0, Z), (X, Y, Z), (X, Y, -Z), wall)        # x=+X, normal -x
    w = 0.05
    b.quad((-X, Y, -Z), (-w, Y, -Z), (-w, Y, Z), (-X, Y, Z), wall)    # roof, normal -y
    b.quad((w, Y, -Z), (X, Y, -Z), (X, Y, Z), (w, Y, Z), wall)
    cam = Camera((-5.0, 4.0, 0.0), (32.0, 3.0, 0.0), (0.0, 1.0, 0.0), 40.0)
    return b.scene("slit_enclosure", cam, width, height, spp, max_depth, env=s.env)


def city(seed: int = 5, width=3840, height=2160, spp=1024, max_depth=16,
         blocks=64, target_tris=16_000_000, emissive_cells=5000) -> Scene:
    """Procedural city of extruded boxes whose facades are split into 1 x 1.5 window cells."""
    rng = SplitMix64(seed)
    nb = blocks * blocks
    fw = rng.uniform(nb, 4.0, 20.0)
    fd = rng.uniform(nb, 4.0, 20.0)
    hh = rng.uniform(nb, 10.0, 120.0)
    # scale heights so the facade cell count lands near the triangle target
    cells = lambda h: (np.ceil(fw / 1.0) * 2 + np.ceil(fd / 1.0) * 2) * np.ceil(h / 1.5)
    scale = min(1.0, target_tris / (2.0 * cells(hh).sum()))
    hh = np.maximum(10.0, hh * scale)
    spacing = 24.0
    b = _Builder()
    ground = b.material((0.3, 0.3, 0.3))
    facade_mats = [b.material(rng.uniform(3, 0.2, 0.7), roughness=float(rng.uniform(1, 0.1, 0.6)[0]),
                              flags=MAT_GGX) for _ in range(8)]
    L = blocks * spacing * 0.5 + 20
    b.quad((-L, 0, -L), (-L, 0, L), (L, 0, L), (L, 0, -L), ground)
    pos_chunks, idx_chunks, mat_chunks = [], [], []
    nv = 4
    facades = []   # (first triangle after the ground plane, cells) per facade
    ntri = 0
    for k in range(nb):
        gx, gz = k % blocks, k // blocks
        cx = (gx - blocks / 2 + 0.5) * spacing
        cz = (gz - blocks / 2 + 0.5) * spacing
        w, d, h = fw[k], fd[k], hh[k]
        nx, nz, ny = int(math.ceil(w)), int(math.ceil(d)), int(math.ceil(h / 1.5))
        corners = [(cx - w / 2, cz - d / 2), (cx + w / 2, cz - d / 2),
                   (cx + w / 2, cz + d / 2), (cx - w / 2, cz + d / 2)]
        mat = facade_mats[k % 8]
        for f in range(4):
            (x0, z0), (x1, z1) = corners[f], corners[(f + 1) % 4]
            nseg = nx if f % 2 == 0 else nz
            s = np.linspace(0, 1, nseg + 1)
            yv = np.linspace(0, h, ny + 1)
            S, Yv = np.meshgrid(s, yv, indexing="ij")
            P = np.stack([x0 + (x1 - x0) * S, Yv, z0 + (z1 - z0) * S], -1).reshape(-1, 3)
            i = np.arange(nseg)[:, None] * (ny + 1) + np.arange(ny)[None, :]
            q0, q1, q2, q3 = i, i + (ny + 1), i + (ny + 2), i + 1
            # outward normal: edge (x1-x0) x up points outward for a counter-clockwise footprint seen from below
            t = np.concatenate([np.stack([q0, q3, q2], -1).reshape(-1, 3),
                                np.stack([q0, q2, q1], -1).reshape(-1, 3)])
            facades.append((ntri, nseg * ny))   # first triangle, cells (triangle j and j + cells)
            ntri += t.shape[0]
            pos_chunks.append(P)
            idx_chunks.append(t + nv)
            mat_chunks.append(np.full(t.shape[0], mat, np.int64))
            nv += P.shape[0]
        # roof
        P = np.array([[corners[j][0], h, corners[j][1]] for j in range(4)])
        pos_chunks.append(P)
        idx_chunks.append(np.array([[0, 2, 1], [0, 3, 2]]) + nv)
        mat_chunks.append(np.full(2, mat, np.int64))
        nv += 4
        ntri += 2
    pos = np.concatenate([np.concatenate(b.pos)] + pos_chunks)
    idx = np.concatenate([np.concatenate(b.idx)] + idx_chunks)
    mat = np.concatenate([np.concatenate(b.mat)] + mat_chunks)
    # emissive window cells: both triangles of a picked facade cell get that
    # cell's own material (lognormal intensity, warm tint)
    starts = np.array([f[0] for f in facades], np.int64)
    cells = np.array([f[1] for f in facades], np.int64)
    first_cell = np.concatenate([[0], np.cumsum(cells)[:-1]])
    total = int(cells.sum())
    pick = np.unique(rng.uniform(emissive_cells * 2, 0, total).astype(np.int64))[:emissive_cells]
    face = np.searchsorted(first_cell, pick, side="right") - 1
    local = pick - first_cell[face]
    tri_a = 2 + starts[face] + local                 # the ground plane's 2 triangles come first
    tri_b = tri_a + cells[face]
    tint = np.array([1.0, 0.8, 0.55])
    E = np.exp(math.log(5.0) + 1.2 * rng.normal(pick.shape[0]))
    base_m = len(b.albedo)
    for j in range(pick.shape[0]):
        b.material((0.0, 0.0, 0.0), emission=E[j] * tint)
    mat[tri_a] = base_m + np.arange(pick.shape[0])
    mat[tri_b] = base_m + np.arange(pick.shape[0])
    b.pos, b.idx, b.mat, b.nv = [pos], [idx], [mat], pos.shape[0]
    cam = Camera((0.0, 260.0, -900.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0)
    return b.scene("city_16m", cam, width, height, spp, max_depth)


# ------------------------------------------------------------- test scenes

def furnace(E=1.0, rho=0.5, width=8, height=8, max_depth=8) -> Scene:
    """Closed cube [-1,1]^3, every face emitting E and reflecting rho; camera inside."""
    b = _Builder()
    m = b.material((rho, rho, rho), emission=(E, E, E))
    v, t = box_mesh((0, 0, 0), (2.0, 2.0, 2.0), 0.0, subdiv=1, inward=True)
    b.mesh(v, t, m)
    cam = Camera((0.1, -0.2, 0.05), (0.3, 0.2, 1.0), (0.0, 1.0, 0.0), 70.0)
    return b.scene("furnace", cam, width, height, 1, max_depth)


def convex_under_env(rho=0.6, E=2.0, width=8, height=8, max_depth=4) -> Scene:
    """A Lambert box seen from outside under a constant environment of radiance E."""
    b = _Builder()
    m = b.material((rho, rho, rho))
    v, t = box_mesh((0, 0, 0), (1.0, 1.0, 1.0), 30.0, subdiv=2)
    b.mesh(v, t, m)
    cam = Camera((0.4, 0.5, -3.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0)
    return b.scene("convex_env", cam, width, height, 1, max_depth, env=constant_env((E, E, E)))


def quad_over_plane(rho=0.7, Le=4.0, width=1, height=1, max_depth=2, subdiv=1) -> Scene:
    """A one-sided square emitter above a Lambert plane; a narrow camera looks at one point.
    subdiv > 1 splits the emitter into subdiv x subdiv cells (two triangles each)."""
    b = _Builder()
    m = b.material((rho, rho, rho))
    light = b.material((0, 0, 0), emission=(Le, Le, Le))
    L = 10.0
    b.quad((-L, 0, -L), (-L, 0, L), (L, 0, L), (L, 0, -L), m)
    y = 1.0
    xs = np.linspace(-0.3, 0.5, subdiv + 1)
    zs = np.linspace(-0.2, 0.4, subdiv + 1)
    for i in range(subdiv):
        for j in range(subdiv):
            b.quad((xs[i], y, zs[j]), (xs[i + 1], y, zs[j]), (xs[i + 1], y, zs[j + 1]), (xs[i], y, zs[j + 1]),
                   light)
    cam = Camera((3.0, 2.0, 0.0), (0.2, 0.0, 0.1), (0.0, 1.0, 0.0), 0.002)
    s = b.scene("quad_over_plane", cam, width, height, 1, max_depth)
    s.extra["target"] = (0.2, 0.0, 0.1)
    s.extra["light_quad"] = [(-0.3, y, -0.2), (0.5, y, -0.2), (0.5, y, 0.4), (-0.3, y, 0.4)]
    return s


def light_field(seed: int = 11, n_lights=2000, width=64, height=48, max_depth=6, env=False) -> Scene:
    """Many small one-sided triangle lights of random orientation, size and
    power (log-uniform over two decades) above a Lambert floor with a few
    boxes: about half of them face away from the floor. The setting of a
    light hierarchy: the flux-proportional choice wastes most shadow rays."""
    rng = SplitMix64(seed)
    b = _Builder()
    floor = b.material((0.6, 0.6, 0.6))
    grey = b.material((0.5, 0.45, 0.4))
    L = 20.0
    b.quad((-L, 0, -L), (-L, 0, L), (L, 0, L), (L, 0, -L), floor)
    for k in range(6):
        c = (rng.uniform(1, -12, 12)[0], 1.0, rng.uniform(1, -12, 12)[0])
        v, t = box_mesh(c, (2.0, 2.0, 2.0), float(rng.uniform(1, 0, 90)[0]))
        b.mesh(v, t, grey)
    cen = np.stack([rng.uniform(n_lights, -15, 15), rng.uniform(n_lights, 0.5, 6.0),
                    rng.uniform(n_lights, -15, 15)], 1)
    nrm = np.stack([rng.normal(n_lights) for _ in range(3)], 1)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    size = rng.uniform(n_lights, 0.1, 0.4)
    power = 10.0 ** rng.uniform(n_lights, -0.3, 1.7)
    hue = rng.uniform(n_lights, 0.5, 1.0)
    # two tangents per light; corners counter-clockwise seen from the front
    a = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(nrm, a)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    for k in range(n_lights):
        m = b.material((0, 0, 0), emission=(power[k], power[k] * hue[k], power[k] * hue[k] * hue[k]))
        p0 = cen[k] + size[k] * t1[k]
        p1 = cen[k] + size[k] * (-0.5 * t1[k] + 0.866 * t2[k])
        p2 = cen[k] + size[k] * (-0.5 * t1[k] - 0.866 * t2[k])
        b.mesh(np.array([p0, p1, p2]), np.array([[0, 1, 2]]), m)
    cam = Camera((0.0, 14.0, -26.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0)
    e = sky_env(64, 32) * 0.2 if env else None
    return b.scene("light_field", cam, width, height, 1, max_depth, env=e)


# ----------------------------------------------------------- guide inputs

GUIDE_SIZES = (32, 64, 64, 64, 40)


def guide_init(seed: int = 7) -> np.ndarray:
    """Initial FP32 parameters of the 32-64-64-64-40 network, He-uniform weights
    (bound sqrt(6 / fan_in)) and zero biases, packed layer by layer as W (in x out,
    row-major) then b. These are input data drawn from the seeded generator."""
    rng = SplitMix64(seed)
    out = []
    for fi, fo in zip(GUIDE_SIZES[:-1], GUIDE_SIZES[1:]):
        lim = math.sqrt(6.0 / fi)
        out.append(rng.uniform(fi * fo, -lim, lim))
        out.append(np.zeros(fo))
    return np.concatenate(out).astype(np.float32)


def guide_frozen(seed: int = 5, gain: float = 3.0, kappa_bias: float = 4.0) -> np.ndarray:
    """Parameters of a fixed, untrained network whose mixtures are far from
    uniform: He-uniform hidden layers as in guide_init, the output layer's
    weights scaled by `gain` (uneven lobe weights, varied concentrations) and
    `kappa_bias` on every lobe's concentration output (median kappa about 4).
    Input data for parity tests of guided rendering."""
    p = guide_init(seed).astype(np.float64)
    o = sum(fi * fo + fo for fi, fo in zip(GUIDE_SIZES[:-2], GUIDE_SIZES[1:-1]))
    fi, fo = GUIDE_SIZES[-2], GUIDE_SIZES[-1]
    p[o:o + fi * fo] *= gain
    p[o + fi * fo + 4:o + fi * fo + fo:5] = kappa_bias
    return p.astype(np.float32)


# the named workloads, each with its fixed seed; the slit enclosure reuses the
# instanced scene's seed (it is that scene plus a roof)
WORKLOADS = {
    "cornell": (cornell, 1),
    "grid_1m": (grid_scene, 2),
    "instanced_env_4m": (instanced_env_scene, 3),
    "slit_enclosure": (slit_scene, 3),
    "city_16m": (city, 5),
}


def workload(name: str, **kw) -> Scene:
    """One of the named workload scenes, from its fixed seed."""
    fn, seed = WORKLOADS[name]
    kw.setdefault("seed", seed)
    return fn(**kw)
