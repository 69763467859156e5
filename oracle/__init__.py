"""CPU oracle for the progressive QMC path tracer -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package. It shares no code with the GPU
library; both read their inputs from :mod:`scenegen`.

The arithmetic lives in ``qpt_oracle.c`` (plain C, FP64 path tracing, exact
128-bit radical inverses, FP32 brute-force watertight hits) and, for the
learned proposal, in :mod:`oracle.guide` (numpy, FP64).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qpt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fused multiply-add contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        u32, u64, i32 = C.c_uint32, C.c_uint64, C.c_int
        L.or_dim_base.argtypes = [u32]
        L.or_dim_base.restype = u32
        L.or_scramble_mult.argtypes = [u32]
        L.or_scramble_mult.restype = u32
        L.or_ri_bits.argtypes = [u64, u32, u32]
        L.or_ri_bits.restype = u32
        L.or_enum_params.argtypes = [u32, u32, P, P, P]
        L.or_pixel_index.argtypes = [u32, u32, u32, u32, u64]
        L.or_pixel_index.restype = u64
        L.or_sample_bits.argtypes = [u64, u32, u32, u32, i32]
        L.or_sample_bits.restype = u32
        L.or_sample_bits_batch.argtypes = [P, P, u32, u32, u32, i32, P]
        L.or_trace_f32.argtypes = [P, P, u32, P, u32, i32, P, P, P]
        L.or_alias_build.argtypes = [u32, P, P, P]
        L.or_scene_create.argtypes = [u32, P, u32, P, P, u32, P, P, P, P, u32, u32, P, P,
                                      u32, u32, i32]
        L.or_scene_create.restype = P
        L.or_scene_destroy.argtypes = [P]
        L.or_scene_num_emitters.argtypes = [P]
        L.or_scene_num_emitters.restype = u32
        L.or_scene_lights.argtypes = [P, P, P, P, P, P]
        L.or_scene_env_tables.argtypes = [P, P, P, P]
        L.or_trace64.argtypes = [P, P, u32, i32, i32, P, P]
        L.or_render.argtypes = [P, u32, u32, u32, u32, P, u32, u64, u32, P, P, P, u32]
        L.or_render.restype = u64
        L.or_camera_ray.argtypes = [P, C.c_double, C.c_double, P, P]
        L.or_bsdf.argtypes = [P, u32, P, P, P, P, P]
        L.or_bsdf_sample.argtypes = [P, u32, P, P, C.c_double, C.c_double, C.c_double, P]
        L.or_bsdf_sample.restype = i32
        L.or_env_lookup.argtypes = [P, P, P]
        L.or_env_lookup.restype = C.c_double
        L.or_bsdf_batch.argtypes = [P, u32, P, P, P, u32, P, P]
        L.or_bsdf_sample_batch.argtypes = [P, u32, P, P, P, u32, P, P]
        L.or_debug_path.argtypes = [P, u32, u32, u32, u32, u32, u32, u64, P, P, u32]
        L.or_debug_path.restype = u32
        L.or_env_pyramid.argtypes = [P, P, P, P, P, P]
        L.or_env_descend.argtypes = [P, P, P, P, i32, u32, P, P, P]
        L.or_env_bin.argtypes = [P]
        L.or_env_bin.restype = u32
        L.or_light_tree.argtypes = [P, P, P, P, P, P, P, P]
        L.or_light_tree.restype = u32
        L.or_light_tree_sample.argtypes = [P, P, P, P, u32, P, P]
        L.or_light_tree_sizes.argtypes = [P, P, P, P]
        L.or_light_tree_estimate.argtypes = [P, u32, P, P]
        L.or_light_tree_estimate.restype = C.c_float
        L.or_light_tree_left_q.argtypes = [P, u32, P, P]
        L.or_light_tree_left_q.restype = u32
        L.or_ggx_D.argtypes = [C.c_double, C.c_double]
        L.or_ggx_D.restype = C.c_double
        L.or_round_bf16.argtypes = [C.c_double]
        L.or_round_bf16.restype = C.c_double
        L.or_round_fp16.argtypes = [C.c_double]
        L.or_round_fp16.restype = C.c_double
        L.or_guide_set.argtypes = [P, P, u32, u32, u32]
        L.or_guide_mix.argtypes = [P, P, P, u32, P]
        L.or_guide_forward.argtypes = [P, P, P, u32, P, P]
        L.or_guide_mix_eval.argtypes = [P, P, P, u32, P, P]
        L.or_plant.argtypes = [i32]
        L.or_rec_hash.argtypes = [u64, u32]
        L.or_rec_hash.restype = u32
        L.or_records.argtypes = [P, u32, u32, u32, u32, P, u32, u64, u32, P, P, u32, P, u32]
        L.or_records.restype = u32
        _lib = L
    return _lib


ENV_BINS = 256  # normal bins of the environment pyramid (16 x 16 octahedral)


def env_bin(n) -> int:
    """Normal bin of an FP32 normal (octahedral map, +y up)."""
    n = np.ascontiguousarray(n, np.float32)
    return int(lib().or_env_bin(_p(n)))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


# ----------------------------------------------------------------- Halton

def dim_base(d: int) -> int:
    return lib().or_dim_base(d)


def scramble_mult(b: int) -> int:
    return lib().or_scramble_mult(b)


def ri_bits(i: int, b: int, f: int = 1) -> int:
    """floor(2^32 * scrambled radical inverse of i in base b)."""
    return lib().or_ri_bits(i, b, f)


def enum_params(W: int, H: int):
    k, l, S = C.c_uint32(), C.c_uint32(), C.c_uint64()
    lib().or_enum_params(W, H, C.byref(k), C.byref(l), C.byref(S))
    return k.value, l.value, S.value


def pixel_index(W: int, H: int, px: int, py: int, j: int) -> int:
    return lib().or_pixel_index(W, H, px, py, j)


def pixel_indices(W: int, H: int, j: int) -> np.ndarray:
    out = np.empty(W * H, np.uint64)
    L = lib()
    for py in range(H):
        for px in range(W):
            out[py * W + px] = L.or_pixel_index(W, H, px, py, j)
    return out


def sample_bits(idx: np.ndarray, dim: np.ndarray, W: int, H: int, scramble: bool = True) -> np.ndarray:
    idx = np.ascontiguousarray(idx, np.uint64)
    dim = np.ascontiguousarray(dim, np.uint32)
    out = np.empty(idx.shape[0], np.uint32)
    lib().or_sample_bits_batch(_p(idx), _p(dim), idx.shape[0], W, H, int(scramble), _p(out))
    return out


# ------------------------------------------------------------ intersection

def trace_f32(scene, rays: np.ndarray, any_hit: bool = False):
    """Brute-force FP32 watertight closest hit (or occlusion) for n x 8 float rays."""
    rays = np.ascontiguousarray(rays, np.float32)
    n = rays.shape[0]
    t = np.empty(n, np.float32)
    tri = np.empty(n, np.uint32)
    b = np.empty((n, 2), np.float32)
    pos = np.ascontiguousarray(scene.positions, np.float32)
    idx = np.ascontiguousarray(scene.indices, np.uint32)
    lib().or_trace_f32(_p(pos), _p(idx), idx.shape[0], _p(rays), n, int(any_hit), _p(t), _p(tri), _p(b))
    return t, tri, b


def alias_build(w: np.ndarray):
    w = np.ascontiguousarray(w, np.float64)
    prob = np.empty_like(w)
    alias = np.empty(w.shape[0], np.uint32)
    lib().or_alias_build(w.shape[0], _p(w), _p(prob), _p(alias))
    return prob, alias


# ------------------------------------------------------------- the scene

class Scene:
    """The oracle's own copy of a scenegen scene (FP64, own BVH and tables)."""

    def __init__(self, sc, build_bvh: bool = True):
        L = lib()
        self.sc = sc
        self._keep = []
        pos = np.ascontiguousarray(sc.positions, np.float32)
        idx = np.ascontiguousarray(sc.indices, np.uint32)
        tm = np.ascontiguousarray(sc.tri_material, np.uint32)
        alb = np.ascontiguousarray(sc.albedo, np.float32)
        rough = np.ascontiguousarray(sc.roughness, np.float32)
        emis = np.ascontiguousarray(sc.emission, np.float32)
        flags = np.ascontiguousarray(sc.mat_flags, np.uint32)
        cam = np.array(list(sc.camera.eye) + list(sc.camera.look) + list(sc.camera.up)
                       + [sc.camera.vfov_deg], np.float64)
        if sc.env is not None:
            env = np.ascontiguousarray(sc.env, np.float32)
            eh, ew = env.shape[:2]
        else:
            env, eh, ew = None, 0, 0
        self._keep = [pos, idx, tm, alb, rough, emis, flags, cam, env]
        self.h = L.or_scene_create(pos.shape[0], _p(pos), idx.shape[0], _p(idx), _p(tm), alb.shape[0],
                                   _p(alb), _p(rough), _p(emis), _p(flags), ew, eh, _p(env), _p(cam),
                                   sc.width, sc.height, int(build_bvh))
        self.W, self.H = sc.width, sc.height

    def __del__(self):
        try:
            if self.h:
                lib().or_scene_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def lights(self):
        L = lib()
        ne = L.or_scene_num_emitters(self.h)
        tri = np.empty(ne, np.uint32)
        flux = np.empty(ne, np.float64)
        prob = np.empty(ne, np.float64)
        alias = np.empty(ne, np.uint32)
        pmf = np.empty(ne, np.float64)
        L.or_scene_lights(self.h, _p(tri), _p(flux), _p(prob), _p(alias), _p(pmf))
        return dict(tri=tri, flux=flux, prob=prob, alias=alias, pmf=pmf)

    def env_pyramid(self):
        """The environment pyramid's tables (Sec. 2.1.2; see the C source)."""
        L = lib()
        m, top, root = C.c_uint32(), C.c_uint32(), C.c_uint32()
        L.or_env_pyramid(self.h, C.byref(m), C.byref(top), C.byref(root), None, None)
        m, top, root = m.value, top.value, root.value
        if not m:
            return dict(m=0)
        q = np.empty(4 * (2 * (4 ** m - 1) // 3), np.uint32)
        oq = np.empty(ENV_BINS * 4 * (1 + 2 * (4 ** top - 1) // 3), np.uint32)
        L.or_env_pyramid(self.h, C.byref(C.c_uint32()), C.byref(C.c_uint32()), C.byref(C.c_uint32()), _p(q), _p(oq))
        return dict(m=m, top=top, root=root, q=q, oq=oq.reshape(ENV_BINS, -1))

    def env_descend(self, bins, u=None, v=None, rows=None, cols=None):
        """Pyramid descents: with u, v sample; with rows, cols steer to those
        texels. Returns rows, cols and the final intervals (ru, su, rv, sv)."""
        bins = np.ascontiguousarray(bins, np.int32)
        n = bins.shape[0]
        steer = rows is not None
        u = np.ascontiguousarray(np.zeros(n) if u is None else u, np.uint32)
        v = np.ascontiguousarray(np.zeros(n) if v is None else v, np.uint32)
        r = np.ascontiguousarray(np.zeros(n) if rows is None else rows, np.uint32)
        c = np.ascontiguousarray(np.zeros(n) if cols is None else cols, np.uint32)
        iv = np.empty((n, 4), np.uint64)
        lib().or_env_descend(self.h, _p(bins), _p(u), _p(v), int(steer), n, _p(r), _p(c), _p(iv))
        return r, c, iv

    def light_tree(self):
        """The light tree's tables (Sec. 2.1.1 hierarchy, see the C source)."""
        L = lib()
        nn = L.or_light_tree(self.h, None, None, None, None, None, None, None)
        ne = L.or_scene_num_emitters(self.h)
        t = dict(center=np.empty((nn, 4), np.float32), flux=np.empty((nn, 6), np.float32),
                 left=np.empty(nn, np.int32), first=np.empty(nn, np.uint32), count=np.empty(nn, np.uint32),
                 emit=np.empty(ne, np.uint32), w=np.empty(ne, np.uint32))
        if nn:
            L.or_light_tree(self.h, _p(t["center"]), _p(t["flux"]), _p(t["left"]), _p(t["first"]),
                            _p(t["count"]), _p(t["emit"]), _p(t["w"]))
        return t

    def light_tree_sample(self, S, x, n):
        S = np.ascontiguousarray(S, np.uint64)
        x = np.ascontiguousarray(x, np.float32).reshape(-1, 3)
        n = np.ascontiguousarray(n, np.float32).reshape(-1, 3)
        e = np.empty(S.shape[0], np.uint32)
        size = np.empty(S.shape[0], np.uint64)
        lib().or_light_tree_sample(self.h, _p(S), _p(x), _p(n), S.shape[0], _p(e), _p(size))
        return e, size

    def light_tree_sizes(self, x, n):
        """Interval size (selection probability times 2^63) of every emitter."""
        x = np.ascontiguousarray(x, np.float32)
        n = np.ascontiguousarray(n, np.float32)
        out = np.empty(lib().or_scene_num_emitters(self.h), np.uint64)
        lib().or_light_tree_sizes(self.h, _p(x), _p(n), _p(out))
        return out

    def light_tree_estimate(self, node, x, n):
        x = np.ascontiguousarray(x, np.float32)
        n = np.ascontiguousarray(n, np.float32)
        return float(lib().or_light_tree_estimate(self.h, node, _p(x), _p(n)))

    def light_tree_left_q(self, node, x, n):
        x = np.ascontiguousarray(x, np.float32)
        n = np.ascontiguousarray(n, np.float32)
        return int(lib().or_light_tree_left_q(self.h, node, _p(x), _p(n)))

    def env_tables(self):
        env = self.sc.env
        eh, ew = env.shape[:2]
        rq = np.empty(eh + 1, np.uint64)
        cq = np.empty(eh * (ew + 1), np.uint64)
        pdf = np.empty(eh * ew, np.float64)
        lib().or_scene_env_tables(self.h, _p(rq), _p(cq), _p(pdf))
        return rq, cq.reshape(eh, ew + 1), pdf.reshape(eh, ew)

    def trace64(self, rays: np.ndarray, any_hit=False, brute=False):
        rays = np.ascontiguousarray(rays, np.float64)
        n = rays.shape[0]
        t = np.empty(n, np.float64)
        tri = np.empty(n, np.int64)
        lib().or_trace64(self.h, _p(rays), n, int(any_hit), int(brute), _p(t), _p(tri))
        return t, tri

    def guide_set(self, params, alpha: float = 0.0, max_vertex: int = 0, rec_thr: int = 0xFFFFFFFF):
        """Load a frozen guide (13032 FP32 parameters, rounded to BF16 here),
        mixed in with probability alpha (its integer threshold round(alpha 2^32))
        at vertices 1..max_vertex (0 = all) when a render passes guide=True."""
        par = np.ascontiguousarray(params, np.float32)
        assert par.shape == (13032,)
        thr = min(int(round(float(alpha) * 2.0 ** 32)), 0xFFFFFFFF)
        lib().or_guide_set(self.h, _p(par), thr, int(max_vertex), int(rec_thr))
        self.guide_alpha_thr = thr

    def guide_mix(self, x, wo):
        """The frozen guide's mixture at vertices x with outgoing wo: weights (n x 8),
        means (n x 8 x 3), concentrations (n x 8), after the FP16 storage step."""
        x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
        wo = np.ascontiguousarray(wo, np.float64).reshape(-1, 3)
        out = np.empty((x.shape[0], 40))
        lib().or_guide_mix(self.h, _p(x), _p(wo), x.shape[0], _p(out))
        lob = out[:, 8:].reshape(-1, 8, 4)
        return out[:, :8], lob[:, :, :3], lob[:, :, 3]

    def guide_forward(self, x, wo):
        """Features (n x 32) and network outputs (n x 40) of the frozen guide."""
        x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
        wo = np.ascontiguousarray(wo, np.float64).reshape(-1, 3)
        f = np.empty((x.shape[0], 32))
        o = np.empty((x.shape[0], 40))
        lib().or_guide_forward(self.h, _p(x), _p(wo), x.shape[0], _p(f), _p(o))
        return f, o

    def records(self, pixels=None, pass0=0, npasses=1, max_depth=None, rr=True, mode=0, scramble=True,
                guide=True, nthreads=None, cap=1 << 22):
        """Render like `render` and return (sums, counts, records): the
        training records of every path (pixel, pass, vertex, x, wo, wi, pdf,
        weight, and nee: the luminance-weighted quotient of the vertex's own
        next-event estimate that the weight leaves out), in no particular order."""
        sc = self.sc
        mode = int(mode) | (0x1000 if guide else 0)
        pix = None if pixels is None else np.ascontiguousarray(pixels, np.uint32)
        npix = sc.width * sc.height if pix is None else pix.shape[0]
        s = np.zeros((npix, 3))
        cnt = np.zeros(npix, np.uint32)
        out = np.empty((cap, 15))
        n = lib().or_records(self.h, max_depth or sc.max_depth, int(rr), mode, int(scramble), _p(pix), npix,
                             pass0, npasses, _p(s), _p(cnt), nthreads or os.cpu_count() or 1, _p(out), cap)
        assert n <= cap, "record buffer too small"
        o = out[:n]
        rec = dict(pixel=o[:, 0].astype(np.int64), pass_=o[:, 1].astype(np.int64), vertex=o[:, 2].astype(np.int64),
                   x=o[:, 3:6], wo=o[:, 6:9], wi=o[:, 9:12], pdf=o[:, 12], weight=o[:, 13], nee=o[:, 14])
        return s, cnt, rec

    def render(self, pixels=None, pass0=0, npasses=1, max_depth=None, rr=True, mode=0,
               scramble=True, nthreads=None, light_tree=False, env_sampling=0, gauss=False, guide=False):
        """FP64 sums, sums of squares and counts for the listed pixel ids (y*W+x).
        light_tree selects triangle lights through the light tree instead of
        the flux alias table; env_sampling 1 / 2 samples the environment by its
        pyramid (2: with normal-weighted top levels) instead of the 2D CDF;
        gauss draws film samples from the Gaussian pixel filter; guide mixes in
        the frozen guide of `guide_set`."""
        mode = (int(mode) | (0x100 if light_tree else 0) | (int(env_sampling) << 9) | (0x800 if gauss else 0)
                | (0x1000 if guide else 0))
        sc = self.sc
        if max_depth is None:
            max_depth = sc.max_depth
        if pixels is None:
            pix = None
            npix = sc.width * sc.height
        else:
            pix = np.ascontiguousarray(pixels, np.uint32)
            npix = pix.shape[0]
        s = np.zeros((npix, 3), np.float64)
        s2 = np.zeros((npix, 3), np.float64)
        cnt = np.zeros(npix, np.uint32)
        nth = nthreads or os.cpu_count() or 1
        rays = lib().or_render(self.h, max_depth, int(rr), mode, int(scramble), _p(pix), npix, pass0,
                               npasses, _p(s), _p(s2), _p(cnt), nth)
        return s, s2, cnt, int(rays)

    def camera_ray(self, fx, fy):
        o = np.empty(3)
        d = np.empty(3)
        lib().or_camera_ray(self.h, fx, fy, _p(o), _p(d))
        return o, d

    def bsdf(self, m, n, wo, wi):
        n, wo, wi = (np.ascontiguousarray(v, np.float64) for v in (n, wo, wi))
        f = np.empty(3)
        pdf = np.empty(1)
        lib().or_bsdf(self.h, m, _p(n), _p(wo), _p(wi), _p(f), _p(pdf))
        return f, float(pdf[0])

    def bsdf_sample(self, m, n, wo, u3, u4, u5):
        n, wo = (np.ascontiguousarray(v, np.float64) for v in (n, wo))
        wi = np.empty(3)
        ok = lib().or_bsdf_sample(self.h, m, _p(n), _p(wo), u3, u4, u5, _p(wi))
        return bool(ok), wi

    def bsdf_batch(self, m, n, wo, wi):
        n, wo = (np.ascontiguousarray(v, np.float64) for v in (n, wo))
        wi = np.ascontiguousarray(wi, np.float64).reshape(-1, 3)
        f = np.empty_like(wi)
        pdf = np.empty(wi.shape[0])
        lib().or_bsdf_batch(self.h, m, _p(n), _p(wo), _p(wi), wi.shape[0], _p(f), _p(pdf))
        return f, pdf

    def bsdf_sample_batch(self, m, n, wo, u):
        n, wo = (np.ascontiguousarray(v, np.float64) for v in (n, wo))
        u = np.ascontiguousarray(u, np.float64).reshape(-1, 3)
        wi = np.empty_like(u)
        ok = np.empty(u.shape[0], np.int32)
        lib().or_bsdf_sample_batch(self.h, m, _p(n), _p(wo), _p(u), u.shape[0], _p(wi), _p(ok))
        return ok.astype(bool), wi

    def debug_path(self, px, py, pass_, max_depth=None, rr=True, mode=0, scramble=True, light_tree=False,
                   env_sampling=0):
        mode = int(mode) | (0x100 if light_tree else 0) | (int(env_sampling) << 9)
        L = np.empty(3)
        log = np.zeros(8 * 256)
        n = lib().or_debug_path(self.h, max_depth or self.sc.max_depth, int(rr), mode, int(scramble), px, py,
                                pass_, _p(L), _p(log), log.shape[0])
        return L, log[:n].reshape(-1, 8)

    def env_lookup(self, w):
        w = np.ascontiguousarray(w, np.float64)
        rgb = np.empty(3)
        pdf = lib().or_env_lookup(self.h, _p(w), _p(rgb))
        return rgb, pdf


def ggx_D(cos_h: float, alpha: float) -> float:
    return lib().or_ggx_D(cos_h, alpha)


def round_bf16(x: float) -> float:
    """Nearest BF16 value (ties to even) of an FP64 number."""
    return lib().or_round_bf16(float(x))


def round_fp16(x: float) -> float:
    """Nearest FP16 value (ties to even) of an FP64 number."""
    return lib().or_round_fp16(float(x))


def plant(which: int) -> None:
    """Plant a known mistake in the oracle (tests of the pins only; 0 = none):
    1 = the guide's mixture density reported twice too large, 2 = record
    weights not divided by the throughput before their vertex, 3 = record
    weights that keep their vertex's own next-event estimate."""
    lib().or_plant(int(which))


def rec_hash(idx: int, v: int) -> int:
    """The training-record hash of a path's sample index and a depth."""
    return lib().or_rec_hash(int(idx), int(v))


def guide_mix_eval(w, mu, kappa, dirs=None, u=None):
    """Density at dirs and samples from u (n x 3) of n explicit mixtures
    (weights n x 8, means n x 8 x 3, concentrations n x 8)."""
    w = np.asarray(w, np.float64).reshape(-1, 8)
    n = w.shape[0]
    mix = np.empty((n, 40))
    mix[:, :8] = w
    lob = np.concatenate([np.asarray(mu, np.float64).reshape(n, 8, 3),
                          np.asarray(kappa, np.float64).reshape(n, 8, 1)], axis=2)
    mix[:, 8:] = lob.reshape(n, 32)
    mix = np.ascontiguousarray(mix)
    d = None if dirs is None else np.ascontiguousarray(dirs, np.float64).reshape(n, 3)
    uu = None if u is None else np.ascontiguousarray(u, np.float64).reshape(n, 3)
    pdf = np.empty(n) if d is not None else None
    smp = np.empty((n, 3)) if uu is not None else None
    lib().or_guide_mix_eval(_p(mix), _p(d), _p(uu), n, _p(pdf), _p(smp))
    return pdf, smp


def image_parity(gpu_sum, oracle_sum):
    """Per-pixel error e_p = sum_c |g-o| / (sum_c |o| + eps), eps = 1e-3 mean_p sum_c o.

    Returns (mean e_p, fraction of pixels with e_p > 1e-3, e_p array).
    """
    g = np.asarray(gpu_sum, np.float64).reshape(-1, 3)
    o = np.asarray(oracle_sum, np.float64).reshape(-1, 3)
    eps = 1e-3 * np.mean(np.sum(o, axis=1))
    e = np.sum(np.abs(g - o), axis=1) / (np.sum(np.abs(o), axis=1) + eps)
    return float(np.mean(e)), float(np.mean(e > 1e-3)), e
