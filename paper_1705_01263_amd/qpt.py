"""Thin ctypes binding of libqpt (include/qpt.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; PyTorch provides
the device memory (the workspace) and the stream. If the compiled library is
missing this module raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpt.so")

QPT_OK = 0
QPT_E_INVALID, QPT_E_STATE, QPT_E_NOMEM, QPT_E_HIP, QPT_E_UNSUPPORTED, QPT_E_ABORTED = -1, -2, -3, -4, -5, -6
QPT_MAT_GGX = 1
QPT_MAT_EMIT_TEXTURE = 2


class qpt_material(C.Structure):
    _fields_ = [("albedo", C.c_float * 3), ("roughness", C.c_float), ("emission", C.c_float * 3),
                ("flags", C.c_uint32)]


class qpt_camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("look", C.c_float * 3), ("up", C.c_float * 3), ("vfov_deg", C.c_float)]


class qpt_scene_desc(C.Structure):
    _fields_ = [("num_vertices", C.c_uint32), ("positions", C.c_void_p), ("num_triangles", C.c_uint32),
                ("indices", C.c_void_p), ("tri_material", C.c_void_p), ("num_materials", C.c_uint32),
                ("materials", C.c_void_p), ("env_width", C.c_uint32), ("env_height", C.c_uint32),
                ("env_rgb", C.c_void_p), ("camera", qpt_camera), ("width", C.c_uint32), ("height", C.c_uint32)]


class qpt_bvh_opts(C.Structure):
    _fields_ = [("max_leaf_size", C.c_uint32), ("sah_bins", C.c_uint32), ("builder", C.c_uint32),
                ("node_format", C.c_uint32), ("scratch", C.c_void_p), ("scratch_bytes", C.c_size_t)]


class qpt_bvh_stats(C.Structure):
    _fields_ = [("num_nodes", C.c_uint32), ("num_leaves", C.c_uint32), ("max_depth", C.c_uint32),
                ("node_bytes", C.c_uint32), ("sah_cost", C.c_double), ("build_ms", C.c_double)]


class qpt_render_opts(C.Structure):
    _fields_ = [("max_depth", C.c_uint32), ("rr", C.c_uint32), ("mode", C.c_uint32), ("scramble", C.c_uint32),
                ("light_tree", C.c_uint32), ("single_stream", C.c_uint32), ("env_sampling", C.c_uint32),
                ("filter", C.c_uint32), ("tail_depth", C.c_uint32), ("regen_paths", C.c_uint32),
                ("compress_state", C.c_uint32)]


class qpt_stats(C.Structure):
    _fields_ = [("rays_extension", C.c_uint64), ("rays_shadow", C.c_uint64), ("paths", C.c_uint64),
                ("passes", C.c_uint64), ("nodes_extension", C.c_uint64), ("tris_extension", C.c_uint64),
                ("nodes_shadow", C.c_uint64), ("tris_shadow", C.c_uint64)]


class qpt_guide_opts(C.Structure):
    _fields_ = [("alpha", C.c_float), ("lr", C.c_float), ("batch", C.c_uint32), ("train", C.c_uint32),
                ("warmup_steps", C.c_uint32), ("seed", C.c_uint32), ("max_vertex", C.c_uint32)]


class qpt_kernel_time(C.Structure):
    _fields_ = [("launches", C.c_uint32), ("reserved", C.c_uint32), ("total_ms", C.c_double)]


KERNEL_KINDS = ["clear", "generate", "trace", "shade", "shadow", "accumulate", "shade_guided", "guide_train", "tail"]
GUIDE_PARAMS = 13032


EXPORTS = [
    "qpt_create", "qpt_destroy", "qpt_last_error", "qpt_build_scene", "qpt_build_bvh", "qpt_build_bvh_noalloc",
    "qpt_bvh_scratch_size", "qpt_set_streams", "qpt_workspace_size",
    "qpt_bind_workspace", "qpt_render_pass", "qpt_readback", "qpt_reset_accum", "qpt_get_stats",
    "qpt_debug_sample_bits", "qpt_debug_wave_sum", "qpt_debug_pixel_index", "qpt_debug_trace", "qpt_debug_light_tables",
    "qpt_abort", "qpt_load_accum", "qpt_guide_get_state", "qpt_guide_set_state",
    "qpt_debug_light_tree", "qpt_debug_light_sample", "qpt_debug_env_pyramid", "qpt_debug_env_sample",
    "qpt_debug_env_tables", "qpt_debug_bvh_nodes", "qpt_profile", "qpt_profile_read", "qpt_guide_config",
    "qpt_guide_set_weights", "qpt_guide_get_weights", "qpt_guide_debug_forward", "qpt_guide_debug_eval", "qpt_guide_debug_grad",
    "qpt_guide_debug_train", "qpt_guide_debug_mixture", "qpt_guide_debug_records", "qpt_guide_loss",
]

_lib = None


class QptError(RuntimeError):
    pass


def lib():
    """Load libqpt.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1705_01263_amd.build")
        L = C.CDLL(LIB_PATH)
        P, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
        sig = {
            "qpt_create": ([i32, P, C.POINTER(P)], i32),
            "qpt_destroy": ([P], None),
            "qpt_last_error": ([P], C.c_char_p),
            "qpt_build_scene": ([P, C.POINTER(qpt_scene_desc)], i32),
            "qpt_build_bvh": ([P, C.POINTER(qpt_bvh_opts), C.POINTER(qpt_bvh_stats)], i32),
            "qpt_build_bvh_noalloc": ([P, C.POINTER(qpt_bvh_opts), C.POINTER(qpt_bvh_stats)], i32),
            "qpt_bvh_scratch_size": ([P, C.POINTER(C.c_size_t)], i32),
            "qpt_set_streams": ([P, P], i32),
            "qpt_workspace_size": ([P, u32, C.POINTER(C.c_size_t)], i32),
            "qpt_bind_workspace": ([P, P, C.c_size_t, u32], i32),
            "qpt_render_pass": ([P, u64, u32, C.POINTER(qpt_render_opts)], i32),
            "qpt_readback": ([P, P, P, i32], i32),
            "qpt_reset_accum": ([P], i32),
            "qpt_get_stats": ([P, C.POINTER(qpt_stats)], i32),
            "qpt_debug_sample_bits": ([P, P, P, u32, i32, P], i32),
            "qpt_debug_wave_sum": ([P, P, u32, P], i32),
            "qpt_debug_pixel_index": ([P, u64, P], i32),
            "qpt_debug_trace": ([P, P, u32, i32, i32, P, P, P, P], i32),
            "qpt_debug_light_tables": ([P, P, P, P, P, P], i32),
            "qpt_abort": ([P], i32),
            "qpt_load_accum": ([P, P, P, i32], i32),
            "qpt_guide_get_state": ([P, P, P, P, C.POINTER(C.c_uint32)], i32),
            "qpt_guide_set_state": ([P, P, P, P, u32], i32),
            "qpt_debug_light_tree": ([P, P, P, P, P, P, P, P, C.POINTER(C.c_uint32)], i32),
            "qpt_debug_light_sample": ([P, P, P, P, u32, P, P, P], i32),
            "qpt_debug_env_pyramid": ([P, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), P, P],
                                      i32),
            "qpt_debug_env_sample": ([P, P, P, u32, u32, P, P, P], i32),
            "qpt_debug_env_tables": ([P, P, P, P], i32),
            "qpt_debug_bvh_nodes": ([P, P, P, P], i32),
            "qpt_profile": ([P, i32], i32),
            "qpt_guide_config": ([P, C.POINTER(qpt_guide_opts)], i32),
            "qpt_guide_set_weights": ([P, P], i32),
            "qpt_guide_get_weights": ([P, P, C.POINTER(C.c_uint32)], i32),
            "qpt_guide_debug_forward": ([P, P, u32, P], i32),
            "qpt_guide_debug_eval": ([P, P, P, u32, P], i32),
            "qpt_guide_debug_grad": ([P, P, P, P, u32, P], i32),
            "qpt_guide_debug_train": ([P, P, P, P, u32, C.c_float, P], i32),
            "qpt_guide_debug_mixture": ([P, P, P, P, u32, P, P], i32),
            "qpt_guide_debug_records": ([P, P, P, u32, C.POINTER(C.c_uint32)], i32),
            "qpt_guide_loss": ([P, C.POINTER(C.c_double), C.POINTER(C.c_double)], i32),
            "qpt_profile_read": ([P, C.POINTER(qpt_kernel_time)], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())  # torch tensor


class Context:
    """One qpt_ctx. device < 0 makes a host-only context (scene and BVH builders only)."""

    def __init__(self, device: int = 0, stream=None):
        self.L = lib()
        self.h = C.c_void_p()
        s = None if stream is None else C.c_void_p(stream)
        rc = self.L.qpt_create(device, s, C.byref(self.h))
        if rc != QPT_OK:
            raise QptError(f"qpt_create failed ({rc})")
        self._keep = []

    def close(self):
        if self.h:
            self.L.qpt_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int, what: str):
        if rc != QPT_OK:
            msg = self.L.qpt_last_error(self.h)
            raise QptError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    # ---- the boundary calls, same names as the C-ABI
    def build_scene(self, sc) -> None:
        pos = np.ascontiguousarray(sc.positions, np.float32)
        idx = np.ascontiguousarray(sc.indices, np.uint32)
        tm = np.ascontiguousarray(sc.tri_material, np.uint32)
        nm = sc.albedo.shape[0]
        mats = (qpt_material * nm)()
        for m in range(nm):
            mats[m].albedo[:] = [float(x) for x in sc.albedo[m]]
            mats[m].roughness = float(sc.roughness[m])
            mats[m].emission[:] = [float(x) for x in sc.emission[m]]
            mats[m].flags = int(sc.mat_flags[m])
        env = None if sc.env is None else np.ascontiguousarray(sc.env, np.float32)
        d = qpt_scene_desc()
        d.num_vertices = pos.shape[0]
        d.positions = pos.ctypes.data
        d.num_triangles = idx.shape[0]
        d.indices = idx.ctypes.data
        d.tri_material = tm.ctypes.data
        d.num_materials = nm
        d.materials = C.cast(mats, C.c_void_p)
        if env is not None:
            d.env_height, d.env_width = env.shape[0], env.shape[1]
            d.env_rgb = env.ctypes.data
        cam = sc.camera
        d.camera.eye[:] = list(cam.eye)
        d.camera.look[:] = list(cam.look)
        d.camera.up[:] = list(cam.up)
        d.camera.vfov_deg = cam.vfov_deg
        d.width, d.height = sc.width, sc.height
        self.check(self.L.qpt_build_scene(self.h, C.byref(d)), "qpt_build_scene")
        self.W, self.H = sc.width, sc.height

    def build_bvh(self, max_leaf_size: int = 0, sah_bins: int = 0, builder: int = 0, scratch=None,
                  scratch_bytes: int = 0, node_format: int = 0) -> qpt_bvh_stats:
        """builder 0: binned SAH on the host; 1: linear BVH on the GPU, its temporaries in the
        caller's device memory `scratch` (a pointer, at least bvh_scratch_size() bytes). Zero
        sizes take the library's defaults (leaves of up to 3 triangles, 16 bins). node_format
        0: quantised 64-byte nodes on the device, 1: full-precision 128-byte nodes."""
        o = qpt_bvh_opts(max_leaf_size, sah_bins, builder, node_format, scratch, scratch_bytes)
        st = qpt_bvh_stats()
        self.check(self.L.qpt_build_bvh(self.h, C.byref(o), C.byref(st)), "qpt_build_bvh")
        return st

    def build_bvh_noalloc(self, max_leaf_size: int = 0) -> qpt_bvh_stats:
        o = qpt_bvh_opts(max_leaf_size, 0, 1, 0, None, 0)
        st = qpt_bvh_stats()
        self.check(self.L.qpt_build_bvh_noalloc(self.h, C.byref(o), C.byref(st)), "qpt_build_bvh_noalloc")
        return st

    def bvh_scratch_size(self) -> int:
        n = C.c_size_t()
        self.check(self.L.qpt_bvh_scratch_size(self.h, C.byref(n)), "qpt_bvh_scratch_size")
        return n.value

    def set_streams(self, lane_stream: int) -> None:
        self.check(self.L.qpt_set_streams(self.h, C.c_void_p(lane_stream)), "qpt_set_streams")

    def workspace_size(self, pool_paths: int = 0) -> int:
        n = C.c_size_t()
        self.check(self.L.qpt_workspace_size(self.h, pool_paths, C.byref(n)), "qpt_workspace_size")
        return n.value

    def bind_workspace(self, ptr: int, nbytes: int, pool_paths: int = 0) -> None:
        self.check(self.L.qpt_bind_workspace(self.h, C.c_void_p(ptr), nbytes, pool_paths), "qpt_bind_workspace")

    def render_pass(self, first_pass: int, num_passes: int, max_depth: int, rr: bool = True, mode: int = 0,
                    scramble: bool = True, light_tree: bool = False, single_stream: bool = False,
                    env_sampling: int = 0, gauss: bool = False, tail_depth: int = 0, regen_paths: int = 0,
                    compress_state: bool = False) -> None:
        o = qpt_render_opts(max_depth, int(rr), mode, int(scramble), int(light_tree), int(single_stream),
                            int(env_sampling), int(gauss), int(tail_depth), int(regen_paths), int(compress_state))
        self.check(self.L.qpt_render_pass(self.h, first_pass, num_passes, C.byref(o)), "qpt_render_pass")

    def readback(self, sum_rgb=None, counts=None, dst_is_device: bool = False) -> bool:
        """Fill the buffers; True if rendering had been aborted (the request is then cleared)."""
        rc = self.L.qpt_readback(self.h, _p(sum_rgb), _p(counts), int(dst_is_device))
        if rc == QPT_E_ABORTED:
            return True
        self.check(rc, "qpt_readback")
        return False

    def abort(self) -> None:
        self.check(self.L.qpt_abort(self.h), "qpt_abort")

    def load_accum(self, sum_rgb, counts, src_is_device: bool = False) -> None:
        self.check(self.L.qpt_load_accum(self.h, _p(sum_rgb), _p(counts), int(src_is_device)), "qpt_load_accum")

    def guide_get_state(self):
        """(params, m, v, steps) of the guide's optimiser."""
        p, m, v = (np.empty(GUIDE_PARAMS, np.float32) for _ in range(3))
        st = C.c_uint32()
        self.check(self.L.qpt_guide_get_state(self.h, _p(p), _p(m), _p(v), C.byref(st)), "qpt_guide_get_state")
        return p, m, v, st.value

    def guide_set_state(self, params, m, v, steps) -> None:
        p, m, v = (np.ascontiguousarray(a, np.float32) for a in (params, m, v))
        assert p.shape == m.shape == v.shape == (GUIDE_PARAMS,)
        self.check(self.L.qpt_guide_set_state(self.h, _p(p), _p(m), _p(v), int(steps)), "qpt_guide_set_state")

    def reset_accum(self) -> None:
        self.check(self.L.qpt_reset_accum(self.h), "qpt_reset_accum")

    def get_stats(self) -> qpt_stats:
        s = qpt_stats()
        self.check(self.L.qpt_get_stats(self.h, C.byref(s)), "qpt_get_stats")
        return s

    def profile(self, enable: bool) -> None:
        self.check(self.L.qpt_profile(self.h, int(enable)), "qpt_profile")

    def profile_read(self) -> dict:
        arr = (qpt_kernel_time * len(KERNEL_KINDS))()
        self.check(self.L.qpt_profile_read(self.h, arr), "qpt_profile_read")
        return {k: (arr[i].launches, arr[i].total_ms) for i, k in enumerate(KERNEL_KINDS)}

    # ---- learned proposal
    def guide_config(self, alpha=0.5, lr=1e-3, batch=1 << 18, train=True, warmup_steps=1, seed=0,
                     max_vertex=0) -> None:
        # train: Adam steps per batch of passes; max_vertex: guide vertices 1..max_vertex (0 = all)
        o = qpt_guide_opts(alpha, lr, batch, int(train), warmup_steps, seed, max_vertex)
        self.check(self.L.qpt_guide_config(self.h, C.byref(o)), "qpt_guide_config")

    def guide_set_weights(self, params) -> None:
        p = np.ascontiguousarray(params, np.float32)
        assert p.shape == (GUIDE_PARAMS,)
        self.check(self.L.qpt_guide_set_weights(self.h, _p(p)), "qpt_guide_set_weights")

    def guide_get_weights(self):
        p = np.empty(GUIDE_PARAMS, np.float32)
        st = C.c_uint32()
        self.check(self.L.qpt_guide_get_weights(self.h, _p(p), C.byref(st)), "qpt_guide_get_weights")
        return p, st.value

    def guide_debug_forward(self, x, n, out) -> None:
        self.check(self.L.qpt_guide_debug_forward(self.h, _p(x), n, _p(out)), "qpt_guide_debug_forward")

    def guide_debug_eval(self, x, wo, n, mix) -> None:
        self.check(self.L.qpt_guide_debug_eval(self.h, _p(x), _p(wo), n, _p(mix)), "qpt_guide_debug_eval")

    def guide_debug_grad(self, x, dirs, w, n, grad) -> None:
        self.check(self.L.qpt_guide_debug_grad(self.h, _p(x), _p(dirs), _p(w), n, _p(grad)), "qpt_guide_debug_grad")

    def guide_debug_train(self, x, dirs, w, n, lr, grad=None) -> None:
        self.check(self.L.qpt_guide_debug_train(self.h, _p(x), _p(dirs), _p(w), n, lr, _p(grad)),
                   "qpt_guide_debug_train")

    def guide_debug_mixture(self, out40, dirs, u, n, pdf, sample) -> None:
        self.check(self.L.qpt_guide_debug_mixture(self.h, _p(out40), _p(dirs), _p(u), n, _p(pdf), _p(sample)),
                   "qpt_guide_debug_mixture")

    def guide_debug_records(self, ident, rec, cap) -> int:
        n = C.c_uint32()
        self.check(self.L.qpt_guide_debug_records(self.h, _p(ident), _p(rec), cap, C.byref(n)),
                   "qpt_guide_debug_records")
        return n.value

    def guide_loss(self):
        l, w = C.c_double(), C.c_double()
        self.check(self.L.qpt_guide_loss(self.h, C.byref(l), C.byref(w)), "qpt_guide_loss")
        return l.value, w.value

    def debug_sample_bits(self, idx, dim, n, scramble, out) -> None:
        self.check(self.L.qpt_debug_sample_bits(self.h, _p(idx), _p(dim), n, int(scramble), _p(out)),
                   "qpt_debug_sample_bits")

    def debug_wave_sum(self, inp, n: int, out) -> None:
        self.check(self.L.qpt_debug_wave_sum(self.h, _p(inp), n, _p(out)), "qpt_debug_wave_sum")

    def debug_pixel_index(self, pass_: int, out) -> None:
        self.check(self.L.qpt_debug_pixel_index(self.h, pass_, _p(out)), "qpt_debug_pixel_index")

    def debug_trace(self, rays, n, any_hit, brute_force, t, tri, b12, stack_max=None) -> None:
        self.check(self.L.qpt_debug_trace(self.h, _p(rays), n, int(any_hit), int(brute_force), _p(t), _p(tri),
                                          _p(b12), _p(stack_max)), "qpt_debug_trace")

    def debug_light_tree(self):
        """The light tree's host tables (same keys as the oracle's)."""
        nn = C.c_uint32()
        self.check(self.L.qpt_debug_light_tree(self.h, None, None, None, None, None, None, None, C.byref(nn)),
                   "qpt_debug_light_tree")
        n = nn.value
        ne = self.debug_light_tables()["tri"].shape[0]
        t = dict(center=np.empty((n, 4), np.float32), flux=np.empty((n, 6), np.float32),
                 left=np.empty(n, np.int32), first=np.empty(n, np.uint32), count=np.empty(n, np.uint32),
                 emit=np.empty(ne, np.uint32), w=np.empty(ne, np.uint32))
        self.check(self.L.qpt_debug_light_tree(self.h, _p(t["center"]), _p(t["flux"]), _p(t["left"]),
                                               _p(t["first"]), _p(t["count"]), _p(t["emit"]), _p(t["w"]),
                                               C.byref(nn)), "qpt_debug_light_tree")
        return t

    def debug_env_pyramid(self):
        """The environment pyramid's host tables (same keys as the oracle's)."""
        m, top, root = C.c_uint32(), C.c_uint32(), C.c_uint32()
        self.check(self.L.qpt_debug_env_pyramid(self.h, C.byref(m), C.byref(top), C.byref(root), None, None),
                   "qpt_debug_env_pyramid")
        m, top, root = m.value, top.value, root.value
        if not m:
            return dict(m=0)
        q = np.empty(4 * (2 * (4 ** m - 1) // 3), np.uint32)
        oq = np.empty(256 * 4 * (1 + 2 * (4 ** top - 1) // 3), np.uint32)
        self.check(self.L.qpt_debug_env_pyramid(self.h, C.byref(C.c_uint32()), C.byref(C.c_uint32()),
                                                C.byref(C.c_uint32()), _p(q), _p(oq)), "qpt_debug_env_pyramid")
        return dict(m=m, top=top, root=root, q=q, oq=oq.reshape(256, -1))

    def debug_env_sample(self, uv, nrm, n, mode, texel, iv, iv_hit) -> None:
        """Device buffers: uv (2n uint32), nrm (3n float32) in; texel (n
        uint32), iv (4n uint64), iv_hit (2n uint64) out."""
        self.check(self.L.qpt_debug_env_sample(self.h, _p(uv), _p(nrm), n, mode, _p(texel), _p(iv), _p(iv_hit)),
                   "qpt_debug_env_sample")

    def debug_light_sample(self, S, x, nrm, n, emitter, size, size_hit) -> None:
        """Device buffers: S (n uint64), x and nrm (3n float32) in; emitter
        (n uint32), size and size_hit (n uint64) out."""
        self.check(self.L.qpt_debug_light_sample(self.h, _p(S), _p(x), _p(nrm), n, _p(emitter), _p(size),
                                                 _p(size_hit)), "qpt_debug_light_sample")

    def debug_light_tables(self):
        cnt = C.c_uint32()
        self.check(self.L.qpt_debug_light_tables(self.h, None, None, None, None, C.byref(cnt)),
                   "qpt_debug_light_tables")
        n = cnt.value
        tri = np.empty(n, np.uint32)
        prob = np.empty(n, np.float64)
        alias = np.empty(n, np.uint32)
        pmf = np.empty(n, np.float64)
        self.check(self.L.qpt_debug_light_tables(self.h, _p(tri), _p(prob), _p(alias), _p(pmf), C.byref(cnt)),
                   "qpt_debug_light_tables")
        return dict(tri=tri, prob=prob, alias=alias, pmf=pmf)

    def debug_env_tables(self, eh: int, ew: int):
        rq = np.empty(eh, np.uint32)
        cq = np.empty(eh * ew, np.uint32)
        pdf = np.empty(eh * ew, np.float32)
        self.check(self.L.qpt_debug_env_tables(self.h, _p(rq), _p(cq), _p(pdf)), "qpt_debug_env_tables")
        return rq, cq.reshape(eh, ew), pdf.reshape(eh, ew)

    def debug_bvh_nodes(self):
        nn = C.c_uint32()
        self.check(self.L.qpt_debug_bvh_nodes(self.h, None, None, C.byref(nn)), "qpt_debug_bvh_nodes")
        nodes = np.empty((nn.value, 32), np.float32)
        order = np.empty(self.ntri, np.uint32) if hasattr(self, "ntri") else None
        self.check(self.L.qpt_debug_bvh_nodes(self.h, _p(nodes), _p(order), C.byref(nn)), "qpt_debug_bvh_nodes")
        return nodes, order


class Renderer:
    """Scene + BVH + a torch-owned workspace on one GPU; renders 1-spp passes."""

    def __init__(self, sc, device: int = 0, pool_paths: int = 0, stream=None, bvh_builder: int = 0,
                 node_format: int = 0, lane_stream=None):
        import torch

        self.torch = torch
        self.sc = sc
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = Context(device, self.stream.cuda_stream)
        # the second batch in flight: on the library's own stream unless one is
        # given (torch's stream pool hands out streams round-robin over the
        # device's few hardware queues, so a pool stream can share the
        # caller's queue, and the two batches then run one after the other)
        self.lane_stream = lane_stream
        if lane_stream is not None:
            self.ctx.set_streams(lane_stream.cuda_stream)
        self.ctx.ntri = sc.num_triangles
        self.ctx.build_scene(sc)
        if bvh_builder == 1:
            nb = self.ctx.bvh_scratch_size()
            tmp = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            self.bvh_stats = self.ctx.build_bvh(builder=1, scratch=(tmp.data_ptr() + 255) & ~255, scratch_bytes=nb,
                                                node_format=node_format)
            del tmp
        else:
            self.bvh_stats = self.ctx.build_bvh(builder=bvh_builder, node_format=node_format)
        self.pool_paths = pool_paths
        nbytes = self.ctx.workspace_size(pool_paths)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) & ~255
        self.ctx.bind_workspace(ptr, nbytes, pool_paths)
        self.W, self.H = sc.width, sc.height

    def render(self, first_pass: int, num_passes: int, max_depth=None, rr=True, mode=0, scramble=True,
               light_tree=False, single_stream=False, env_sampling=0, gauss=False, tail_depth=0, regen_paths=0,
               compress_state=False):
        self.ctx.render_pass(first_pass, num_passes, max_depth or self.sc.max_depth, rr, mode, scramble, light_tree,
                             single_stream, env_sampling, gauss, tail_depth, regen_paths, compress_state)

    def readback(self):
        """FP64 sums and counts; `self.aborted` tells whether rendering had been aborted."""
        s = np.empty((self.H * self.W, 3), np.float64)
        c = np.empty(self.H * self.W, np.uint32)
        self.aborted = self.ctx.readback(s, c)
        return s, c

    def reset(self):
        self.ctx.reset_accum()

    def stats(self):
        return self.ctx.get_stats()
