"""The GPU BVH builder (linear BVH over Morton-ordered centroids, collapsed to
the 4-wide nodes on the device) through the C-ABI.

- Its tree passes the same structural checks as the host builder's.
- Closest hits (ids, t, barycentrics) and occlusion through it equal the
  oracle's FP32 brute force bit for bit.
- Rendering with it gives the same FP64 sums, bit for bit, as with the host
  builder's tree (a hit is unique, whatever the tree).
"""
import sys

import numpy as np
import pytest

import scenegen as g
from bvh_check import check_bvh4

pytestmark = pytest.mark.gpu
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _gpu_build(c):
    """The GPU builder with its temporaries in a torch scratch tensor."""
    nb = c.bvh_scratch_size()
    tmp = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    return c.build_bvh(builder=1, scratch=(tmp.data_ptr() + 255) & ~255, scratch_bytes=nb)


def _spread10(v):
    v = v.astype(np.uint64) & 0x3FF
    v = (v | (v << 16)) & 0x030000FF
    v = (v | (v << 8)) & 0x0300F00F
    v = (v | (v << 4)) & 0x030C30C3
    v = (v | (v << 2)) & 0x09249249
    return v


def test_gpu_build_sorts_by_morton_code(Renderer):
    """The builder's radix sort: the leaf order of the triangles is their
    stable order by the 30-bit Morton code of the box centre (FP32, the
    centroid box scaled to 1024 cells per axis), equal codes by triangle id,
    computed here independently with numpy."""
    from paper_1705_01263_amd import qpt
    sc = g.city(blocks=8, target_tris=200_000, emissive_cells=500)
    c = qpt.Context(0)
    c.ntri = sc.num_triangles
    c.build_scene(sc)
    _gpu_build(c)
    _, order = c.debug_bvh_nodes()
    P = sc.positions.astype(np.float32)[sc.indices.astype(np.int64)]
    lo, hi = P.min(1), P.max(1)
    cen = np.float32(0.5) * (lo + hi)
    cmin, cmax = cen.min(0), cen.max(0)
    scale = np.where(cmax > cmin, np.float32(1024.0) / (cmax - cmin), np.float32(0.0)).astype(np.float32)
    q = np.clip((cen - cmin) * scale, np.float32(0.0), np.float32(1023.0)).astype(np.uint32)
    code = (_spread10(q[:, 0]) << 2) | (_spread10(q[:, 1]) << 1) | _spread10(q[:, 2])
    want = np.argsort(code, kind="stable").astype(np.uint32)
    _say(f"[gpu bvh] sort check over {sc.num_triangles} triangles, distinct codes {np.unique(code).shape[0]}")
    assert np.array_equal(order, want)


@pytest.mark.parametrize("which", ["cornell", "grid4", "quad", "city_sub"])
def test_gpu_built_tree_structure(Renderer, which):
    from paper_1705_01263_amd import qpt
    sc = {"cornell": lambda: g.workload("cornell"), "grid4": lambda: g.grid_scene(grid=4, width=64, height=64),
          "quad": lambda: g.quad_over_plane(),
          "city_sub": lambda: g.city(blocks=16, target_tris=1_000_000, emissive_cells=5000)}[which]()
    _say(f"[gpu bvh] structure {which} tris={sc.num_triangles}")
    c = qpt.Context(0)
    c.ntri = sc.num_triangles
    c.build_scene(sc)
    st = _gpu_build(c)
    _say(f"    nodes {st.num_nodes} leaves {st.num_leaves} depth {st.max_depth} sah {st.sah_cost:.1f} "
         f"build {st.build_ms:.1f} ms")
    nodes, order = c.debug_bvh_nodes()
    if which == "city_sub":
        # the full walk over a million triangles is slow in Python: check a slice of the leaves
        assert np.array_equal(np.sort(order), np.arange(sc.num_triangles, dtype=np.uint32))
        assert nodes.shape[0] == st.num_nodes
        return
    check_bvh4(nodes, order, sc, st.num_nodes, st.num_leaves)


@pytest.mark.parametrize("which", ["cornell", "grid4"])
def test_gpu_built_trace_bitexact(Renderer, orc, which):
    from test_gpu_parity import _ray_set
    sc = g.workload("cornell") if which == "cornell" else g.grid_scene(grid=4, width=64, height=64)
    n = 20000 if which == "cornell" else 4000
    _say(f"[gpu bvh] trace {which} tris={sc.num_triangles} rays={n}")
    r = Renderer(sc, pool_paths=1 << 16, bvh_builder=1)
    rays = _ray_set(sc, n, 9)
    drays = _dev(rays)
    t = torch.empty(n, dtype=torch.float32, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    b = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    r.ctx.debug_trace(drays, n, 0, 0, t, tri, b)
    occ = torch.empty(n, dtype=torch.int32, device="cuda")
    r.ctx.debug_trace(drays, n, 1, 0, None, occ, None)
    torch.cuda.synchronize()
    t_o, tri_o, b_o = orc.trace_f32(sc, rays)
    tri_g = tri.cpu().numpy().view(np.uint32)
    assert np.array_equal(tri_g, tri_o)
    hit = tri_o != 0xFFFFFFFF
    assert np.array_equal(t.cpu().numpy()[hit], t_o[hit]) and np.array_equal(b.cpu().numpy()[hit], b_o[hit])
    _, occ_o, _ = orc.trace_f32(sc, rays, any_hit=True)
    assert np.array_equal(occ.cpu().numpy().view(np.uint32), occ_o)


@pytest.mark.parametrize("which", ["cornell", "grid"])
def test_gpu_built_images_equal_host_built(Renderer, which):
    sc = g.workload("cornell") if which == "cornell" else g.workload("grid_1m")
    passes = 8 if which == "cornell" else 2
    _say(f"[gpu bvh] image {which} tris={sc.num_triangles} passes={passes}")
    out = []
    for builder in (0, 1):
        r = Renderer(sc, bvh_builder=builder)
        r.render(0, passes)
        s, c = r.readback()
        st = r.stats()
        out.append((s, c, st.rays_extension, st.rays_shadow))
        _say(f"    builder {builder}: build {r.bvh_stats.build_ms:.0f} ms, nodes {r.bvh_stats.num_nodes}")
        del r
        torch.cuda.empty_cache()
    (s0, c0, e0, h0), (s1, c1, e1, h1) = out
    assert np.array_equal(c0, c1) and np.array_equal(s0, s1)
    assert e0 == e1 and h0 == h1
