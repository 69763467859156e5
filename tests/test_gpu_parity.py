"""GPU parity through the C-ABI: HIP path vs the CPU oracle on identical inputs.

- Halton sample bits and pixel indices: bit-exact (integer work).
- Closest-hit ids, t and barycentrics: bit-exact against the oracle's FP32
  brute force (both decide in FP32 with the same watertight test); BVH
  traversal equals brute-force traversal on the GPU.
- Images at identical sample indices: mean relative pixel error <= 1e-4 and
  at most 0.1% of pixels above 1e-3 (per-pixel error sum_c |g-o| /
  (sum_c |o| + 1e-3 * mean_p sum_c o)).
- Closed forms on the GPU: white furnace per path; split pass ranges give
  bit-identical FP64 sums.
"""
import math
import sys

import numpy as np
import pytest

import scenegen as g

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


# ------------------------------------------------------------------ Halton

@pytest.mark.parametrize("W,H", [(128, 128), (1920, 1080)])
def test_sample_bits_bitexact(Renderer, orc, W, H):
    _say(f"[sample_bits] W={W} H={H}")
    sc = g.cornell(width=W, height=H)
    r = Renderer(sc, pool_paths=1 << 16)
    rng = np.random.default_rng(W + H)
    n = 1 << 16
    bits = rng.choice([8, 20, 34, 40, 48, 56, 63, 64], n)
    idx = (rng.integers(0, 2 ** 63, n, dtype=np.uint64) >> (64 - bits).astype(np.uint64)).astype(np.uint64)
    idx[:4] = [0, 1, 2 ** 64 - 1, 2 ** 34 + 5]
    dim = rng.integers(0, 256, n).astype(np.uint32)
    dim[:256] = np.arange(256)
    for scramble in (False, True):
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        r.ctx.debug_sample_bits(_dev(idx.view(np.int64)), _dev(dim.view(np.int32)), n, scramble, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        want = orc.sample_bits(idx, dim, W, H, scramble)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (scramble, idx[bad[:5]], dim[bad[:5]], got[bad[:5]], want[bad[:5]])


@pytest.mark.parametrize("W,H,passes", [(128, 128, (0, 1, 15, 1 << 20)), (1920, 1080, (0, 63, 1 << 30)),
                                        (3840, 2160, (0, 1023, 1 << 30)), (5, 4, (0, 7))])
def test_pixel_index_bitexact(Renderer, orc, W, H, passes):
    _say(f"[pixel_index] W={W} H={H}")
    sc = g.cornell(width=W, height=H)
    r = Renderer(sc, pool_paths=1 << 16)
    rng = np.random.default_rng(1)
    pix = rng.integers(0, W * H, min(W * H, 4000))
    for j in passes:
        out = torch.empty(W * H, dtype=torch.int64, device="cuda")
        r.ctx.debug_pixel_index(j, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint64)
        want = np.array([orc.pixel_index(W, H, int(p % W), int(p // W), j) for p in pix], np.uint64)
        assert np.array_equal(got[pix], want), j


# ------------------------------------------------------------------ tracing

def _ray_set(sc, n, seed):
    rng = np.random.default_rng(seed)
    lo = sc.positions.min(0).astype(np.float64)
    hi = sc.positions.max(0).astype(np.float64)
    ext = hi - lo
    o = lo - 0.1 * ext + rng.uniform(0, 1, (n, 3)) * 1.2 * ext
    # half random directions, half aimed at triangle vertices and edge midpoints
    d = rng.normal(size=(n, 3))
    k = n // 2
    tri = rng.integers(0, sc.num_triangles, k)
    w = rng.choice([0.0, 0.5, 1.0], (k, 2))
    p = sc.positions[sc.indices[tri]].astype(np.float64)
    tgt = p[:, 0] + w[:, :1] * (p[:, 1] - p[:, 0]) + w[:, 1:] * 0.5 * (p[:, 2] - p[:, 0])
    d[:k] = tgt - o[:k]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = o
    rays[:, 3] = np.where(rng.uniform(size=n) < 0.2, rng.uniform(0.1, 1.0, n) * np.linalg.norm(ext), np.inf)
    rays[:, 4:7] = d
    return rays


@pytest.mark.parametrize("which", ["cornell", "grid4"])
def test_trace_bitexact(Renderer, orc, which):
    sc = g.workload("cornell") if which == "cornell" else g.grid_scene(grid=4, width=64, height=64)
    n = 20000 if which == "cornell" else 4000
    _say(f"[trace] {which} tris={sc.num_triangles} rays={n}")
    r = Renderer(sc, pool_paths=1 << 16)
    rays = _ray_set(sc, n, 5)
    drays = _dev(rays)
    res = {}
    for brute in (0, 1):
        t = torch.empty(n, dtype=torch.float32, device="cuda")
        tri = torch.empty(n, dtype=torch.int32, device="cuda")
        b = torch.empty((n, 2), dtype=torch.float32, device="cuda")
        r.ctx.debug_trace(drays, n, 0, brute, t, tri, b)
        torch.cuda.synchronize()
        res[brute] = (t.cpu().numpy(), tri.cpu().numpy().view(np.uint32), b.cpu().numpy())
    t_o, tri_o, b_o = orc.trace_f32(sc, rays)
    for brute in (0, 1):
        t_g, tri_g, b_g = res[brute]
        bad = np.nonzero(tri_g != tri_o)[0]
        assert bad.size == 0, (brute, bad[:5], tri_g[bad[:5]], tri_o[bad[:5]])
        hit = tri_o != 0xFFFFFFFF
        assert np.array_equal(t_g[hit], t_o[hit])
        assert np.array_equal(b_g[hit], b_o[hit])
    assert np.mean(tri_o != 0xFFFFFFFF) > 0.3
    # occlusion
    for brute in (0, 1):
        occ = torch.empty(n, dtype=torch.int32, device="cuda")
        r.ctx.debug_trace(drays, n, 1, brute, None, occ, None)
        torch.cuda.synchronize()
        _, occ_o, _ = orc.trace_f32(sc, rays, any_hit=True)
        assert np.array_equal(occ.cpu().numpy().view(np.uint32), occ_o)


def _with_degenerate_triangles(sc):
    """The scene plus a zero-area triangle (one point) and a collinear one
    inside the room, and a sliver, all with the first material."""
    extra = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.5, 0.5, 0.5],
                      [0.2, 0.7, 0.3], [0.4, 0.7, 0.5], [0.6, 0.7, 0.7],
                      [0.1, 0.2, 0.9], [0.9, 0.2, 0.9], [0.5, 0.2 + 1e-7, 0.9]], np.float32)
    nv = sc.positions.shape[0]
    sc.positions = np.concatenate([sc.positions, extra])
    sc.indices = np.concatenate([sc.indices, (np.arange(9, dtype=np.uint32) + nv).reshape(3, 3)])
    sc.tri_material = np.concatenate([sc.tri_material, np.zeros(3, np.uint32)])
    sc.validate()
    return sc


def test_trace_axis_rays_and_degenerate_triangles(Renderer, orc):
    """Rays exactly along +-x, +-y, +-z (reciprocal directions of 1e20 in the slab
    test) and rays aimed at a point-like, a collinear and a sliver triangle:
    ids, t and barycentrics bit-exact against the oracle's FP32 brute force."""
    sc = _with_degenerate_triangles(g.workload("cornell"))
    rng = np.random.default_rng(21)
    n = 6000
    o = rng.uniform(0.02, 0.98, (n, 3))
    axes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float64)
    d = axes[rng.integers(0, 6, n)]
    k = n // 3
    tgt = sc.positions[-9:].astype(np.float64)[rng.integers(0, 9, k)]
    d[:k] = tgt - o[:k]
    d[:k] /= np.linalg.norm(d[:k], axis=1, keepdims=True)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = o
    rays[:, 3] = np.inf
    rays[:, 4:7] = d
    r = Renderer(sc, pool_paths=1 << 14)
    t = torch.empty(n, dtype=torch.float32, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    b = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    r.ctx.debug_trace(_dev(rays), n, 0, 0, t, tri, b)
    torch.cuda.synchronize()
    t_o, tri_o, b_o = orc.trace_f32(sc, rays)
    tri_g = tri.cpu().numpy().view(np.uint32)
    assert np.array_equal(tri_g, tri_o)
    hit = tri_o != 0xFFFFFFFF
    assert np.array_equal(t.cpu().numpy()[hit], t_o[hit])
    assert np.array_equal(b.cpu().numpy()[hit], b_o[hit])
    assert not np.any(tri_o == sc.num_triangles - 3)  # three equal vertices: never hit


def test_single_pixel_per_path(Renderer, orc):
    """A 1 x 1 frame (enumeration stride 1): each pass is one path, compared
    path by path. A path whose FP32 and FP64 geometry decide differently (a
    ray grazing an edge) may legitimately differ; such paths must stay rare."""
    sc = g.cornell(width=1, height=1, max_depth=8)
    r = Renderer(sc, pool_paths=1 << 10)
    S = orc.Scene(sc)
    prev = np.zeros(3)
    agree = 0
    n = 64
    for j in range(n):
        r.render(j, 1)
        s, c = r.readback()
        got = s[0] - prev
        prev = s[0].copy()
        so, _, co, _ = S.render(pass0=j, npasses=1)
        want = so[0]
        assert c[0] == j + 1 and co[0] == 1
        agree += np.allclose(got, want, rtol=1e-4, atol=1e-6)
    _say(f"[image] 1x1: {agree} of {n} paths agree")
    assert agree >= n - 2


@pytest.mark.parametrize("W,H,D,passes", [(7, 5, 32, 16), (13, 11, 1, 8)])
def test_image_parity_edge_sizes(Renderer, orc, W, H, D, passes):
    """A ragged 7 x 5 frame at the largest depth (32 vertices, 250 sample
    dimensions) and depth 1 (camera vertex only)."""
    sc = g.cornell(width=W, height=H, max_depth=D)
    _say(f"[image] cornell {W}x{H} D={D} passes={passes}")
    s, c, _ = _render(Renderer, sc, passes)
    so, _, co, _ = orc.Scene(sc).render(npasses=passes)
    assert np.all(c == passes) and np.all(co == passes)
    mean_e, frac, e = orc.image_parity(s, so)
    _say(f"    mean rel err {mean_e:.3e}, max {e.max():.3e}")
    assert mean_e <= 1e-4 and frac <= 1e-3


def test_render_pass_rejects_index_overflow(Renderer):
    from paper_1705_01263_amd import QptError
    r = Renderer(g.cornell(width=16, height=16), pool_paths=1 << 12)
    with pytest.raises(QptError):
        r.render(2 ** 64 // (2 ** 4 * 3 ** 3), 1)   # S = 2^4 3^3 for 16 x 16: last index beyond 2^64
    r.render(0, 1)  # the context stays usable
    _, c = r.readback()
    assert np.all(c == 1)


# ------------------------------------------------------------------ images

def _render(Renderer, sc, passes, **kw):
    r = Renderer(sc, pool_paths=kw.pop("pool_paths", 0))
    r.render(0, passes, **kw)
    s, c = r.readback()
    return s, c, r


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_image_parity_cornell(Renderer, orc, mode):
    sc = g.workload("cornell")
    _say(f"[image] cornell 128x128x16 D=8 mode={mode}")
    s, c, _ = _render(Renderer, sc, sc.spp, mode=mode)
    assert np.all(c == sc.spp)
    so, _, co, _ = orc.Scene(sc).render(npasses=sc.spp, mode=mode)
    mean_e, frac, e = orc.image_parity(s, so)
    _say(f"    mean rel err {mean_e:.3e}, pixels > 1e-3: {frac:.4%}, max {e.max():.3e}")
    assert mean_e <= 1e-4 and frac <= 1e-3


def test_image_parity_grid_subset(Renderer, orc):
    """The 0.97M-triangle grid workload (GGX, textured emitters) at 1920 x 1080 on every 8th pixel, 2 passes."""
    sc = g.workload("grid_1m")
    _say(f"[image] grid 1920x1080 tris={sc.num_triangles} passes=2 D=12")
    s, c, _ = _render(Renderer, sc, 2)
    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(0, H, 8), np.arange(0, W, 8), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    so, _, co, _ = orc.Scene(sc).render(pixels=pix, npasses=2)
    mean_e, frac, e = orc.image_parity(s[pix], so)
    _say(f"    mean rel err {mean_e:.3e}, pixels > 1e-3: {frac:.4%}, max {e.max():.3e}")
    assert np.all(c[pix] == 2)
    assert mean_e <= 1e-4 and frac <= 1e-3


def test_image_parity_env_subset(Renderer, orc):
    """4M-triangle instanced scene under the sun-and-sky map (2D CDF sampling), every 8th pixel."""
    sc = g.workload("instanced_env_4m")
    _say(f"[image] env 1920x1080 tris={sc.num_triangles} passes=2 D=16")
    s, c, _ = _render(Renderer, sc, 2)
    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(0, H, 8), np.arange(0, W, 8), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    so, _, co, _ = orc.Scene(sc).render(pixels=pix, npasses=2)
    mean_e, frac, e = orc.image_parity(s[pix], so)
    _say(f"    mean rel err {mean_e:.3e}, pixels > 1e-3: {frac:.4%}, max {e.max():.3e}")
    assert np.all(c[pix] == 2)
    assert mean_e <= 1e-4 and frac <= 1e-3


def test_image_parity_slit_full_size(Renderer, orc):
    """The 4M-triangle slit enclosure (sun and sky through a 0.1-wide roof slit, the
    equal-time workload) at 1920 x 1080 with the default pool, every 8th pixel. Most light
    arrives over several bounces, so 64 passes, for enough lit samples (about 10% of the
    pixels) to compare."""
    sc = g.workload("slit_enclosure")
    P = 64
    _say(f"[image] slit 1920x1080 tris={sc.num_triangles} passes={P} D={sc.max_depth}")
    s, c, _ = _render(Renderer, sc, P)
    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(3, H, 8), np.arange(5, W, 8), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    so, _, co, _ = orc.Scene(sc).render(pixels=pix, npasses=P)
    mean_e, frac, e = orc.image_parity(s[pix], so)
    lit = float(np.mean(np.any(so > 0, axis=1)))
    _say(f"    lit pixels {lit:.1%}, mean rel err {mean_e:.3e}, pixels > 1e-3: {frac:.4%}, max {e.max():.3e}")
    assert np.all(c == P) and np.all(co == P)
    assert lit > 0.05
    assert mean_e <= 1e-4 and frac <= 1e-3


def test_image_parity_city_subset(Renderer, orc):
    """The city generator at 1/16 of its blocks (about 1M triangles, 5,000 emissive window cells
    as triangle pairs, alias-table light selection) at the full 3840 x 2160: a pass exceeds the
    path pool, so every pass is rendered in pixel chunks. Every 16th pixel, 2 passes."""
    sc = g.city(blocks=16, target_tris=1_000_000, emissive_cells=5000)
    _say(f"[image] city 3840x2160 tris={sc.num_triangles} passes=2 D=16")
    s, c, _ = _render(Renderer, sc, 2, pool_paths=1 << 21)
    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(0, H, 16), np.arange(0, W, 16), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    so, _, co, _ = orc.Scene(sc).render(pixels=pix, npasses=2)
    mean_e, frac, e = orc.image_parity(s[pix], so)
    _say(f"    mean rel err {mean_e:.3e}, pixels > 1e-3: {frac:.4%}, max {e.max():.3e}")
    assert np.all(c == 2)
    assert mean_e <= 1e-4 and frac <= 1e-3


def test_image_parity_city_full_size(Renderer, orc):
    """The 16M-triangle city at 3840 x 2160 in the benchmark's launch configuration (the
    default pool: eight-frame batches, two in flight), 2 passes, every 16th pixel in x
    and y (32,400 pixels). The oracle builds its own BVH over all 16M triangles (about a
    minute)."""
    sc = g.workload("city_16m")
    _say(f"[image] city 3840x2160 tris={sc.num_triangles} passes=2 D=16, default pool")
    s, c, _ = _render(Renderer, sc, 2)
    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(5, H, 16), np.arange(3, W, 16), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    _say("    oracle BVH build and render")
    so, _, co, _ = orc.Scene(sc).render(pixels=pix, npasses=2)
    mean_e, frac, e = orc.image_parity(s[pix], so)
    _say(f"    mean rel err {mean_e:.3e}, pixels > 1e-3: {frac:.4%}, max {e.max():.3e}")
    assert np.all(c == 2) and np.all(co == 2)
    assert mean_e <= 1e-4 and frac <= 1e-3


def test_constant_sky_every_path(Renderer):
    """Convex Lambert box under a constant sky: BSDF-sampled paths that hit it carry rho E exactly."""
    rho, E = 0.6, 2.0
    sc = g.convex_under_env(rho, E, width=32, height=32, max_depth=4)
    _say("[sky] convex box under constant env, BSDF only")
    s, c, _ = _render(Renderer, sc, 8, rr=False, mode=1)
    m = s / c[:, None]
    r32 = float(np.float32(rho))
    frac = (E - m) / (E - r32 * E)
    assert np.all(frac > -1e-5) and np.all(frac < 1 + 1e-5)
    full = np.all(np.abs(frac - 1.0) < 1e-5, axis=1)
    assert full.sum() > 100
    # with NEE of the sky and MIS the object pixels still average rho E
    s, c, _ = _render(Renderer, sc, 64, rr=False, mode=0)
    m = (s / c[:, None])[full].mean(0)
    assert np.allclose(m, r32 * E, rtol=2e-3), m


def test_furnace_every_path(Renderer):
    E, rho, D = 1.0, 0.5, 8
    sc = g.furnace(E, rho, width=32, height=32, max_depth=D)
    _say("[furnace] 32x32 D=8 BSDF only")
    s, c, _ = _render(Renderer, sc, 8, rr=False, mode=1)
    want = E * (1 - rho ** D) / (1 - rho)
    assert np.allclose(s / c[:, None], want, rtol=2e-6)


@pytest.mark.parametrize("W,H", [(64, 48), (61, 45)])
def test_pass_split_is_bit_identical(Renderer, W, H):
    """Whole-frame batches (pixels in 8 x 8 tile order, ragged tiles at the
    right and bottom edges when W or H is not a multiple of 8) and pixel
    chunks in scanline order give the same sums and counts bit for bit."""
    sc = g.cornell(width=W, height=H)
    _say(f"[split] cornell {W}x{H}, passes [0,8) vs [0,3)+[3,8) vs small pool")
    a, ca, r = _render(Renderer, sc, 8)
    r.reset()
    r.render(0, 3)
    r.render(3, 5)
    b, cb = r.readback()
    c_, cc, _ = _render(Renderer, sc, 8, pool_paths=1000)  # pixel chunks of 1000
    assert np.all(ca == 8)
    assert np.array_equal(ca, cb) and np.array_equal(ca, cc)
    assert np.array_equal(a, b)
    assert np.array_equal(a, c_)


@pytest.mark.parametrize("pool", [1 << 12, 1 << 9])
def test_two_lanes_bit_identical(Renderer, pool):
    """Consecutive batches alternate between two streams with their own path
    pools; the FP64 sums, counts and ray statistics equal one-stream rendering
    bit for bit, also when a pass is split into pixel chunks (pool < frame)."""
    sc = g.cornell(width=32, height=32)
    _say(f"[lanes] cornell 32x32 pool={pool}")
    out = []
    for single in (True, False):
        r = Renderer(sc, pool_paths=pool)
        r.render(0, 21, single_stream=single)
        r.render(21, 6, single_stream=single)
        s, c = r.readback()
        st = r.stats()
        out.append((s, c, (st.rays_extension, st.rays_shadow, st.paths)))
    (s1, c1, t1), (s2, c2, t2) = out
    assert np.all(c1 == 27) and np.array_equal(c1, c2)
    assert np.array_equal(s1, s2)
    assert t1 == t2


def test_wave_sum_dpp(Renderer):
    """The wavefront reduction the traversal kernels add their lanes' node
    and triangle counts with (DPP row moves, then the four row sums) equals
    numpy's sums modulo 2^32: random counts, sums that wrap, one lane set,
    all lanes at the maximum."""
    from paper_1705_01263_amd import qpt
    rng = np.random.default_rng(11)
    waves = 4096
    a = rng.integers(0, 1 << 20, size=(waves, 64), dtype=np.uint64)
    a[1] = rng.integers(0, 1 << 32, size=64, dtype=np.uint64)   # wraps modulo 2^32
    a[2] = 0
    a[2, 37] = 12345                                            # one lane
    a[3] = (1 << 32) - 1                                        # every lane at the maximum
    a[4] = np.arange(64, dtype=np.uint64) << np.uint64(20)      # lane-dependent, no two equal
    want = (a.sum(axis=1) % (1 << 32)).astype(np.uint32)
    inp = torch.from_numpy(a.astype(np.uint32).reshape(-1).view(np.int32)).cuda()
    out = torch.zeros(waves, dtype=torch.int32, device="cuda")
    ctx = qpt.Context(0, torch.cuda.current_stream(0).cuda_stream)
    ctx.debug_wave_sum(inp, waves * 64, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)
    with pytest.raises(qpt.QptError):
        ctx.debug_wave_sum(inp, 100, out)   # not whole waves


def test_caller_lane_stream_bit_identical(Renderer):
    """The second batch in flight on a stream the caller provides
    (qpt_set_streams) renders the same sums and counts as on the library's
    own; the context's own stream is refused for it."""
    from paper_1705_01263_amd import qpt
    sc = g.cornell(width=64, height=48)
    base, cb, _ = _render(Renderer, sc, 40)
    lane = torch.cuda.Stream(0)
    r = Renderer(sc, lane_stream=lane)
    r.render(0, 40)
    s, c = r.readback()
    assert np.array_equal(c, cb) and np.array_equal(s, base)
    ctx = qpt.Context(0, torch.cuda.current_stream(0).cuda_stream)
    with pytest.raises(qpt.QptError):
        ctx.set_streams(torch.cuda.current_stream(0).cuda_stream)


def test_counts_and_stats(Renderer):
    sc = g.cornell(width=32, height=32)
    _, c, r = _render(Renderer, sc, 5)
    st = r.stats()
    assert np.all(c == 5)
    assert st.paths == 32 * 32 * 5 and st.passes == 5
    assert st.rays_extension >= st.paths and st.rays_shadow > 0
