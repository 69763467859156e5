"""GPU parity of the light tree (the many-light hierarchy of Sec. 2.1.1)
through the C-ABI.

- The renderer's descent (FP32 importance, 24-bit child probabilities,
  63-bit integer interval arithmetic) chooses the oracle's emitter with the
  oracle's interval size, bit for bit, at random points, normals and
  samples; the descent steered to the chosen emitter (an emitter hit's MIS
  weight) finds the same size.
- Images rendered with tree selection (MIS and NEE only, with and without an
  environment, and the city's 10,000 emissive triangles) match the oracle's
  tree images at identical sample indices: mean relative pixel error
  <= 1e-4 and at most 0.1% of pixels above 1e-3.
"""
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


def _city_subset():
    return g.city(blocks=16, target_tris=1_000_000, emissive_cells=5000)


@pytest.mark.parametrize("which", ["field", "field_env", "city"])
def test_light_sample_bitexact(Renderer, orc, which):
    sc = {"field": lambda: g.light_field(n_lights=2000),
          "field_env": lambda: g.light_field(n_lights=300, env=True),
          "city": _city_subset}[which]()
    _say(f"[light tree] sampling {which}, tris={sc.num_triangles}")
    r = Renderer(sc, pool_paths=1 << 14)
    n = 100_003
    rng = np.random.default_rng(5)
    lo, hi = sc.positions.min(0), sc.positions.max(0)
    x = rng.uniform(lo, hi, (n, 3)).astype(np.float32)
    nrm = rng.normal(size=(n, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    S = rng.integers(0, 1 << 63, n, dtype=np.uint64)
    S[:4] = [0, (1 << 63) - 1, 1 << 62, 12345]
    e = torch.empty(n, dtype=torch.int32, device="cuda")
    z = torch.empty(n, dtype=torch.int64, device="cuda")
    zh = torch.empty(n, dtype=torch.int64, device="cuda")
    r.ctx.debug_light_sample(_dev(S.view(np.int64)), _dev(x), _dev(nrm), n, e, z, zh)
    torch.cuda.synchronize()
    ge = e.cpu().numpy().view(np.uint32)
    gz = z.cpu().numpy().view(np.uint64)
    gzh = zh.cpu().numpy().view(np.uint64)
    oe, oz = orc.Scene(sc, build_bvh=False).light_tree_sample(S, x, nrm)
    agree = np.mean((ge == oe) & (gz == oz))
    _say(f"    emitter and size agree on {agree:.6f} of {n}")
    assert np.array_equal(ge, oe) and np.array_equal(gz, oz)
    assert np.array_equal(gzh, gz)


def _parity(Renderer, orc, sc, passes, pix=None, **kw):
    r = Renderer(sc, pool_paths=kw.pop("pool_paths", 0))
    r.render(0, passes, light_tree=True, **kw)
    s, c = r.readback()
    assert np.all(c == passes)
    so, _, co, _ = orc.Scene(sc).render(pixels=pix, npasses=passes, light_tree=True, **kw)
    if pix is not None:
        s = s[pix]
    mean_e, frac, e = orc.image_parity(s, so)
    _say(f"    mean rel err {mean_e:.3e}, pixels > 1e-3: {frac:.4%}, max {e.max():.3e}")
    assert mean_e <= 1e-4 and frac <= 1e-3


@pytest.mark.parametrize("env,mode", [(False, 0), (False, 2), (True, 0)])
def test_image_parity_light_field(Renderer, orc, env, mode):
    sc = g.light_field(n_lights=2000, width=96, height=64, max_depth=6, env=env)
    _say(f"[light tree] image light_field 96x64 D=6 env={env} mode={mode}")
    _parity(Renderer, orc, sc, 16, mode=mode)


def test_image_parity_city_subset(Renderer, orc):
    """The city at 1/16 of its blocks (10,000 emissive triangles) at 3840 x 2160,
    tree selection; every 16th pixel, 2 passes, pixel-chunked passes."""
    sc = _city_subset()
    _say(f"[light tree] image city 3840x2160 tris={sc.num_triangles} passes=2 D=16")
    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(0, H, 16), np.arange(0, W, 16), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    _parity(Renderer, orc, sc, 2, pix=pix, pool_paths=1 << 21)


def test_render_rejects_bad_light_option(Renderer):
    from paper_1705_01263_amd import QptError
    r = Renderer(g.cornell(width=16, height=16), pool_paths=1 << 12)
    with pytest.raises(QptError):
        r.ctx.render_pass(0, 1, 4, light_tree=2)
    r.render(0, 1, light_tree=True)
    _, c = r.readback()
    assert np.all(c == 1)
