"""GPU parity of the environment pyramid (Sec. 2.1.2) through the C-ABI.

- The renderer's descent (24-bit shares, 32-bit integer intervals, FP32
  normal bins) finds the oracle's texel and intervals bit for bit, with and
  without the normal-weighted top levels, on a small sky map and on the
  2048 x 1024 sun-and-sky map; the descent steered to that texel (an
  environment hit's MIS weight) finds the same interval sizes.
- Images with pyramid sampling (MIS and NEE only, with and without the
  normal weighting) match the oracle's at identical sample indices: mean
  relative pixel error <= 1e-4 and at most 0.1% of pixels above 1e-3.
- A map of other shape is refused for pyramid sampling.
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


@pytest.mark.parametrize("env", [(64, 32), (2048, 1024)])
@pytest.mark.parametrize("mode", [1, 2])
def test_env_sample_bitexact(Renderer, orc, env, mode):
    sc = g.instanced_env_scene(width=16, height=16, target_tris=2000, env_size=env)
    _say(f"[env pyramid] sampling env={env} mode={mode}")
    r = Renderer(sc, pool_paths=1 << 12)
    n = 30_011
    rng = np.random.default_rng(7)
    uv = rng.integers(0, 1 << 32, (n, 2), dtype=np.uint64).astype(np.uint32)
    uv[0], uv[1] = (0, 0), (0xFFFFFFFF, 0xFFFFFFFF)
    nrm = rng.normal(size=(n, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    nrm[2:8] = [[0, 1, 0], [0, -1, 0], [1, 0, 0], [-1, 0, 0], [0, 0, 1], [0, 0, -1]]
    texel = torch.empty(n, dtype=torch.int32, device="cuda")
    iv = torch.empty((n, 4), dtype=torch.int64, device="cuda")
    iv_hit = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    r.ctx.debug_env_sample(_dev(uv), _dev(nrm), n, mode, texel, iv, iv_hit)
    torch.cuda.synchronize()
    gt = texel.cpu().numpy().view(np.uint32)
    giv = iv.cpu().numpy().view(np.uint64)
    ghit = iv_hit.cpu().numpy().view(np.uint64)
    S = orc.Scene(sc, build_bvh=False)
    bins = np.array([orc.env_bin(v) if mode == 2 else -1 for v in nrm], np.int32)
    rows, cols, oiv = S.env_descend(bins, u=uv[:, 0], v=uv[:, 1])
    W = sc.env.shape[1]
    agree = np.mean((gt == rows * W + cols) & np.all(giv == oiv, axis=1))
    _say(f"    texel and intervals agree on {agree:.6f}")
    assert np.array_equal(gt, rows * W + cols) and np.array_equal(giv, oiv)
    assert np.array_equal(ghit[:, 0], giv[:, 0]) and np.array_equal(ghit[:, 1], giv[:, 2])


def _parity(Renderer, orc, sc, passes, pix=None, **kw):
    r = Renderer(sc, pool_paths=kw.pop("pool_paths", 0))
    r.render(0, passes, **kw)
    s, c = r.readback()
    assert np.all(c == passes)
    so, _, co, _ = orc.Scene(sc).render(pixels=pix, npasses=passes, **kw)
    if pix is not None:
        s = s[pix]
    mean_e, frac, e = orc.image_parity(s, so)
    _say(f"    mean rel err {mean_e:.3e}, pixels > 1e-3: {frac:.4%}, max {e.max():.3e}")
    assert mean_e <= 1e-4 and frac <= 1e-3


@pytest.mark.parametrize("env_sampling,mode", [(1, 0), (2, 0), (2, 2)])
def test_image_parity_sky(Renderer, orc, env_sampling, mode):
    sc = g.instanced_env_scene(width=96, height=64, target_tris=20_000, env_size=(256, 128), max_depth=6)
    _say(f"[env pyramid] image 96x64 env 256x128 env_sampling={env_sampling} mode={mode}")
    _parity(Renderer, orc, sc, 16, env_sampling=env_sampling, mode=mode)


def test_image_parity_env_subset(Renderer, orc):
    """The 4M-triangle instanced scene under the 2048 x 1024 sun-and-sky map,
    normal-weighted pyramid, every 8th pixel, 2 passes."""
    sc = g.workload("instanced_env_4m")
    _say(f"[env pyramid] image env 1920x1080 tris={sc.num_triangles} passes=2 D=16")
    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(0, H, 8), np.arange(0, W, 8), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    _parity(Renderer, orc, sc, 2, pix=pix, env_sampling=2)


def test_pyramid_needs_power_of_two_map(Renderer):
    from paper_1705_01263_amd import QptError
    sc = g.instanced_env_scene(width=16, height=16, target_tris=2000, env_size=(96, 48))
    r = Renderer(sc, pool_paths=1 << 12)
    with pytest.raises(QptError):
        r.render(0, 1, env_sampling=2)
    r.render(0, 1)  # the 2D CDF still works
    _, c = r.readback()
    assert np.all(c == 1)
