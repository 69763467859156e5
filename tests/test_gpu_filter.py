"""GPU parity of the Gaussian pixel filter (Appendix A.1) through the C-ABI:
images with filter importance sampling match the oracle's at identical
sample indices (mean relative pixel error <= 1e-4, at most 0.1% of pixels
above 1e-3), and an emitter edge across the view gives Le times the normal
CDF of the pixel centre's distance to it."""
import math
import sys

import numpy as np
import pytest

import scenegen as g
from test_oracle_filter import _edge_film_x, _edge_scene, _phi

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


@pytest.mark.parametrize("mode", [0, 2])
def test_image_parity_gauss(Renderer, orc, mode):
    sc = g.workload("cornell")
    _say(f"[filter] cornell 128x128x16 gauss mode={mode}")
    r = Renderer(sc)
    r.render(0, sc.spp, mode=mode, gauss=True)
    s, c = r.readback()
    assert np.all(c == sc.spp)
    so, _, co, _ = orc.Scene(sc).render(npasses=sc.spp, mode=mode, gauss=True)
    mean_e, frac, e = orc.image_parity(s, so)
    _say(f"    mean rel err {mean_e:.3e}, pixels > 1e-3: {frac:.4%}, max {e.max():.3e}")
    assert mean_e <= 1e-4 and frac <= 1e-3


def test_edge_closed_form_gpu(Renderer):
    W, H, Le = 12, 4, 2.0
    x_edge = 0.3137
    sc = _edge_scene(W, H, x_edge, Le)
    r = Renderer(sc, pool_paths=1 << 16)
    r.render(0, 16384, rr=False, gauss=True)
    s, c = r.readback()
    img = (s[:, 0] / c).reshape(H, W)
    e = _edge_film_x(sc, x_edge)
    want = np.array([Le * _phi((px + 0.5 - e) / 0.5) for px in range(W)])
    assert np.allclose(img, want[None, :], atol=2e-3 * Le), (img, want)
