"""What the trained network gains over the plain tracer (GPU, through the C-ABI).

Slit workload at 480 x 270 (1M triangles, depth 16; the camera sees only
indirectly lit surfaces). A guide trained online for 512 passes (one Adam
step per pass, alpha 0.7, vertices 1-2) and then frozen renders 256 passes; the plain tracer renders
the same 256 passes. Both are compared with a 4096-pass plain reference from
an independent pass range, which is itself checked against the FP64 CPU
oracle on a pixel sample. Equal passes rather than equal time keep the test
deterministic (seeded Halton sampling, no timing); the equal-time comparison
is reported by bench.py.
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


def _rmse(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)))


def test_trained_guide_lowers_error(orc):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01263_amd import Renderer

    sc = g.slit_scene(width=480, height=270, target_tris=1_000_000, max_depth=16)
    r = Renderer(sc)
    _say("[gain] reference: plain, 4096 passes")
    r.render(1 << 24, 4096)
    s, c = r.readback()
    ref = s / c[:, None]
    r.reset()
    r.render(0, 256)
    s, c = r.readback()
    plain = s / c[:, None]
    r.reset()
    _say("[gain] training the guide for 512 passes")
    r.ctx.guide_set_weights(g.guide_init(1))
    r.ctx.guide_config(alpha=0.7, lr=1e-3, batch=1 << 16, train=1, warmup_steps=8, seed=1, max_vertex=2)
    r.render(1 << 20, 512)
    r.reset()
    r.ctx.guide_config(alpha=0.7, lr=1e-3, batch=1 << 16, train=0, warmup_steps=0, seed=1, max_vertex=2)
    r.render(0, 256)
    s, c = r.readback()
    guided = s / c[:, None]
    _, steps = r.ctx.guide_get_weights()
    e_p, e_g = _rmse(plain, ref), _rmse(guided, ref)
    _say(f"[gain] {steps} Adam steps; RMSE over 256 passes: plain {e_p:.6f}, guided {e_g:.6f} ({e_g / e_p:.3f}x)")
    assert steps == 512
    assert e_g < 0.95 * e_p
    # the reference against the FP64 oracle on a pixel sample: with 4096
    # reference, 2048 oracle and 256 plain passes the expected ratio of the
    # two errors is sqrt((1/2048 + 1/4096) / (1/2048 + 1/256)) = 0.41
    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(4, H, 16), np.arange(8, W, 16), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    S = orc.Scene(sc)
    so, _, co, _ = S.render(pixels=pix, pass0=1 << 25, npasses=2048, nthreads=16)
    o_ref = so / co[:, None]
    e_ref = _rmse(ref[pix], o_ref)
    e_plain_o = _rmse(plain[pix], o_ref)
    _say(f"[gain] on {pix.shape[0]} px vs the oracle (2048 passes): reference {e_ref:.6f}, plain {e_plain_o:.6f}")
    assert e_ref < 0.6 * e_plain_o
