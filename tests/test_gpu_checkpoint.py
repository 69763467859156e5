"""Checkpoint and resume through the C-ABI: the framebuffer saved by
qpt_readback and loaded into a fresh context continues the progressive image
bit for bit; the guide's optimiser state (weights, Adam moments, step count)
round-trips and a restored guide takes the same Adam step as the original."""
import numpy as np
import pytest

import scenegen as g
from oracle import guide as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def Renderer():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01263_amd import Renderer as R
    return R


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def test_framebuffer_resume(Renderer):
    sc = g.workload("cornell")
    a = Renderer(sc)
    a.render(0, 10)
    s, c = a.readback()
    del a
    b = Renderer(sc)               # a fresh context, as after a restart
    b.ctx.load_accum(s, c)
    b.render(10, 14)
    s2, c2 = b.readback()
    ref = Renderer(sc)
    ref.render(0, 24)
    s3, c3 = ref.readback()
    assert np.all(c2 == 24) and np.array_equal(c2, c3) and np.array_equal(s2, s3)


def test_guide_state_resume(Renderer):
    sc = g.cornell(width=16, height=16)
    rng = np.random.default_rng(3)
    n = 1024
    x = rng.uniform(-1, 1, (n, 3))
    wo = rng.normal(size=(n, 3))
    wo /= np.linalg.norm(wo, axis=1, keepdims=True)
    X = G.encode(x, wo, [-1, -1, -1], [2, 2, 2])
    w = rng.normal(size=(n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    wt = rng.uniform(0.5, 1.5, n)
    grad = torch.empty(G.NPARAM, dtype=torch.float32, device="cuda")
    a = Renderer(sc, pool_paths=1 << 12)
    a.ctx.guide_set_weights(g.guide_init(4))
    for _ in range(3):
        a.ctx.guide_debug_train(_dev(X), _dev(w), _dev(wt), n, 1e-3, grad)
    p, m, v, steps = a.ctx.guide_get_state()
    assert steps == 3 and np.any(m != 0) and np.all(v >= 0)
    b = Renderer(sc, pool_paths=1 << 12)
    b.ctx.guide_set_state(p, m, v, steps)
    p2, m2, v2, steps2 = b.ctx.guide_get_state()
    assert steps2 == 3 and np.array_equal(p, p2) and np.array_equal(m, m2) and np.array_equal(v, v2)
    for r in (a, b):
        r.ctx.guide_debug_train(_dev(X), _dev(w), _dev(wt), n, 1e-3, grad)
    pa, ma, va, sa = a.ctx.guide_get_state()
    pb, mb, vb, sb = b.ctx.guide_get_state()
    assert sa == sb == 4
    assert np.array_equal(pa, pb) and np.array_equal(ma, mb) and np.array_equal(va, vb)
