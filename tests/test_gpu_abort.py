"""Stopping enqueued rendering through the host-mapped abort word (the
driver-timeout recovery of Appendix A.4), forced from the host: passes are
done whole or not at all, the counts show the progress, and rendering the
remaining passes gives the uninterrupted image bit for bit (whole-pass
batches and pixel-chunked passes alike)."""
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


def test_abort_before_render(Renderer):
    from paper_1705_01263_amd import QptError
    sc = g.cornell(width=32, height=32)
    r = Renderer(sc, pool_paths=1 << 12)
    r.render(0, 8)
    r.ctx.abort()
    with pytest.raises(QptError):
        r.render(8, 8)  # refused while the request stands
    s, c = r.readback()
    assert r.aborted and np.all(c == 8)
    r.render(8, 8)
    s, c = r.readback()
    assert not r.aborted and np.all(c == 16)
    ref = Renderer(sc, pool_paths=1 << 12)
    ref.render(0, 16)
    s2, c2 = ref.readback()
    assert np.array_equal(s, s2) and np.array_equal(c, c2)


@pytest.mark.parametrize("pool", [1 << 13, 1 << 11])  # two passes per batch; two pixel chunks per pass
def test_abort_midway_and_resume(Renderer, pool):
    sc = g.cornell(width=64, height=64, max_depth=8)
    total = 240
    _say(f"[abort] cornell 64x64 pool={pool} passes={total}")
    r = Renderer(sc, pool_paths=pool)
    r.render(0, total)   # enqueued; returns at once
    r.ctx.abort()        # most batches have not started yet
    s, c = r.readback()
    done = int(c[0])
    _say(f"    aborted={r.aborted}, passes done {done}")
    assert np.all(c == done) and done <= total
    if pool == 1 << 13:
        assert done % 2 == 0
    r.render(done, total - done)
    s, c = r.readback()
    assert not r.aborted and np.all(c == total)
    ref = Renderer(sc, pool_paths=pool)
    ref.render(0, total)
    s2, c2 = ref.readback()
    assert np.array_equal(s, s2)
