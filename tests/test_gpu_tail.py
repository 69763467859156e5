"""The megakernel tail (render option tail_depth, Sec. 3.1.3): from depth k on,
one launch takes every path still alive to its end with the same per-vertex
code as the per-depth kernels. The FP64 sums, counts and ray counters equal
the per-depth wavefront's bit for bit, with one batch at a time and with two
in flight, from the first depth (the whole batch in one launch) to a late one."""
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


def _render(r, passes, **kw):
    r.reset()
    st0 = r.stats()
    r.render(0, passes, **kw)
    s, c = r.readback()
    st = r.stats()
    return s, c, (st.rays_extension - st0.rays_extension, st.rays_shadow - st0.rays_shadow, st.paths - st0.paths)


@pytest.mark.parametrize("case", ["cornell", "grid", "env"])
def test_tail_bit_identical(Renderer, case):
    if case == "cornell":
        sc, passes = g.workload("cornell"), 16
    elif case == "grid":
        sc, passes = g.grid_scene(grid=8, width=320, height=180), 8
    else:
        sc, passes = g.light_field(n_lights=300, width=96, height=64, max_depth=8, env=True), 8
    r = Renderer(sc)
    base = _render(r, passes)
    _say(f"[tail] {case}: {sc.num_triangles} triangles, rays {base[2]}")
    for k in (1, 3, sc.max_depth):
        for single in (True, False):
            got = _render(r, passes, tail_depth=k, single_stream=single)
            _say(f"    tail_depth {k} single_stream {single}: rays {got[2]}")
            assert np.array_equal(got[1], base[1])
            assert np.array_equal(got[0], base[0]), (k, single)
            assert got[2] == base[2]


def _records(r):
    cap = 1 << 20
    ident = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
    rec = torch.empty((cap, 11), dtype=torch.float32, device="cuda")
    n = r.ctx.guide_debug_records(ident, rec, cap)
    ident = ident[:n].cpu().numpy().view(np.uint32).astype(np.int64)
    rec = rec[:n].cpu().numpy()
    key = (ident[:, 0] << 24) + (ident[:, 1] << 6) + ident[:, 2]
    o = np.argsort(key, kind="stable")
    return key[o], rec[o]


def test_tail_guided_bit_identical(Renderer):
    """With the guide sampling vertices 1-2 (alpha 0.7, frozen weights) and
    training records on, a tail from depth 3 (past the guided vertices)
    leaves the image, the ray counts and every record (identity, fields and
    weight) as the per-depth kernels do; a tail at a guided depth is
    ignored."""
    sc = g.cornell(width=128, height=128, max_depth=8)
    r = Renderer(sc, pool_paths=1 << 18)
    r.ctx.guide_set_weights(g.guide_frozen(5))
    r.ctx.guide_config(alpha=0.7, lr=1e-3, batch=1 << 12, train=1, warmup_steps=0, seed=1, max_vertex=2)
    passes = 16  # one batch: the image does not depend on the training that follows it
    base = _render(r, passes)
    kb, rb = _records(r)
    _say(f"[tail guided] rays {base[2]}, records {kb.shape[0]}")
    assert kb.shape[0] > 1000
    for k in (2, 3, sc.max_depth):
        r.ctx.guide_set_weights(g.guide_frozen(5))
        got = _render(r, passes, tail_depth=k)
        kg, rg = _records(r)
        _say(f"    tail_depth {k}: rays {got[2]}, records {kg.shape[0]}")
        assert np.array_equal(got[1], base[1]) and np.array_equal(got[0], base[0]), k
        assert got[2] == base[2]
        assert np.array_equal(kg, kb) and np.array_equal(rg.view(np.uint32), rb.view(np.uint32)), k
