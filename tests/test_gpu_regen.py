"""Regeneration of terminated paths (render option regen_paths, Sec. 3.1.3):
a batch's paths run through fewer state slots than the batch has paths, and
once more than half of the slots are free the free ones start the batch's
next paths, each iteration tracing and shading live paths of every depth.
The FP64 sums, counts and ray counters equal those of the per-depth
wavefront (one slot per path) bit for bit: from a live pool of one wave to
one larger than the batch, with several batches per call, the Gaussian pixel
filter, the light tree and the environment pyramid."""
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


def _render(r, passes, first=0, **kw):
    r.reset()
    st0 = r.stats()
    r.render(first, passes, **kw)
    s, c = r.readback()
    st = r.stats()
    return s, c, (st.rays_extension - st0.rays_extension, st.rays_shadow - st0.rays_shadow, st.paths - st0.paths)


def _same(got, base, tag):
    assert np.array_equal(got[1], base[1]), tag
    assert np.array_equal(got[0], base[0]), tag
    assert got[2] == base[2], (tag, got[2], base[2])


@pytest.mark.parametrize("case", ["cornell", "grid", "env"])
def test_regen_bit_identical(Renderer, case):
    if case == "cornell":
        sc, passes = g.workload("cornell"), 16
    elif case == "grid":
        sc, passes = g.grid_scene(grid=8, width=320, height=180), 8
    else:
        sc, passes = g.light_field(n_lights=300, width=96, height=64, max_depth=8, env=True), 8
    npaths = sc.width * sc.height * passes
    pool = 1 << 16
    while pool < npaths:
        pool <<= 1
    r = Renderer(sc, pool_paths=pool)
    base = _render(r, passes, single_stream=True)
    _say(f"[regen] {case}: {sc.num_triangles} triangles, {sc.width}x{sc.height}, rays {base[2]}")
    for live in (64, 1000, 1 << 14, npaths // 3, npaths, pool):
        got = _render(r, passes, regen_paths=live)
        _say(f"    regen_paths {live}: rays {got[2]}")
        _same(got, base, (case, live))


def test_regen_options_and_batches(Renderer):
    """Several batches per call (a pool of 2^16 paths holds four frames of
    128 x 128: 20 passes are five batches), the Gaussian filter, the light
    tree, the environment pyramid, and a pass range that does not start at 0."""
    sc = g.light_field(n_lights=400, width=128, height=128, max_depth=6, env=True)
    r = Renderer(sc, pool_paths=1 << 16)
    for kw in ({}, {"gauss": True}, {"light_tree": True}, {"env_sampling": 2}):
        base = _render(r, 20, first=1000, single_stream=True, **kw)
        got = _render(r, 20, first=1000, regen_paths=5000, **kw)
        _say(f"[regen] light field, 20 passes in batches of 4 frames, {kw}: rays {got[2]}")
        _same(got, base, kw)


def test_regen_ignored_for_guided_and_validated(Renderer):
    from paper_1705_01263_amd import qpt
    sc = g.cornell(width=64, height=64, max_depth=8)
    r = Renderer(sc, pool_paths=1 << 16)
    with pytest.raises(qpt.QptError, match="regen_paths"):
        r.render(0, 1, regen_paths=32)
    with pytest.raises(qpt.QptError, match="regen_paths"):
        r.render(0, 1, regen_paths=(1 << 16) + 1)
    # a frozen guide samples: regeneration does not apply, the image is the guided one
    r.ctx.guide_set_weights(g.guide_frozen(5))
    r.ctx.guide_config(alpha=0.5, lr=1e-3, batch=1 << 12, train=0, warmup_steps=0, seed=1, max_vertex=0)
    a = _render(r, 4, single_stream=True)
    b = _render(r, 4, regen_paths=256)
    _same(b, a, "guided")
