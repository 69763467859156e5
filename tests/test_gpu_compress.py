"""Compressed path state (render option compress_state, Sec. 3.1.1): the
next ray's direction as an octahedral pair of 16-bit values, throughput and
sampling density in half precision, barycentrics as 16-bit fixed point.

- The compressed estimator is unbiased: against the oracle's full-precision
  render from a disjoint pass range, every 16 x 16 block mean within 3
  standard errors (Cornell box with MIS and with BSDF sampling only, a light
  field under an environment map, the grid at 320 x 180).
- At identical sample indices it differs from the full-precision image only
  by paths that the quantisation sends elsewhere (reported, gross bounds).
- The schedules stay interchangeable: one stream, two batches in flight,
  the megakernel tail and regeneration give the same compressed image bit
  for bit.
"""
import sys

import numpy as np
import pytest

import oracle
import scenegen as g
from blocks import block_test

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


def _scene(case):
    if case.startswith("cornell"):
        return g.cornell(width=128, height=128, max_depth=8), (0 if case == "cornell_mis" else 1), 64
    if case == "light_field_env":
        return g.light_field(n_lights=300, width=64, height=48, max_depth=6, env=True), 0, 256
    return g.grid_scene(grid=8, width=320, height=180), 0, 32


@pytest.mark.parametrize("case", ["cornell_mis", "cornell_bsdf", "light_field_env", "grid"])
def test_compressed_unbiased(Renderer, case):
    sc, mode, n = _scene(case)
    _say(f"[compress] {case}: {sc.width}x{sc.height}, {sc.num_triangles} triangles, {n} passes, mode {mode}")
    r = Renderer(sc)
    r.render(1 << 20, n, mode=mode, compress_state=True)
    sg, cg = r.readback()
    assert np.all(cg == n)
    S = oracle.Scene(sc)
    so, sq, co, _ = S.render(npasses=n, mode=mode)
    assert np.all(co == n)
    block_test(sg / n, so / n, so, sq, n, n, sc.width, sc.height, block=16, tag=f"compress {case}")
    # identical indices: full precision against compressed
    r.reset()
    r.render(0, 16, mode=mode)
    sf, _ = r.readback()
    r.reset()
    r.render(0, 16, mode=mode, compress_state=True)
    sc_, _ = r.readback()
    mean_e, frac_bad, _ = oracle.image_parity(sc_, sf)
    tot = abs(float(sc_.sum()) - float(sf.sum())) / max(float(sf.sum()), 1e-30)
    _say(f"[compress] {case}: identical indices vs full precision: mean rel err {mean_e:.2e}, "
         f"pixels > 1e-3 {frac_bad:.3%}, totals {tot:.2e}")
    assert tot <= 0.02


def test_compressed_schedules_bit_identical(Renderer):
    sc = g.light_field(n_lights=400, width=128, height=128, max_depth=8, env=True)
    r = Renderer(sc, pool_paths=1 << 16)

    def run(**kw):
        r.reset()
        r.render(0, 12, compress_state=True, **kw)
        return r.readback()

    base = run(single_stream=True)
    for kw in ({}, {"single_stream": True, "tail_depth": 3}, {"regen_paths": 5000}):
        s, c = run(**kw)
        _say(f"[compress] schedule {kw}")
        assert np.array_equal(c, base[1]) and np.array_equal(s, base[0]), kw
