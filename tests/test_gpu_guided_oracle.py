"""GPU guided rendering and training records against the CPU oracle's guided
branch (the learned proposal mixed one-sided with BSDF sampling under MIS,
an extension of Sec. 2.1-2.2), through the C-ABI at identical sample indices.

- Training records at alpha = 0 (paths identical to plain): the set of
  records that enter the replay ring (positive, finite weight), keyed by
  (pixel, pass, vertex), equals the oracle's; positions, directions and
  densities agree to FP32 rounding; weights meet the image tolerance
  (mean relative error <= 1e-4, <= 0.1% of records above 1e-3).
- A frozen guide at alpha = 0.7 on every vertex: GPU images against the
  oracle's guided images at the image tolerance (Cornell box with MIS and
  with BSDF sampling only; a many-light field under an environment map).
- Records of a guided batch (alpha = 0.7, the frozen guide's first batch):
  records and their mixture densities against the oracle's.
"""
import sys

import numpy as np
import pytest

import oracle
import scenegen as g

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ALPHA = 0.7


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Renderer():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01263_amd import Renderer as R
    return R


def _gpu_records(r):
    cap = 1 << 20
    ident = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
    rec = torch.empty((cap, 11), dtype=torch.float32, device="cuda")
    n = r.ctx.guide_debug_records(ident, rec, cap)
    assert n <= cap
    ident = ident[:n].cpu().numpy().view(np.uint32).astype(np.int64)
    rec = rec[:n].cpu().numpy().astype(np.float64)
    return dict(pixel=ident[:, 0], pass_=ident[:, 1], vertex=ident[:, 2], x=rec[:, 0:3], wo=rec[:, 3:6],
                wi=rec[:, 6:9], pdf=rec[:, 9], weight=rec[:, 10])


def _key(rec):
    return rec["pixel"] * (1 << 24) + rec["pass_"] * 64 + rec["vertex"]


def _compare_records(gr, orc_rec, tag):
    sel_g = np.isfinite(gr["weight"]) & (gr["weight"] > 0)
    sel_o = np.isfinite(orc_rec["weight"]) & (orc_rec["weight"] > 0)
    kg, ko = _key(gr), _key(orc_rec)
    assert np.unique(kg).shape[0] == kg.shape[0], "one record per (pixel, pass, vertex)"
    # the replay ring's set: identical
    sg, so = set(kg[sel_g].tolist()), set(ko[sel_o].tolist())
    only_g, only_o = len(sg - so), len(so - sg)
    _say(f"[{tag}] records gpu {kg.shape[0]} oracle {ko.shape[0]}, selected gpu {len(sg)} oracle {len(so)}, "
         f"only gpu {only_g}, only oracle {only_o}")
    # a record exists on one side only where a path decided differently in
    # FP32 and FP64 (a grazing hit, a roulette or lobe choice at a tie)
    paths_g = set((gr["pixel"] * (1 << 24) + gr["pass_"] * 64).tolist())
    diff = (sg ^ so)
    diff_paths = {k - (k % 64) for k in diff}
    assert len(diff_paths) <= 1e-3 * max(len(paths_g), 1), (len(diff_paths), len(paths_g))
    # fields of the records both sides hold
    common, ig, io = np.intersect1d(kg, ko, return_indices=True)
    assert common.shape[0] >= 0.999 * min(kg.shape[0], ko.shape[0])
    for f, tol in (("x", 1e-4), ("wo", 1e-4), ("wi", 1e-4)):
        err = np.abs(gr[f][ig] - orc_rec[f][io]).max(1)
        bad = np.mean(err > tol)
        _say(f"[{tag}] {f}: max err {err.max():.2e}, fraction above {tol:g}: {bad:.2e}")
        assert bad <= 1e-3
    pg, po = gr["pdf"][ig], orc_rec["pdf"][io]
    rel = np.abs(pg - po) / np.maximum(np.abs(po), 1e-30)
    _say(f"[{tag}] pdf: median rel err {np.median(rel):.2e}, fraction above 1e-3: {np.mean(rel > 1e-3):.2e}")
    assert np.mean(rel > 1e-3) <= 1e-3
    wg, wo_ = gr["weight"][ig], orc_rec["weight"][io]
    eps = 1e-3 * np.mean(np.abs(wo_))
    e = np.abs(wg - wo_) / (np.abs(wo_) + eps)
    _say(f"[{tag}] weight: mean rel err {e.mean():.2e}, fraction above 1e-3: {np.mean(e > 1e-3):.2e}")
    assert e.mean() <= 1e-4 and np.mean(e > 1e-3) <= 1e-3


def test_records_alpha_zero(Renderer):
    sc = g.cornell(width=64, height=64, max_depth=8)
    theta = g.guide_frozen(5)
    r = Renderer(sc)
    r.ctx.guide_set_weights(theta)
    # recording on (one Adam step per pass), sampling off: paths as plain
    r.ctx.guide_config(alpha=0.0, lr=1e-3, batch=1 << 12, train=1, warmup_steps=0, seed=1, max_vertex=0)
    npass = 4
    r.render(0, npass)
    torch.cuda.synchronize()
    gr = _gpu_records(r)
    s, c = r.readback()
    S = oracle.Scene(sc)
    S.guide_set(theta, alpha=0.0)
    so, co, orc_rec = S.records(npasses=npass, guide=True)
    assert np.array_equal(c, co)
    mean_e, frac_bad, _ = oracle.image_parity(s, so)
    _say(f"[records alpha 0] image mean rel err {mean_e:.2e}, pixels > 1e-3 {frac_bad:.4%}")
    assert mean_e <= 1e-4 and frac_bad <= 1e-3
    _compare_records(gr, orc_rec, "records alpha 0")


@pytest.mark.parametrize("case", ["cornell_mis", "cornell_bsdf", "light_field_env"])
def test_frozen_guide_image_parity(Renderer, case):
    if case.startswith("cornell"):
        sc = g.cornell(width=128, height=128, max_depth=8)
        npass, mode = 16, (0 if case == "cornell_mis" else 1)
    else:
        sc = g.light_field(n_lights=300, width=64, height=48, max_depth=6, env=True)
        npass, mode = 32, 0
    theta = g.guide_frozen(5)
    _say(f"[frozen guide {case}] {sc.width}x{sc.height} passes {npass} mode {mode}")
    r = Renderer(sc)
    r.ctx.guide_set_weights(theta)
    r.ctx.guide_config(alpha=ALPHA, lr=1e-3, batch=1 << 12, train=0, warmup_steps=0, seed=1, max_vertex=0)
    r.render(0, npass, mode=mode)
    s, c = r.readback()
    assert np.all(c == npass)
    S = oracle.Scene(sc)
    S.guide_set(theta, alpha=ALPHA)
    so, _, co, _ = S.render(npasses=npass, mode=mode, guide=True)
    mean_e, frac_bad, _ = oracle.image_parity(s, so)
    # the plain image at the same indices differs by far more than the tolerance
    sp, _, _, _ = S.render(npasses=npass, mode=mode)
    mean_p, _, _ = oracle.image_parity(sp, so)
    _say(f"[frozen guide {case}] mean rel err {mean_e:.2e}, pixels > 1e-3 {frac_bad:.4%} "
         f"(plain vs guided oracle: {mean_p:.2e})")
    assert mean_p > 1e-2
    assert mean_e <= 1e-4 and frac_bad <= 1e-3


def test_records_guided_first_batch(Renderer):
    """The first batch of a training run renders with the weights it was
    given (training steps publish into the other buffer), so its image and
    records are those of the frozen guide."""
    sc = g.cornell(width=64, height=64, max_depth=8)
    theta = g.guide_frozen(5)
    r = Renderer(sc)
    r.ctx.guide_set_weights(theta)
    r.ctx.guide_config(alpha=ALPHA, lr=1e-3, batch=1 << 12, train=1, warmup_steps=0, seed=1, max_vertex=0)
    npass = 4
    r.render(0, npass)
    torch.cuda.synchronize()
    gr = _gpu_records(r)
    s, c = r.readback()
    S = oracle.Scene(sc)
    S.guide_set(theta, alpha=ALPHA)
    so, co, orc_rec = S.records(npasses=npass, guide=True)
    mean_e, frac_bad, _ = oracle.image_parity(s, so)
    _say(f"[records guided] image mean rel err {mean_e:.2e}, pixels > 1e-3 {frac_bad:.4%}")
    assert mean_e <= 1e-4 and frac_bad <= 1e-3
    _compare_records(gr, orc_rec, "records guided")
