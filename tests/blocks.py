"""Block test of two Monte Carlo images (shared by GPU tests)."""
import sys

import numpy as np


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def block_test(g_mean, o_mean, o_sum, o_sumsq, n_o, n_g, W, H, pix=None, block=16, tag=""):
    """Unbiasedness of a GPU estimator against the oracle's: both images
    from disjoint pass ranges, per channel the mean of every block of
    block x block pixels (of the listed pixels, by their frame position)
    within 3 standard errors of the difference, the errors from the oracle's
    per-pixel sample variance (the QMC points spread more evenly than
    independent samples, so this is conservative). At most 1% of the
    block-channel pairs, and at least one, may fall outside."""
    var = np.maximum(o_sumsq / n_o - (o_sum / n_o) ** 2, 0.0)   # per-sample variance per pixel
    if pix is None:
        ys, xs = np.divmod(np.arange(W * H), W)
    else:
        ys, xs = np.divmod(pix.astype(np.int64), W)
    bid = (ys // block) * ((W + block - 1) // block) + xs // block
    nb = int(bid.max()) + 1
    cnt = np.bincount(bid, minlength=nb).astype(np.float64)
    bad = total = 0
    worst = 0.0
    for c in range(3):
        gm = np.bincount(bid, g_mean[:, c], nb) / np.maximum(cnt, 1)
        om = np.bincount(bid, o_mean[:, c], nb) / np.maximum(cnt, 1)
        # standard error of a block mean: sqrt(sum of pixel variances / n) / pixels
        se = np.sqrt(np.bincount(bid, var[:, c], nb) * (1.0 / n_o + 1.0 / n_g)) / np.maximum(cnt, 1)
        used = cnt > 0
        z = np.abs(gm - om)[used] / np.maximum(se[used], 1e-12 * np.abs(om[used]).max() + 1e-30)
        bad += int(np.sum(z > 3.0))
        total += int(used.sum())
        worst = max(worst, float(z.max()))
    _say(f"[{tag}] block test: {bad} of {total} block-channel means beyond 3 sigma, largest {worst:.2f} sigma")
    assert bad <= max(1, int(0.01 * total)), (bad, total)


