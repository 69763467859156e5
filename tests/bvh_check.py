"""Structural check of the renderer's 4-wide BVH (shared by the host-built
and GPU-built tree tests)."""
import numpy as np


def check_bvh4(nodes, order, sc, num_nodes, num_leaves):
    """Every triangle in exactly one leaf and inside its box, every child box
    inside its parent's slot box, 2-4 used slots per node (1 when the whole
    tree is one leaf), siblings stored together, every node but the root
    referenced once."""
    assert nodes.shape[0] == num_nodes
    assert np.array_equal(np.sort(order), np.arange(sc.num_triangles, dtype=np.uint32))
    lo = nodes[:, 0:12].reshape(-1, 3, 4)   # [node, axis, child]
    hi = nodes[:, 12:24].reshape(-1, 3, 4)
    refs = nodes[:, 24:28].copy().view(np.int32)
    used = nodes[:, 28:29].copy().view(np.int32)[:, 0]
    pos = sc.positions[sc.indices[order]]  # leaf order, (nt, 3, 3)
    seen = np.zeros(sc.num_triangles, np.int32)
    parents = np.zeros(nodes.shape[0], np.int32)
    leaves = 0
    for k in range(nodes.shape[0]):
        nu = int(used[k])
        assert (2 <= nu <= 4) or (nodes.shape[0] == 1 and nu == 1)
        for ch in range(4):
            r = int(refs[k, ch])
            if ch >= nu:
                assert r == -(2 ** 31)
                continue
            assert r != -(2 ** 31)
            blo, bhi = lo[k, :, ch], hi[k, :, ch]
            if r >= 0:
                parents[r] += 1
                cu = int(used[r])
                assert np.all(lo[r, :, :cu] >= blo[:, None]) and np.all(hi[r, :, :cu] <= bhi[:, None])
            else:
                p = ~np.int64(r) & 0xFFFFFFFF
                first, cnt = p >> 3, (p & 7) + 1
                tri = pos[first:first + cnt]
                assert np.all(tri >= blo) and np.all(tri <= bhi)
                seen[first:first + cnt] += 1
                leaves += 1
        kids = [int(x) for x in refs[k, :nu] if x >= 0]
        if kids:
            assert max(kids) - min(kids) == len(kids) - 1  # siblings contiguous
    assert np.all(seen == 1)
    assert parents[0] == 0 and np.all(parents[1:] == 1)
    assert leaves == num_leaves
