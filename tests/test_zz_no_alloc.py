"""The allocation-free GPU BVH build (qpt_build_bvh_noalloc: temporaries in
the library's fixed device region) against the GPU builder with caller
scratch (qpt_build_bvh, builder = 1) through the C-ABI: the same tree (child
boxes and leaf ranges bit for bit; node numbers aside, which follow the order
in which the builder's threads claim them) and the same leaf order, on two
calls in a row on one context, the second with a smaller scene; a scene beyond the region's size is refused with a
message; the tree renders the same image as the caller-scratch tree."""
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
def qpt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_01263_amd import qpt as q
    return q


def _same_tree(a, b):
    """The two device trees are the same tree: from the roots down, the same
    used slots, child boxes (bit for bit) and leaf ranges in every node. Node
    numbers are not compared: the GPU builder numbers nodes in the order its
    threads claim them, which varies from build to build."""
    la, lb = a.view(np.uint32), b.view(np.uint32)
    todo = [(0, 0)]
    seen = 0
    while todo:
        i, j = todo.pop()
        seen += 1
        na, nb = la[i], lb[j]
        used = int(na[28])
        assert used == int(nb[28]), (i, j)
        for c in range(4):
            for axis in range(6):
                assert na[axis * 4 + c] == nb[axis * 4 + c], (i, j, c, axis)
            ra, rb = int(na[24 + c]), int(nb[24 + c])
            if ra >= 1 << 31:   # leaf (negative reference) or an unused slot
                assert ra == rb, (i, j, c)
            else:
                assert rb < 1 << 31, (i, j, c)
                todo.append((ra, rb))
    assert seen == a.shape[0] == b.shape[0]


def _with_scratch(c):
    nb = c.bvh_scratch_size()
    tmp = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    st = c.build_bvh(builder=1, scratch=(tmp.data_ptr() + 255) & ~255, scratch_bytes=nb)
    torch.cuda.synchronize()
    return st, c.debug_bvh_nodes()


def test_noalloc_build_matches_scratch_build(qpt):
    c = qpt.Context(0)
    ref = qpt.Context(0)
    scenes = [g.grid_scene(grid=6, width=64, height=64), g.workload("cornell")]
    assert scenes[1].num_triangles < scenes[0].num_triangles
    for sc in scenes:
        _say(f"[noalloc] {sc.name} tris={sc.num_triangles}")
        c.ntri = ref.ntri = sc.num_triangles
        c.build_scene(sc)
        ref.build_scene(sc)
        need = c.bvh_scratch_size()
        assert need <= 64 << 20
        st = c.build_bvh_noalloc()
        nodes, order = c.debug_bvh_nodes()
        st_r, (nodes_r, order_r) = _with_scratch(ref)
        _say(f"    nodes {st.num_nodes} vs {st_r.num_nodes}, scratch {need} bytes")
        assert st.num_nodes == st_r.num_nodes and st.num_leaves == st_r.num_leaves and st.max_depth == st_r.max_depth
        _same_tree(nodes, nodes_r)
        assert np.array_equal(order, order_r)
        assert np.array_equal(np.sort(order), np.arange(sc.num_triangles, dtype=np.uint32))


def test_noalloc_refuses_large_scene(qpt):
    c = qpt.Context(0)
    sc = g.city(blocks=8, target_tris=400_000, emissive_cells=500)
    c.ntri = sc.num_triangles
    c.build_scene(sc)
    assert c.bvh_scratch_size() > 64 << 20
    with pytest.raises(qpt.QptError, match="too large"):
        c.build_bvh_noalloc()


def test_noalloc_tree_renders(qpt):
    from paper_1705_01263_amd import Renderer
    sc = g.workload("cornell")
    r = Renderer(sc, bvh_builder=1)
    r.render(0, 4)
    s_ref, c_ref = r.readback()
    r.ctx.build_bvh_noalloc()
    nbytes = r.ctx.workspace_size(0)
    assert nbytes <= r.ws.numel() - 256
    r.ctx.bind_workspace((r.ws.data_ptr() + 255) & ~255, nbytes, 0)
    r.render(0, 4)
    s, c = r.readback()
    assert np.array_equal(c, c_ref) and np.array_equal(s, s_ref)
