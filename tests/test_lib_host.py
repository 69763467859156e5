"""CPU checks of libqpt: it loads, exports every symbol of include/qpt.h, and its
host-side builders (alias table, light pmf, environment CDFs, BVH) agree with
the independent oracle and are structurally valid. No compute call here
needs a GPU: a context on device -1 only runs the host builders.
"""
import os
import re

import numpy as np
import pytest

import scenegen as g
from bvh_check import check_bvh4

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def qpt():
    from paper_1705_01263_amd import qpt as q
    q.lib()
    return q


def _declared():
    txt = open(os.path.join(ROOT, "include", "qpt.h")).read()
    return sorted(set(re.findall(r"\b(qpt_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(qpt):
    L = qpt.lib()
    names = _declared()
    assert "qpt_render_pass" in names and "qpt_build_bvh" in names
    for n in names:
        assert hasattr(L, n), n
    assert sorted(qpt.EXPORTS) == names


def test_call_order_and_errors(qpt):
    c = qpt.Context(-1)
    with pytest.raises(qpt.QptError):
        c.build_bvh()  # before build_scene
    sc = g.workload("cornell")
    sc2 = g.workload("cornell")
    sc2.indices = sc2.indices.copy()
    sc2.indices[0, 0] = 10_000  # out of range
    with pytest.raises(qpt.QptError):
        c.build_scene(sc2)
    c.build_scene(sc)
    with pytest.raises(qpt.QptError):
        c.workspace_size()  # before build_bvh
    c.build_bvh()
    assert c.workspace_size(1 << 16) > 0
    with pytest.raises(qpt.QptError):
        c.bind_workspace(0x1000, 1 << 30)  # host-only context: no device
    with pytest.raises(qpt.QptError):
        c.render_pass(0, 1, 8)


@pytest.mark.parametrize("make", [lambda: g.workload("cornell"), lambda: g.grid_scene(grid=2)])
def test_light_tables_match_oracle(qpt, orc, make):
    sc = make()
    c = qpt.Context(-1)
    c.build_scene(sc)
    mine = c.debug_light_tables()
    ref = orc.Scene(sc, build_bvh=False).lights()
    assert np.array_equal(mine["tri"], ref["tri"])
    assert np.array_equal(mine["alias"], ref["alias"])
    assert np.array_equal(mine["prob"], ref["prob"])   # bit-identical FP64 tables
    assert np.array_equal(mine["pmf"], ref["pmf"])


def test_env_tables_match_oracle(qpt, orc):
    sc = g.instanced_env_scene(target_tris=1000, env_size=(256, 128))
    c = qpt.Context(-1)
    c.build_scene(sc)
    eh, ew = sc.env.shape[:2]
    rq, cq, pdf = c.debug_env_tables(eh, ew)
    orq, ocq, opdf = orc.Scene(sc, build_bvh=False).env_tables()
    assert np.array_equal(rq.astype(np.uint64), orq[:eh])
    assert np.array_equal(cq.astype(np.uint64), ocq[:, :ew])
    assert np.array_equal(pdf, opdf.astype(np.float32))


@pytest.mark.parametrize("make", [lambda: g.workload("cornell"), lambda: g.grid_scene(grid=4),
                                  lambda: g.quad_over_plane()])
def test_bvh_structure(qpt, make):
    """The 4-wide tree: every triangle in exactly one leaf and inside its
    box, every child box inside its parent's slot box, 2-4 used slots per
    node (1 when the whole tree is one leaf), siblings stored together."""
    sc = make()
    c = qpt.Context(-1)
    c.ntri = sc.num_triangles
    c.build_scene(sc)
    st = c.build_bvh()
    assert st.max_depth < 32
    nodes, order = c.debug_bvh_nodes()
    check_bvh4(nodes, order, sc, st.num_nodes, st.num_leaves)


TOP_NODES = 64  # nodes the traversal kernels keep in LDS


@pytest.mark.parametrize("make", [lambda: g.grid_scene(grid=4), lambda: g.city(blocks=4, target_tris=60_000,
                                                                              emissive_cells=50)])
def test_bvh_top_levels_first(qpt, make):
    """The host builder numbers the tree breadth-first until TOP_NODES nodes
    exist: the first TOP_NODES node numbers go to whole top levels in level
    order (depth never decreases along them, and every node above the
    deepest of them is among them), the root is node 0, and every node is
    reachable from it exactly once (check_bvh4 covers the rest)."""
    sc = make()
    c = qpt.Context(-1)
    c.build_scene(sc)
    st = c.build_bvh()
    nodes, _ = c.debug_bvh_nodes()
    assert st.num_nodes > 2 * TOP_NODES
    refs = nodes[:, 24:28].copy().view(np.int32)
    used = nodes[:, 28:29].copy().view(np.int32)[:, 0]
    depth = np.full(nodes.shape[0], -1, np.int64)
    depth[0] = 0
    frontier = [0]
    while frontier:
        nxt = []
        for k in frontier:
            for r in refs[k, :used[k]]:
                if r >= 0:
                    assert depth[r] == -1
                    depth[r] = depth[k] + 1
                    nxt.append(int(r))
        frontier = nxt
    assert np.all(depth >= 0)
    top = depth[:TOP_NODES]
    assert np.all(np.diff(top) >= 0), "the first nodes are in level order"
    assert np.all(np.nonzero(depth < top[-1])[0] < TOP_NODES), "whole levels above the last staged one"


@pytest.mark.parametrize("make", [lambda: g.light_field(n_lights=700), lambda: g.light_field(n_lights=300, env=True),
                                  lambda: g.grid_scene(grid=2), lambda: g.quad_over_plane(subdiv=12),
                                  lambda: g.light_field(n_lights=5)])
def test_light_tree_matches_oracle(qpt, orc, make):
    """The library's light tree, built by its own code, equals the oracle's
    table for table, bit for bit (same split rule, same FP64 sums in the
    same order, same FP32 rounding)."""
    sc = make()
    c = qpt.Context(-1)
    c.build_scene(sc)
    mine = c.debug_light_tree()
    ref = orc.Scene(sc, build_bvh=False).light_tree()
    assert mine["left"].shape == ref["left"].shape
    for k in ("center", "flux", "left", "first", "count", "emit", "w"):
        assert np.array_equal(mine[k].view(np.uint32), ref[k].view(np.uint32)), k


@pytest.mark.parametrize("env", [(64, 32), (16, 8), (2048, 1024)])
def test_env_pyramid_matches_oracle(qpt, orc, env):
    """The library's environment pyramid, built by its own code, equals the
    oracle's table for table, bit for bit."""
    if env == (16, 8):
        sc = g.convex_under_env()
    else:
        sc = g.instanced_env_scene(width=8, height=8, target_tris=2000, env_size=env)
    c = qpt.Context(-1)
    c.build_scene(sc)
    mine = c.debug_env_pyramid()
    ref = orc.Scene(sc, build_bvh=False).env_pyramid()
    assert mine["m"] == ref["m"] > 0 and mine["top"] == ref["top"] and mine["root"] == ref["root"]
    assert np.array_equal(mine["q"], ref["q"])
    assert np.array_equal(mine["oq"], ref["oq"])


def test_env_pyramid_absent_for_other_shapes(qpt):
    sc = g.instanced_env_scene(width=8, height=8, target_tris=2000, env_size=(96, 48))
    c = qpt.Context(-1)
    c.build_scene(sc)
    assert c.debug_env_pyramid()["m"] == 0


def test_binding_struct_layout_matches_header(qpt, tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C header gives its counterpart (gcc, C99), so the argument
    marshalling passes what the library reads."""
    import ctypes as C
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = [n for n in dir(qpt) if n.startswith("qpt_") and isinstance(getattr(qpt, n), type)
               and issubclass(getattr(qpt, n), C.Structure)]
    assert "qpt_render_opts" in structs and "qpt_guide_opts" in structs
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qpt.h"', "int main(void) {"]
    for n in structs:
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for f, _ in getattr(qpt, n)._fields_:
            lines.append(f'  printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.check_call([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(root, "include"), str(src), "-o",
                           str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for n in structs:
        cls = getattr(qpt, n)
        assert int(got[f"{n} size"]) == C.sizeof(cls), n
        for f, _ in cls._fields_:
            assert int(got[f"{n} {f}"]) == getattr(cls, f).offset, (n, f)
