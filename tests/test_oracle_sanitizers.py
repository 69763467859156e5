"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
driver built with gcc renders a light field under a sky (BVH, alias table,
light tree, 2D CDF and pyramid, box and Gaussian filters, every estimator
mode) and must finish without a report."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import scenegen as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_scene(sc, path):
    env = sc.env
    eh, ew = (env.shape[0], env.shape[1]) if env is not None else (0, 0)
    with open(path, "wb") as f:
        np.array([sc.positions.shape[0], sc.num_triangles, sc.albedo.shape[0], ew, eh, sc.width, sc.height,
                  sc.max_depth], np.uint32).tofile(f)
        np.ascontiguousarray(sc.positions, np.float32).tofile(f)
        np.ascontiguousarray(sc.indices, np.uint32).tofile(f)
        np.ascontiguousarray(sc.tri_material, np.uint32).tofile(f)
        np.ascontiguousarray(sc.albedo, np.float32).tofile(f)
        np.ascontiguousarray(sc.roughness, np.float32).tofile(f)
        np.ascontiguousarray(sc.emission, np.float32).tofile(f)
        np.ascontiguousarray(sc.mat_flags, np.uint32).tofile(f)
        if env is not None:
            np.ascontiguousarray(env, np.float32).tofile(f)
        np.array(list(sc.camera.eye) + list(sc.camera.look) + list(sc.camera.up) + [sc.camera.vfov_deg],
                 np.float64).tofile(f)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_driver"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off",
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "qpt_oracle.c"),
           "-o", str(exe), "-lm", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    sc = g.light_field(n_lights=300, width=12, height=8, max_depth=5, env=True)
    scene = tmp_path / "scene.bin"
    _write_scene(sc, scene)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([str(exe), str(scene)], capture_output=True, text=True, timeout=600, env=env)
    assert p.returncode == 0, p.stderr[-3000:]
    assert "runtime error" not in p.stderr and "ERROR: AddressSanitizer" not in p.stderr, p.stderr[-3000:]
