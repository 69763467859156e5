"""The library's host side under AddressSanitizer and UndefinedBehaviorSanitizer
on the CPU: qpt_host.cpp built with g++ (host code only; the device entry
points it calls are replaced by stubs generated from their declarations,
which a host-only context never reaches), driven on a host-only context over
scenes with triangle lights, many lights, an environment map and its pyramid:
scene ingest, light tables, light tree, environment CDFs and pyramid, the
binned-SAH BVH at several leaf sizes, workspace sizing, the host-table hooks
and the documented argument and call-order errors. It must finish without a
report."""
import os
import re
import shutil
import subprocess

import pytest

import scenegen as g
from test_oracle_sanitizers import _write_scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1705_01263_amd", "csrc")


def _stubs(path):
    """Definitions returning an error for every device entry point declared in
    the internal header (kernel launchers, the GPU builder, the static region)."""
    hdr = open(os.path.join(CSRC, "qpt_internal.h")).read()
    decls = re.findall(r"^((?:hipError_t|size_t) (?:launch_\w+|gpu_\w+|static_scratch)\([^;]*\));", hdr, re.M)
    assert len(decls) >= 20
    with open(path, "w") as f:
        f.write('#include "qpt_internal.h"\nnamespace qpt {\n')
        for d in decls:
            ret = "0" if d.startswith("size_t") else "hipErrorNotSupported"
            f.write(f"{d}\n{{\n    return {ret};\n}}\n")
        f.write("}  // namespace qpt\n")


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the ROCm headers are not available")
def test_host_library_clean_under_sanitizers(tmp_path):
    stubs = tmp_path / "device_stubs.cpp"
    _stubs(stubs)
    exe = tmp_path / "host_driver"
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", "/opt/rocm/include", "-w"]
    cmd = ["g++", *flags, os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), os.path.join(CSRC, "qpt_host.cpp"),
           str(stubs), "-o", str(exe), "-L/opt/rocm/lib", "-lamdhip64", "-lpthread"]
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stderr[-3000:]
    scenes = [g.workload("cornell"), g.light_field(n_lights=300, width=12, height=8, max_depth=5, env=True),
              g.grid_scene(grid=3, width=16, height=16), g.quad_over_plane(subdiv=8),
              g.city(blocks=4, target_tris=20_000, emissive_cells=300)]
    files = []
    for k, sc in enumerate(scenes):
        f = tmp_path / f"scene{k}.bin"
        _write_scene(sc, f)
        files.append(str(f))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               LD_LIBRARY_PATH="/opt/rocm/lib:" + os.environ.get("LD_LIBRARY_PATH", ""))
    p = subprocess.run([str(exe), *files], capture_output=True, text=True, timeout=900, env=env)
    assert p.returncode == 0, (p.stdout[-2000:], p.stderr[-3000:])
    assert "runtime error" not in p.stderr and "ERROR: AddressSanitizer" not in p.stderr, p.stderr[-3000:]
    assert p.stdout.count(": ok") == len(files)
