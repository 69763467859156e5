#!/usr/bin/env python3
"""Throughput of the progressive QMC path tracer on one MI355X.

One step = one pass of the whole hot path over the frame (one sample per
pixel: enumeration, Halton samples, camera rays, closest hit, emission with
MIS, next-event estimation, BSDF sampling, roulette, occlusion, FP64
accumulation), through the C-ABI on torch's current stream.

Workload: the seeded 0.97M-triangle grid of spheres and boxes (GGX over
Lambert, 256 textured emitters), 1920x1080, max depth 12. Inputs are
resident in HBM before the timed region starts.

Prints one JSON line: Mrays/s (extension + shadow rays per second) as
`value`, Mpaths/s, a roofline entry for the dominant kernel (per-launch
algorithmic bytes over its average launch time, HIP events inside the
library on the launch stream) and the CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s and Mpaths/s per GPU; equal-time RMSE, guided vs plain vs FP64 oracle"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes per unit of work ("Measurement")
NODE_BYTES, TRI_BYTES = 128, 48   # 4-wide node (four child boxes + references), triangle
TRACE_RAY_BYTES = 4 + 32 + 16        # queue entry, ray (o, tmax, d), hit record
SHADOW_RAY_BYTES = 48 + 32           # shadow ray + contribution, radiance read-modify-write
SHADE_VERTEX_BYTES = 4 + 16 + 16 + 16 + 16 + 8 + 48 + 32 + 16   # reads + radiance write
SHADE_CONTINUE_BYTES = 16 + 16 + 16 + 4                           # next ray, throughput, queue
SHADE_NEE_BYTES = 4 + 48 + 48 + 8 + 4 + 4                         # shadow record, light tri, alias, pmf


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    src = os.path.join(ROOT, "paper_1705_01263_amd", "csrc", "qpt_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def pmc_traffic(kernel: str, workload_tag: str):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload_tag}.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha:\s*([0-9a-f]+)", txt)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_sha():
        return None
    return float(t.group(1))


def cpu_baseline(sc, seconds: float):
    """The FP64 oracle on every 8th pixel in x and y, passes until `seconds` of work."""
    import numpy as np

    import oracle

    t0 = time.perf_counter()
    S = oracle.Scene(sc)
    build_s = time.perf_counter() - t0
    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(0, H, 8), np.arange(0, W, 8), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = min(threads, 16)
    rays = 0
    passes = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        _, _, _, r = S.render(pixels=pix, pass0=passes, npasses=4, nthreads=threads)
        rays += r
        passes += 4
    dt = time.perf_counter() - t0
    return {
        "value": rays / dt / 1e6,
        "unit": "Mrays/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"every 8th pixel in x and y ({pix.shape[0]} px) of the {W}x{H} frame, passes 0..{passes - 1}, "
                  f"FP64 oracle, {rays} rays in {dt:.1f} s, BVH build ({build_s:.1f} s) excluded",
        "mpaths_per_s": pix.shape[0] * passes / dt / 1e6,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-sized buffer once (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenegen
    from paper_1705_01263_amd import Renderer

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        _say(f"bench: copied {n} bytes for counter calibration")
        del src, dst
    sc = scenegen.make_config(1)
    D = sc.max_depth
    _say(f"bench: scene {sc.name} tris={sc.num_triangles} {sc.width}x{sc.height} D={D}")
    r = Renderer(sc, device=0)
    bs = r.bvh_stats
    _say(f"bench: bvh nodes={bs.num_nodes} leaves={bs.num_leaves} depth={bs.max_depth} build={bs.build_ms:.0f} ms")
    for j in range(args.warmup):
        r.render(j, 1)
    torch.cuda.synchronize()
    _say(f"bench: warmup {args.warmup} passes done")
    st0 = r.stats()
    if not args.no_profile:
        r.ctx.profile(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for j in range(args.steps):
        r.render(args.warmup + j, 1)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not args.no_profile:
        r.ctx.profile(False)
    gpu_ms = ev0.elapsed_time(ev1)
    st1 = r.stats()
    ext = st1.rays_extension - st0.rays_extension
    sh = st1.rays_shadow - st0.rays_shadow
    paths = st1.paths - st0.paths
    secs = wall
    mrays = (ext + sh) / secs / 1e6
    mpaths = paths / secs / 1e6
    _say(f"bench: {args.steps} passes in {wall * 1e3:.1f} ms wall ({gpu_ms:.1f} ms events): "
         f"{mrays:.1f} Mrays/s, {mpaths:.2f} Mpaths/s, rays/path {(ext + sh) / paths:.2f}")

    roof = None
    kernels = None
    if not args.no_profile:
        prof = r.ctx.profile_read()
        kernels = {k: {"launches": n, "ms": round(ms, 3)} for k, (n, ms) in prof.items()}
        dn = st1.nodes_extension - st0.nodes_extension
        dt_ = st1.tris_extension - st0.tris_extension
        sn = st1.nodes_shadow - st0.nodes_shadow
        stt = st1.tris_shadow - st0.tris_shadow
        byts = {
            "trace": ext * TRACE_RAY_BYTES + dn * NODE_BYTES + dt_ * TRI_BYTES,
            "shadow": sh * SHADOW_RAY_BYTES + sn * NODE_BYTES + stt * TRI_BYTES,
            "shade": ext * SHADE_VERTEX_BYTES + (ext - paths) * SHADE_CONTINUE_BYTES + sh * SHADE_NEE_BYTES,
        }
        dom = max(byts, key=lambda k: prof[k][1])
        n_l, ms = prof[dom]
        per_launch = byts[dom] / n_l
        achieved = per_launch / (ms / n_l * 1e-3) / 1e9
        roof = {"kernel": f"k_{dom}", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": pmc_traffic(f"k_{dom}", "grid_1m"),
                "bytes_per_launch": round(per_launch), "avg_launch_ms": round(ms / n_l, 4),
                "nodes_per_ray": round(dn / max(ext, 1), 2), "tris_per_ray": round(dt_ / max(ext, 1), 2),
                "shadow_nodes_per_ray": round(sn / max(sh, 1), 2),
                "shadow_tris_per_ray": round(stt / max(sh, 1), 2)}
        _say(f"bench: kernels {kernels}")
        _say(f"bench: roofline {roof}")

    cpu = None
    if not args.no_cpu_baseline:
        _say(f"bench: CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        cpu = cpu_baseline(sc, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": round(mrays, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "grid of 400 tessellated spheres/boxes, 0.97M triangles, 256 textured emitters, "
                               "1920x1080, 1 spp per step, max depth 12, NEE+MIS, roulette",
                   "triangles": sc.num_triangles, "pixels": sc.width * sc.height, "max_depth": D,
                   "parallelism": "single GPU"},
        "mpaths_per_s": round(mpaths, 3),
        "rays_per_path": round((ext + sh) / paths, 3),
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
