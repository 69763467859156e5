#!/usr/bin/env python3
"""Throughput of the progressive QMC path tracer on one MI355X.

One step = one pass of the whole hot path over the frame (one sample per
pixel: enumeration, Halton samples, camera rays, closest hit, emission with
MIS, next-event estimation, BSDF sampling, roulette, occlusion, FP64
accumulation), through the C-ABI on torch's current stream; the library runs
two batches of passes at a time (that stream and one of its own, each with a
path pool of up to sixteen frames) and keeps the framebuffer updates in pass
order.

Workload (default): the seeded 16M-triangle procedural city with 10,000
emissive window triangles (alias-table light selection), 3840x2160, max
depth 16; `--workload grid` runs the 0.97M-triangle 1080p grid instead.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line: Mrays/s (extension + shadow rays per second) as
`value`, Mpaths/s, a roofline entry for the dominant kernel (per-launch
algorithmic bytes over its average launch time, HIP events inside the
library on the launch stream, timed on one stream right after the timed
region because launches of the two batches in flight share the GPU), the CPU
oracle's rate on a bounded sample, and the equal-time RMSE of the guided and
the plain tracer (slit enclosure at 1080p and the city at 4K).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import sqlite3
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s and Mpaths/s per GPU; equal-time RMSE, guided vs plain vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "grid": ("grid_1m", "grid of 400 tessellated spheres/boxes, 0.97M triangles, 256 textured emitters, 1920x1080, "
                "1 spp per step (passes in nearly equal batches of at most sixteen frames, two batches in flight), max "
                "depth 12, "
                "NEE+MIS, roulette"),
    "city": ("city_16m", "procedural city, 16.0M triangles, 5,000 emissive window cells (10k triangles, alias-table light "
                "selection), 3840x2160, 1 spp per step (passes in nearly equal batches of at most sixteen frames, two "
                "batches in flight), max depth 16, NEE+MIS, roulette"),
}
# the guided tracer's settings in the equal-time legs
GUIDE = {"alpha": 0.7, "warmup": 16, "max_vertex": 2, "lr": 2e-3, "batch": 1 << 17}

# algorithmic bytes per unit of work
TRI_BYTES = 48   # triangle (three float4 corners); a 4-wide node is 64 bytes quantised, 128 in full (bvh stats)
TRACE_RAY_BYTES = 4 + 32 + 16        # queue entry, ray (o, tmax, d), hit record
SHADOW_RAY_BYTES = 48 + 32           # shadow ray + contribution, radiance read-modify-write
SHADE_VERTEX_BYTES = 4 + 16 + 16 + 16 + 16 + 8 + 48 + 32 + 16   # reads + radiance write
SHADE_CONTINUE_BYTES = 16 + 16 + 16 + 4                           # next ray, throughput, queue
SHADE_NEE_BYTES = 48 + 48 + 8 + 4 + 4                             # shadow record, light tri, alias, pmf
# the same with the compressed path state: direction 8 (octahedral pair and
# previous vertex), throughput and density 8, hit record 12
TRACE_RAY_BYTES_C = 4 + 16 + 8 + 12
SHADE_VERTEX_BYTES_C = 4 + 12 + 8 + 8 + 16 + 8 + 48 + 32 + 16
SHADE_CONTINUE_BYTES_C = 16 + 8 + 8 + 4


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha() -> str:
    """SHA of the path kernels and of the host side that builds the tree they
    traverse and launches them: counters taken on other sources are stale."""
    h = hashlib.sha256()
    for f in ("qpt_kernels.hip", "qpt_host.cpp"):
        h.update(open(os.path.join(ROOT, "paper_1705_01263_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


# ---------------------------------------------- rocprofv3 summaries and
# profiling workloads (`python bench.py summarize ...`, `--sweep`, `--profile-guided`)

def guide_sha() -> str:
    """SHA of the guide's kernels (training, inference and the mixture code)."""
    h = hashlib.sha256()
    for f in ("qpt_guide.hip", "qpt_guide_mlp.h", "qpt_guide_dev.h"):
        h.update(open(os.path.join(ROOT, "paper_1705_01263_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("qpt::(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    name = name.split("(")[0] if "(" in name else name
    return name.split("<")[0]  # template instances under one name


def kernel_durations(path: str):
    """{kernel: [durations in ns]} from a rocprofv3 results.db or kernel_trace.csv."""
    out = collections.defaultdict(list)
    if path.endswith(".db"):
        con = sqlite3.connect(path)
        for name, dur in con.execute("select name, duration from kernels"):
            out[_short(name)].append(float(dur))
    else:
        for r in csv.DictReader(open(path)):
            out[_short(r["Kernel_Name"])].append(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
    return out


def summarize_trace(path: str, out_txt: str, cmd: str) -> str:
    d = kernel_durations(path)
    total = sum(sum(v) for v in d.values())
    lines = [f"# rocprofv3 kernel trace summary", f"command: {cmd}", f"kernel_source_sha: {kernel_sha()}",
             "", f"{'kernel':<28} {'calls':>6} {'total_us':>12} {'avg_us':>10} {'pct':>6}"]
    for k, v in sorted(d.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{k:<28} {len(v):>6} {sum(v) / 1e3:>12.1f} {sum(v) / len(v) / 1e3:>10.2f} "
                     f"{100 * sum(v) / total:>6.2f}")
    txt = "\n".join(lines) + "\n"
    open(out_txt, "w").write(txt)
    return txt


def _pmc(dirpath: str, counter: str):
    f = glob.glob(os.path.join(dirpath, "**", "*counter_collection.csv"), recursive=True)[0]
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(f)):
        if r["Counter_Name"] == counter:
            vals[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def summarize_pmc(fetch_dir: str, write_dir: str, kernel: str, out_txt: str, calib_mib: int, cmd: str,
                  calib_kernel: str = "__amd_rocclr_copyBuffer") -> str:
    fe = _pmc(fetch_dir, "FETCH_SIZE")
    wr = _pmc(write_dir, "WRITE_SIZE")
    # the copy moves calib_mib MiB in and out, split over its dispatches
    want_kib = calib_mib * 1024.0
    f_scale = want_kib / sum(fe[calib_kernel])
    w_scale = want_kib / sum(wr[calib_kernel])
    fk = sum(fe[kernel]) / len(fe[kernel]) * f_scale * 1024.0
    wk = sum(wr[kernel]) / len(wr[kernel]) * w_scale * 1024.0
    lines = [f"# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE summary for {kernel}", f"command: {cmd}",
             f"kernel_source_sha: {kernel_sha()}",
             f"calibration: {calib_kernel} copying {calib_mib} MiB reads FETCH_SIZE x{1 / f_scale:.4f}, "
             f"WRITE_SIZE x{1 / w_scale:.4f} of the true bytes; factors applied: fetch {f_scale:.4f}, "
             f"write {w_scale:.4f}",
             f"dispatches: {len(fe[kernel])}",
             f"fetch_bytes_per_launch: {fk:.0f}", f"write_bytes_per_launch: {wk:.0f}",
             f"hbm_bytes_per_launch: {fk + wk:.0f}", "", "all kernels (scaled bytes per dispatch):"]
    for k in sorted(fe):
        if k in wr:
            lines.append(f"  {k:<28} fetch {sum(fe[k]) / len(fe[k]) * f_scale * 1024:>14.0f}  "
                         f"write {sum(wr[k]) / len(wr[k]) * w_scale * 1024:>14.0f}  n={len(fe[k])}")
    txt = "\n".join(lines) + "\n"
    open(out_txt, "w").write(txt)
    return txt


def summarize_mfma(pmc_dir: str, kernels, out_txt: str, cmd: str, simds: int = 1024, xcds: int = 8) -> str:
    """Per-dispatch MFMA and VALU activity of `kernels` from one rocprofv3
    --pmc run with SQ_INSTS_VALU_MFMA_MOPS_BF16, SQ_VALU_MFMA_BUSY_CYCLES,
    SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_BUSY_CU_CYCLES and GRBM_GUI_ACTIVE.
    MFMA FLOPs = MOPS_BF16 x 512. GRBM_GUI_ACTIVE comes summed over the
    chip's XCDs (its value over a dispatch's duration is xcds x the clock),
    so the dispatch's elapsed cycles are GRBM_GUI_ACTIVE / xcds, and MFMA
    utilisation = MFMA busy cycles over (elapsed cycles x SIMDs), 256 CUs x
    4 SIMDs on MI355X."""
    f = glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True)[0]
    per = collections.defaultdict(lambda: collections.defaultdict(dict))  # kernel -> dispatch -> counter
    dur = collections.defaultdict(dict)
    for r in csv.DictReader(open(f)):
        k = _short(r["Kernel_Name"])
        d = r["Dispatch_Id"]
        per[k][d][r["Counter_Name"]] = float(r["Counter_Value"])
        dur[k][d] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    lines = ["# rocprofv3 --pmc MFMA / VALU summary", f"command: {cmd}", f"kernel_source_sha: {kernel_sha()}",
             f"guide_source_sha: {guide_sha()}",
             f"SIMDs: {simds}", ""]
    for k in kernels:
        if k not in per:
            lines.append(f"{k}: no dispatches")
            continue
        ds = list(per[k])
        avg = lambda c: sum(per[k][d].get(c, 0.0) for d in ds) / len(ds)
        t_ns = sum(dur[k][d] for d in ds) / len(ds)
        flops = avg("SQ_INSTS_VALU_MFMA_MOPS_BF16") * 512
        busy, gui = avg("SQ_VALU_MFMA_BUSY_CYCLES"), avg("GRBM_GUI_ACTIVE")
        cyc = gui / xcds
        lines += [f"{k}: dispatches {len(ds)}, avg duration {t_ns / 1e3:.2f} us",
                  f"  BF16 MFMA FLOP per dispatch {flops:.4g} -> {flops / t_ns / 1e3:.2f} TFLOP/s "
                  f"({100 * flops / t_ns / 1e3 / 2500.0:.2f}% of the 2.5 PFLOP/s dense BF16 peak)",
                  f"  MFMA busy {100 * busy / max(cyc * simds, 1):.2f}% of SIMD cycles "
                  f"(SQ_VALU_MFMA_BUSY_CYCLES {busy:.4g}; GRBM_GUI_ACTIVE {gui:.4g}, summed over {xcds} XCDs: "
                  f"{cyc:.4g} cycles, {cyc / t_ns:.2f} GHz)",
                  f"  SQ_INSTS_VALU {avg('SQ_INSTS_VALU'):.4g}, SQ_ACTIVE_INST_VALU {avg('SQ_ACTIVE_INST_VALU'):.4g}, "
                  f"SQ_BUSY_CU_CYCLES {avg('SQ_BUSY_CU_CYCLES'):.4g}"]
    txt = "\n".join(lines) + "\n"
    open(out_txt, "w").write(txt)
    return txt


def summarize_counters(pmc_dirs, kernels, out_txt: str, cmd: str) -> str:
    """Per-kernel averages over dispatches of every counter in one or more
    rocprofv3 --pmc runs (one counter group per run), with the launch
    duration; rocprofv3's derived metrics (VALUBusy, VALUUtilization,
    MemUnitBusy, L2CacheHit, OccupancyPercent and the like) are listed under
    their own names and units."""
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    dur = collections.defaultdict(list)
    runs = []
    for dpath in pmc_dirs:
        files = glob.glob(os.path.join(dpath, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            continue
        names = set()
        seen = set()
        for r in csv.DictReader(open(files[0])):
            k = _short(r["Kernel_Name"])
            per[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
            names.add(r["Counter_Name"])
            key = (k, r["Dispatch_Id"])
            if key not in seen:
                seen.add(key)
                dur[k].append(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
        runs.append(f"{os.path.basename(os.path.normpath(dpath))}: {', '.join(sorted(names))}")
    lines = ["# rocprofv3 --pmc counter summary (average per dispatch)", f"command: {cmd}",
             f"kernel_source_sha: {kernel_sha()}", "runs:"] + [f"  {r}" for r in runs] + [""]
    for k in kernels:
        if k not in per:
            lines.append(f"{k}: no dispatches")
            continue
        lines.append(f"{k}: {len(dur[k]) // max(1, len(runs))} dispatches per run, "
                     f"avg duration {sum(dur[k]) / len(dur[k]) / 1e3:.2f} us")
        for c in sorted(per[k]):
            v = per[k][c]
            lines.append(f"  {c:<28} {sum(v) / len(v):>16.6g}")
    txt = "\n".join(lines) + "\n"
    open(out_txt, "w").write(txt)
    return txt


def run_guided(width: int, height: int, tris: int, passes: int, alpha: float = 0.7, max_vertex: int = 2) -> None:
    """A guided workload to profile: the slit scene with the guide training
    one Adam step per pass from its first pass, two batches in flight and the
    megakernel tail from half the maximum depth (the equal-time leg's
    schedule)."""
    import torch

    import scenegen
    from paper_1705_01263_amd import Renderer

    sc = scenegen.slit_scene(width=width, height=height, target_tris=tris, max_depth=16)
    r = Renderer(sc)
    r.ctx.guide_set_weights(scenegen.guide_init(1))
    r.ctx.guide_config(alpha=alpha, lr=1e-3, batch=1 << 18, train=1, warmup_steps=0, seed=1, max_vertex=max_vertex)
    r.render(0, passes, tail_depth=sc.max_depth // 2)
    torch.cuda.synchronize()
    _, steps = r.ctx.guide_get_weights()
    print(f"guided: {passes} passes of {sc.name} {width}x{height}, {steps} Adam steps", flush=True)


def run_sweep(out_txt: str, min_log2: int, max_log2: int, cmd: str) -> str:
    """Passes per launch sequence against throughput (the paper's Table 1 in
    kind): the grid workload at 1080p with path pools from 2^min_log2 to
    2^max_log2 slots; per pool: one batch at a time, two in flight, the
    megakernel tail from depth 4 (one stream and two in flight), and, for
    pools of whole frames, regeneration through a quarter of the pool's slots. Each setting renders
    two pools' worth of passes (at least 8) after one untimed batch."""
    import time

    import torch

    import scenegen
    from paper_1705_01263_amd import Renderer

    sc = scenegen.workload("grid_1m")
    npix = sc.width * sc.height
    lines = ["# passes per launch sequence against throughput (grid, 0.97M triangles, 1920x1080, depth 12)",
             f"command: {cmd}", f"kernel_source_sha: {kernel_sha()}", "",
             "Mrays/s per schedule: one batch at a time; two batches in flight; one at a time with the",
             "megakernel tail from depth 4; two in flight with that tail; regeneration with live slots =",
             "pool / 4 (whole-frame batches only)", "",
             f"{'pool (paths)':>14} {'frames/batch':>13} {'passes':>7} {'one stream':>11} {'two in flight':>14} "
             f"{'tail from 4':>12} {'two + tail':>11} {'regeneration':>13} {'Mpaths/s (best)':>16}"]
    for lg in range(min_log2, max_log2 + 1):
        pool = 1 << lg
        frames = pool / npix
        per = max(1, pool // npix)
        passes = max(8, 2 * per)
        r = Renderer(sc, pool_paths=pool)
        schedules = [{"single_stream": True}, {"single_stream": False}, {"single_stream": True, "tail_depth": 4},
                     {"single_stream": False, "tail_depth": 4}]
        if pool >= npix:
            schedules.append({"regen_paths": pool // 4})
        res = []
        for kw in schedules:
            r.reset()
            r.render(0, per, **kw)
            torch.cuda.synchronize()
            st0 = r.stats()
            t0 = time.perf_counter()
            r.render(per, passes, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st1 = r.stats()
            rays = (st1.rays_extension - st0.rays_extension) + (st1.rays_shadow - st0.rays_shadow)
            res.append((rays / dt / 1e6, passes * npix / dt / 1e6))
        del r
        torch.cuda.empty_cache()
        cols = [f"{x[0]:.1f}" for x in res] + ["--"] * (5 - len(res))
        lines.append(f"{'2^%d' % lg:>14} {frames:>13.3f} {passes:>7} {cols[0]:>11} {cols[1]:>14} {cols[2]:>12} "
                     f"{cols[3]:>11} {cols[4]:>13} {max(x[1] for x in res):>16.1f}")
        print(lines[-1], flush=True)
    txt = "\n".join(lines) + "\n"
    open(out_txt, "w").write(txt)
    return txt


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


def oracle_scene(sc):
    """The FP64 oracle's own copy of the scene (its BVH build timed)."""
    import oracle

    t0 = time.perf_counter()
    S = oracle.Scene(sc)
    return S, time.perf_counter() - t0


def cpu_baseline(S, sc, seconds: float, build_s: float):
    """The FP64 oracle on every 8th pixel in x and y, passes until `seconds` of work."""
    import numpy as np

    W, H = sc.width, sc.height
    ys, xs = np.meshgrid(np.arange(0, H, 8), np.arange(0, W, 8), indexing="ij")
    pix = (ys * W + xs).reshape(-1).astype(np.uint32)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = min(threads, 16)
    rays = 0
    passes = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        _, _, _, r = S.render(pixels=pix, pass0=passes, npasses=2, nthreads=threads)
        rays += r
        passes += 2
    dt = time.perf_counter() - t0
    return {
        "value": rays / dt / 1e6,
        "unit": "Mrays/s",
        "cores": threads,
        "host_cpu": _host_cpu(),
        "kind": "oracle",
        "sample": f"every 8th pixel in x and y ({pix.shape[0]} px) of the {W}x{H} frame, passes 0..{passes - 1}, "
                  f"FP64 oracle, {rays} rays in {dt:.1f} s, BVH build ({build_s:.1f} s) excluded",
        "mpaths_per_s": pix.shape[0] * passes / dt / 1e6,
    }


def _host_cpu():
    """CPU model and threads per core of this host, from /proc/cpuinfo."""
    model, siblings, cores = "unknown", None, None
    try:
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and model == "unknown":
                model = v
            elif k == "siblings" and siblings is None:
                siblings = int(v)
            elif k == "cpu cores" and cores is None:
                cores = int(v)
    except OSError:
        pass
    tpc = siblings // cores if siblings and cores else None
    return {"model": model, "threads_per_core": tpc, "logical_cpus": os.cpu_count()}


def equal_time(sc, views, seconds: float, ref_passes: int, per_call: int, oracle_scene=None,
               oracle_seconds: float = 0.0, oracle_stride=(32, 16), guide=None, tail_depth=None):
    """Equal-time RMSE of the plain and the guided tracer on one scene.

    Both runs of a pair get the same wall time on the same GPU, the guided
    one including its online training from an untrained network. Two
    budgets: the plain tracer's time for 64 passes, and `seconds`. For each
    camera in `views` the error is measured against the plain tracer at
    2 x `ref_passes` passes from two independent pass ranges (FP64
    accumulation, whole frame), with the reference's own error (estimated
    from the difference of its halves) taken out of the squared errors
    (`rmse`; the raw figure is `rmse_vs_gpu_reference`), and, for the first
    camera, against the FP64 CPU oracle on a
    bounded pixel sample (every `oracle_stride` pixels, also from an
    independent pass range), whose own error against the GPU reference is
    reported beside it. `per_call` passes go to the library per call (two
    batches in flight), with the next call enqueued before the host waits
    for the previous one. A timed run starts another call only while the
    mean call time so far says it would end within half a call of the
    budget, so both runs overshoot it by about the same fraction; the
    ratio is also reported scaled by sqrt(guided time / plain time)
    (`time_adjusted`), which removes what difference in wall time is left,
    since RMSE falls as one over the square root of the passes. Both
    tracers (and the references) render with the megakernel tail from
    `tail_depth` (default: half the maximum depth, past the guided
    vertices), as the throughput leg does.
    """
    import numpy as np
    import torch

    import scenegen
    from paper_1705_01263_amd import Renderer

    g = dict(GUIDE)
    if guide:
        g.update(guide)
    td = sc.max_depth // 2 if tail_depth is None else tail_depth
    width, height = sc.width, sc.height
    rmse = lambda a, b: float(np.sqrt(np.mean((a - b) ** 2)))
    out = {"workload": f"{sc.name}: {sc.num_triangles} triangles, {width}x{height}, max depth {sc.max_depth}",
           "guide": {"alpha": g["alpha"], "guided_vertices": g["max_vertex"], "lr": g["lr"], "batch": g["batch"],
                     "adam_steps_per_pass": 1, "warmup_steps": g["warmup"]},
           "passes_per_call": per_call, "tail_depth": td, "views": []}
    for vi, (vname, cam) in enumerate(views):
        if cam is not None:
            sc.camera = cam
        r = Renderer(sc, device=0)

        def run(budget=None, passes=None, guided=False):
            r.reset()
            if guided:
                r.ctx.guide_set_weights(scenegen.guide_init(1))
                r.ctx.guide_config(alpha=g["alpha"], lr=g["lr"], batch=g["batch"], train=1,
                                   warmup_steps=g["warmup"], seed=1, max_vertex=g["max_vertex"])
            else:
                r.ctx.guide_config(alpha=0.0, lr=1e-3, batch=1 << 18, train=0, warmup_steps=0, seed=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = 0
            # one call stays in flight while the host waits for the one before
            # it, so the GPU renders without a gap between calls (as a
            # progressive renderer would). With a time budget, another call is
            # started only if it is expected to end within half a call of the
            # budget (one call is still in flight; a call's duration is the
            # mean so far), so a run ends near the budget however long its
            # calls are; the wall time includes the last call
            prev, done, d = None, 0, 0.0
            while True:
                if passes is not None and n >= passes:
                    break
                if budget is not None and done and time.perf_counter() - t0 + 1.5 * d > budget:
                    break
                r.render(n, per_call, tail_depth=td)
                n += per_call
                ev = torch.cuda.Event()
                ev.record()
                if prev is not None:
                    prev.synchronize()
                    done += 1
                    d = (time.perf_counter() - t0) / done
                prev = ev
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            s, c = r.readback()
            steps = r.ctx.guide_get_weights()[1] if guided else 0
            return s / c[:, None], n, dt, steps

        r.render(0, 4)  # warm-up (module load, first launches)
        torch.cuda.synchronize()
        r.ctx.guide_config(alpha=0.0, lr=1e-3, batch=1 << 18, train=0, warmup_steps=0, seed=0)
        # two references from disjoint pass ranges: their mean is the
        # reference, and half their difference estimates its own error, which
        # is removed from the squared errors compared (an error of the
        # reference adds to every image's squared error alike and would pull
        # every ratio toward 1)
        t0 = time.perf_counter()
        refs = []
        for first in (1 << 24, (1 << 24) + (1 << 23)):
            r.reset()
            r.render(first, ref_passes, tail_depth=td)
            s, c = r.readback()
            refs.append(s / c[:, None])
        ref = 0.5 * (refs[0] + refs[1])
        ref_mse = np.mean((refs[0] - refs[1]) ** 2) / 4.0
        del refs
        t_ref = time.perf_counter() - t0
        rmse_c = lambda a: float(np.sqrt(max(np.mean((a - ref) ** 2) - ref_mse, 0.0)))
        view = {"camera": vname, "gpu_reference": {"passes": 2 * ref_passes, "first_passes": [1 << 24,
                                                                                            (1 << 24) + (1 << 23)],
                                                   "seconds": round(t_ref, 2),
                                                   "own_rmse_estimate": float(np.sqrt(ref_mse))}, "budgets": []}
        img = {}
        for label, kw in (("plain tracer's time for 64 passes", {"passes": 64}), (f"{seconds:g} s", {"budget": seconds})):
            plain, n_p, t_p, _ = run(**kw)
            guided, n_g, t_g, steps = run(budget=t_p, guided=True)
            img[label] = (plain, guided)
            view["budgets"].append({
                "budget": label, "seconds": round(t_p, 3),
                "plain": {"passes": n_p, "rmse_vs_gpu_reference": rmse(plain, ref), "rmse": rmse_c(plain)},
                "guided": {"passes": n_g, "seconds": round(t_g, 3), "adam_steps": int(steps),
                           "rmse_vs_gpu_reference": rmse(guided, ref), "rmse": rmse_c(guided),
                           "final_loss": round(r.ctx.guide_loss()[0], 4)},
                "guided_over_plain_rmse": round(rmse_c(guided) / max(rmse_c(plain), 1e-30), 4),
                # the same ratio with each error scaled to the plain run's exact wall time
                # (an error falls as one over the square root of the time spent)
                "time_adjusted": round(rmse_c(guided) / max(rmse_c(plain), 1e-30) * (t_g / t_p) ** 0.5, 4)})
            _say(f"bench: equal time [{sc.name}, {vname}, {label}] plain {n_p} passes, guided {n_g} passes, "
                 f"ratio {view['budgets'][-1]['guided_over_plain_rmse']}")
        del r
        torch.cuda.empty_cache()
        if vi == 0 and oracle_scene is not None and oracle_seconds > 0:
            sy, sx = oracle_stride[1], oracle_stride[0]
            ys, xs = np.meshgrid(np.arange(height // (2 * sy), height, sy),
                                 np.arange(width // (2 * sx), width, sx), indexing="ij")
            pix = (ys * width + xs).reshape(-1).astype(np.uint32)
            threads = min(len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1, 16)
            acc = np.zeros((pix.shape[0], 3))
            n_o = 0
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < oracle_seconds:
                s_o, _, cnt, _ = oracle_scene.render(pixels=pix, pass0=(1 << 25) + n_o, npasses=16, nthreads=threads)
                acc += s_o
                n_o += 16
            o_ref = acc / n_o
            view["oracle_reference"] = {"pixels": int(pix.shape[0]), "passes": n_o, "first_pass": 1 << 25,
                                        "threads": threads, "seconds": round(time.perf_counter() - t0, 1),
                                        "gpu_reference_rmse": rmse(ref[pix], o_ref)}
            for bud in view["budgets"]:
                plain, guided = img[bud["budget"]]
                bud["plain"]["rmse_vs_oracle_sample"] = rmse(plain[pix], o_ref)
                bud["guided"]["rmse_vs_oracle_sample"] = rmse(guided[pix], o_ref)
        out["views"].append(view)
    return out


def light_select_equal_time(r, sc, seconds: float, ref_passes: int):
    """Equal-time RMSE of triangle-light selection by the flux alias table and
    by the light tree, on the renderer's own scene (the city: 10,000 emissive
    window triangles). Reference: both estimators at `ref_passes` passes each
    from an independent pass range, averaged (FP64 sums, whole frame). Each
    contender renders whole two-frame batches from pass 0 until `seconds`
    have passed (the tree gets the alias run's wall time). Also the shading
    kernel's time per pass with each selector."""
    import numpy as np
    import torch

    W, H = sc.width, sc.height
    lum = np.array([0.2126, 0.7152, 0.0722])
    ref = np.zeros((W * H, 3))
    t_ref = {}
    for tree in (False, True):
        r.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.render(1 << 24, ref_passes, light_tree=tree)
        s, c = r.readback()
        t_ref[tree] = round(time.perf_counter() - t0, 2)
        ref += 0.5 * s / c[:, None]
    lit = ref @ lum > 0
    out = {"reference": {"passes_each": ref_passes, "first_pass": 1 << 24, "seconds": t_ref[False] + t_ref[True],
                         "lit_pixel_fraction": round(float(lit.mean()), 4)}}
    budget = seconds
    for name, tree in (("alias_table", False), ("light_tree", True)):
        # shading kernel per pass, event-timed over 8 passes on one stream
        r.reset()
        r.ctx.profile(True)
        r.render(1 << 26, 8, light_tree=tree, single_stream=True)
        r.ctx.profile(False)
        prof = r.ctx.profile_read()
        r.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget:
            r.render(n, 2, light_tree=tree)
            n += 2
            torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if not tree:
            budget = dt
        s, c = r.readback()
        img = s / c[:, None]
        e = img - ref
        out[name] = {"passes": n, "seconds": round(dt, 3), "ms_per_pass": round(dt * 1e3 / n, 3),
                     "shade_ms_per_pass": round(prof["shade"][1] / 8, 3),
                     "rmse": float(np.sqrt(np.mean(e ** 2))),
                     "rel_rmse_lit": float(np.sqrt(np.mean(((e @ lum)[lit] / np.maximum((ref @ lum)[lit], 1e-3)) ** 2)))}
        _say(f"bench: light selection {name}: {n} passes in {dt:.2f} s, rmse {out[name]['rmse']:.5f}")
    out["tree_over_alias_rmse"] = round(out["light_tree"]["rmse"] / out["alias_table"]["rmse"], 4)
    out["tree_over_alias_rel_rmse_lit"] = round(out["light_tree"]["rel_rmse_lit"] / out["alias_table"]["rel_rmse_lit"], 4)
    return out


def env_select_equal_time(seconds: float, ref_passes: int, width: int, height: int, tris: int):
    """Equal-time RMSE of the three environment samplers: the 2D CDF, the
    texel pyramid, and the pyramid with normal-weighted top levels (Sec.
    2.1.2), on the sun-and-sky scene (open) and on the slit enclosure (the sky
    reaches the inside through a slit). Reference: the 2D CDF and the
    weighted pyramid at `ref_passes` passes each from pass 2^24, averaged.
    Each sampler renders as many passes as fit in `seconds` (measured per
    pass first, rounded down to whole four-pass batches)."""
    import numpy as np
    import torch

    import scenegen
    from paper_1705_01263_amd import Renderer

    lum = np.array([0.2126, 0.7152, 0.0722])
    out = []
    for name, make in (("sun and sky, open", lambda: scenegen.instanced_env_scene(width=width, height=height,
                                                                                    target_tris=tris)),
                       ("slit enclosure", lambda: scenegen.slit_scene(width=width, height=height, target_tris=tris,
                                                                      max_depth=16))):
        sc = make()
        _say(f"bench: environment samplers on {sc.name} tris={sc.num_triangles} {width}x{height}")
        r = Renderer(sc, device=0)
        ref = np.zeros((width * height, 3))
        t0 = time.perf_counter()
        for es in (0, 2):
            r.reset()
            r.render(1 << 24, ref_passes, env_sampling=es)
            s, c = r.readback()
            ref += 0.5 * s / c[:, None]
        res = {"scene": f"{sc.name}: {sc.num_triangles} triangles, {width}x{height}, max depth {sc.max_depth}, "
                        "2048x1024 sun (peak 5e4, 0.5 degrees) and sky",
               "reference": {"passes_each": ref_passes, "first_pass": 1 << 24,
                             "seconds": round(time.perf_counter() - t0, 2)}}
        lit = ref @ lum > 0
        for label, es in (("cdf_2d", 0), ("pyramid", 1), ("pyramid_normal_weighted", 2)):
            r.reset()
            r.render(1 << 26, 4, env_sampling=es)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r.render(1 << 26, 16, env_sampling=es)
            torch.cuda.synchronize()
            per = (time.perf_counter() - t1) / 16
            n = max(4, int(seconds / per) // 4 * 4)
            r.reset()
            st0 = r.stats()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r.render(0, n, env_sampling=es)
            s, c = r.readback()
            dt = time.perf_counter() - t1
            st1 = r.stats()
            e = s / c[:, None] - ref
            res[label] = {"passes": n, "seconds": round(dt, 3), "ms_per_pass": round(dt * 1e3 / n, 3),
                          "shadow_rays_per_path": round((st1.rays_shadow - st0.rays_shadow) / (st1.paths - st0.paths), 3),
                          "rmse": float(np.sqrt(np.mean(e ** 2))),
                          "rel_rmse_lit": float(np.sqrt(np.mean(((e @ lum)[lit] / np.maximum((ref @ lum)[lit], 1e-3)) ** 2)))}
            _say(f"bench: {name} {label}: {n} passes in {dt:.2f} s, rmse {res[label]['rmse']:.6f}")
        for label in ("pyramid", "pyramid_normal_weighted"):
            res[f"{label}_over_cdf_rmse"] = round(res[label]["rmse"] / res["cdf_2d"]["rmse"], 4)
        out.append(res)
        del r
        torch.cuda.empty_cache()
    return out


def summarize_main(argv):
    """`python bench.py summarize trace|pmc|mfma|counters ...`: rocprofv3 output
    -> the text summaries committed under profiles/."""
    ap = argparse.ArgumentParser(prog="bench.py summarize")
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("src")
    t.add_argument("out")
    t.add_argument("--cmd", required=True)
    p = sub.add_parser("pmc")
    p.add_argument("fetch_dir")
    p.add_argument("write_dir")
    p.add_argument("kernel")
    p.add_argument("out")
    p.add_argument("--calib-mib", type=int, required=True)
    p.add_argument("--cmd", required=True)
    m = sub.add_parser("mfma")
    m.add_argument("pmc_dir")
    m.add_argument("out")
    m.add_argument("--kernels", default="k_shade_guided,k_guide_train")
    m.add_argument("--cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("pmc_dirs", nargs="+")
    c.add_argument("--kernels", default="k_trace,k_shade,k_shadow")
    c.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    if a.what == "trace":
        print(summarize_trace(a.src, a.out, a.cmd))
    elif a.what == "pmc":
        print(summarize_pmc(a.fetch_dir, a.write_dir, a.kernel, a.out, a.calib_mib, a.cmd))
    elif a.what == "mfma":
        print(summarize_mfma(a.pmc_dir, a.kernels.split(","), a.out, a.cmd))
    else:
        print(summarize_counters(a.pmc_dirs, a.kernels.split(","), a.out, a.cmd))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        summarize_main(sys.argv[2:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=24, help="timed passes (24 = two batches of twelve at 4K)")
    ap.add_argument("--warmup", type=int, default=8, help="untimed passes (8 = one batch)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="city",
                    help="city: the 16M-triangle 4K city (default); grid: the 0.97M-triangle 1080p scene")
    ap.add_argument("--no-equal-time", action="store_true", help="skip the guided vs plain equal-time RMSE leg")
    ap.add_argument("--et-seconds", type=float, default=4.0, help="wall time of each equal-time run")
    ap.add_argument("--et-ref-passes", type=int, default=2048)
    ap.add_argument("--et-oracle-seconds", type=float, default=10.0)
    ap.add_argument("--et-size", type=str, default="1920x1080")
    ap.add_argument("--et-tris", type=int, default=4_000_000)
    ap.add_argument("--et-city-seconds", type=float, default=4.0, help="wall time of each equal-time run on the city")
    ap.add_argument("--et-city-ref-passes", type=int, default=512)
    ap.add_argument("--no-et-city", action="store_true", help="skip the guided vs plain equal-time leg on the city")
    ap.add_argument("--node-format", type=int, choices=(0, 1), default=0,
                    help="device tree: 0: quantised 64-byte nodes, 1: full-precision 128-byte nodes")
    ap.add_argument("--bvh-builder", type=int, choices=(0, 1), default=0,
                    help="0: binned SAH on the host, 1: linear BVH built on the GPU")
    ap.add_argument("--single-stream", action="store_true",
                    help="render the timed passes one batch at a time on one stream")
    ap.add_argument("--tail-depth", type=int, default=-1,
                    help="megakernel for every path still alive from this depth on (0: none; default: half the "
                         "workload's maximum depth, measured +4%% on the city and the grid against none)")
    ap.add_argument("--compress-state", action="store_true",
                    help="path state in the compressed layout (octahedral directions, half-precision throughput)")
    ap.add_argument("--no-light-select", action="store_true",
                    help="skip the alias table vs light tree equal-time leg (city workload only)")
    ap.add_argument("--ls-seconds", type=float, default=2.0, help="wall time of each light-selection run")
    ap.add_argument("--ls-ref-passes", type=int, default=512, help="reference passes per selector")
    ap.add_argument("--env-select", action="store_true",
                    help="also compare the environment samplers at equal time (sun-and-sky and slit scenes)")
    ap.add_argument("--es-seconds", type=float, default=1.0)
    ap.add_argument("--es-ref-passes", type=int, default=2048)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy a MIB-sized buffer once (reference kernel for HBM counters)")
    ap.add_argument("--sweep", metavar="OUT", help="only the passes-per-launch sweep (grid workload), written to OUT")
    ap.add_argument("--sweep-log2", default="15,26", help="smallest and largest pool (log2 paths) of the sweep")
    ap.add_argument("--profile-guided", metavar="WxH", help="only a guided, training run of the slit scene (to profile)")
    ap.add_argument("--profile-passes", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is designed but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenegen
    from paper_1705_01263_amd import Renderer

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.sweep:
        lo, hi = (int(v) for v in args.sweep_log2.split(","))
        print(run_sweep(args.sweep, lo, hi, " ".join(["python", "bench.py"] + sys.argv[1:])))
        return
    if args.profile_guided:
        w, h = (int(v) for v in args.profile_guided.split("x"))
        run_guided(w, h, args.et_tris, args.profile_passes)
        return
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        _say(f"bench: copied {n} bytes for counter calibration")
        del src, dst
    sc = scenegen.workload(WORKLOADS[args.workload][0])
    D = sc.max_depth
    _say(f"bench: scene {sc.name} tris={sc.num_triangles} {sc.width}x{sc.height} D={D}")
    r = Renderer(sc, device=0, bvh_builder=args.bvh_builder, node_format=args.node_format)
    bs = r.bvh_stats
    _say(f"bench: bvh nodes={bs.num_nodes} leaves={bs.num_leaves} depth={bs.max_depth} build={bs.build_ms:.0f} ms")
    # the passes go to the library as one range, which renders them in batches
    # of as many whole passes as its path pool holds (sixteen frames' worth)
    cs = args.compress_state
    td = args.tail_depth if args.tail_depth >= 0 else D // 2
    r.render(0, args.warmup, single_stream=args.single_stream, compress_state=cs, tail_depth=td)
    torch.cuda.synchronize()
    _say(f"bench: warmup {args.warmup} passes done")
    st0 = r.stats()
    if not args.no_profile:
        r.ctx.profile(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    r.render(args.warmup, args.steps, single_stream=args.single_stream, compress_state=cs, tail_depth=td)
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

        def kernel_bytes(a, b):
            e, h = b.rays_extension - a.rays_extension, b.rays_shadow - a.rays_shadow
            dn, dt_ = b.nodes_extension - a.nodes_extension, b.tris_extension - a.tris_extension
            sn, stt = b.nodes_shadow - a.nodes_shadow, b.tris_shadow - a.tris_shadow
            nb = r.bvh_stats.node_bytes
            tr_b, sv_b, sc_b = ((TRACE_RAY_BYTES_C, SHADE_VERTEX_BYTES_C, SHADE_CONTINUE_BYTES_C) if cs else
                                (TRACE_RAY_BYTES, SHADE_VERTEX_BYTES, SHADE_CONTINUE_BYTES))
            byts = {"trace": e * tr_b + dn * nb + dt_ * TRI_BYTES,
                    "shadow": h * SHADOW_RAY_BYTES + sn * nb + stt * TRI_BYTES,
                    "shade": e * sv_b + (e - (b.paths - a.paths)) * sc_b + h * SHADE_NEE_BYTES}
            stream = {"trace": e * tr_b, "shadow": h * SHADOW_RAY_BYTES, "shade": byts["shade"]}
            counts = {"nodes_per_ray": round(dn / max(e, 1), 2), "tris_per_ray": round(dt_ / max(e, 1), 2),
                      "shadow_nodes_per_ray": round(sn / max(h, 1), 2), "shadow_tris_per_ray": round(stt / max(h, 1), 2)}
            return byts, stream, counts

        # Per-launch durations are taken on one stream: with two batches in
        # flight a launch's events also span its wait for the other batch's
        # kernels. When the timed region ran two batches at a time, the same
        # number of passes follows on one stream for the roofline, and the
        # dominant kernel is the one with the most time there.
        if args.single_stream and not td:
            r_prof, r0, r1 = prof, st0, st1
        else:
            r0 = r.stats()
            r.ctx.profile(True)
            # without the megakernel tail, whose launches would trace and shade
            # rays the per-depth kernels' byte counts could not tell apart
            r.render(args.warmup + args.steps, args.steps, single_stream=True, compress_state=cs)
            r.ctx.profile(False)
            r_prof = r.ctx.profile_read()
            r1 = r.stats()
        rb, rstream, counts = kernel_bytes(r0, r1)
        dom = max(rb, key=lambda k: r_prof[k][1])
        n_l, ms = r_prof[dom]
        launch_s = ms / n_l * 1e-3
        per_launch = rb[dom] / n_l
        achieved = per_launch / launch_s / 1e9
        # the committed counter summaries were taken with the full-precision state
        traffic = None if cs else pmc_traffic(f"k_{dom}", WORKLOADS[args.workload][0])
        roof = {"kernel": f"k_{dom}", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                # compulsory streaming bytes only (no node or triangle fetches), and the
                # HBM bytes the counters measured, over the same launch time
                "frac_stream": round(rstream[dom] / n_l / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                "frac_measured": round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                "bytes_per_launch": round(per_launch), "avg_launch_ms": round(ms / n_l, 4),
                "launches": n_l, "timed_on": "one stream, %d passes after the timed region, per-depth kernels "
                "to the end (no megakernel tail)" % args.steps
                if (not args.single_stream or td) else "the timed region (one stream)", **counts}
        if not args.single_stream and prof[dom][0]:
            o_l, o_ms = prof[dom]
            roof["two_batches_in_flight"] = {"launches": o_l, "avg_launch_event_ms": round(o_ms / o_l, 4),
                                             "note": "event span per launch in the timed region, including "
                                                     "waits for the other batch's kernels"}
        _say(f"bench: kernels {kernels}")
        _say(f"bench: roofline {roof}")

    cpu = None
    S = None
    if not args.no_cpu_baseline:
        _say("bench: CPU oracle: building its scene")
        S, build_s = oracle_scene(sc)
        _say(f"bench: CPU oracle baseline (~{args.cpu_seconds:.0f} s after a {build_s:.1f} s build)")
        cpu = cpu_baseline(S, sc, args.cpu_seconds, build_s)

    ls = None
    if args.workload == "city" and not args.no_light_select:
        _say("bench: alias table vs light tree at equal time")
        ls = light_select_equal_time(r, sc, args.ls_seconds, args.ls_ref_passes)
        _say(f"bench: light selection {ls}")

    es_out = None
    if args.env_select:
        r = None
        torch.cuda.empty_cache()
        w, h = (int(v) for v in args.et_size.split("x"))
        es_out = env_select_equal_time(args.es_seconds, args.es_ref_passes, w, h, args.et_tris)
        _say(f"bench: environment samplers {es_out}")

    et = None
    if not args.no_equal_time:
        r = None
        torch.cuda.empty_cache()
        et = []
        if args.workload == "city" and not args.no_et_city:
            _say("bench: equal time, guided vs plain, on the city")
            et.append(equal_time(sc, [("the workload's camera", None)], args.et_city_seconds, args.et_city_ref_passes,
                                 32, oracle_scene=S, oracle_seconds=args.et_oracle_seconds, oracle_stride=(64, 64)))
            torch.cuda.empty_cache()
        S = None
        w, h = (int(v) for v in args.et_size.split("x"))
        slit = scenegen.slit_scene(width=w, height=h, target_tris=args.et_tris, max_depth=16)
        _say(f"bench: equal-time workload {slit.name} tris={slit.num_triangles} {w}x{h} D=16")
        S_slit = None
        if args.et_oracle_seconds > 0:
            S_slit, _ = oracle_scene(slit)
        et.append(equal_time(slit, [("indirectly lit half (the workload's camera)", None),
                                    ("along the enclosure, sunlit strip in view",
                                     scenegen.Camera((0.0, 4.0, -28.0), (0.0, 2.0, 0.0), (0.0, 1.0, 0.0), 40.0))],
                             args.et_seconds, args.et_ref_passes, 32, oracle_scene=S_slit,
                             oracle_seconds=args.et_oracle_seconds, oracle_stride=(64, 64)))
        del S_slit
        _say(f"bench: equal time {et}")

    out = {
        "metric": METRIC, "value": round(mrays, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload][1],
                   "triangles": sc.num_triangles, "pixels": sc.width * sc.height, "max_depth": D,
                   "path_state": "compressed" if cs else "full precision",
                   "megakernel_tail_from_depth": td or None,
                   "parallelism": "single GPU"},
        "mpaths_per_s": round(mpaths, 3),
        "rays_per_path": round((ext + sh) / paths, 3),
        "bvh": {"builder": "GPU linear BVH (Morton, collapsed to 4-wide)" if args.bvh_builder else
                "host binned SAH (collapsed to 4-wide)", "build_ms": round(bs.build_ms, 1),
                "nodes": bs.num_nodes, "node_bytes": bs.node_bytes, "leaves": bs.num_leaves, "depth": bs.max_depth,
                "sah_cost": round(bs.sah_cost, 2)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "equal_time_rmse": et,
        "light_selection_equal_time": ls,
        "env_sampling_equal_time": es_out,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
