"""Summaries of rocprofv3 output for the committed profiles.

`python -m paper_1705_01263_amd.profiling trace <results.db|kernel_trace.csv> <out.txt> --cmd "..."`
writes per-kernel launch counts and durations.

`python -m paper_1705_01263_amd.profiling pmc <fetch_dir> <write_dir> <kernel> <out.txt> --calib-mib N --cmd "..."`
turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch) into HBM bytes per launch of
`kernel`, each counter scaled by what it reads for the calibration copy
kernel of known size in the same run.

`python -m paper_1705_01263_amd.profiling mfma <pmc_dir> <out.txt> --cmd "..."` summarises
BF16 MFMA FLOPs and MFMA busy cycles of the network kernels.

`python -m paper_1705_01263_amd.profiling sweep <out.txt> [--min-log2 A --max-log2 B]` measures
throughput against the path pool size, one batch at a time and two in flight.

`python -m paper_1705_01263_amd.profiling guided [--size WxH --tris N --passes K]`
runs a guided, training workload on the slit scene to be profiled.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import os
import sqlite3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_sha() -> str:
    """SHA of the path kernels and of the host side that builds the tree they
    traverse and launches them: counters taken on other sources are stale."""
    h = hashlib.sha256()
    for f in ("qpt_kernels.hip", "qpt_host.cpp"):
        h.update(open(os.path.join(ROOT, "paper_1705_01263_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def guide_sha() -> str:
    src = os.path.join(ROOT, "paper_1705_01263_amd", "csrc", "qpt_guide.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("qpt::(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(")[0] if "(" in name else name


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


def summarize_mfma(pmc_dir: str, kernels, out_txt: str, cmd: str, simds: int = 1024) -> str:
    """Per-dispatch MFMA and VALU activity of `kernels` from one rocprofv3
    --pmc run with SQ_INSTS_VALU_MFMA_MOPS_BF16, SQ_VALU_MFMA_BUSY_CYCLES,
    SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_BUSY_CU_CYCLES and GRBM_GUI_ACTIVE.
    MFMA FLOPs = MOPS_BF16 x 512; utilisation = MFMA busy cycles over
    GRBM_GUI_ACTIVE x SIMDs (256 CUs x 4 on MI355X)."""
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
        lines += [f"{k}: dispatches {len(ds)}, avg duration {t_ns / 1e3:.2f} us",
                  f"  BF16 MFMA FLOP per dispatch {flops:.4g} -> {flops / t_ns / 1e3:.2f} TFLOP/s "
                  f"({100 * flops / t_ns / 1e3 / 2500.0:.2f}% of the 2.5 PFLOP/s dense BF16 peak)",
                  f"  MFMA busy {100 * busy / max(gui * simds, 1):.2f}% of SIMD cycles "
                  f"(SQ_VALU_MFMA_BUSY_CYCLES {busy:.4g}, GRBM_GUI_ACTIVE {gui:.4g})",
                  f"  SQ_INSTS_VALU {avg('SQ_INSTS_VALU'):.4g}, SQ_ACTIVE_INST_VALU {avg('SQ_ACTIVE_INST_VALU'):.4g}, "
                  f"SQ_BUSY_CU_CYCLES {avg('SQ_BUSY_CU_CYCLES'):.4g}"]
    txt = "\n".join(lines) + "\n"
    open(out_txt, "w").write(txt)
    return txt


def run_guided(width: int, height: int, tris: int, passes: int, alpha: float = 0.7, max_vertex: int = 2) -> None:
    """A guided workload to profile: the slit scene with the guide training
    one step per batch of passes from its first pass."""
    import torch

    import scenegen
    from paper_1705_01263_amd import Renderer

    sc = scenegen.slit_scene(width=width, height=height, target_tris=tris, max_depth=16)
    r = Renderer(sc)
    r.ctx.guide_set_weights(scenegen.guide_init(1))
    r.ctx.guide_config(alpha=alpha, lr=1e-3, batch=1 << 18, train=1, warmup_steps=0, seed=1, max_vertex=max_vertex)
    r.render(0, passes)
    torch.cuda.synchronize()
    _, steps = r.ctx.guide_get_weights()
    print(f"guided: {passes} passes of {sc.name} {width}x{height}, {steps} Adam steps", flush=True)


def run_sweep(out_txt: str, min_log2: int, max_log2: int, cmd: str) -> str:
    """Passes per launch sequence against throughput (the paper's Table 1 in
    kind): the grid workload at 1080p with path pools from 2^min_log2 to
    2^max_log2 slots, one batch at a time and two in flight; each setting
    renders two pools' worth of passes (at least 8) after one untimed batch."""
    import time

    import torch

    import scenegen
    from paper_1705_01263_amd import Renderer

    sc = scenegen.workload("grid_1m")
    npix = sc.width * sc.height
    lines = ["# passes per launch sequence against throughput (grid, 0.97M triangles, 1920x1080, depth 12)",
             f"command: {cmd}", f"kernel_source_sha: {kernel_sha()}", "",
             f"{'pool (paths)':>14} {'frames/batch':>13} {'passes':>7} {'one stream Mrays/s':>19} "
             f"{'two in flight Mrays/s':>22} {'Mpaths/s (two)':>15}"]
    for lg in range(min_log2, max_log2 + 1):
        pool = 1 << lg
        frames = pool / npix
        per = max(1, pool // npix)
        passes = max(8, 2 * per)
        r = Renderer(sc, pool_paths=pool)
        res = []
        for single in (True, False):
            r.reset()
            r.render(0, per, single_stream=single)
            torch.cuda.synchronize()
            st0 = r.stats()
            t0 = time.perf_counter()
            r.render(per, passes, single_stream=single)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st1 = r.stats()
            rays = (st1.rays_extension - st0.rays_extension) + (st1.rays_shadow - st0.rays_shadow)
            res.append((rays / dt / 1e6, passes * npix / dt / 1e6))
        del r
        torch.cuda.empty_cache()
        lines.append(f"{'2^%d' % lg:>14} {frames:>13.3f} {passes:>7} {res[0][0]:>19.1f} {res[1][0]:>22.1f} "
                     f"{res[1][1]:>15.1f}")
        print(lines[-1], flush=True)
    txt = "\n".join(lines) + "\n"
    open(out_txt, "w").write(txt)
    return txt


def main():
    ap = argparse.ArgumentParser()
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
    m.add_argument("--kernels", default="k_guide_eval,k_guide_train")
    m.add_argument("--cmd", required=True)
    sw = sub.add_parser("sweep")
    sw.add_argument("out")
    sw.add_argument("--min-log2", type=int, default=15)
    sw.add_argument("--max-log2", type=int, default=25)
    gd = sub.add_parser("guided")
    gd.add_argument("--size", default="1920x1080")
    gd.add_argument("--tris", type=int, default=4_000_000)
    gd.add_argument("--passes", type=int, default=8)
    gd.add_argument("--max-vertex", type=int, default=2)
    a = ap.parse_args()
    if a.what == "trace":
        print(summarize_trace(a.src, a.out, a.cmd))
    elif a.what == "pmc":
        print(summarize_pmc(a.fetch_dir, a.write_dir, a.kernel, a.out, a.calib_mib, a.cmd))
    elif a.what == "sweep":
        cmd = ("python -u -m paper_1705_01263_amd.profiling sweep " + a.out +
               f" --min-log2 {a.min_log2} --max-log2 {a.max_log2}")
        print(run_sweep(a.out, a.min_log2, a.max_log2, cmd))
    elif a.what == "mfma":
        print(summarize_mfma(a.pmc_dir, a.kernels.split(","), a.out, a.cmd))
    else:
        w, h = (int(v) for v in a.size.split("x"))
        run_guided(w, h, a.tris, a.passes, max_vertex=a.max_vertex)


if __name__ == "__main__":
    main()
