"""Summaries of rocprofv3 output for the committed profiles.

`python -m paper_1705_01263_amd.profiling trace <results.db|kernel_trace.csv> <out.txt> --cmd "..."`
writes per-kernel launch counts and durations.

`python -m paper_1705_01263_amd.profiling pmc <fetch_dir> <write_dir> <kernel> <out.txt> --calib-mib N --cmd "..."`
turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch) into HBM bytes per launch of
`kernel`, each counter scaled by what it reads for the calibration copy
kernel of known size in the same run.
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
    src = os.path.join(ROOT, "paper_1705_01263_amd", "csrc", "qpt_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("qpt::(anonymous namespace)::", "")
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
    a = ap.parse_args()
    if a.what == "trace":
        print(summarize_trace(a.src, a.out, a.cmd))
    else:
        print(summarize_pmc(a.fetch_dir, a.write_dir, a.kernel, a.out, a.calib_mib, a.cmd))


if __name__ == "__main__":
    main()
