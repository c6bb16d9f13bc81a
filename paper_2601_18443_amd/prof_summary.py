"""Text summaries of rocprofv3 CSV output (``-f csv``) for the kernels of liblbr.

Two reports:

``stats DIR``
    the per-kernel table of ``--kernel-trace --stats`` (``*kernel_stats.csv``),
    plus a per-launch-size breakdown of the step kernels from
    ``*kernel_trace.csv``;
``traffic``
    HBM bytes per step-kernel dispatch from two ``--pmc`` runs (FETCH_SIZE, then
    WRITE_SIZE, in KiB per dispatch), each scaled by what the same counter reads
    for a device copy of known size (``bench.py --copy-calibration``);
``gaps``
    the idle time between consecutive step-kernel dispatches of a stream of
    super steps (``*kernel_trace.csv``): per super step of M launches, the span
    from the first start to the last end, the summed kernel durations and the
    summed gaps, the part of the span a single persistent launch could at most
    remove by running the same work without launch boundaries.

Usage::

    python -m paper_2601_18443_amd.prof_summary stats DIR --cmd "..." > out.txt
    python -m paper_2601_18443_amd.prof_summary traffic --fetch D1 --write D2 \\
        --cal-fetch D3 --cal-write D4 --copy-bytes N --storage f32 \\
        --alg-bytes B --cmd "..." > out.txt
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import sys
from collections import defaultdict

_HERE = os.path.dirname(os.path.abspath(__file__))
# the kernels and the host code that lays out their launches
SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("lbr_kernels.hip", "lbr_host.cpp")]


def kernel_source_hash():
    """Hash of the code (comments and whitespace stripped) of the kernels and
    of the host code that lays out their launches."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(f) as fh:
            text = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def short_name(name):
    """k_step<float, float> from a demangled kernel signature."""
    name = name.strip().strip('"')
    m = re.search(r"(k_[a-z_]+)<([^()]*)>", name)
    if m:
        return f"{m.group(1)}<{m.group(2).replace('__hip_bfloat16', 'bf16').replace('__half', 'half')}>"
    m = re.search(r"(k_[a-z_]+)", name)
    if m:
        return m.group(1)
    return name.split("(")[0][:60]


def _find(directory, pattern):
    hits = sorted(glob.glob(os.path.join(directory, "**", pattern), recursive=True))
    if not hits:
        sys.exit(f"no {pattern} under {directory}")
    return hits


def _col(row, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError(f"none of {names} in {list(row)}")


def stats(directory, cmd, tail=0):
    out = [f"# rocprofv3 kernel statistics", f"# command: {cmd}", ""]
    rows = []
    for path in _find(directory, "*kernel_stats.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                rows.append((short_name(_col(r, "Name", "KernelName")), int(_col(r, "Calls")),
                             float(_col(r, "TotalDurationNs")), float(_col(r, "AverageNs")),
                             float(_col(r, "MinNs")), float(_col(r, "MaxNs")),
                             float(_col(r, "Percentage"))))
    rows.sort(key=lambda r: -r[2])
    out.append(f"{'kernel':34s} {'calls':>7s} {'total ms':>10s} {'avg us':>9s} {'min us':>9s} "
               f"{'max us':>9s} {'%':>6s}")
    for n, calls, tot, avg, mn, mx, pct in rows:
        out.append(f"{n:34s} {calls:7d} {tot / 1e6:10.3f} {avg / 1e3:9.2f} {mn / 1e3:9.2f} "
                   f"{mx / 1e3:9.2f} {pct:6.2f}")
    traces = glob.glob(os.path.join(directory, "**", "*kernel_trace.csv"), recursive=True)
    if traces:
        per = defaultdict(list)
        seq = []
        for path in traces:
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    n = short_name(_col(r, "Kernel_Name"))
                    if not n.startswith("k_step"):
                        continue
                    g = int(_col(r, "Grid_Size_X", "Grid_Size", "Grid_X"))
                    t0 = float(_col(r, "Start_Timestamp"))
                    d = float(_col(r, "End_Timestamp")) - t0
                    per[(n, g)].append(d)
                    seq.append((t0, d))
        if tail and seq:
            seq.sort()
            last = [d for _, d in seq[-tail:]]
            out += ["", f"step kernels, the last {len(last)} dispatches (the direct launches that "
                    f"bench.py times with dispatch events): average {sum(last) / len(last) / 1e3:.2f} us"]
        out += ["", "step kernels by launch size (the 20 largest)",
                f"{'kernel':34s} {'threads':>9s} {'blocks':>7s} {'calls':>7s} {'avg us':>9s} {'median us':>10s}"]
        for (n, g), v in sorted(per.items(), key=lambda kv: -kv[0][1])[:20]:
            v.sort()
            out.append(f"{n:34s} {g:9d} {g // 256:7d} {len(v):7d} {sum(v) / len(v) / 1e3:9.2f} "
                       f"{v[len(v) // 2] / 1e3:10.2f}")
    return "\n".join(out) + "\n"


def _counter(directory, counter, match):
    """Per-dispatch values of one counter for kernels whose short name starts with match."""
    vals = defaultdict(float)
    for path in _find(directory, "*counter_collection.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if _col(r, "Counter_Name") != counter:
                    continue
                n = short_name(_col(r, "Kernel_Name"))
                if not match(n):
                    continue
                key = (path, _col(r, "Dispatch_Id", "Correlation_Id"))
                vals[key] += float(_col(r, "Counter_Value"))
    return list(vals.values())


def traffic(a):
    is_step = lambda n: n.split("<")[0] == a.kernel                  # noqa: E731
    is_copy = lambda n: "copy" in n.lower()                           # noqa: E731
    fetch = _counter(a.fetch, "FETCH_SIZE", is_step)
    write = _counter(a.write, "WRITE_SIZE", is_step)
    cf = _counter(a.cal_fetch, "FETCH_SIZE", is_copy)
    cw = _counter(a.cal_write, "WRITE_SIZE", is_copy)
    if not (fetch and write and cf and cw):
        sys.exit("missing counter rows")
    f_kib = sum(fetch) / len(fetch)
    w_kib = sum(write) / len(write)
    ffac = a.copy_bytes / (max(cf) * 1024.0)
    wfac = a.copy_bytes / (max(cw) * 1024.0)
    hbm = f_kib * 1024.0 * ffac + w_kib * 1024.0 * wfac
    lines = [
        f"# HBM traffic of {a.kernel} (all levels), rocprofv3 --pmc, per dispatch",
        f"# fetch run: {a.cmd_fetch}",
        f"# write run: {a.cmd_write}",
        f"# calibration runs: {a.cmd_cal}",
        f"# FETCH_SIZE / WRITE_SIZE are averaged over the {a.kernel} dispatches and scaled by",
        "# copy bytes / counter reading of a device copy of known size.",
        f"source_sha256 = {kernel_source_hash()}",
        f"storage = {a.storage}",
        f"kernel = {a.kernel}",
        f"dispatches = {len(fetch)}",
        f"fetch_kib_per_dispatch = {f_kib:.1f}",
        f"write_kib_per_dispatch = {w_kib:.1f}",
        f"copy_bytes = {a.copy_bytes}",
        f"copy_fetch_kib = {max(cf):.1f}",
        f"copy_write_kib = {max(cw):.1f}",
        f"fetch_scale = {ffac:.4f}",
        f"write_scale = {wfac:.4f}",
        f"hbm_bytes_per_launch = {hbm:.0f}",
        f"alg_bytes_per_launch = {a.alg_bytes:.0f}",
        f"hbm_over_alg = {hbm / a.alg_bytes:.3f}",
    ]
    return "\n".join(lines) + "\n"


def gaps(a):
    """Idle gaps between the first a.first dispatches of a.kernel (by start time),
    grouped into super steps of a.per_step launches."""
    rows = []
    for path in _find(a.dir, "*kernel_trace.csv"):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                n = short_name(_col(r, "Kernel_Name"))
                if n.split("<")[0] != a.kernel:
                    continue
                rows.append((float(_col(r, "Start_Timestamp")), float(_col(r, "End_Timestamp"))))
    rows.sort()
    rows = rows[a.skip:a.skip + a.first]
    m = a.per_step
    nsup = len(rows) // m
    if nsup < 1:
        sys.exit("fewer dispatches than one super step")
    span = busy = inner = between = 0.0
    for k in range(nsup):
        grp = rows[k * m:(k + 1) * m]
        span += grp[-1][1] - grp[0][0]
        busy += sum(e - s for s, e in grp)
        inner += sum(max(0.0, grp[j + 1][0] - grp[j][1]) for j in range(m - 1))
        if k + 1 < nsup:
            between += max(0.0, rows[(k + 1) * m][0] - grp[-1][1])
    lines = [
        f"# dispatch gaps of {a.kernel}, rocprofv3 --kernel-trace",
        f"# command: {a.cmd}",
        f"source_sha256 = {kernel_source_hash()}",
        f"kernel = {a.kernel}",
        f"dispatches = {nsup * m} (dispatch {a.skip} on, {nsup} super steps of {m} launches)",
        f"span_us_per_super_step = {span / nsup / 1e3:.2f}",
        f"kernel_us_per_super_step = {busy / nsup / 1e3:.2f}",
        f"gaps_inside_us_per_super_step = {inner / nsup / 1e3:.2f}",
        f"gap_between_super_steps_us = {between / max(nsup - 1, 1) / 1e3:.2f}",
        f"gaps_over_span = {(inner + between) / (span + between):.4f}",
    ]
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--cmd", required=True)
    s.add_argument("--tail", type=int, default=0,
                   help="also average the last TAIL step-kernel dispatches")
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "cal_fetch", "cal_write"):
        t.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--storage", required=True)
    t.add_argument("--alg-bytes", type=float, required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--cmd-cal", required=True)
    t.add_argument("--kernel", default="k_step_batch",
                   help="kernel whose dispatches are averaged (k_step_batch: the merged schedule)")
    g = sub.add_parser("gaps")
    g.add_argument("dir")
    g.add_argument("--cmd", required=True)
    g.add_argument("--kernel", default="k_step_batch")
    g.add_argument("--skip", type=int, default=0, help="dispatches to skip first (warm-up)")
    g.add_argument("--first", type=int, required=True, help="dispatches to analyse")
    g.add_argument("--per-step", type=int, required=True, help="launches per super step")
    a = ap.parse_args(argv)
    if a.what == "stats":
        sys.stdout.write(stats(a.dir, a.cmd, a.tail))
    elif a.what == "gaps":
        sys.stdout.write(gaps(a))
    else:
        sys.stdout.write(traffic(a))


if __name__ == "__main__":
    main()
