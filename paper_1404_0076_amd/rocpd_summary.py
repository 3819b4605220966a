"""Summarise rocprofv3 output databases (rocpd SQLite) as short text.

    python -m paper_1404_0076_amd.rocpd_summary trace  DIR   [--kernel NAME] [--last N]
    python -m paper_1404_0076_amd.rocpd_summary counters DIR [--kernel NAME] [--last N]
    python -m paper_1404_0076_amd.rocpd_summary phases DIR
    python -m paper_1404_0076_amd.rocpd_summary hbm --fetch DIR --write DIR
        --copy-fetch DIR --copy-write DIR --copy-bytes N --bench-json FILE --sources-hash H

``trace``: per-kernel calls / total / average duration from a --kernel-trace
run, plus the last N dispatches of the selected kernel.  ``counters``: the
per-dispatch value of every collected counter (summed over its instances) for
the selected kernel's last N dispatches.  ``phases``: the paper-pipeline
ablation's kernel time split into its loop's phases.  ``hbm``: HBM bytes per launch of the
bench's reduce kernel from one FETCH_SIZE run and one WRITE_SIZE run, each
scaled by what the same counter reads for a plain device copy of known size;
the output carries the meta lines (kernel source hash, workload key, bytes per
launch) that bench.py matches before it reports the figure.
"""
from __future__ import annotations

import argparse
import glob
import os
import sqlite3
import sys


def _dbs(path):
    if os.path.isfile(path):
        return [path]
    return sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True))


def trace(path, kernel, last):
    out = []
    for db in _dbs(path):
        con = sqlite3.connect(db)
        out.append(f"# {os.path.basename(db)}")
        out.append(f"{'kernel':70s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>12s}")
        # the top_kernels view reports microseconds; the kernels table nanoseconds
        for name, calls, total, avg, pct in con.execute(
                "select name, total_calls, total_duration, average, percentage from top_kernels"):
            out.append(f"{name[:70]:70s} {calls:6d} {total / 1e3:10.3f} {avg:12.3f}")
        if kernel:
            rows = con.execute("select name, duration, grid_x, workgroup_x, lds_size, vgpr_count "
                               "from kernels where instr(name, ?) > 0 order by start",
                               (kernel,)).fetchall()
            out.append(f"last {min(last, len(rows))} dispatches of {kernel}: "
                       "duration_us grid workgroup lds vgpr")
            for name, dur, gx, wx, lds, vgpr in rows[-last:]:
                out.append(f"  {dur / 1e3:12.3f} {gx // max(wx, 1):7d} {wx:5d} {lds:7d} {vgpr:4d}")
    return "\n".join(out)


def counters(path, kernel, last):
    out = []
    for db in _dbs(path):
        con = sqlite3.connect(db)
        rows = con.execute(
            "select dispatch_id, kernel_name, counter_name, sum(value), grid_size, duration "
            "from counters_collection where instr(kernel_name, ?) > 0 "
            "group by dispatch_id, counter_name order by start", (kernel,)).fetchall()
        out.append(f"# {os.path.basename(db)}: last {min(last, len(rows))} dispatches of {kernel}")
        out.append("  dispatch counter value(KiB for *_SIZE) grid duration_us")
        for d, name, cname, val, grid, dur in rows[-last:]:
            out.append(f"  {d:6d} {cname:12s} {val:16.1f} {grid:9d} {dur / 1e3:12.3f}")
    return "\n".join(out)


def _counter_rows(path, kernel, counter):
    rows = []
    for db in _dbs(path):
        con = sqlite3.connect(db)
        rows += con.execute(
            "select dispatch_id, sum(value), duration from counters_collection "
            "where instr(kernel_name, ?) > 0 and counter_name = ? group by dispatch_id order by start",
            (kernel, counter)).fetchall()
    if not rows:
        raise SystemExit(f"no {counter} rows for {kernel!r} under {path}")
    return rows


def hbm(a):
    import json
    bench = None
    with open(a.bench_json) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{"):
                bench = json.loads(line)
    if bench is None:
        raise SystemExit(f"no JSON line in {a.bench_json}")
    roof = bench["roofline"]
    kernel = roof["kernel"]
    fetch = _counter_rows(a.fetch, kernel, "FETCH_SIZE")[-1]
    write = _counter_rows(a.write, kernel, "WRITE_SIZE")[-1]
    cf = [v for _, v, _ in _counter_rows(a.copy_fetch, "copyBuffer", "FETCH_SIZE")[-3:]]
    cw = [v for _, v, _ in _counter_rows(a.copy_write, "copyBuffer", "WRITE_SIZE")[-3:]]
    kib = a.copy_bytes / 1024.0
    ff, fw = kib / (sum(cf) / len(cf)), kib / (sum(cw) / len(cw))
    fb, wb = fetch[1] * 1024.0 * ff, write[1] * 1024.0 * fw
    alg = roof["algorithmic_bytes"]
    out = [
        f"# {kernel} -- {bench['config']['workload']}: HBM counters of the last dispatch",
        f"# kernel_sources_sha256: {a.sources_hash}",
        f"# workload_key: {roof['workload_key']}",
        f"# traffic_bytes_per_launch: {fb + wb:.6e}",
        f"# FETCH_SIZE {fetch[1]:.1f} KiB (dispatch {fetch[0]}, {fetch[2] / 1e3:.3f} us), "
        f"WRITE_SIZE {write[1]:.1f} KiB (dispatch {write[0]}, {write[2] / 1e3:.3f} us)",
        f"# copy calibration: {a.copy_bytes} B copied; FETCH_SIZE reads "
        f"{', '.join(f'{v:.1f}' for v in cf)} KiB (factor {ff:.3f}), WRITE_SIZE reads "
        f"{', '.join(f'{v:.1f}' for v in cw)} KiB (factor {fw:.3f})",
        f"# traffic per launch: fetch {fb:.4e} B + write {wb:.4e} B = {fb + wb:.4e} B",
        f"# algorithmic bytes per launch (bench.py): {alg:.4e} B; traffic / algorithmic = "
        f"{(fb + wb) / alg:.2f}",
    ]
    return "\n".join(out)


# kernels of the paper-pipeline ablation that open a phase of its loop; the
# primitives' own scan and reduction kernels belong to the phase that launched
# them (the latest one opened)
_PHASE_OPEN = (("k_pp_need", "int"), ("KeepIfNot", "filter"), ("k_pp_key", "com: sort"),
               ("RunHead", "com: reduce by key"))
_PHASES = ("int", "filter", "com: sort", "com: reduce by key", "copies and fills", "other")


def _phase_of(name, cur):
    for mark, ph in _PHASE_OPEN:
        if mark in name:
            return ph, ph
    if "k_pp_int" in name:
        return "int", "int"
    if "k_rs_" in name:
        return "com: sort", cur
    if "k_tile_" in name:
        return cur or "other", cur
    if "copyBuffer" in name or "fillBuffer" in name:
        return "copies and fills", cur
    return "other", cur


def phases(path):
    """Kernel time of the paper pipeline's loop split by phase: int (need,
    allocation scan, the interaction kernel), filter (dummy removal), com
    (key, radix sort; reduce by key), and the copies and fills between them
    (counts to the host, list moves).  The net engine's own launches in the
    same process (sizing runs) are left out."""
    out = []
    for db in _dbs(path):
        con = sqlite3.connect(db)
        tot = dict.fromkeys(_PHASES, 0.0)
        calls = dict.fromkeys(_PHASES, 0)
        int_kernel = 0.0
        cur = ""
        for name, dur in con.execute("select name, duration from kernels order by start"):
            if "inet_grid" in name or "inet_static" in name or "k_jump" in name \
                    or "k_reset" in name or "k_zero" in name:
                continue
            ph, cur = _phase_of(name, cur)
            tot[ph] += dur / 1e6
            calls[ph] += 1
            if "k_pp_int" in name:
                int_kernel += dur / 1e6
        all_ms = sum(tot.values())
        out.append(f"# {os.path.basename(db)}: paper-pipeline kernel time by phase")
        out.append(f"{'phase':22s} {'dispatches':>10s} {'ms':>10s} {'share':>7s}")
        for ph in _PHASES:
            out.append(f"{ph:22s} {calls[ph]:10d} {tot[ph]:10.3f} {tot[ph] / max(all_ms, 1e-9):7.1%}")
        out.append(f"{'total':22s} {sum(calls.values()):10d} {all_ms:10.3f}")
        out.append(f"interaction kernel alone (k_pp_int): {int_kernel:.3f} ms = "
                   f"{int_kernel / max(all_ms, 1e-9):.2%} of the loop's kernel time")
        if int_kernel > 0:
            out.append(f"filter / interaction kernel = {tot['filter'] / int_kernel:.2f}; "
                       f"(filter + com) / interaction kernel = "
                       f"{(tot['filter'] + tot['com: sort'] + tot['com: reduce by key']) / int_kernel:.2f}")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "counters", "hbm", "phases"])
    ap.add_argument("path", nargs="?", default="")
    ap.add_argument("--kernel", default="")
    ap.add_argument("--last", type=int, default=5)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--bench-json")
    ap.add_argument("--sources-hash", default="")
    a = ap.parse_args(argv)
    if a.mode == "hbm":
        print(hbm(a))
    elif a.mode == "trace":
        print(trace(a.path, a.kernel, a.last))
    elif a.mode == "phases":
        print(phases(a.path))
    else:
        print(counters(a.path, a.kernel, a.last))


if __name__ == "__main__":
    sys.exit(main())
