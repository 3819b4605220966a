"""Summarise rocprofv3 output databases (rocpd SQLite) as short text.

    python -m paper_1404_0076_amd.rocpd_summary trace  DIR   [--kernel NAME] [--last N]
    python -m paper_1404_0076_amd.rocpd_summary counters DIR [--kernel NAME] [--last N]

``trace``: per-kernel calls / total / average duration from a --kernel-trace
run, plus the last N dispatches of the selected kernel.  ``counters``: the
per-dispatch value of every collected counter (summed over its instances) for
the selected kernel's last N dispatches.
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
                               "from kernels where name like ? order by start",
                               (f"%{kernel}%",)).fetchall()
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
            "from counters_collection where kernel_name like ? group by dispatch_id, counter_name "
            "order by start", (f"%{kernel}%",)).fetchall()
        out.append(f"# {os.path.basename(db)}: last {min(last, len(rows))} dispatches of {kernel}")
        out.append("  dispatch counter value(KiB for *_SIZE) grid duration_us")
        for d, name, cname, val, grid, dur in rows[-last:]:
            out.append(f"  {d:6d} {cname:12s} {val:16.1f} {grid:9d} {dur / 1e3:12.3f}")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["trace", "counters"])
    ap.add_argument("path")
    ap.add_argument("--kernel", default="")
    ap.add_argument("--last", type=int, default=5)
    a = ap.parse_args(argv)
    print(trace(a.path, a.kernel, a.last) if a.mode == "trace" else counters(a.path, a.kernel, a.last))


if __name__ == "__main__":
    sys.exit(main())
