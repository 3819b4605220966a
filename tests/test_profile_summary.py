"""Host-side checks of the profile summariser (rocpd SQLite databases), on
small databases written here with the tables and columns it reads."""
import os
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1404_0076_amd import rocpd_summary as rs  # noqa: E402


def kernels_db(path, rows):
    """rows: (name, duration_ns) in launch order."""
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, duration integer, grid_x integer,"
                " workgroup_x integer, lds_size integer, vgpr_count integer)")
    for i, (name, dur) in enumerate(rows):
        con.execute("insert into kernels values (?, ?, ?, 256, 256, 0, 8)", (name, 1000 * i, dur))
    con.commit()
    con.close()


def test_phases_assign_primitives_to_the_phase_that_launched_them(tmp_path):
    # one loop iteration of the paper pipeline: int (need, scan, interaction),
    # filter (count, scan, emit), com (key, four radix passes of hist / scan /
    # scatter, then reduce by key: count, scan, emit), copies; the net
    # engine's sizing launch is left out
    it = [("inet::k_pp_need", 2000), ("inet::prim::k_tile_scan<unsigned long long>", 3000),
          ("inet::k_pp_int", 5000),
          ("inet::prim::k_flag_count<inet::prim::KeepIfNot>", 1000),
          ("inet::prim::k_tile_scan<unsigned int>", 1000),
          ("inet::prim::k_flag_emit<inet::prim::KeepIfNot, x>", 1000),
          ("__amd_rocclr_copyBuffer", 7000),
          ("inet::k_pp_key", 500)]
    for _ in range(4):
        it += [("inet::prim::k_rs_hist", 100), ("inet::prim::k_tile_scan<unsigned int>", 100),
               ("inet::prim::k_rs_scatter<unsigned long long>", 300)]
    it += [("inet::prim::k_flag_count<inet::prim::RunHead>", 400),
           ("inet::prim::k_tile_scan<unsigned int>", 400),
           ("inet::prim::k_flag_emit<inet::prim::RunHead, y>", 400),
           ("__amd_rocclr_fillBufferAligned", 600)]
    db = tmp_path / "pipe_results.db"
    kernels_db(str(db), [("inet_grid_1024", 10**6)] + it + it)
    out = rs.phases(str(db))
    rows = {line[:22].strip(): line.split() for line in out.splitlines()[2:8]}
    # dispatches and milliseconds per phase, two iterations
    assert rows["int"][-3:-1] == ["6", "0.020"]
    assert rows["filter"][-3:-1] == ["6", "0.006"]
    assert rows["com: sort"][-3:-1] == ["26", "0.005"]  # key + 4 x 3 per iteration
    assert rows["com: reduce by key"][-3:-1] == ["6", "0.002"]
    assert rows["copies and fills"][-3:-1] == ["4", "0.015"]
    assert rows["other"][-3:-1] == ["0", "0.000"]
    assert "interaction kernel alone (k_pp_int): 0.010 ms" in out


def test_trace_lists_the_last_dispatches_of_a_kernel(tmp_path):
    db = tmp_path / "t_results.db"
    kernels_db(str(db), [("inet_static_1024", 1000 * k) for k in range(1, 8)] + [("k_zero", 5)])
    con = sqlite3.connect(str(db))
    con.execute("create view top_kernels as select name, count(*) as total_calls,"
                " sum(duration) / 1000.0 as total_duration, avg(duration) / 1000.0 as average,"
                " 0.0 as percentage from kernels group by name")
    con.commit()
    con.close()
    out = rs.trace(str(db), "inet_static_1024", 3)
    lines = out.splitlines()
    assert "last 3 dispatches of inet_static_1024" in out
    assert [float(l.split()[0]) for l in lines[-3:]] == [5.0, 6.0, 7.0]
