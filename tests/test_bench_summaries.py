"""The benchmark's profile summarisers on small synthetic rocprofv3-style
databases (no GPU): the busy fraction of a kernel trace is the union of the
kernel intervals, overlaps counted once, per window and overall; the last
call of a batched launch is the last group of overlapping dispatches."""
import os
import sqlite3
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

S = 10 ** 9


def _db(tmp_path, rows, extra_cols=False):
    db = str(tmp_path / "trace.db")
    con = sqlite3.connect(db)
    if extra_cols:
        con.execute("create table kernels (name text, start integer, end integer, grid_x integer, "
                    "workgroup_x integer, vgpr_count integer, accum_vgpr_count integer, lds_size integer)")
        con.executemany("insert into kernels values (?,?,?,?,?,?,?,?)", rows)
    else:
        con.execute("create table kernels (name text, start integer, end integer)")
        con.executemany("insert into kernels values (?,?,?)", rows)
    con.commit()
    con.close()
    return db


def test_union_counts_overlaps_once():
    spans = [(0, 4), (1, 2), (3, 6), (8, 9)]
    assert bench._union_ns(spans, 0, 10) == 7
    assert bench._union_ns(spans, 2, 5) == 3
    assert bench._union_ns(spans, 6, 8) == 0
    assert bench._union_ns([], 0, 10) == 0


def test_busy_table(tmp_path):
    rows = [("void jsvd::gpair_kernel<true>(x)", 0, 2 * S), ("void jsvd::batched_kernel<1>(y)", 1 * S, 3 * S),
            ("jsvd::fold_kernel(z)", 6 * S, 7 * S), ("void jsvd::gpair_kernel<false>(x)", 8 * S, 10 * S)]
    out = bench.busy_table(_db(tmp_path, rows))
    assert "device busy 0.600" in out
    assert "| 0.0–5.0 | 0.600 |" in out and "| 5.0–10.0 | 0.600 |" in out
    # families: template arguments dropped, summed over dispatches
    assert "| `jsvd::gpair_kernel` | 4.00 |" in out
    assert out.index("gpair_kernel` |") < out.index("batched_kernel` |") < out.index("fold_kernel` |")


def test_busy_table_empty(tmp_path):
    with pytest.raises(SystemExit):
        bench.busy_table(_db(tmp_path, []))


def test_last_call_is_the_last_overlapping_group(tmp_path):
    # two tuner launches one after another, then a call of three concurrent classes
    rows = [("batched_kernel<1>", 0, 10, 256, 64, 40, 0, 100),
            ("batched_kernel<2>", 20, 30, 256, 64, 40, 0, 100),
            ("batched_kernel<1>", 40, 100, 512, 64, 40, 0, 100),
            ("batched_kernel<2>", 45, 90, 512, 128, 60, 0, 200),
            ("batched_kernel<4>", 50, 120, 256, 256, 80, 0, 400),
            ("other_kernel", 60, 70, 1, 1, 1, 0, 0)]
    out = bench.last_call_table(_db(tmp_path, rows, extra_cols=True), "batched_kernel")
    assert out.startswith("Last call: 3 dispatches")
    assert "span 0.1 us" in out   # 40 .. 120 ns
    assert out.count("| `batched_kernel<") == 3
