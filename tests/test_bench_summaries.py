"""The benchmark's profile summarisers on small synthetic rocprofv3-style
databases (no GPU): the busy fraction of a kernel trace is the union of the
kernel intervals, overlaps counted once, per window and overall; the last
call of a batched launch is the last group of overlapping dispatches; the
byte counters are scaled by what they read for a plain copy of known size
(the arithmetic behind the headline's traffic figure)."""
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


def _counter_db(tmp_path, name, rows):
    db = str(tmp_path / name)
    con = sqlite3.connect(db)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, grid_size integer, "
                "value real)")
    con.executemany("insert into counters_collection values (?,?,?,?)",
                    [(i, nm, g, v) for i, (nm, g, v) in enumerate(rows)])
    con.commit()
    con.close()
    return db


def test_counters_are_scaled_by_the_calibration_copy(tmp_path):
    """A copy of 512 MiB that FETCH_SIZE reads as half its bytes (one read per
    64 B line counted as 32 B, say) and WRITE_SIZE as all of them: FETCH is
    scaled by 2, WRITE by 1; a kernel's scaled bytes per dispatch are the
    means of its dispatches, scaled; with last_of only the last dispatch of a
    matching kernel counts."""
    mib = 512
    fetch = [("__amd_rocclr_copyBuffer", 0, mib * 1024 / 2), ("kern_a", 0, 100.0), ("kern_a", 0, 300.0),
             ("kern_b", 0, 50.0), ("__amd_rocclr_copyBuffer", 0, 1.0)]
    write = [("__amd_rocclr_copyBuffer", 0, mib * 1024), ("kern_a", 0, 10.0), ("kern_a", 0, 30.0),
             ("kern_b", 0, 5.0), ("__amd_rocclr_copyBuffer", 0, 2.0)]
    fdb, wdb = _counter_db(tmp_path, "f.db", fetch), _counter_db(tmp_path, "w.db", write)
    out = bench.counters_table(fdb, wdb, mib)
    # kern_a: mean fetch 200 KiB x 2 + mean write 20 KiB x 1 = 420 KiB = 0.430 MB
    assert "| `kern_a` | 2 | 200.0 | 20.0 | 0.430 |" in out
    assert "| `kern_b` | 1 | 50.0 | 5.0 | 0.108 |" in out
    assert "scale factors 2.0000 and 1.0000" in out
    # only the last dispatch of kern_a: 300 x 2 + 30 = 630 KiB
    out = bench.counters_table(fdb, wdb, mib, last_of="kern_a")
    assert "| `kern_a` | 1 | 300.0 | 30.0 | 0.645 |" in out


def test_counters_need_the_calibration_copy(tmp_path):
    rows = [("kern_a", 0, 1.0)]
    with pytest.raises(SystemExit):
        bench.counters_table(_counter_db(tmp_path, "f.db", rows), _counter_db(tmp_path, "w.db", rows), 512)


def test_evd_traffic_record(tmp_path):
    """The EVD kernels' bytes per launch: the last dispatch of each kernel,
    each counter scaled by the first copy; the record names the sources it
    was taken for."""
    r = 1 << 26
    real, cplx = bench.evd_kernel_name(r, False), bench.evd_kernel_name(r, True)
    fetch = [("__amd_rocclr_copyBuffer", 0, 262144.0), (real, 0, 1.0), (real, 0, 1000.0), (cplx, 0, 2000.0)]
    write = [("__amd_rocclr_copyBuffer", 0, 524288.0), (real, 0, 1.0), (real, 0, 3000.0), (cplx, 0, 4000.0)]
    rec, md = bench.traffic_from(_counter_db(tmp_path, "f.db", fetch), _counter_db(tmp_path, "w.db", write), 512, r)
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["real"]["bytes"] == (1000.0 * 2 + 3000.0) * 1024
    assert rec["complex"]["bytes"] == (2000.0 * 2 + 4000.0) * 1024
    assert len(rec["kernel_sources_sha256"]) == 64
    assert real in md and cplx in md
