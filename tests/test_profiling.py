"""The rocprofv3 summaries bench.py and profiles/ rely on, checked on small
synthetic result databases (no GPU)."""

import sqlite3

from paper_2001_11220_amd import profiling as PR


def _db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_scales_kernel_counters_by_the_calibration_copy(tmp_path):
    gib = 1 << 30
    k = "void etd::k_mid_s<8, 2, 32, 2, true, double>(double const*, double*)"
    # the copy of 1 GiB reads half its bytes on FETCH_SIZE and all on WRITE_SIZE
    _db(tmp_path / "f.db", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", gib / 2048),
                            (k, "FETCH_SIZE", 100.0), (k, "FETCH_SIZE", 110.0), (k, "FETCH_SIZE", 90.0),
                            ("at::native::other", "FETCH_SIZE", 5.0)])
    _db(tmp_path / "w.db", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", gib / 1024),
                            (k, "WRITE_SIZE", 50.0)])
    r = PR.traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"), gib)
    assert abs(r["fetch_scale"] - 2.0) < 1e-12 and abs(r["write_scale"] - 1.0) < 1e-12
    rec = r["kernels"]["k_mid_s<8, 2, 32, 2, true, double>"]
    assert rec["fetch_bytes"] == 100.0 * 1024 * 2  # median of the dispatches
    assert rec["write_bytes"] == 50.0 * 1024
    assert rec["bytes_per_launch"] == rec["fetch_bytes"] + rec["write_bytes"]
    assert list(r["kernels"]) == ["k_mid_s<8, 2, 32, 2, true, double>"]  # only the library's kernels


def test_kernel_times_and_names(tmp_path):
    con = sqlite3.connect(tmp_path / "k.db")
    con.execute("create table kernels (name text, start integer, end integer)")
    con.executemany("insert into kernels values (?, ?, ?)",
                    [("void etd::k_first_s<8, 2, 32, 2, true, false, double>(double const*)", 0, 250000),
                     ("void etd::k_first_s<8, 2, 32, 2, true, false, double>(double const*)", 0, 260000)])
    con.commit()
    con.close()
    t = PR.kernel_times(str(tmp_path / "k.db"))
    (name, v), = t.items()
    assert PR.short_name(name) == "k_first_s<8, 2, 32, 2, true, false, double>"
    assert v == [250.0, 260.0]
    assert len(PR.kernel_rev()) == 12
