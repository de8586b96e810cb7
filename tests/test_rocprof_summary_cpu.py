"""Host checks of the rocprofv3 summaries on small synthetic counter databases: the traffic
scaling by the copy kernel and the memory-interface view (request sizes, Little's law)."""
import os
import sqlite3
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2211_02435_amd import rocprof_summary as R  # noqa: E402

COPY = "lbm::copy_kernel(unsigned int __vector(4)*, unsigned int __vector(4) const*, unsigned long)"
SWEEP = "void lbm::sweep_kernel<2, 2, 0, true, float, float, 0, false, false>(lbm::SweepArgs<float, float>)"


def _db(path, rows):
    """rows: (kernel, dispatch, counter, value); the counters_collection view's columns."""
    con = sqlite3.connect(path)
    con.execute("create table pmc_info (name text)")
    con.execute("create table counters_collection (kernel_name text, dispatch_id int, counter_name text, value real)")
    for name in sorted({r[2] for r in rows}):
        con.execute("insert into pmc_info values (?)", (name,))
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    return path


def test_traffic_is_scaled_by_the_copy_kernel(tmp_path):
    gib4 = 4 * 2 ** 30
    # the copy moves 4 GiB each way; FETCH_SIZE reads half of it, WRITE_SIZE all of it (KiB)
    f = _db(str(tmp_path / "f.db"), [(COPY, 1, "FETCH_SIZE", gib4 / 2048), (SWEEP, 2, "FETCH_SIZE", 1000.0),
                                     (SWEEP, 3, "FETCH_SIZE", 1002.0), (SWEEP, 4, "FETCH_SIZE", 5000.0)])
    w = _db(str(tmp_path / "w.db"), [(COPY, 1, "WRITE_SIZE", gib4 / 1024), (SWEEP, 2, "WRITE_SIZE", 700.0)])
    t = R.traffic(f, w, "sweep_kernel", gib4, "x")
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["fetch_bytes_per_launch"] == pytest.approx(1002.0 * 1024 * 2)  # median of the dispatches
    assert t["bytes_per_launch"] == pytest.approx(1002.0 * 2048 + 700.0 * 1024)
    assert t["kernel_source_sha"] == R.kernel_source_hash()


def test_memory_view_applies_littles_law(tmp_path):
    gib4 = 4 * 2 ** 30
    cycles = 8 * 1.0e6           # GRBM_GUI_ACTIVE over 8 XCDs: 1e6 cycles each
    rd, wr = 2.0e6, 4.0e6        # requests
    vals = {"FETCH_SIZE": 256e6 / 2048, "WRITE_SIZE": 256e6 / 1024,
            "TCC_EA0_RDREQ_sum": rd, "TCC_EA0_RDREQ_LEVEL_sum": rd * 2500.0,
            "TCC_EA0_WRREQ_sum": wr, "TCC_EA0_WRREQ_LEVEL_sum": wr * 500.0,
            "TCC_EA0_WRREQ_64B_sum": wr, "TCC_EA0_WRREQ_STALL_sum": 0.01 * 1e6 * 128,
            "TCC_EA0_RDREQ_DRAM_CREDIT_STALL_sum": 0.0, "TCC_EA0_WRREQ_DRAM_CREDIT_STALL_sum": 0.0,
            "GRBM_GUI_ACTIVE": cycles}
    rows = [(SWEEP, 2, k, v) for k, v in vals.items()]
    rows += [(COPY, 1, "FETCH_SIZE", gib4 / 2048), (COPY, 1, "WRITE_SIZE", gib4 / 1024)]
    rows += [(COPY, 1, k, 1.0) for k in vals if k not in ("FETCH_SIZE", "WRITE_SIZE")]
    db = _db(str(tmp_path / "m.db"), rows)
    view = {r["kernel"]: r for r in R.memory_view([db], gib4)}
    s = view[SWEEP]
    assert s["fetch_GB"] == pytest.approx(0.256) and s["write_GB"] == pytest.approx(0.256)
    assert s["bytes_per_read_req"] == pytest.approx(128.0)
    assert s["bytes_per_write_req"] == pytest.approx(64.0)
    assert s["write_64B_fraction"] == pytest.approx(1.0)
    assert s["read_latency_cycles"] == pytest.approx(2500.0)
    assert s["write_latency_cycles"] == pytest.approx(500.0)
    # in flight = level / cycles per XCD: rd * 2500 / 1e6 = 5000 reads
    assert s["reads_in_flight"] == pytest.approx(5000.0)
    assert s["write_stall_fraction"] == pytest.approx(0.01)
    assert COPY in view


def test_memory_view_takes_given_scales_without_a_copy_kernel(tmp_path):
    vals = {"FETCH_SIZE": 1000.0, "WRITE_SIZE": 3000.0, "TCC_EA0_RDREQ_sum": 16.0, "TCC_EA0_RDREQ_LEVEL_sum": 1.0,
            "TCC_EA0_WRREQ_sum": 48.0, "TCC_EA0_WRREQ_LEVEL_sum": 1.0, "TCC_EA0_WRREQ_64B_sum": 48.0,
            "TCC_EA0_WRREQ_STALL_sum": 0.0, "TCC_EA0_RDREQ_DRAM_CREDIT_STALL_sum": 0.0,
            "TCC_EA0_WRREQ_DRAM_CREDIT_STALL_sum": 0.0, "GRBM_GUI_ACTIVE": 8.0}
    db = _db(str(tmp_path / "s.db"), [(SWEEP, 2, k, v) for k, v in vals.items()])
    with pytest.raises(SystemExit):
        R.memory_view([db], None)
    s = R.memory_view([db], None, scales=(2.0, 1.0))[0]
    assert s["fetch_GB"] == pytest.approx(1000.0 * 1024 * 2 / 1e9)
    assert s["write_GB"] == pytest.approx(3000.0 * 1024 / 1e9)
    assert s["bytes_per_read_req"] == pytest.approx(1000.0 * 1024 * 2 / 16)
