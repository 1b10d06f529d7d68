"""Host logic of the profile summaries in bench.py (no GPU).

The summaries read rocprofv3 result databases; here small stand-ins hold only
the tables and columns their queries read, filled with known values, and the
figures they produce (bytes per node, calibration factors, instructions per
node, dispatch statistics) are checked against the arithmetic done by hand.
"""
import os
import sqlite3
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

NODES = 512 ** 3
K16 = "void lbpf::step_kernel<1, 12, lbpf::StF16, false, false, false, 1>(lbpf::SimDev, lbpf::TileDev)"
K64 = "void lbpf::step_kernel<1, 4, lbpf::StF64, false, false, false, 1>(lbpf::SimDev, lbpf::TileDev)"
KCOPY = "void at::native::vectorized_elementwise_kernel<4, copy>(int)"


def _pmc_db(d, rows):
    """rows: (kernel name, dispatch id, counter, value); several rows of one
    dispatch and counter stand for the per-instance values of that counter."""
    os.makedirs(d, exist_ok=True)
    con = sqlite3.connect(os.path.join(d, "run_results.db"))
    con.execute("CREATE TABLE pmc_events (name TEXT, dispatch_id INTEGER, counter_name TEXT, counter_value REAL)")
    con.executemany("INSERT INTO pmc_events VALUES (?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    return d


def test_pmc_sums_instances_and_averages_dispatches(tmp_path):
    d = _pmc_db(str(tmp_path / "p"), [
        (K16, 1, "FETCH_SIZE", 100.0), (K16, 1, "FETCH_SIZE", 50.0),  # one dispatch: 150
        (K16, 2, "FETCH_SIZE", 200.0), (K16, 2, "FETCH_SIZE", 50.0),  # another: 250
    ])
    v = bench._pmc(d)
    assert list(v) == ["step_kernel<1, 12, StF16, false, false, false, 1>"]
    assert v[bench._short(K16)]["FETCH_SIZE"] == pytest.approx(200.0)


def test_traffic_scaled_by_the_copy_calibration(tmp_path):
    copy_bytes = 1 << 30
    # the copy reads FETCH_SIZE = half its bytes in KiB and WRITE_SIZE = its bytes in KiB
    cf = _pmc_db(str(tmp_path / "cf"), [(KCOPY, 1, "FETCH_SIZE", copy_bytes / 2048)])
    cw = _pmc_db(str(tmp_path / "cw"), [(KCOPY, 1, "WRITE_SIZE", copy_bytes / 1024)])
    fe = _pmc_db(str(tmp_path / "fe"), [(K16, 1, "FETCH_SIZE", 1000.0), (K64, 2, "FETCH_SIZE", 4000.0)])
    wr = _pmc_db(str(tmp_path / "wr"), [(K16, 1, "WRITE_SIZE", 500.0), (K64, 2, "WRITE_SIZE", 3000.0)])
    res, md = bench.summarize_traffic(fe, wr, cf, cw, copy_bytes, "cmd")
    assert res["factor_fetch"] == pytest.approx(2048.0) and res["factor_write"] == pytest.approx(1024.0)
    k16 = res["kernels"][bench.traffic_key("D3Q19_D3Q7", "fp16")]
    assert k16["read_bytes"] == pytest.approx(1000.0 * 2048) and k16["write_bytes"] == pytest.approx(500.0 * 1024)
    assert k16["bytes_per_node"] == pytest.approx((1000.0 * 2048 + 500.0 * 1024) / NODES)
    k64 = res["kernels"][bench.traffic_key("D3Q19_D3Q7", "fp64")]
    assert k64["bytes_per_launch"] == pytest.approx(4000.0 * 2048 + 3000.0 * 1024)
    assert res["kernel_sha"] == bench.kernel_sha() and k16["kernel_sha"] == res["kernel_sha"]
    assert "cmd" in md and res["kernel_sha"] in md


def test_instruction_mix_per_node(tmp_path):
    waves = 65536.0
    p1 = {"SQ_WAVES": waves, "SQ_INSTS_VALU": 800.0 * NODES / 64, "SQ_INSTS_LDS": 96.0 * NODES / 64,
          "SQ_INSTS_VMEM_RD": 50.0 * NODES / 64, "SQ_INSTS_VMEM_WR": 28.0 * NODES / 64,
          "SQ_INSTS_SALU": 380.0 * NODES / 64, "SQ_WAVE_CYCLES": 1000.0 * waves, "SQ_BUSY_CYCLES": 1.0}
    p2 = {"SQ_WAIT_INST_ANY": 1.0, "SQ_ACTIVE_INST_VALU": 200.0 * waves, "SQ_ACTIVE_INST_LDS": 20.0 * waves,
          "SQ_LDS_BANK_CONFLICT": 0.5 * 96.0 * NODES / 64, "SQ_WAIT_ANY": 420.0 * waves,
          "SQ_ACTIVE_INST_ANY": 1.0, "SQ_INSTS_SMEM": 1.0, "SQ_ACTIVE_INST_SCA": 90.0 * waves}
    d1 = _pmc_db(str(tmp_path / "s1"), [(K16, 1, c, v) for c, v in p1.items()])
    d2 = _pmc_db(str(tmp_path / "s2"), [(K16, 1, c, v) for c, v in p2.items()])
    md = bench.summarize_sq(d1, d2, "cmd")
    row = next(line for line in md.splitlines() if line.startswith("| `step_kernel<1, 12"))
    cells = [c.strip() for c in row.strip("|").split("|")]
    # kernel | waves | VALU | SALU | LDS | VMEM rd | VMEM wr | VALU act | SALU act | LDS act | waiting | conflicts
    assert cells[1:7] == ["65536", "800", "380", "96", "50.0", "28.0"]
    assert cells[7:12] == ["0.20", "0.09", "0.02", "0.42", "0.500"]


def test_counter_table_per_node(tmp_path):
    d = _pmc_db(str(tmp_path / "c"), [(K64, 1, "TCC_EA0_RDREQ_128B_sum", 2.5 * NODES),
                                      (K64, 2, "TCC_EA0_RDREQ_128B_sum", 3.5 * NODES),
                                      (KCOPY, 3, "TCC_EA0_RDREQ_128B_sum", 7.0)])
    md = bench.summarize_counters([d], "cmd", "title")
    assert "| `step_kernel<1, 4, StF64, false, false, false, 1>` |" in md
    assert "/ 3.000 |" in md  # mean of 2.5 and 3.5 per node
    assert "vectorized" not in md  # only the step kernels of the 3D workload


def test_trace_statistics(tmp_path):
    d = str(tmp_path / "t")
    os.makedirs(d)
    con = sqlite3.connect(os.path.join(d, "bench_results.db"))
    con.execute("CREATE TABLE rocpd_info_kernel_symbol (id INTEGER, guid TEXT, display_name TEXT)")
    con.execute("CREATE TABLE rocpd_kernel_dispatch (kernel_id INTEGER, guid TEXT, start INTEGER, end INTEGER)")
    con.executemany("INSERT INTO rocpd_info_kernel_symbol VALUES (?, ?, ?)", [(1, "g", K16), (2, "g", KCOPY)])
    con.executemany("INSERT INTO rocpd_kernel_dispatch VALUES (?, ?, ?, ?)",
                    [(1, "g", 0, 5_000_000), (1, "g", 10_000_000, 16_000_000), (2, "g", 0, 1_000_000)])
    con.commit()
    con.close()
    md = bench.summarize_trace(d, "cmd")
    row = next(line for line in md.splitlines() if "step_kernel" in line and line.startswith("| `"))
    cells = [c.strip() for c in row.strip("|").split("|")]
    assert cells[1:] == ["2", "5.5000", "5.0000", "6.0000", "11.000"]
