"""Host logic of the benchmark's counter summaries: HBM traffic from the
FETCH_SIZE / WRITE_SIZE runs (scaled by the calibration copy) and the
rasteriser's VALU / LDS use, on small synthetic counter files in rocprofv3's
CSV layout, plus the argument check for more than one GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (disp, name, counter, value, t0, t1) in enumerate(rows):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": disp, "Agent_Id": "Agent 1", "Queue_Id": 1,
                        "Process_Id": 1, "Thread_Id": 1, "Grid_Size": 1, "Kernel_Id": 1, "Kernel_Name": name,
                        "Workgroup_Size": 256, "LDS_Block_Size": 0, "Scratch_Size": 0, "VGPR_Count": 8,
                        "Accum_VGPR_Count": 0, "SGPR_Count": 8, "Counter_Name": counter, "Counter_Value": value,
                        "Start_Timestamp": t0, "End_Timestamp": t1})


RASTER = "void gsr::(anonymous namespace)::k_raster<16, 64, false>(gsr::SceneDev, gsr::ChunkDev, gsr::RasterParams)"


def test_traffic_summary_scales_by_the_calibration_copy(tmp_path):
    kib = bench.CALIB_BYTES / 1024.0
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    # the copy reads 1 GiB but FETCH_SIZE shows half of it (factor 2); WRITE_SIZE shows all of it
    level2 = "gsr::(anonymous namespace)::k_rowtile_rank(gsr::ChunkDev, int, int, unsigned int const*, int)"
    _write_counters(fetch, [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", kib / 2, 0, 10),
                            (2, RASTER, "FETCH_SIZE", 1000.0, 10, 20), (3, RASTER, "FETCH_SIZE", 3000.0, 20, 30),
                            (4, level2, "FETCH_SIZE", 100.0, 30, 40)])
    _write_counters(write, [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", kib, 0, 10),
                            (2, RASTER, "WRITE_SIZE", 500.0, 10, 20), (3, RASTER, "WRITE_SIZE", 700.0, 20, 30),
                            (4, level2, "WRITE_SIZE", 50.0, 30, 40)])
    out = tmp_path / "pmc.json"
    bench.pmc_summary(str(fetch), str(write), str(out), "cmd")
    s = json.loads(out.read_text())
    assert s["fetch_dispatches"] == 2 and s["write_dispatches"] == 2
    assert s["fetch_factor"] == pytest.approx(2.0)
    assert s["write_factor"] == pytest.approx(1.0)
    assert s["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2)
    assert s["write_bytes_per_launch"] == pytest.approx(600.0 * 1024)
    assert s["traffic_bytes_per_launch"] == pytest.approx(2000.0 * 2048 + 600.0 * 1024)
    assert s["source_sha256"] == bench.raster_source_hash()
    # every kernel's calibrated bytes per dispatch, the copy excluded
    assert set(s["kernels"]) == {"k_raster<16, 64, false>", "k_rowtile_rank"}
    assert s["kernels"]["k_rowtile_rank"]["fetch_bytes_per_dispatch"] == pytest.approx(100.0 * 2048)
    assert s["kernels"]["k_rowtile_rank"]["write_bytes_per_dispatch"] == pytest.approx(50.0 * 1024)
    assert s["kernels"]["k_raster<16, 64, false>"]["dispatches"] == 2


def test_traffic_summary_rejects_a_bad_calibration(tmp_path):
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    _write_counters(fetch, [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 10.0, 0, 10),
                            (2, RASTER, "FETCH_SIZE", 1000.0, 10, 20)])
    _write_counters(write, [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 10.0, 0, 10),
                            (2, RASTER, "WRITE_SIZE", 500.0, 10, 20)])
    with pytest.raises(SystemExit):
        bench.pmc_summary(str(fetch), str(write), str(tmp_path / "pmc.json"), "cmd")


def test_valu_lds_summary(tmp_path):
    agent = tmp_path / "agent.csv"
    with open(agent, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Agent_Type", "Num_Xcc", "Cu_Count", "Simd_Per_Cu", "Max_Engine_Clk_Fcompute"])
        w.writerow(["CPU", 1, 16, 0, 5000])
        w.writerow(["GPU", 8, 256, 4, 2400])
    counters = tmp_path / "util.csv"
    ns = 10_000_000                       # a 10 ms launch
    clocks = 2.0 * ns                     # at 2 GHz
    rows = [(5, RASTER, "GRBM_GUI_ACTIVE", clocks * 8, 0, ns),            # summed over 8 XCDs
            (5, RASTER, "SQ_ACTIVE_INST_VALU", 0.75 * 1024 * clocks / 4, 0, ns),   # quad-cycles, 75 % busy
            (5, RASTER, "SQ_BUSY_CU_CYCLES", 1024 * clocks / 4, 0, ns),
            (5, RASTER, "SQ_LDS_IDX_ACTIVE", 0.5 * 256 * clocks, 0, ns),
            (5, RASTER, "SQ_INSTS_LDS_LOAD_BANDWIDTH", 1e12 / 64, 0, ns),  # 1 TB read
            (5, RASTER, "SQ_INSTS_VALU", 0.9 * 1024 * clocks / 4, 0, ns),  # wave64 instructions: 90 % of issue
            (6, "k_project<0, 3>", "GRBM_GUI_ACTIVE", 1.0, 0, 1)]
    # a 1 ms launch of another kernel at half the VALU issue rate
    ns2, clocks2 = 1_000_000, 2.0 * 1_000_000
    rows += [(7, "k_rowtile_rank", "GRBM_GUI_ACTIVE", clocks2 * 8, ns, ns + ns2),
             (7, "k_rowtile_rank", "SQ_ACTIVE_INST_VALU", 0.5 * 1024 * clocks2 / 4, ns, ns + ns2),
             (7, "k_rowtile_rank", "SQ_BUSY_CU_CYCLES", 1024 * clocks2 / 4, ns, ns + ns2),
             (7, "k_rowtile_rank", "SQ_LDS_IDX_ACTIVE", 0.25 * 256 * clocks2, ns, ns + ns2),
             (7, "k_rowtile_rank", "SQ_INSTS_LDS_LOAD_BANDWIDTH", 1e9 / 64, ns, ns + ns2),
             (7, "k_rowtile_rank", "SQ_INSTS_VALU", 0.5 * 1024 * clocks2 / 4, ns, ns + ns2)]
    _write_counters(counters, rows)
    out = tmp_path / "util.json"
    bench.util_summary(str(counters), str(agent), str(out), "cmd")
    s = json.loads(out.read_text())
    assert s["dispatches"] == 1
    assert s["clock_ghz"] == pytest.approx(2.0)
    assert s["valu_busy"] == pytest.approx(0.75)
    assert s["cu_busy"] == pytest.approx(1.0)
    assert s["lds_busy"] == pytest.approx(0.5)
    assert s["lds_read_gbs"] == pytest.approx(1e12 / 0.01 / 1e9)
    assert s["lds_peak_gbs"] == pytest.approx(256 * 256 * 2.4)
    assert s["lds_read_frac"] == pytest.approx(s["lds_read_gbs"] / s["lds_peak_gbs"])
    assert s["valu_issue_frac"] == pytest.approx(0.9)
    assert s["valu_instr_per_launch"] == pytest.approx(0.9 * 1024 * clocks / 4)
    # per-kernel figures: complete launches only (the project row lacks counters)
    assert set(s["kernels"]) == {"k_raster<16, 64, false>", "k_rowtile_rank"}
    k = s["kernels"]["k_rowtile_rank"]
    assert k["dispatches"] == 1 and k["avg_ms"] == pytest.approx(1.0)
    assert k["valu_issue_frac"] == pytest.approx(0.5)
    assert k["lds_busy"] == pytest.approx(0.25)
    assert s["kernels"]["k_raster<16, 64, false>"]["valu_issue_frac"] == pytest.approx(0.9)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout
