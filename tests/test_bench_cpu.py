"""Host logic of the benchmark and the profile summaries (no GPU)."""

import csv
import json
import os
import subprocess
import sys

import pytest

from paper_2306_08514_amd import rocprof_summary as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in rec["error"] and rec["n_gpus_requested"] == 2


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, disp, val in rows:
            w.writerow({"Kernel_Name": name, "Dispatch_Id": disp, "Counter_Name": counter, "Counter_Value": val})


def test_clock_is_the_xcd_mean_cycle_count_over_the_dispatch_span(tmp_path):
    """GRBM_GUI_ACTIVE is summed over the 8 XCDs (per-instance records of one
    dispatch add up); divided by 8 and by the dispatch's span it gives the
    clock: 8 x 2.4e6 cycles over 1 ms is 2.4 GHz."""
    d = tmp_path / "clk"
    os.makedirs(d)
    fd = "_ZN3srp12_GLOBAL__N_19gemm_fd16IDF16bEEvPKT_lS4_lPfliiifiil"
    with open(d / "pmc_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value",
                                          "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for disp, t0, cyc in ((1, 0, 4 * 2.4e6), (1, 0, 4 * 2.4e6), (2, 5_000_000, 8 * 1.8e6)):
            w.writerow({"Kernel_Name": fd, "Dispatch_Id": disp, "Counter_Name": "GRBM_GUI_ACTIVE",
                        "Counter_Value": cyc, "Start_Timestamp": t0, "End_Timestamp": t0 + 1_000_000})
    c = rs.clocks(str(d))[fd]
    assert sorted(round(g, 6) for _, g in c) == [1.8, 2.4]
    assert rs._dtype(fd) == "bf16"
    assert rs._dtype("void srp::(anonymous namespace)::gemm_fd16<float>(float const*, long)") == "f32"
    assert rs._dtype("void srp::gemm_fd16<srp::fp8>(srp::fp8 const*)") == "fp8"
    md = rs._md_clock(str(d), "t", "cmd")
    assert "| gemm_fd (bf16) | 2 | 1.000 | 2.10 | 1.80 | 2.40 |" in md


def test_traffic_is_calibrated_by_the_copy_and_summed_over_instances(tmp_path):
    """A 1 GiB copy that reads 2^19 FETCH units and writes 2^20 WRITE units
    fixes 2048 B and 1024 B per unit; a kernel's per-dispatch value is the
    sum of its per-instance records, and the median over dispatches is kept."""
    copy = "__amd_rocclr_copyBuffer"
    fd = "void srp::gemm_nt<float, 128, 128, 2, 256, false>(srp::GemmBatch const*)"
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE",
                    [(copy, 1, 2 ** 19), (copy, 2, 2 ** 19), (fd, 3, 600.0), (fd, 3, 400.0), (fd, 4, 1000.0)])
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE",
                    [(copy, 1, 2 ** 20), (copy, 2, 2 ** 20), (fd, 3, 100.0), (fd, 4, 100.0)])
    rec = rs.traffic(str(tmp_path / "f"), str(tmp_path / "w"))
    assert rec["calibration"]["fetch_bytes_per_unit"] == 2048.0
    assert rec["calibration"]["write_bytes_per_unit"] == 1024.0
    k = rec["kernels"]["gemm_fd"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes"] == 1000.0 * 2048 and k["write_bytes"] == 100.0 * 1024
    assert k["bytes_per_launch"] == 1000.0 * 2048 + 100.0 * 1024
    assert rec["source_sha256"] == rs.source_sha256()


def test_kernel_tags():
    assert rs.tag("void srp::gemm_nt<float, 128, 128, 2, 256, false>(x)") == "gemm_fd"
    assert rs.tag("void srp::gemm_nt<float, 256, 128, 2, 128, false>(x)") == "gemm_tall"
    assert rs.tag("void srp::gemm_nt<__bf16, 256, 256, 2, 128, false>(x)") == "gemm_fd"
    assert rs.tag("void srp::gemm_nt<__bf16, 128, 128, 2, 256, false>(x)") == "gemm_tall"
    assert rs.tag("_ZN3srp7gemm_ntIDF16bLi256ELi256ELi2ELi128ELb0EEEvPKNS_9GemmBatchE") == "gemm_fd"
    assert rs.tag("_ZN3srp7gemm_ntIDF16bLi128ELi128ELi2ELi256ELb0EEEvPKNS_9GemmBatchE") == "gemm_tall"
    assert rs.tag("_ZN3srp7tall_wsIDF16bLi16ELi8ELb0EEEvPKT_liS3_lPflilfiiiPKiS6_") == "gemm_tall"
    assert rs.tag("void srp::tall_ws<__bf16, 16, 8, false>(__bf16 const*, long)") == "gemm_tall"
    # the tall kernel reading a per-tile chunk table: dense-window SSPI
    assert rs.tag("_ZN3srp7tall_wsIDF16bLi32ELi8ELb1EEEvPKT_liS3_lPflilfiiiPKiS6_") == "sspi_dense"
    assert rs.tag("void srp::tall_ws<__bf16, 32, 8, true>(__bf16 const*, long)") == "sspi_dense"
    assert rs.tag("void srp::xi_to_frames<__bf16>(float const*, long)") == "xi_to_frames"
    assert rs.tag("void srp::sspi_gather<__bf16, 4, 32, true>(x)") == "sspi_gather"
    assert rs.tag("void srp::gcc_direct<1>(HIP_vector_type<float, 2u> const*, int)") == "gcc_direct"
    assert rs.tag("_ZN3srp13slri_fat_mfmaIDF16bEEvPKfliPKiS4_S2_iiS2_iPT_i") == "slri_fat"
    assert rs.tag("_ZN3srp20slri_fat_global_mfmaIDF16bEEvPKfliiS2_iS2_PT_") == "slri_fat_global"
    assert rs.tag("_ZN3srp9sspi_bandILi2ELi128EEEvPKDF16_liPKiPKjPKNS_8BandDescEPKtS4_iliiPfl") == "sspi_band"
    assert rs.tag("_ZN3srp17sspi_band_recordsIDF16bEEvPKiPKT_iiliiS2_PiPj") == "sspi_band_records (plan)"
    assert rs.tag("_ZN3srp11rows_to_f16EPKfliiiPDF16_l") == "xi_to_frames"
    assert rs.tag("void srp::lam_gemm_f64<true>(double const*, long)") == "lam_gemm_f64 (plan)"
    assert rs.tag("srp::split_reduce(float const*, int, long)") == "split_reduce"
    assert rs.tag("_ZN3srp12_GLOBAL__N_19gemm_fd16IDF16bEEvPKT_lS4_lPfliiifiil") == "gemm_fd"
    assert rs.tag("_ZN3srp8fd_gen16IDF16bLi256EEEvPKT_lPKdliiPfliifiiil") == "gemm_fd_gen"
    assert rs.tag("void srp::gcc_direct<1, true>(HIP_vector_type<float, 2u> const*, int)") == "gcc_direct"
    tags = rs.unique_tags(["void srp::sspi_gather<__bf16, 3, 32, true>(float const*)",
                           "void srp::sspi_gather<__bf16, 5, 32, true>(float const*)", "srp::gcc_direct<1>(x)"])
    assert tags["srp::gcc_direct<1>(x)"] == "gcc_direct"
    assert tags["void srp::sspi_gather<__bf16, 3, 32, true>(float const*)"] == "sspi_gather <__bf16, 3, 32, true>"


def test_traffic_record_round_trips_through_the_summary(tmp_path):
    md = tmp_path / "t.md"
    md.write_text("# x\n\n```json\n" + json.dumps({"source_sha256": "abc", "kernels": {}}) + "\n```\n")
    assert rs.read_traffic_record(str(md)) == {"source_sha256": "abc", "kernels": {}}
    assert rs.read_traffic_record(str(tmp_path / "missing.md")) is None
