"""Host-side checks of bench.py that need no GPU: the one-GPU rule, the
algorithmic byte count behind the roofline line, and the rocprofv3 summary
(calibrated traffic) on a small synthetic set of profiler CSV files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_algorithmic_bytes():
    # 2D fp32: per point 2 coordinates + permutation + complex strength = 20 B, grid 8 B per cell
    assert bench.algorithmic_bytes("spread", 2, 10_000_000, 2048 * 2048, 4) == \
        10_000_000 * 20 + 2048 * 2048 * 8
    # 3D fp64: 3 x 8 + 4 + 16 = 44 B per point, 16 B per cell
    assert bench.algorithmic_bytes("interp", 3, 1000, 64 ** 3, 8) == 1000 * 44 + 64 ** 3 * 16


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_profiles_calibrates_traffic(tmp_path):
    d = str(tmp_path)
    spread = "void mn::detail::k_spread_smp<float, 2, 6, false>(mn::Geom, int const*)"
    interp = "void mn::detail::k_interp_sm<float, 2, 6, false>(mn::Geom, int const*)"
    _write(f"{d}/stats/run_kernel_stats.csv", ["Name", "Calls", "AverageNs", "Percentage"],
           [[spread, 2, 250000, 40.0], [interp, 2, 240000, 38.0]])
    cc = ["Kernel_Name", "Counter_Value"]
    _write(f"{d}/fetch/run_counter_collection.csv", cc, [[spread, 600000], [spread, 600000],
                                                          [interp, 100000]])
    _write(f"{d}/write/run_counter_collection.csv", cc, [[spread, 40000], [interp, 300000]])
    # a 256 MiB copy reads half its bytes on FETCH_SIZE and all on WRITE_SIZE
    _write(f"{d}/cf/run_counter_collection.csv", cc, [["__amd_rocclr_copyBuffer", 131072]])
    _write(f"{d}/cw/run_counter_collection.csv", cc, [["__amd_rocclr_copyBuffer", 262144]])
    traffic = f"{d}/traffic.json"
    md = f"{d}/summary.md"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-profiles",
                        "--stats-dir", f"{d}/stats", "--fetch-dir", f"{d}/fetch",
                        "--write-dir", f"{d}/write", "--cal-fetch-dir", f"{d}/cf",
                        "--cal-write-dir", f"{d}/cw", "--workload", "2d", "--md-out", md,
                        "--traffic-out", traffic], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    t = json.load(open(traffic))
    e = t["2d:k_spread_smp"]
    assert e["cal_fetch"] == pytest.approx(2.0) and e["cal_write"] == pytest.approx(1.0)
    assert e["bytes_per_launch"] == pytest.approx((600000 * 2.0 + 40000) * 1024)
    assert e["source_hash"] == bench.kernel_source_hash()
    assert t["2d:k_interp_sm"]["bytes_per_launch"] == pytest.approx((100000 * 2.0 + 300000) * 1024)
    text = open(md).read()
    assert "k_spread_smp<float, 2, 6, false>" in text and "250.0" in text


def test_summarize_profiles_sq_fractions(tmp_path):
    """SQ counters -> utilisation fractions: cycles are one XCD's
    GRBM_GUI_ACTIVE (the CSV sums eight), fractions are per CU and cycle."""
    d = str(tmp_path)
    spread = "void mn::detail::k_spread_smp<float, 3, 6, false>(mn::Geom, int const*)"
    _write(f"{d}/stats/run_kernel_stats.csv", ["Name", "Calls", "AverageNs", "Percentage"],
           [[spread, 1, 1000000, 50.0]])
    cyc = 2_400_000  # 1 ms at 2.4 GHz on each XCD
    rows = [[spread, "GRBM_GUI_ACTIVE", 8 * cyc],
            [spread, "SQ_ACTIVE_INST_VALU", 0.5 * 256 * cyc],
            [spread, "SQ_INSTS_VALU", 0.25 * 256 * cyc],
            [spread, "SQ_LDS_IDX_ACTIVE", 0.75 * 256 * cyc],
            [spread, "SQ_LDS_BANK_CONFLICT", 0.25 * 256 * cyc],
            [spread, "SQ_WAVE_CYCLES", 16 * 256 * cyc / 4]]
    _write(f"{d}/sq/run_counter_collection.csv", ["Kernel_Name", "Counter_Name", "Counter_Value"],
           rows)
    out = f"{d}/counters.json"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-profiles",
                        "--stats-dir", f"{d}/stats", "--sq-dir", f"{d}/sq", "--workload", "3d",
                        "--md-out", f"{d}/s.md", "--counters-out", out],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    e = json.load(open(out))["3d:k_spread_smp"]
    assert e["valu_busy"] == pytest.approx(0.5) and e["lds_util"] == pytest.approx(0.75)
    assert e["lds_bank_conflict"] == pytest.approx(0.25)
    assert e["valu_insts_per_cu_cycle"] == pytest.approx(0.25)
    assert e["occupancy"] == pytest.approx(0.5)
    assert e["source_hash"] == bench.kernel_source_hash()
    assert "| `k_spread_smp` | 0.50 | 0.25 | 0.75 | 0.25 | 0.50 |" in open(f"{d}/s.md").read()


def test_summarize_profiles_rows_per_instantiation(tmp_path):
    """Two instantiations of one kernel (the add-back's two passes) get a row
    each, with their own counters, not one row averaging both."""
    d = str(tmp_path)
    light = "void mn::detail::k_tile_sum<float, 3, false>(mn::Geom, int const*)"
    heavy = "void mn::detail::k_tile_sum<float, 3, true>(mn::Geom, int const*)"
    spread = "void mn::detail::k_spread_smp<float, 3, 6, false>(mn::Geom, int const*)"
    _write(f"{d}/stats/run_kernel_stats.csv", ["Name", "Calls", "AverageNs", "Percentage"],
           [[spread, 1, 1000000, 80.0], [light, 1, 180000, 15.0], [heavy, 1, 4000, 1.0]])
    cc = ["Kernel_Name", "Counter_Value"]
    _write(f"{d}/fetch/run_counter_collection.csv", cc,
           [[spread, 500000], [light, 280000], [heavy, 20]])
    _write(f"{d}/write/run_counter_collection.csv", cc,
           [[spread, 550000], [light, 131072], [heavy, 0]])
    _write(f"{d}/cf/run_counter_collection.csv", cc, [["__amd_rocclr_copyBuffer", 131072]])
    _write(f"{d}/cw/run_counter_collection.csv", cc, [["__amd_rocclr_copyBuffer", 262144]])
    cyc = 1_000_000
    sq = []
    for name, busy in ((spread, 0.5), (light, 0.75), (heavy, 0.0)):
        sq += [[name, "GRBM_GUI_ACTIVE", 8 * cyc], [name, "SQ_ACTIVE_INST_VALU", busy * 256 * cyc],
               [name, "SQ_INSTS_VALU", busy * 256 * cyc], [name, "SQ_LDS_IDX_ACTIVE", 0],
               [name, "SQ_LDS_BANK_CONFLICT", 0]]
    _write(f"{d}/sq/run_counter_collection.csv", ["Kernel_Name", "Counter_Name", "Counter_Value"],
           sq)
    md = f"{d}/s.md"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--summarize-profiles",
                        "--stats-dir", f"{d}/stats", "--fetch-dir", f"{d}/fetch",
                        "--write-dir", f"{d}/write", "--cal-fetch-dir", f"{d}/cf",
                        "--cal-write-dir", f"{d}/cw", "--sq-dir", f"{d}/sq", "--workload", "3d",
                        "--kernels", "k_spread_smp,k_tile_sum", "--md-out", md,
                        "--traffic-out", f"{d}/traffic.json", "--counters-out", f"{d}/c.json"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    text = open(md).read()
    # traffic: 280000 KiB x 2 + 131072 KiB for the first pass alone
    assert "| `k_tile_sum<float, 3, false>` | 180.0 | 280000 | 131072 | %.1f | - |" % (
        (280000 * 2.0 + 131072) * 1024 / 1e6) in text
    assert "| `k_tile_sum<float, 3, true>` | 4.0 | 20 | 0 |" in text
    # utilisation: one row per pass, and a single spreading kernel under its plain name
    assert "| `k_tile_sum<float, 3, false>` | 0.75 |" in text
    assert "| `k_tile_sum<float, 3, true>` | 0.00 |" in text
    assert "| `k_spread_smp` | 0.50 |" in text
    c = json.load(open(f"{d}/c.json"))
    assert set(c) == {"3d:k_spread_smp"}
    t = json.load(open(f"{d}/traffic.json"))
    assert set(t) == {"3d:k_spread_smp"}
