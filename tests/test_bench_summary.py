"""bench.py --summarize: rocprofv3 kernel-trace and counter CSVs into the
per-kernel tables committed with the profiles (CPU only, synthetic CSVs)."""
import csv
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402

TRACE_COLS = ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id", "Dispatch_Id", "Kernel_Id", "Kernel_Name",
              "Correlation_Id", "Start_Timestamp", "End_Timestamp", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
              "Accum_VGPR_Count", "SGPR_Count", "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z",
              "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
PMC_COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
            "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
            "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
SWEEP = ("void cs::(anonymous namespace)::k_sweep<float, 8, 8, false, false, false, 256>"
         "(long, long, int const*, long const*, int const*, int const*, float const*, float const*)")


def _write(path, cols, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow({c: r.get(c, 0) for c in cols})


def test_short_kernel_names():
    assert bench._short_kernel(SWEEP) == "k_sweep<float, 8, 8, false, false, false, 256>"
    assert bench._short_kernel("void cs::k_gram_mfma8(int, int const*)") == "k_gram_mfma8"
    assert bench._short_kernel("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_trace_summary_groups_by_kernel_and_grid(tmp_path):
    rows = []
    # two grids of the same kernel: 3 launches of 60/70/80 us and 1 of 5 us
    for k, (t0, dt, grid) in enumerate([(0, 60000, 2097152), (100000, 70000, 2097152), (200000, 80000, 2097152),
                                        (300000, 5000, 32768)]):
        rows.append(dict(Kind="KERNEL_DISPATCH", Kernel_Name=SWEEP, Start_Timestamp=t0, End_Timestamp=t0 + dt,
                         Grid_Size_X=grid, Grid_Size_Y=1, Grid_Size_Z=1))
    rows.append(dict(Kind="KERNEL_DISPATCH", Kernel_Name="__amd_rocclr_copyBuffer", Start_Timestamp=0,
                     End_Timestamp=10000, Grid_Size_X=512, Grid_Size_Y=1, Grid_Size_Z=1))
    p = tmp_path / "run_kernel_trace.csv"
    _write(p, TRACE_COLS, rows)
    out = bench.summarize_rocprof(str(p)).splitlines()
    body = [l for l in out if l.startswith("| `")]
    assert body[0].startswith("| `k_sweep<float, 8, 8, false, false, false, 256>` | 2097152 | 3 | 70.00 | 60.00 | 80.00 |")
    assert any(l.startswith("| `k_sweep<float, 8, 8, false, false, false, 256>` | 32768 | 1 | 5.00 |") for l in body)
    total = 60 + 70 + 80 + 5 + 10
    share = float(body[0].split("|")[8])
    assert abs(share - 100.0 * 210 / total) < 0.01


def test_counter_summary_means_max_and_sums(tmp_path):
    rows = []
    for v in (161000.0, 162000.0):
        rows.append(dict(Kernel_Name=SWEEP, Grid_Size=2097152, Counter_Name="FETCH_SIZE", Counter_Value=v,
                         Start_Timestamp=0, End_Timestamp=65000))
    rows.append(dict(Kernel_Name="__amd_rocclr_copyBuffer", Grid_Size=131072, Counter_Name="FETCH_SIZE",
                     Counter_Value=524320.0, Start_Timestamp=0, End_Timestamp=400000))
    p = tmp_path / "run_counter_collection.csv"
    _write(p, PMC_COLS, rows)
    body = [l for l in bench.summarize_rocprof(str(p)).splitlines() if l.startswith("| `")]
    sweep = [l for l in body if "k_sweep" in l][0].split("|")
    assert [c.strip() for c in sweep[2:8]] == ["2097152", "FETCH_SIZE", "2", "161500", "162000", "323000"]
    assert abs(float(sweep[8]) - 65.0) < 1e-9
    copy = [l for l in body if "copyBuffer" in l][0].split("|")
    assert copy[6].strip() == "524320"


def test_setup_windows(tmp_path):
    # three setups (prescale ... E update) each followed by a solve kernel
    rows, t = [], 0

    def add(name, dt):
        nonlocal t
        rows.append(dict(Kind="KERNEL_DISPATCH", Kernel_Name=f"void cs::(anonymous namespace)::{name}(int)",
                         Start_Timestamp=t, End_Timestamp=t + dt, Grid_Size_X=256, Grid_Size_Y=1, Grid_Size_Z=1))
        t += dt + 1000

    add("k_sweep<float, 8, 8, false, false, false, 256>", 5000)   # before any setup: ignored
    for k in range(3):
        add("k_prescale_w", 1000)
        add("k_rowprod_nb<8>", 10000 * (k + 1))
        add("k_eupdate<8>", 2000)
        add("k_sweep<float, 8, 8, true, false, false, 256>", 5000)
    p = tmp_path / "run_kernel_trace.csv"
    _write(p, TRACE_COLS, rows)
    out = bench.summarize_setups(str(p), first=1, count=2)
    assert out.startswith("3 setups in the trace; setups 1-2:")
    body = [l for l in out.splitlines() if l.startswith("| `")]
    assert body[0] == "| `k_rowprod_nb<8>` | 1 | 0.03 |"     # (20 + 30) / 2 us -> 0.025 ms
    assert "| `k_eupdate<8>` | 1 | 0.00 |" in body
    # span: prescale start to E update end = 1000 + 1000 + rowprod + 1000 + 2000
    assert "span 0.03 ms" in out
