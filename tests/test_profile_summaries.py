"""Host checks of the profiler summaries (paper_2405_18982_amd.profile_run):
per-dispatch means of counters and per-grid duration statistics, on small
synthetic CSV files in rocprofv3's column layout; no GPU needed."""
import csv

from paper_2405_18982_amd import profile_run


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_counter_means_per_kernel_and_grid(tmp_path, capsys):
    hdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Workgroup_Size", "Counter_Name", "Counter_Value"]
    rows = [
        [1, "k_a", 256, 64, "SQ_WAVES", 4], [1, "k_a", 256, 64, "SQ_INSTS_VALU", 400],
        [2, "k_a", 256, 64, "SQ_WAVES", 4], [2, "k_a", 256, 64, "SQ_INSTS_VALU", 600],
        [3, "k_a", 128, 64, "SQ_WAVES", 2], [3, "k_a", 128, 64, "SQ_INSTS_VALU", 50],
        [4, "k_b", 256, 64, "SQ_WAVES", 4], [4, "k_b", 256, 64, "SQ_INSTS_VALU", 7],
    ]
    p = tmp_path / "c.csv"
    _write(p, hdr, rows)
    profile_run.summarize(str(p))
    out = capsys.readouterr().out
    blocks = {}
    cur = None
    for line in out.splitlines():
        if "grid=" in line:
            cur = line.split()[0] + " " + line.split("grid=")[1].split()[0]
            blocks[cur] = {"head": line}
        elif cur and line.startswith("    "):
            name, val = line.split()
            blocks[cur][name] = float(val)
    assert "dispatches=2" in blocks["k_a 256"]["head"]
    assert blocks["k_a 256"]["SQ_INSTS_VALU"] == 500.0 and blocks["k_a 256"]["SQ_WAVES"] == 4.0
    assert blocks["k_a 128"]["SQ_INSTS_VALU"] == 50.0
    assert blocks["k_b 256"]["SQ_INSTS_VALU"] == 7.0


def test_trace_durations_per_kernel_and_grid(tmp_path, capsys):
    hdr = ["Kernel_Name", "Grid_Size", "Workgroup_Size", "Start_Timestamp", "End_Timestamp"]
    rows = [["k_a", 256, 64, 1000, 11000], ["k_a", 256, 64, 20000, 50000], ["k_a", 128, 64, 0, 4000],
            ["k_b", 256, 64, 0, 1000]]
    p = tmp_path / "t.csv"
    _write(p, hdr, rows)
    profile_run.summarize_trace(str(p))
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.strip().endswith(("k_a", "k_b"))]
    first = lines[0].split()  # largest total first: k_a on grid 256
    assert first[0] == "2" and abs(float(first[1]) - 40.0) < 1e-9 and abs(float(first[2]) - 20.0) < 1e-9
    assert abs(float(first[3]) - 10.0) < 1e-9 and abs(float(first[4]) - 30.0) < 1e-9
    assert first[6] == "256" and first[-1] == "k_a"
    assert any(ln.split()[6] == "128" and float(ln.split()[2]) == 4.0 for ln in lines)


def test_run_options_parse():
    """The profiler driver's run command takes the right-hand side count and
    the V-cycle mode (parsed on the host; no GPU call is made here)."""
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-m", "paper_2405_18982_amd.profile_run", "run", "--help"],
                         capture_output=True, text=True, cwd=root, timeout=120)
    assert out.returncode == 0
    assert "--nrhs" in out.stdout and "--vcycle" in out.stdout and "--smooth-only" in out.stdout
