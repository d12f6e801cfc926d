"""The rocprofv3 solve-phase summariser on a synthetic trace: it must pick
the last large burst (optionally the one holding a named kernel) and report
per-solve launch counts and times."""
import csv

from paper_1503_01287_amd.trace_summary import summarise

FIELDS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_solve_phase_table(tmp_path):
    rows, t = [], 0
    # setup burst: 1,200 launches of "k_setup" (2 us each, 1 us apart)
    for _ in range(1200):
        rows.append({"Kernel_Name": "amgp2::k_setup", "Start_Timestamp": t, "End_Timestamp": t + 2000})
        t += 3000
    t += 5_000_000  # idle gap > 1 ms ends the burst
    # solve burst: 2 solves x (600 "k_a" of 4 us + 300 "k_b" of 10 us)
    for _ in range(2):
        for _ in range(600):
            rows.append({"Kernel_Name": "amgp2::k_a", "Start_Timestamp": t, "End_Timestamp": t + 4000})
            t += 5000
        for _ in range(300):
            rows.append({"Kernel_Name": "amgp2::k_b", "Start_Timestamp": t, "End_Timestamp": t + 10000})
            t += 11000
    path = tmp_path / "trace.csv"
    _write(path, rows)
    text = summarise(str(path), 2)
    lines = text.splitlines()
    assert lines[0].startswith("solve phase: 1800 kernels in 2 solves")
    # k_b: 300 per solve, 3.0 ms per solve, 10 us each; k_a: 600, 2.4 ms, 4 us
    assert "300.0     3.000    10.00  k_b" in text
    assert "600.0     2.400     4.00  k_a" in text
    assert "k_setup" not in text
    named = summarise(str(path), 1, "k_setup")
    assert "k_setup: 1200 launches in the solve phase, mean 2.00 us" in named
