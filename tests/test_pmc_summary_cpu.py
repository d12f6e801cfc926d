"""Traffic summariser on synthetic rocprofv3 --pmc runs: calibration from
the three copies, the solve phase and the dominant kernel's per-launch
bytes (largest grid of the named kernel)."""
import csv

from paper_1503_01287_amd.pmc_summary import summarise

FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value", "Start_Timestamp",
          "End_Timestamp"]


def _run(path, counter, copy_kib, kib_of):
    rows, t, d = [], 0, 0

    def add(name, grid, kib):
        nonlocal t, d
        d += 1
        # a counter may come in several rows per dispatch (per XCD): split it
        for part in (0.25, 0.75):
            rows.append(dict(Dispatch_Id=d, Kernel_Name=name, Grid_Size=grid, Counter_Name=counter,
                             Counter_Value=kib * part, Start_Timestamp=t, End_Timestamp=t + 1000))
        t += 2000
    for _ in range(3):
        add("__amd_rocclr_copyBuffer", 1024, copy_kib)
    t += 5_000_000
    for _ in range(1100):  # setup
        add("k_setup", 256, 1.0)
    t += 5_000_000
    for _ in range(2):  # 2 solves: level-0 and level-1 launches of the same kernel
        for _ in range(500):
            add("k_gs<3, 32>", 4096, kib_of(4096))
            add("k_gs<3, 32>", 512, kib_of(512))
            add("k_other", 256, 2.0)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        w.writerows(rows)


def test_traffic_summary(tmp_path):
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _run(fp, "FETCH_SIZE", 131072.0, lambda g: 10.0 if g == 4096 else 3.0)   # fetch reads half
    _run(wp, "WRITE_SIZE", 262144.0, lambda g: 4.0 if g == 4096 else 1.0)   # write reads all
    r = summarise(str(fp), str(wp), "k_gs", 2, "largest")
    assert abs(r["fetch"]["scale"] - 2.0) < 1e-12 and abs(r["write"]["scale"] - 1.0) < 1e-12
    assert r["fetch"]["grid"] == 4096 and r["fetch"]["launches"] == 1000
    assert abs(r["fetch"]["kib"] - 10.0) < 1e-12 and abs(r["write"]["kib"] - 4.0) < 1e-12
    # per solve: 500 x (10 + 3 + 2) KiB fetched x 2, 500 x (4 + 1 + 2) KiB written
    assert abs(r["fetch"]["solve_bytes"] - 500 * 15 * 1024 * 2) < 1e-6
    assert abs(r["write"]["solve_bytes"] - 500 * 7 * 1024) < 1e-6
    # all launches of the kernel (a colour kernel's launches differ in size)
    a = summarise(str(fp), str(wp), "k_gs", 2, "all")
    assert a["fetch"]["launches"] == 2000 and abs(a["fetch"]["kib"] - 6.5) < 1e-12
