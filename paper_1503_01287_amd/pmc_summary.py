"""HBM traffic from two rocprofv3 --pmc runs of profile_run (one with
FETCH_SIZE, one with WRITE_SIZE).

Calibration: profile_run first copies 256 MiB three times; the counters'
reading for those copies against the bytes a copy moves gives the scale of
each counter (FETCH_SIZE reads half of a copy's fetched bytes here,
WRITE_SIZE all of its written bytes). The solve phase is the last burst of
dispatches (no idle gap over 1 ms) with at least 100 dispatches (profile_run
ends with its solves). The dominant kernel's launches are the solve-phase
dispatches whose name matches the given regular expression; with "largest",
only those with the largest grid among them (the finest level of a kernel
that every level runs; a colour kernel's launches differ in size by colour,
so they are taken whole, "all").

    python -m paper_1503_01287_amd.pmc_summary FETCH.csv WRITE.csv "KERNEL REGEX" SOLVES [all|largest]
"""
from __future__ import annotations

import collections
import csv
import re
import sys

COPY_KIB = 256 * 1024


def _dispatches(path: str, counter: str):
    d = collections.OrderedDict()
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        k = int(r["Dispatch_Id"])
        if k not in d:
            d[k] = dict(name=r["Kernel_Name"], grid=int(r["Grid_Size"]), t0=int(r["Start_Timestamp"]),
                        t1=int(r["End_Timestamp"]), kib=0.0)
        d[k]["kib"] += float(r["Counter_Value"])
    return list(d.values())


def _scale(ds):
    copies = sorted((x["kib"] for x in ds if "copyBuffer" in x["name"]), reverse=True)[:3]
    if len(copies) < 3:
        raise SystemExit("no calibration copies in the run")
    return COPY_KIB / (sum(copies) / 3), copies


def _solve_phase(ds):
    ds = sorted(ds, key=lambda x: x["t0"])
    bursts, cur = [], [ds[0]]
    for a, b in zip(ds, ds[1:]):
        if b["t0"] - a["t1"] > 1_000_000:
            bursts.append(cur)
            cur = []
        cur.append(b)
    bursts.append(cur)
    big = [b for b in bursts if len(b) >= 100]
    return big[-1]


def summarise(fetch_csv: str, write_csv: str, kernel: str, solves: int, mode: str = "all") -> dict:
    out = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        ds = _dispatches(path, counter)
        scale, copies = _scale(ds)
        ph = _solve_phase(ds)
        dom = [x for x in ph if re.search(kernel, x["name"])]
        if not dom:
            raise SystemExit(f"no dispatch of {kernel!r} in the solve phase")
        g = max(x["grid"] for x in dom)
        if mode == "largest":
            dom = [x for x in dom if x["grid"] == g]
        out[key] = dict(scale=scale, copies=copies, kib=sum(x["kib"] for x in dom) / len(dom),
                        launches=len(dom), grid=g, name=dom[0]["name"],
                        solve_bytes=scale * 1024 * sum(x["kib"] for x in ph) / solves,
                        solve_dispatches=len(ph))
    return out


def main() -> int:
    if len(sys.argv) < 5:
        print(__doc__, file=sys.stderr)
        return 2
    r = summarise(sys.argv[1], sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5] if len(sys.argv) > 5 else "all")
    for k in ("fetch", "write"):
        v = r[k]
        print(f"{k}: scale {v['scale']:.5f} (copies {', '.join(f'{c:,.0f}' for c in v['copies'])} KiB); "
              f"{v['name']} (largest grid {v['grid']}): {v['launches']} launches, {v['kib']:,.1f} KiB = "
              f"{v['kib'] * 1024 * v['scale']:,.0f} bytes per launch; solve phase {v['solve_dispatches']} "
              f"dispatches, {v['solve_bytes']:,.0f} bytes per solve")
    tot = sum(r[k]["kib"] * 1024 * r[k]["scale"] for k in ("fetch", "write"))
    print(f"bytes_per_launch={round(tot)} solve_bytes={round(r['fetch']['solve_bytes'] + r['write']['solve_bytes'])}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
