"""Per-solve kernel table of the solve phase of a rocprofv3 kernel trace.

The solve phase is taken as the last burst of kernels (no idle gap over
1 ms) that holds more than 1,000 kernels and, if a name is given, at least
one launch of that kernel; its kernels are summed per name and divided by
the number of solves the burst holds.

    python -m paper_1503_01287_amd.trace_summary run_kernel_trace.csv SOLVES OUT.txt [KERNEL]
"""
from __future__ import annotations

import collections
import csv
import sys


def summarise(path: str, nsolves: int, want: str | None = None, top: int = 30) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    bursts, cur = [], [rows[0]]
    for a, b in zip(rows, rows[1:]):
        if int(b["Start_Timestamp"]) - int(a["End_Timestamp"]) > 1_000_000:
            bursts.append(cur)
            cur = []
        cur.append(b)
    bursts.append(cur)
    big = [bl for bl in bursts if len(bl) > 1000]
    if want:
        big = [bl for bl in big if any(want in r["Kernel_Name"] for r in bl)]
    bl = big[-1]
    span = (int(bl[-1]["End_Timestamp"]) - int(bl[0]["Start_Timestamp"])) / 1e6
    busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in bl) / 1e6
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in bl:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        k = r["Kernel_Name"].replace("amgp2::", "")[:100]
        agg[k][0] += 1
        agg[k][1] += d
    out = [f"solve phase: {len(bl)} kernels in {nsolves} solves, span {span:.2f} ms, kernel-busy {busy:.2f} ms",
           "launches/solve  ms/solve   avg_us  kernel"]
    for k, v in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"{v[0] / nsolves:14.1f} {v[1] / nsolves / 1000:9.3f} {v[1] / v[0]:8.2f}  {k}")
    if want:
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in bl if want in r["Kernel_Name"]]
        out.append(f"{want}: {len(d)} launches in the solve phase, mean {sum(d) / len(d):.2f} us")
    return "\n".join(out) + "\n"


def main() -> int:
    if len(sys.argv) < 4:
        print(__doc__, file=sys.stderr)
        return 2
    text = summarise(sys.argv[1], int(sys.argv[2]), sys.argv[4] if len(sys.argv) > 4 else None)
    with open(sys.argv[3], "w") as f:
        f.write(text)
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
