"""Summaries of rocprofv3 output for the profiles/ notes.

  python -m paper_2603_26968_amd.prof kernels <results.db>
      per-kernel table from a --kernel-trace database (rocpd SQLite): calls,
      total / average / min / max duration (us), VGPRs, LDS and scratch bytes.
  python -m paper_2603_26968_amd.prof counters <counter_collection.csv> [--copy NAME BYTES]
      per-kernel average of each counter per dispatch from a --pmc run
      written with --output-format csv.  FETCH_SIZE and WRITE_SIZE are in
      KiB; with --copy, the reading of kernel NAME (a plain copy that moves
      BYTES bytes each way) gives the factor from counter to bytes, and each
      kernel's scaled bytes per dispatch are printed beside its reading.
"""
from __future__ import annotations

import collections
import csv
import sqlite3
import sys


def kernels(path, label=""):
    db = sqlite3.connect(path)
    rows = db.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration), "
        "max(vgpr_count), max(lds_size), max(scratch_size) from kernels group by name "
        "order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    if label:
        print(label)
    print(f"{'kernel':60s} {'calls':>6s} {'total_us':>10s} {'avg_us':>9s} {'min_us':>9s} "
          f"{'max_us':>9s} {'pct':>6s} {'vgpr':>5s} {'lds':>7s} {'scr':>5s}")
    for name, n, tot, avg, mn, mx, vg, lds, scr in rows:
        short = name.replace("(anonymous namespace)::", "").split("(")[0][:60]
        print(f"{short:60s} {n:6d} {tot / 1e3:10.1f} {avg / 1e3:9.2f} {mn / 1e3:9.2f} "
              f"{mx / 1e3:9.2f} {100 * tot / total:6.1f} {vg:5d} {lds:7d} {scr:5d}")


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names)


def counters(path, copy=None):
    acc = collections.defaultdict(lambda: [0.0, 0])
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = _col(row, "Kernel_Name", "kernel_name", "Kernel-Name")
            cname = _col(row, "Counter_Name", "counter_name", "Counter-Name")
            val = float(_col(row, "Counter_Value", "counter_value", "Counter-Value"))
            key = (name.replace("(anonymous namespace)::", "").split("(")[0], cname)
            acc[key][0] += val
            acc[key][1] += 1
    per = {k: v[0] / v[1] for k, v in acc.items()}
    factor = {}
    if copy:
        cname_k, nbytes = copy[0], float(copy[1])
        # the copy is the matching kernel with the largest reading (other
        # element-wise kernels of the run move little)
        best = {}
        for (kname, cname), v in per.items():
            if cname_k in kname and v > best.get(cname, 0.0):
                best[cname] = v
        factor = {c: nbytes / v for c, v in best.items()}
    print(f"{'kernel':60s} {'counter':>12s} {'avg/dispatch':>14s} {'scaled_bytes':>14s}")
    for (kname, cname), v in sorted(per.items()):
        sc = f"{v * factor[cname]:14.0f}" if cname in factor else f"{'':>14s}"
        print(f"{kname[:60]:60s} {cname:>12s} {v:14.1f} {sc}")
    for c, fct in factor.items():
        print(f"factor {c}: {fct:.3f} bytes per unit (from the copy kernel)")


if __name__ == "__main__":
    if len(sys.argv) < 3:
        print(__doc__)
        sys.exit(2)
    if sys.argv[1] == "kernels":
        kernels(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "")
    elif sys.argv[1] == "counters":
        cp = None
        if "--copy" in sys.argv:
            i = sys.argv.index("--copy")
            cp = (sys.argv[i + 1], sys.argv[i + 2])
        counters(sys.argv[2], cp)
    else:
        print(__doc__)
        sys.exit(2)
