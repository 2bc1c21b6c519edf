"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) into a
per-kernel table: calls, total / average / min / max duration (us), VGPRs,
LDS bytes.  Usage: python profiles/summarize_rocpd.py <results.db> [label]"""
import sqlite3
import sys


def main(path, label=""):
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


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else "")
