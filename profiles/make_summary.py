"""Per-kernel duration summary (count, mean/min/max microseconds, total ms) from a rocprofv3 SQLite result file.

Usage: python profiles/make_summary.py <results.db> > profiles/<kernel>_<workload>.txt
"""
import sqlite3
import sys


def main(path):
    con = sqlite3.connect(path)
    rows = con.execute(
        "select name, count(*), avg(end-start), min(end-start), max(end-start), sum(end-start) "
        "from kernels group by name order by sum(end-start) desc").fetchall()
    print(f"{'kernel':70s} {'calls':>5s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>10s}")
    for name, n, avg, lo, hi, tot in rows:
        print(f"{name[:70]:70s} {n:5d} {avg / 1e3:10.1f} {lo / 1e3:10.1f} {hi / 1e3:10.1f} {tot / 1e6:10.3f}")


if __name__ == "__main__":
    main(sys.argv[1])
