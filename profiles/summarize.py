#!/usr/bin/env python3
"""Summarise a rocprofv3 kernel trace (the *_results.db it writes) as a text table.

    python profiles/summarize.py <results.db> "<command that produced it>" > profiles/<name>.txt

Prints per-kernel launch count, total, average, min and max duration (microseconds) from the
`kernels` view of the rocpd SQLite database, highest total first.
"""
import sqlite3
import sys


def main():
    db, cmd = sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else ""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    print(f"# rocprofv3 --kernel-trace --stats summary")
    print(f"# command: {cmd}")
    print(f"# durations in microseconds (from {db.split('/')[-1]})")
    print(f"{'kernel':60s} {'calls':>6s} {'total_us':>11s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s}")
    for name, n, tot, avg, mn, mx in rows:
        short = name if len(name) <= 60 else name[:57] + "..."
        print(f"{short:60s} {n:6d} {tot / 1e3:11.1f} {avg / 1e3:9.2f} {mn / 1e3:9.2f} {mx / 1e3:9.2f}")


if __name__ == "__main__":
    main()
