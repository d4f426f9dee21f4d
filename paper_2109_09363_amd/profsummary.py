"""Per-kernel duration summary (count, total, average, min, max) from a
rocprofv3 trace database (`rocprofv3 --kernel-trace ... -d DIR -o NAME`
writes DIR/NAME_results.db).  Used when the profiler's own --stats report
is not written, e.g. when it exits abnormally after the program finished.

python -m paper_2109_09363_amd.profsummary path/to/run_results.db [--top N]
"""
from __future__ import annotations

import argparse
import sqlite3


def summarize(db: str):
    con = sqlite3.connect(db)
    cur = con.cursor()
    tabs = [r[0] for r in cur.execute("select name from sqlite_master where type='table'")]
    disp = next(t for t in tabs if t.startswith("rocpd_kernel_dispatch"))
    sym = next(t for t in tabs if t.startswith("rocpd_info_kernel_symbol"))
    cols = [r[1] for r in cur.execute(f"pragma table_info({sym})")]
    name_col = "kernel_name" if "kernel_name" in cols else ("display_name" if "display_name" in cols else "name")
    q = (f"select s.{name_col}, count(*), sum(d.end - d.start), avg(d.end - d.start), "
         f"min(d.end - d.start), max(d.end - d.start) from {disp} d join {sym} s "
         f"on d.kernel_id = s.id group by s.{name_col} order by sum(d.end - d.start) desc")
    return list(cur.execute(q))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=25)
    a = ap.parse_args()
    rows = summarize(a.db)
    tot = sum(r[2] for r in rows) or 1
    print(f"{'kernel':70s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'min_us':>9s} {'max_us':>10s} {'pct':>6s}")
    for name, n, s, avg, mn, mx in rows[: a.top]:
        short = name if len(name) <= 70 else name[:67] + "..."
        print(f"{short:70s} {n:7d} {s / 1e6:10.3f} {avg / 1e3:10.2f} {mn / 1e3:9.2f} {mx / 1e3:10.2f} {100 * s / tot:6.2f}")


if __name__ == "__main__":
    main()
