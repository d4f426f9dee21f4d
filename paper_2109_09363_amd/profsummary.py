"""Summaries of rocprofv3 result databases (`rocprofv3 ... -d DIR -o NAME`
writes DIR/NAME_results.db).

python -m paper_2109_09363_amd.profsummary trace DB [--top N]
    per-kernel dispatch count, total, average, min and max duration (used
    when the profiler's own --stats report is not written, e.g. when it exits
    abnormally after the program finished)

python -m paper_2109_09363_amd.profsummary dispatches DB --kernel NAME [--last N]
    average, min and max duration of the (last N) dispatches of kernel NAME

python -m paper_2109_09363_amd.profsummary counters DB --kernel NAME [--last N] [--out FILE]
    mean per dispatch of every counter the database holds for kernels whose
    name contains NAME (one PMC pass, e.g. the SQ_* counters of a kernel)

python -m paper_2109_09363_amd.profsummary traffic --kernel NAME
        --fetch DB --write DB --copy-fetch DB --copy-write DB --copy-bytes B
        [--last N] [--out FILE] [--command TEXT]
    HBM traffic per dispatch of kernel NAME from two counter passes
    (FETCH_SIZE, WRITE_SIZE, in KiB per dispatch), each scaled by what the same
    counter reads for a device-to-device copy of B bytes (B read + B written).
    Writes `key: value` lines, including a hash of the kernel's sources so that
    a stale figure can be recognised.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {
    "jacobi_reg": ["csrc/solvers.hip", "csrc/common.h", "csrc/jacobi_rows.h", "csrc/tile_table.h"],
    "pcg_reg": ["csrc/solvers.hip", "csrc/common.h"],
    "plan_": ["csrc/stencil.hip", "csrc/common.h"],
    "conv_mfma": ["csrc/conv_mfma.h", "csrc/cnn.hip", "csrc/papernets.hip"],
    "jacobi_batch": ["csrc/batched.hip", "csrc/batch.h", "csrc/common.h", "csrc/jacobi_rows.h",
                     "csrc/batch_tile_table.h"],
}


def source_hash(kernel: str) -> str:
    """Hash of the sources of the kernel family whose name `kernel` holds
    (e.g. 'conv_mfma<unsigned short, 3, 64, 64, true, false>')."""
    h = hashlib.sha256()
    fam = next((k for k in KERNEL_SOURCES if k in kernel), None)
    for rel in KERNEL_SOURCES.get(fam, []):
        path = os.path.join(PKG, rel)
        if os.path.exists(path):
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def _tables(cur):
    return [r[0] for r in cur.execute("select name from sqlite_master where type in ('table','view')")]


def summarize(db: str):
    con = sqlite3.connect(db)
    cur = con.cursor()
    tabs = _tables(cur)
    disp = next(t for t in tabs if t.startswith("rocpd_kernel_dispatch"))
    sym = next(t for t in tabs if t.startswith("rocpd_info_kernel_symbol"))
    cols = [r[1] for r in cur.execute(f"pragma table_info({sym})")]
    name_col = "kernel_name" if "kernel_name" in cols else ("display_name" if "display_name" in cols else "name")
    q = (f"select s.{name_col}, count(*), sum(d.end - d.start), avg(d.end - d.start), "
         f"min(d.end - d.start), max(d.end - d.start) from {disp} d join {sym} s "
         f"on d.kernel_id = s.id group by s.{name_col} order by sum(d.end - d.start) desc")
    return list(cur.execute(q))


def counter_per_dispatch(db: str, kernel_substr: str, counter: str, last: int = 0):
    """Mean, count, min, max of a counter (summed over its instances per
    dispatch) over the dispatches whose kernel name contains kernel_substr
    (the last `last` of them in dispatch order, if given)."""
    con = sqlite3.connect(db)
    cur = con.cursor()
    rows = list(cur.execute(
        "select dispatch_id, sum(value) from counters_collection where counter_name = ? and "
        "kernel_name like ? group by dispatch_id order by dispatch_id", (counter, f"%{kernel_substr}%")))
    if last > 0:
        rows = rows[-last:]
    vals = [r[1] for r in rows]
    if not vals:
        raise SystemExit(f"no {counter} records for kernel '{kernel_substr}' in {db}")
    return sum(vals) / len(vals), len(vals), min(vals), max(vals)


def cmd_trace(a):
    rows = summarize(a.db)
    tot = sum(r[2] for r in rows) or 1
    print(f"{'kernel':70s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'min_us':>9s} {'max_us':>10s} {'pct':>6s}")
    for name, n, s, avg, mn, mx in rows[: a.top]:
        short = name if len(name) <= 70 else name[:67] + "..."
        print(f"{short:70s} {n:7d} {s / 1e6:10.3f} {avg / 1e3:10.2f} {mn / 1e3:9.2f} {mx / 1e3:10.2f} {100 * s / tot:6.2f}")


def cmd_dispatches(a):
    """Durations of the (last N) dispatches of the kernels whose name
    contains --kernel, in start order."""
    con = sqlite3.connect(a.db)
    cur = con.cursor()
    tabs = _tables(cur)
    disp = next(t for t in tabs if t.startswith("rocpd_kernel_dispatch"))
    sym = next(t for t in tabs if t.startswith("rocpd_info_kernel_symbol"))
    cols = [r[1] for r in cur.execute(f"pragma table_info({sym})")]
    name_col = "kernel_name" if "kernel_name" in cols else ("display_name" if "display_name" in cols else "name")
    rows = list(cur.execute(
        f"select d.end - d.start from {disp} d join {sym} s on d.kernel_id = s.id "
        f"where s.{name_col} like ? order by d.start", (f"%{a.kernel}%",)))
    if a.last > 0:
        rows = rows[-a.last:]
    us = [r[0] / 1e3 for r in rows]
    if not us:
        raise SystemExit(f"no dispatches of '{a.kernel}' in {a.db}")
    lines = [f"kernel: {a.kernel}", f"source_sha: {source_hash(a.kernel)}",
             f"dispatches: {len(us)}" + (f" (the last {a.last})" if a.last > 0 else ""),
             f"avg_us: {sum(us) / len(us):.2f}", f"min_us: {min(us):.2f}", f"max_us: {max(us):.2f}"]
    if a.command:
        lines.append(f"command: {a.command}")
    text = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text, end="")


def cmd_counters(a):
    con = sqlite3.connect(a.db)
    cur = con.cursor()
    names = [r[0] for r in cur.execute(
        "select distinct counter_name from counters_collection where kernel_name like ?",
        (f"%{a.kernel}%",))]
    lines = [f"kernel: {a.kernel}", f"source_sha: {source_hash(a.kernel)}"]
    for n in sorted(names):
        mean, cnt, mn, mx = counter_per_dispatch(a.db, a.kernel, n, a.last)
        lines.append(f"{n}: {mean:.1f} per dispatch ({cnt} dispatches, min {mn:.1f}, max {mx:.1f})")
    if a.command:
        lines.append(f"command: {a.command}")
    text = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text, end="")


def cmd_traffic(a):
    f_mean, f_n, f_min, f_max = counter_per_dispatch(a.fetch, a.kernel, "FETCH_SIZE", a.last)
    w_mean, w_n, w_min, w_max = counter_per_dispatch(a.write, a.kernel, "WRITE_SIZE", a.last)
    cf, _, _, _ = counter_per_dispatch(a.copy_fetch, "copyBuffer", "FETCH_SIZE")
    cw, _, _, _ = counter_per_dispatch(a.copy_write, "copyBuffer", "WRITE_SIZE")
    kfetch = a.copy_bytes / (cf * 1024.0)   # true bytes per counted byte
    kwrite = a.copy_bytes / (cw * 1024.0)
    traffic = kfetch * f_mean * 1024.0 + kwrite * w_mean * 1024.0
    lines = [
        f"kernel: {a.kernel}",
        f"source_sha: {source_hash(a.kernel)}",
        f"dispatches_fetch_pass: {f_n}",
        f"dispatches_write_pass: {w_n}",
        f"fetch_kib_per_dispatch: {f_mean:.3f} (min {f_min:.3f}, max {f_max:.3f})",
        f"write_kib_per_dispatch: {w_mean:.3f} (min {w_min:.3f}, max {w_max:.3f})",
        f"copy_bytes: {a.copy_bytes}",
        f"copy_fetch_kib: {cf:.3f}",
        f"copy_write_kib: {cw:.3f}",
        f"fetch_scale: {kfetch:.4f}",
        f"write_scale: {kwrite:.4f}",
        f"traffic_bytes_per_dispatch: {traffic:.0f}",
    ]
    if a.command:
        lines.append(f"command: {a.command}")
    text = "\n".join(lines) + "\n"
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text, end="")


def read_traffic(path: str):
    """The `key: value` lines of a traffic summary as a dict of strings."""
    out = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--top", type=int, default=25)
    t.set_defaults(fn=cmd_trace)
    d = sub.add_parser("dispatches")
    d.add_argument("db")
    d.add_argument("--kernel", required=True)
    d.add_argument("--last", type=int, default=0)
    d.add_argument("--out")
    d.add_argument("--command")
    d.set_defaults(fn=cmd_dispatches)
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("--kernel", required=True)
    c.add_argument("--last", type=int, default=0)
    c.add_argument("--out")
    c.add_argument("--command")
    c.set_defaults(fn=cmd_counters)
    r = sub.add_parser("traffic")
    r.add_argument("--kernel", required=True)
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--copy-fetch", required=True)
    r.add_argument("--copy-write", required=True)
    r.add_argument("--copy-bytes", type=float, required=True)
    r.add_argument("--last", type=int, default=0)
    r.add_argument("--out")
    r.add_argument("--command")
    r.set_defaults(fn=cmd_traffic)
    a = ap.parse_args()
    a.fn(a)


if __name__ == "__main__":
    main()
