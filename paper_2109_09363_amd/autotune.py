"""Tile autotuner of the persistent Jacobi kernels.

Single grids: for each grid size, time a number of sweeps (E_1 tested every
--check-every, 384 by default) with every
tile height R that fits the GPU and every block length B (sweeps between
halo exchanges, halo B + 1) of --blocks, and keep the fastest pair; the
result is the C header the library compiles (csrc/tile_table.h), and grids
without an entry use B = 8 and the smallest R that fits.

Batches (--batch): for each grid side, time the batched projection of a
batch of plumes of that side at a fixed sweep count with R = 8 and R = 16
for every instance, and keep the faster (csrc/batch_tile_table.h).

python -m paper_2109_09363_amd.autotune [--sizes 128 192 256 384 512 768 1024]
        [--blocks 8 12 16] [--sweeps 512] [--reps 3] [--batch [--per-batch 16]] [--out HEADER]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import scenes  # noqa: E402
import paper_2109_09363_amd as hp  # noqa: E402
from paper_2109_09363_amd import _lib as L  # noqa: E402

ROWS = (4, 8, 12, 16, 24, 32)


def time_rows(n, rows, sweeps, reps, dev, block=8, check_every=384):
    sc = scenes.plume_scene(n, seed=0, n_obstacles=2)
    u, v = scenes.random_faces(n, n, 0, kind="mixed")
    pr = hp.Projector(n, n, sc.dx, 1.0, 1.0, 0, 0, "fp32", device=dev)
    flags = torch.from_numpy(sc.flags).to(dev)
    pr.plan(flags)
    u0 = torch.from_numpy(u.astype(np.float32)).to(dev)
    v0 = torch.from_numpy(v.astype(np.float32)).to(dev)
    p = torch.empty((n, n), dtype=torch.float32, device=dev)
    out = {}
    for r in rows:
        ts = []
        try:
            for rep in range(reps + 1):
                uu, vv = u0.clone(), v0.clone()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                # the benchmark's pattern: E_1 tested every check_every
                # sweeps (a grid barrier), the others neighbour-synchronised;
                # a zero threshold runs to max_iters, no folds
                pr.project_async(uu, vv, flags, p, 0.0, method="jacobi", max_iters=sweeps,
                                 check_every=check_every, fold_window=1 << 30, tile_rows=r,
                                 block_sweeps=block)
                b.record()
                torch.cuda.synchronize()
                if rep > 0:
                    ts.append(a.elapsed_time(b))
        except L.HypError:
            continue  # these tiles do not fit
        out[r] = float(np.median(ts))
    return out


def write_header(path, entries):
    lines = [
        "// Tuned tiles of the persistent Jacobi kernel: for a grid of nx x ny cells,",
        "// the halo H (H - 1 sweeps between exchanges) and rows per wave R that ran",
        "// fastest on MI355X.  Written by paper_2109_09363_amd/autotune.py (do not",
        "// edit by hand); a grid without an entry uses H = 9 and the smallest R",
        "// whose tiles fit one work-group per CU.",
        "#pragma once",
        "",
        "namespace hyp {",
        "",
        "struct TileEntry {",
        "  int nx, ny, H, R;",
        "};",
        "",
    ]
    if entries:
        lines.append("constexpr TileEntry kTileTable[] = {")
        for (n, b, r, ms) in entries:
            lines.append(f"    {{{n}, {n}, {b + 1}, {r}}},  // {ms:.3f} ms")
        lines.append("};")
        lines.append(f"constexpr int kTileTableSize = {len(entries)};")
    else:
        lines.append("// (no measured entries yet)")
        lines.append("constexpr TileEntry kTileTable[] = {{0, 0, 0, 0}};")
        lines.append("constexpr int kTileTableSize = 0;")
    lines += ["", "}  // namespace hyp", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def time_batch_rows(n, count, sweeps, reps, dev):
    """ms of one batched projection (fixed sweeps) of `count` plumes of side n
    with every instance's tiles at R = 8 and at R = 16."""
    inst = []
    for i in range(count):
        sc = scenes.plume_scene(n, seed=200 + i, n_obstacles=(0, 3))
        u, v = scenes.random_faces(n, n, 200 + i, kind="mixed")
        inst.append(dict(nx=n, ny=n, dx=sc.dx, flags=torch.from_numpy(sc.flags).to(dev),
                         u=torch.from_numpy(u.astype(np.float32)).to(dev),
                         v=torch.from_numpy(v.astype(np.float32)).to(dev),
                         p=torch.zeros((n, n), dtype=torch.float32, device=dev)))
    u0 = [d["u"].clone() for d in inst]
    v0 = [d["v"].clone() for d in inst]
    out = {}
    for r in (8, 16):
        b = hp.Batch(inst, threshold=0.0, method="jacobi", max_iters=sweeps, tile_rows=r, device=dev)
        ts = []
        for rep in range(reps + 1):
            for d, uu, vv in zip(inst, u0, v0):
                d["u"].copy_(uu)
                d["v"].copy_(vv)
            a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            b.project_async()
            e.record()
            torch.cuda.synchronize()
            if rep > 0:
                ts.append(a.elapsed_time(e))
        out[r] = float(np.median(ts))
        del b
    return out


def write_batch_header(path, entries):
    lines = [
        "// Tile rows of the batched (streaming) Jacobi kernel per grid side: for",
        "// batches of grids of nx x ny cells, the rows per wave R (8 or 16) that ran",
        "// fastest on MI355X.  Written by paper_2109_09363_amd/autotune.py --batch",
        "// (do not edit by hand); sides without an entry use R = 16.",
        "#pragma once",
        "",
        "namespace hyp {",
        "",
        "struct BatchTileEntry {",
        "  int nx, ny, R;",
        "};",
        "",
        "constexpr BatchTileEntry kBatchTileTable[] = {",
    ]
    for (n, r, ms) in entries:
        lines.append(f"    {{{n}, {n}, {r}}},  // {ms:.3f} ms")
    lines += ["};", f"constexpr int kBatchTileTableSize = {len(entries)};", "", "}  // namespace hyp", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="*", default=[128, 192, 256, 384, 512, 768, 1024])
    ap.add_argument("--sweeps", type=int, default=512)
    ap.add_argument("--blocks", type=int, nargs="*", default=[8, 12, 16],
                    help="block lengths (sweeps between halo exchanges) to try")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--check-every", type=int, default=384)
    ap.add_argument("--out", default=None)
    ap.add_argument("--batch", action="store_true", help="tune the batched kernel's rows per side")
    ap.add_argument("--per-batch", type=int, default=16, help="--batch: plumes per timed batch")
    a = ap.parse_args()
    dev = torch.device("cuda")
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    if a.batch:
        entries = []
        for n in a.sizes:
            t = time_batch_rows(n, a.per_batch, a.sweeps, a.reps, dev)
            best = min(t, key=t.get)
            entries.append((n, best, t[best]))
            print(json.dumps({"n": n, "instances": a.per_batch, "sweeps": a.sweeps, "ms_by_rows": t,
                              "best_rows": best}), flush=True)
        out = a.out or os.path.join(csrc, "batch_tile_table.h")
        write_batch_header(out, entries)
        print(f"# wrote {out}", file=sys.stderr, flush=True)
        return
    a.out = a.out or os.path.join(csrc, "tile_table.h")
    entries = []
    for n in a.sizes:
        t = {}
        for b in a.blocks:
            times = time_rows(n, ROWS, a.sweeps, a.reps, dev, block=b, check_every=a.check_every)
            for r, ms in times.items():
                t[(b, r)] = ms
        if not t:
            print(json.dumps({"n": n, "fits": False}), flush=True)
            continue
        best = min(t, key=t.get)
        entries.append((n, best[0], best[1], t[best]))
        print(json.dumps({"n": n, "sweeps": a.sweeps,
                          "ms_by_block_rows": {f"B{b}_R{r}": round(ms, 4) for (b, r), ms in sorted(t.items())},
                          "best_block": best[0], "best_rows": best[1],
                          "us_per_sweep": round(1e3 * t[best] / a.sweeps, 3)}), flush=True)
    write_header(a.out, entries)
    print(f"# wrote {a.out}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
