"""Autotuner for the batched EM march: the tile shape per size class.

    python -m paper_2603_07038_amd.tune [--out FILE] [--classes 15-24] [--steps 64]

The batched march works on tiles of 4 waves, cut into z-chunks of
``kchunk`` node planes.  In mixed precision a wave takes either a run of 62
consecutive nodes of the plane numbered x fastest (layout 1) or a 62-node
segment of one row, 4 rows per block (layout 2); in FP64 a tile is 64 x 4
nodes staged in LDS.  Short chunks give more work items (better load balance
when few variants are attached) but stage extra planes per chunk; long
chunks amortise the halo.  Runs leave no lanes idle at row ends; row
segments share the rows j - 1, j + 1 of their neighbours in L2.  For each
size class (floor of log2 of the cell count, the key the batch uses) a
package variant of that size is replicated until the batch holds at least
16 M cells, and every candidate (layout, chunk) is timed over graph-replayed
EM steps.  The choice per class (see ``pick``) is written as
``{"kchunk": {"<class>": k, ...}, "layout": {"<class>": 1 or 2, ...},
"timings_us": {...}, "timings_fp64_us": {...}}`` (a run updates its own
precision's entries), the table ``Batch`` reads (``tune_gfx950.json`` next to
this file by default).  Every layout and chunk gives bitwise the same
results, so the table changes speed only.

An FP64 run records its timings but writes its picks (``"kchunk_fp64"``)
only with ``--fp64-map``: on gfx950 the FP64 chunks are within 1 % of each
other up to 0.75 M cells and 2 planes win above, yet served in batches of
mixed sizes the picks (24 and 2 planes) gave fewer designs per hour than the
batch's own rule for chunks without an entry (10.8 k against 12.7 k at
saturation; uniform 2-plane chunks and the mixed-precision table also lost).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tune_gfx950.json")
CANDIDATES = (2, 4, 6, 8, 12, 16, 24, 32)
LAYOUTS = (1, 2)  # mixed precision: runs over the x-fastest plane, row segments


def class_problem(c: int):
    """A package variant with about 2**c cells (1 um voxels)."""
    import workloads as W
    nz = 32 if c <= 18 else (48 if c <= 21 else 64)
    n = max(8, int(round(math.sqrt(2.0 ** (c + 0.5) / nz))))
    return W.package(n, n, nz, 9000 + c, bump_pitch_um=20.0, bump_cells=6, trace_width=3, trace_pitch=6,
                     n_trace_layers=4, max_traces=16, n_bits=64, steps_per_bit=4, em_per_thermal=1024,
                     name=f"tune{c}")


def time_class(c: int, steps: int, precision: int):
    import torch
    from . import ETM_PREC_MIXED, Batch, Plan, cfl_dt
    p = class_problem(c)
    assert int(math.floor(math.log2(p.n_cells))) == c, (c, p.n_cells)
    copies = max(1, min(32, (16 << 20) // p.n_cells))
    dt = cfl_dt(p)
    J = p.sample_J_half(dt, 4 * steps)
    layouts = LAYOUTS if precision == ETM_PREC_MIXED else (0,)
    plans = [Plan(p, J, dt=dt, precision=precision, n_steps=4 * steps, history=False) for _ in range(copies)]
    res = {}
    for lay in layouts:
        for kc in CANDIDATES:
            if kc > p.nz + 1 and kc != CANDIDATES[0]:
                continue
            table = {"kchunk": {str(c): kc}}
            if lay:
                table["layout"] = {str(c): lay}
            b = Batch(copies + 1, json.dumps(table))
            for pl in plans:
                b.attach(pl)
            s = torch.cuda.Stream()
            b.advance(steps, s)  # warm-up: captures the graph of this segment length
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            b.advance(steps, s)
            e1.record(s)
            e1.synchronize()
            res[(lay, kc)] = e0.elapsed_time(e1) * 1e3 / steps
            for slot in range(copies):
                b.detach(slot)
            del b
            torch.cuda.synchronize()
    del plans
    torch.cuda.synchronize()
    return res, copies, p.n_cells


TIE = 0.02  # candidates within 2 % of the fastest count as tied


def pick(res):
    """The (layout, chunk) to use: among the candidates within TIE of the
    fastest, the longest chunk (fewest work items and least halo traffic: a
    chunk stages one plane beyond its own), runs before row segments.  The
    classes are timed in batches of one size; in a batch of mixed sizes, as
    the server runs, the shorter of two tied chunks measured up to 8 % slower
    per design."""
    best = min(res.values())
    tied = [key for key, v in res.items() if v <= (1.0 + TIE) * best]
    return max(tied, key=lambda key: (key[1], key[0] == 1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--classes", default="15-24")
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--fp64-map", action="store_true", help="write the FP64 picks, not only their timings")
    a = ap.parse_args(argv)
    from . import ETM_PREC_FP64, ETM_PREC_MIXED
    prec = ETM_PREC_MIXED if a.precision == "mixed" else ETM_PREC_FP64
    lo, hi = (int(x) for x in a.classes.split("-"))
    # one table for both precisions: this run replaces its own precision's maps
    table = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            table = json.load(f)
    sfx = "" if a.precision == "mixed" else "_fp64"
    kmap, lmap, tmap = {}, {}, {}
    for c in range(lo, hi + 1):
        res, copies, cells = time_class(c, a.steps, prec)
        lay, kc = pick(res)
        kmap[str(c)] = kc
        if lay:
            lmap[str(c)] = lay
        tmap[str(c)] = {f"{'runs' if l == 1 else 'rows' if l == 2 else 'tile'}/{k}": round(v, 2)
                        for (l, k), v in res.items()}
        print(json.dumps({"class": c, "cells": cells, "copies": copies, "best": [lay, kc],
                          "us_per_step": tmap[str(c)]}), flush=True)
    if a.precision == "mixed":
        table["kchunk"] = kmap
        table["layout"] = lmap
    elif a.fp64_map:
        table["kchunk_fp64"] = kmap
    table["timings" + sfx + "_us"] = tmap
    table["candidates"] = list(CANDIDATES)
    table.pop("precision", None)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote", a.out)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    main()
