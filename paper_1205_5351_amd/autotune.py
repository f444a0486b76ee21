"""Empirical tuning of the LDS Jacobi layout (rows per block, lanes per row
pair) per window shape.

For each shape every valid layout is timed on a batch of seeded low-rank
plus noise matrices through ``tilt_svt_batch`` (the SVT the solver runs at
every inner iteration), and the fastest is recorded.  The table is JSON:
``{"device": ..., "entries": [{"m", "n", "bs", "lpp", "ms", "candidates"}]}``;
``load_tuning`` applies it (the package loads ``tuning/mi355x_svt_layouts.json``
at import when present).

Run on the GPU:  python -m paper_1205_5351_amd.autotune --out table.json
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import tilt as T

DEFAULT_SIDES = (32, 48, 64, 80, 100, 128, 160, 200, 256)


def _inputs(m, n, count, seed):
    rng = np.random.default_rng(seed)
    out = np.empty((count, m, n), np.float32)
    for i in range(count):
        L = rng.standard_normal((m, 4)) @ rng.standard_normal((4, n))
        X = L / np.linalg.norm(L) + 0.03 * np.where(rng.uniform(size=(m, n)) < 0.2, rng.standard_normal((m, n)), 0.0)
        out[i] = X + 0.001 * rng.standard_normal((m, n))
    return out


def tune(shapes, count=256, reps=3, log=print):
    import torch

    ctx = T.Context(0)
    dev = torch.device("cuda:0")
    entries = []
    for (m, n) in shapes:
        layouts = T.svt_layouts(m, n)
        if len(layouts) < 2:
            continue
        M = torch.from_numpy(_inputs(m, n, count, 1000 * m + n)).to(dev)
        A = torch.zeros_like(M)
        eps = np.full(count, 0.01, np.float32)
        times = {}
        for bs, lpp in layouts:
            T.tune_set(m, n, bs, lpp)
            ctx.svt_batch(M.data_ptr(), A.data_ptr(), 0, count, m, n, eps)
            best = math.inf
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.svt_batch(M.data_ptr(), A.data_ptr(), 0, count, m, n, eps)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            times[f"{bs}x{lpp}"] = round(1000 * best, 4)
        key = min(times, key=times.get)
        bs, lpp = (int(x) for x in key.split("x"))
        T.tune_set(m, n, bs, lpp)
        entries.append({"m": m, "n": n, "bs": bs, "lpp": lpp, "ms": times[key], "candidates": times})
        log(f"{m}x{n}: best {key} {times[key]} ms of {times}")
    ctx.close()
    import torch

    return {"device": torch.cuda.get_device_name(0), "batch": count, "entries": entries}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--count", type=int, default=256)
    args = ap.parse_args(argv)
    shapes = [(a, b) for a in DEFAULT_SIDES for b in DEFAULT_SIDES if a <= b]
    T.tune_clear()
    table = tune(shapes, count=args.count, log=lambda s: print(s, file=sys.stderr, flush=True))
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"wrote {len(table['entries'])} entries to {args.out}", file=sys.stderr)


if __name__ == "__main__":
    main()
