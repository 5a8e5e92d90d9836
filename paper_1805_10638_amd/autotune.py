"""Tile-shape autotuner for the assignment kernel.

For each (GEMM precision, X type, d, K) bucket it times the assignment of
one application of G (kmeans_g: the assignment kernel and, where rows are
listed, the pass-wide re-check, from the library's own HIP events) with
every tile shape of the kernel family on seeded synthetic data and keeps
the fastest; the table is written as JSON and applied to every Context
created afterwards (see ``load_table``).

    python -m paper_1805_10638_amd.autotune [--out FILE] [--rows N] [--reps R]

Buckets: K rounds up to a power of two (at least 16) and d to the padded
width of the kernel, exactly as km_set_tile_shape keys them.  The default
bucket list covers the benchmark configurations: the batched mix (d in
{3, 16, 64}, K from 8 to 512), d = 32 / K = 256 float32, d = 128 /
K = 1024 and d = 96 / K = 2048 on bfloat16 rows.  The d = 128 / K = 1024
buckets are timed on the precision workload's own data (4M bfloat16 rows of
512 Gaussian clusters with 5 % outliers), the others on Gaussian mixtures.
"""

from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tiles_gfx950.json")
SHAPES = 4

# (prec, xtype, d, K, rows, data): data "mixture" or "precision"
DEFAULT_BUCKETS = (
    [("f32", "f32", d, k, 200_000, "mixture") for d in (3, 16, 64) for k in (16, 32, 64, 128, 256, 512)]
    + [("f32", "f32", 32, 256, 1_000_000, "mixture"),
       ("bf16", "bf16", 128, 1024, 4_000_000, "precision"), ("f32", "bf16", 128, 1024, 4_000_000, "precision"),
       ("bf16", "bf16", 96, 2048, 500_000, "mixture")]
)


def load_table(path: str = TABLE):
    """Entries of a tuning table, [] when there is none."""
    if not os.path.exists(path):
        return []
    with open(path) as f:
        return json.load(f).get("entries", [])


def apply_table(ctx, entries) -> int:
    n = 0
    for e in entries:
        ctx.set_tile_shape(e["prec"], e["xtype"], int(e["d"]), int(e["K"]), int(e["shape"]))
        n += 1
    return n


def _data(rows, d, k, xtype, seed, kind="mixture"):
    from . import synth
    if kind == "precision":   # bfloat16 rows by construction
        x, _ = synth.precision(rep=1, n=rows, d=d, k=max(2, k // 2))
        if xtype == "f32":
            x = synth.bf16_bits_to_f32(x)
        return x, synth.init_centroids(x, k, seed)
    x, _ = synth.plain_large(rep=seed, n=rows, d=d, k=max(2, k // 2), cfg=200)
    if xtype == "bf16":
        x = synth.to_bf16_bits(x)
    return x, synth.init_centroids(x, k, seed)


def tune(buckets=DEFAULT_BUCKETS, reps=5, rows=None, log=print):
    import torch
    from . import _lib
    ctx = _lib.Context(0, tuned=False)
    ctx.set_timing(True)
    out = []
    for prec, xtype, d, k, n, kind in buckets:
        n = rows or n
        x, c0 = _data(n, d, k, xtype, seed=d * 1000 + k, kind=kind)
        X = torch.from_numpy(x.view(np.int16) if xtype == "bf16" else x).to("cuda")
        C = torch.from_numpy(c0).to("cuda")
        times, whole = [], []
        for sh in range(SHAPES):
            ctx.set_tile_shape(prec, xtype, d, k, sh)
            _lib.kmeans_g(X, C, prec=prec, ctx=ctx)          # warm-up (workspace, code load)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            ms = 0.0
            for _ in range(reps):
                ms += _lib.kmeans_g(X, C, prec=prec, ctx=ctx)[3].assign_ms
            b.record()
            torch.cuda.synchronize()
            times.append(ms * 1e3 / reps)
            whole.append(a.elapsed_time(b) * 1e3 / reps)
        best = int(np.argmin(times))
        ctx.set_tile_shape(prec, xtype, d, k, 0)
        out.append({"prec": prec, "xtype": xtype, "d": d, "K": k, "rows": n, "data": kind, "shape": best,
                    "assign_us": [round(t, 1) for t in times], "us_per_g": [round(t, 1) for t in whole]})
        log(json.dumps(out[-1]), flush=True)
        del X, C
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--rows", type=int, default=None)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    t0 = time.time()
    entries = tune(reps=a.reps, rows=a.rows)
    doc = {"device": "MI355X (gfx950)", "what": "fastest assignment tile shape per bucket, timed by the "
           "library's events around the assignment (and re-check) of kmeans_g calls; us_per_g is the "
           "whole call", "seconds": round(time.time() - t0, 1), "entries": entries}
    with open(a.out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
