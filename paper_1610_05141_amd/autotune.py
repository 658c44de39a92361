"""Autotuner for the sampler's launch geometry and, per class of the batched
workload, its leaf size.

Geometry never changes a sample (the sample is a function of (n, N, seed,
n0, dense_ratio) only): for each size class (variant, floor(log2 n)) the
tuner times the cut-depth bias of the tree kernels (the depth at which the
recursion is handed to threads, Sec. 4.2's Algorithm P cut) and the number
of leaf work-groups per compute unit, and keeps the fastest pair.

The leaf size n0 does change the sample, so it is never applied behind the
caller's back: for the classes (floor(log2 n), dense or sparse) of the
batched workload the tuner times n0 in {1024, 2048, 4096} and records the
fastest; n0_for(n, N) returns the recorded value, which a caller passes with
the instance (and an oracle check passes to the oracle).

    python -m paper_1610_05141_amd.autotune [--out PATH] [--quick]

runs the sweeps on cuda:0 and writes the table with every measurement.
apply_table() pushes the geometry into the library; the binding calls it
when it loads the library.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

_HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(_HERE, "tune_table.json")
DEFAULT_N0 = 4096
DENSE_RATIO = 16
CUT_BIASES = (-2, -1, 0, 1, 2)
LEAF_WGS = (1, 2, 3)
N0_CHOICES = (1024, 2048, 4096)
N_CLASSES = 64

# plain classes timed by the sweep: (variant, log2 n, N)
GEOMETRY_CLASSES = (
    [(0, k, min(1 << 48, 1 << (k + 18))) for k in (10, 13, 16, 19, 22, 25, 28, 30)]
    + [(1, k, 1 << (k + 12)) for k in (12, 16, 20, 24, 28)]
)


def size_class(n: int) -> int:
    return max(0, int(n).bit_length() - 1)


def load_table(path: str = TABLE_PATH):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _nearest(entries, key, value):
    best = None
    for e in entries:
        d = abs(e[key] - value)
        if best is None or d < best[0]:
            best = (d, e)
    return None if best is None else best[1]


def geometry_rows(table):
    """(variant, class, cut_bias, leaf_wgs_per_cu) for all 2 x 64 classes:
    each class takes the measured class of its variant nearest in log2 n."""
    rows = []
    geo = table.get("geometry", []) if table else []
    for variant in (0, 1):
        measured = [e for e in geo if e["variant"] == variant]
        for c in range(N_CLASSES):
            e = _nearest(measured, "log2_n", c)
            if e is not None:
                rows.append((variant, c, int(e["cut_bias"]), int(e["leaf_wgs_per_cu"])))
    return rows


def apply_table(L=None, table=None) -> bool:
    """Push the table's geometry into the library (L: the loaded CDLL)."""
    if table is None:
        table = load_table()
    if not table:
        return False
    if L is None:
        from . import lib
        L = lib()
    for variant, c, cb, w in geometry_rows(table):
        rc = L.dcs_tune_set(variant, c, cb, w)
        if rc != 0:
            raise RuntimeError(f"dcs_tune_set({variant}, {c}, {cb}, {w}) returned {rc}")
    return True


def n0_for(n: int, N: int, table=None) -> int:
    """Recorded leaf size for an instance of the batched workload's classes."""
    if table is None:
        table = load_table()
    rows = (table or {}).get("leaf_size", [])
    dense = DENSE_RATIO * n >= N
    same = [e for e in rows if bool(e["dense"]) == dense] or rows
    e = _nearest(same, "log2_n", size_class(n))
    return int(e["n0"]) if e else DEFAULT_N0


# ---------------------------------------------------------------------------
# sweeps (GPU)
# ---------------------------------------------------------------------------
def _time_ms(run, sync, min_ms: float = 25.0, max_reps: int = 40) -> float:
    run()
    sync()
    reps, t0 = 0, time.perf_counter()
    while True:
        run()
        reps += 1
        if reps >= max_reps or (reps >= 3 and (time.perf_counter() - t0) * 1e3 >= min_ms):
            break
    sync()
    return (time.perf_counter() - t0) * 1e3 / reps


def tune_geometry(classes=GEOMETRY_CLASSES, log=print):
    import torch
    import paper_1610_05141_amd as dcs
    out_rows = []
    for variant, k, N in classes:
        n = 1 << k
        out = torch.empty(n, dtype=torch.int64, device="cuda")
        f = dcs.sample if variant == 0 else dcs.sample_replacement
        ms = {}
        for cb in CUT_BIASES:
            for w in LEAF_WGS:
                dcs.tune_set(variant, k, cb, w)
                ms[f"{cb},{w}"] = _time_ms(lambda: f(n, N, 7, out=out), dcs.synchronize)
        best = min(ms, key=ms.get)
        cb, w = (int(x) for x in best.split(","))
        dcs.tune_set(variant, k, cb, w)
        row = {"variant": variant, "log2_n": k, "N": N, "cut_bias": cb, "leaf_wgs_per_cu": w,
               "best_ms": ms[best], "default_ms": ms["0,3"], "ms": ms}
        out_rows.append(row)
        log(f"[tune] geometry variant={variant} n=2^{k}: cut_bias={cb} wgs={w} "
            f"{ms[best]:.3f} ms (default {ms['0,3']:.3f})")
        del out
        torch.cuda.empty_cache()
    return out_rows


def tune_leaf_size(count: int = 4096, min_group: int = 8, log=print):
    import torch
    import paper_1610_05141_amd as dcs
    from .workloads import batched_instances
    insts = batched_instances(count)
    groups = {}
    for x in insts:
        groups.setdefault((size_class(x.n), DENSE_RATIO * x.n >= x.N), []).append(x)
    stream = torch.cuda.Stream()
    rows = []
    for (k, dense), xs in sorted(groups.items()):
        if len(xs) < min_group:
            continue
        total = sum(x.n for x in xs)
        out = torch.empty(total, dtype=torch.int64, device="cuda")
        ms = {}
        for n0 in N0_CHOICES:
            specs, off = [], 0
            for x in xs:
                specs.append(dcs.InstanceSpec(n=x.n, N=x.N, seed=x.seed, out_offset=off, n0=n0))
                off += x.n
            b = dcs.Batch(specs)

            def run():
                with torch.cuda.stream(stream):
                    b.run(out, use_graph=True, stream=stream)

            ms[str(n0)] = _time_ms(run, lambda: dcs.synchronize(stream))
            b.close()
        best = min(ms, key=ms.get)
        rows.append({"log2_n": k, "dense": dense, "instances": len(xs), "samples": total,
                     "n0": int(best), "best_ms": ms[best], "ms": ms})
        log(f"[tune] leaf size n=2^{k} {'dense' if dense else 'sparse'} ({len(xs)} instances): "
            f"n0={best} {ms[best]:.3f} ms")
        del out
        torch.cuda.empty_cache()
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--quick", action="store_true", help="a few classes only")
    args = ap.parse_args(argv)
    if os.environ.get("DCS_CUT_BIAS") or os.environ.get("DCS_LEAF_GRID"):
        print("unset DCS_CUT_BIAS / DCS_LEAF_GRID: they override the geometry being tuned",
              file=sys.stderr)
        return 2
    import torch
    import paper_1610_05141_amd as dcs
    torch.cuda.set_device(0)
    dcs.lib()
    dcs.tune_reset()
    classes = GEOMETRY_CLASSES if not args.quick else GEOMETRY_CLASSES[::4]
    t0 = time.time()
    geometry = tune_geometry(classes)
    leaf = tune_leaf_size(min_group=8 if not args.quick else 200)
    table = {
        "device": torch.cuda.get_device_name(0),
        "host": platform.node(),
        "date": time.strftime("%Y-%m-%d %H:%M:%S"),
        "command": "python -m paper_1610_05141_amd.autotune" + (" --quick" if args.quick else ""),
        "seconds": round(time.time() - t0, 1),
        "method": "wall-clock ms per call after one warm-up call, at least 3 calls and 25 ms; "
                  "geometry keys are cut_bias,leaf_wgs_per_cu; default geometry is 0,3",
        "geometry": geometry,
        "leaf_size": leaf,
    }
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print(f"[tune] wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
