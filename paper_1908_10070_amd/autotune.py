"""Autotuner for the launch shape of the subset engines: work-item chunk sizes and engine choice.

The library cuts every pattern's subset order into work items: ``chunk_small`` subsets per item
for |Z| <= 8 (the quad and one-tile engines) and ``chunk_large`` for larger subsets (tile
engines). Small chunks balance the persistent launch better; large chunks amortise the per-item
staging of the pattern matrix and the per-wave trace buffers. The best pair depends on n, on the
batch size and on the device, so it is measured:

* a coordinate search -- ``chunk_small`` over its candidates with the default ``chunk_large``,
  then ``chunk_large`` with the best ``chunk_small`` (of chunk sizes within 1% of the fastest, the
  smallest), then the engine of each subset-size band (another engine only if more than 1% faster) in
  turn (``gbs_ctx_set_shape``: for |Z| = 9, 10 and 11, 12 the default engine, the 16x16-tile engine
  or the symmetric quad-tile engine; for |Z| = 13, 14 the 16x16-tile engine or the 7x7 symmetric
  quad-tile engine; where they apply at this n) -- timing the real call
  (``haf_batch`` on the caller's matrices) with HIP events, median of a few repetitions;
* the winner goes to ``gbs_ctx_set_tuning`` / ``gbs_ctx_set_shape`` and to a JSON cache keyed by
  (GPU arch, n), so later contexts load it without measuring (``load_cache``).

Results depend on the chunk sizes only through the order partial sums are added in, i.e. at the
rounding level; within one context every pattern's result is independent of the batch around it.
"""
from __future__ import annotations

import json
import os
import pathlib
import statistics
from typing import Dict, Iterable, Optional, Tuple

DEFAULT_CACHE = pathlib.Path(os.environ.get("GBS_TUNE_CACHE", pathlib.Path.home() / ".cache" / "gbs_tune.json"))

SMALL_CANDIDATES = (128, 256, 512, 1024, 2048, 4096)
LARGE_CANDIDATES = (8, 16, 32, 64, 128, 256, 512)
# chunk sizes within this fraction of the fastest count as tied; the smallest of them is taken, since
# smaller work items spread a call smaller than the tuning batch (a serving step) over more workgroups
TIE = 0.01


def smallest_within(times: Dict[int, float], tol: float = TIE) -> int:
    """The smallest candidate whose time is within (1 + tol) of the fastest one's."""
    best = min(times.values())
    return min(c for c, t in times.items() if t <= best * (1.0 + tol))


def faster_than(current: int, times: Dict[int, float], tol: float = TIE) -> int:
    """The fastest candidate if it beats `current` by more than tol, else `current`."""
    best = min(times, key=times.get)
    return best if times[best] < times[current] * (1.0 - tol) else current


def _arch(ctx) -> str:
    import torch
    return torch.cuda.get_device_properties(ctx.torch_device).gcnArchName.split(":")[0]


def _time_call(fn, reps: int) -> float:
    import torch
    fn()  # warm-up (graph capture for a new shape)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return statistics.median(ts)


def tune(ctx, n: int, A, reps: int = 3, small: Iterable[int] = SMALL_CANDIDATES,
         large: Iterable[int] = LARGE_CANDIDATES, cache: Optional[pathlib.Path] = DEFAULT_CACHE,
         log: Optional[list] = None, shapes=True) -> Tuple[int, int]:
    """Measure chunk sizes, then the engine shape (shapes=True: every shape that differs at n; a
    tuple: those; False: keep the built-in one), for size-n hafnians of the (batch, n, n) CUDA
    tensor A; apply and cache them. Returns the chunk pair (the shape is ctx.get_shape(n))."""
    import torch
    out = torch.empty(A.shape[0], dtype=torch.complex128, device=A.device)
    ctx.set_tuning(n, 0, 0)  # start from the built-in defaults
    d_small, d_large = ctx.get_tuning(n)

    def run(cs, cl):
        ctx.set_tuning(n, cs, cl)
        t = _time_call(lambda: ctx.haf_batch(A, out=out), reps)
        if log is not None:
            log.append({"n": n, "chunk_small": cs, "chunk_large": cl, "ms": t})
        return t

    ctx.set_shape(n, -1)
    d_shape = ctx.get_shape(n)
    best_s = smallest_within({cs: run(cs, d_large) for cs in small})
    best_l = smallest_within({cl: run(best_s, cl) for cl in large})
    ctx.set_tuning(n, best_s, best_l)
    best_shape = d_shape
    if shapes:
        timed = {}

        def run_shape(sh):
            if sh not in timed:
                ctx.set_shape(n, sh)
                timed[sh] = _time_call(lambda: ctx.haf_batch(A, out=out), reps)
                if log is not None:
                    log.append({"n": n, "chunk_small": best_s, "chunk_large": best_l, "shape": sh, "ms": timed[sh]})
            return timed[sh]
        if shapes is True:
            # coordinate search over the bands, starting from the built-in shape; another engine
            # replaces the current one only if it is faster by more than TIE (ties keep the table)
            for band in shape_bands(n):
                mask = sum(band)
                cands = [(best_shape & ~mask) | b for b in band]
                if best_shape not in cands:
                    cands.insert(0, best_shape)
                best_shape = faster_than(best_shape, {c: run_shape(c) for c in cands})
        else:
            best_shape = min(shapes, key=run_shape)
    ctx.set_shape(n, best_shape)
    if cache is not None:
        save_cache({(_arch(ctx), n): (best_s, best_l, best_shape)}, cache)
    return best_s, best_l


def shape_bands(n: int):
    """Engine choices per subset-size band that differ at photon number n, as lists of shape bits (the
    first entry is the default engine): |Z| = 9, 10: 5x5 quad grid, 16x16 tiles (1, k >= 9),
    symmetric quad-tile (8, k >= 11); |Z| = 11, 12: strip / quad-tile, 16x16 tiles (2), symmetric
    quad-tile (4), from k >= 11; |Z| = 13, 14: 16x16 tiles, symmetric quad-tile on a 7x7 grid (16),
    from k >= 13."""
    k = n // 2
    bands = []
    if k >= 9:
        bands.append([0, 1] + ([8] if k >= 11 else []))
    if k >= 11:
        bands.append([0, 2, 4])
    if k >= 13:
        bands.append([0, 16])
    return bands


def shapes_for(n: int) -> Tuple[int, ...]:
    """Every combination of the per-band choices of shape_bands(n)."""
    out = [0]
    for band in shape_bands(n):
        out = [a | b for b in band for a in out]
    return tuple(out)


def save_cache(entries: Dict[tuple, Tuple[int, int]], path: pathlib.Path = DEFAULT_CACHE) -> None:
    path = pathlib.Path(path)
    data = {}
    if path.exists():
        try:
            data = json.loads(path.read_text())
        except (OSError, ValueError):
            data = {}
    for (arch, n), v in entries.items():
        e = {"chunk_small": int(v[0]), "chunk_large": int(v[1])}
        if len(v) > 2:
            e["shape"] = int(v[2])
        data[f"{arch}:{n}"] = e
    path.parent.mkdir(parents=True, exist_ok=True)
    tmp = path.with_suffix(".tmp%d" % os.getpid())
    tmp.write_text(json.dumps(data, indent=1, sort_keys=True))
    os.replace(tmp, path)


def load_cache(ctx, path: pathlib.Path = DEFAULT_CACHE) -> int:
    """Apply every cached entry for this device's arch; returns how many were applied."""
    path = pathlib.Path(path)
    if not path.exists():
        return 0
    try:
        data = json.loads(path.read_text())
    except (OSError, ValueError):
        return 0
    arch = _arch(ctx)
    k = 0
    for key, v in data.items():
        a, _, n = key.rpartition(":")
        if a == arch:
            ctx.set_tuning(int(n), int(v["chunk_small"]), int(v["chunk_large"]))
            if "shape" in v:
                ctx.set_shape(int(n), int(v["shape"]))
            k += 1
    return k


# Batch per n for the table: about 5..350 ms of work per call on one MI355X.
TABLE_BATCH = {16: 16384, 18: 16384, 20: 16384, 22: 8192, 24: 4096, 26: 2048, 28: 1024, 30: 512, 32: 256,
               34: 128, 36: 64, 38: 32, 40: 16, 42: 8, 44: 4, 46: 2}


def tune_table(ns=None, seed: int = 7700, log=None) -> Dict[int, dict]:
    """Tune every n of ``ns`` (default n = 16..46) on random complex-symmetric matrices (seed + n)
    in a fresh context each; returns {n: {chunk_small, chunk_large, shape, streams, best_ms}} -- the
    library's built-in table (kDefaultShape in the runtime) is this output."""
    import numpy as np
    import torch
    from paper_1908_10070_amd import gbs, inputs
    out = {}
    for n in (ns or sorted(TABLE_BATCH)):
        ctx = gbs.Context(0)
        A = torch.from_numpy(inputs.random_symmetric(n, TABLE_BATCH[n], np.random.default_rng(seed + n))).cuda()
        lg = []
        cs, cl = tune(ctx, n, A, reps=3 if n <= 40 else 1, cache=None, log=lg)
        # then the stream count: two (the context default) unless one is faster by more than TIE
        res = torch.empty(A.shape[0], dtype=torch.complex128, device=A.device)
        ts = {}
        for s in (2, 1):
            ctx.set_streams(s)
            ts[s] = _time_call(lambda: ctx.haf_batch(A, out=res), 3 if n <= 40 else 1)
        out[n] = {"batch": TABLE_BATCH[n], "chunk_small": cs, "chunk_large": cl, "shape": ctx.get_shape(n),
                  "streams": faster_than(2, ts), "best_ms": min(r["ms"] for r in lg)}
        if log is not None:
            log.extend(lg)
        print(f"n={n}: chunks {cs}/{cl} shape {out[n]['shape']} streams {out[n]['streams']} "
              f"({out[n]['best_ms']:.3f} ms)", flush=True)
        ctx.close()
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="autotune the launch shape for every n and print the table")
    ap.add_argument("--table", action="store_true", required=True)
    ap.add_argument("ns", nargs="*", type=int)
    a = ap.parse_args()
    print(json.dumps(tune_table(a.ns or None), indent=1))
