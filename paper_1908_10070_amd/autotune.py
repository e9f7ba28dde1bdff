"""Autotuner for the work-item chunk sizes of the subset engines.

The library cuts every pattern's subset order into work items: ``chunk_small`` subsets per item
for |Z| <= 8 (the quad and one-tile engines) and ``chunk_large`` for larger subsets (tile
engines). Small chunks balance the persistent launch better; large chunks amortise the per-item
staging of the pattern matrix and the per-wave trace buffers. The best pair depends on n, on the
batch size and on the device, so it is measured:

* a coordinate search -- ``chunk_small`` over its candidates with the default ``chunk_large``,
  then ``chunk_large`` with the best ``chunk_small`` -- timing the real call (``haf_batch`` on the
  caller's matrices) with HIP events, median of a few repetitions;
* the winner goes to ``gbs_ctx_set_tuning`` and to a JSON cache keyed by (GPU arch, n), so later
  contexts load it without measuring (``load_cache``).

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
LARGE_CANDIDATES = (8, 16, 32, 64, 128)


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
         log: Optional[list] = None) -> Tuple[int, int]:
    """Measure chunk sizes for size-n hafnians of the (batch, n, n) CUDA tensor A; apply and cache them."""
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

    best_s = min(small, key=lambda cs: run(cs, d_large))
    best_l = min(large, key=lambda cl: run(best_s, cl))
    ctx.set_tuning(n, best_s, best_l)
    if cache is not None:
        save_cache({(_arch(ctx), n): (best_s, best_l)}, cache)
    return best_s, best_l


def save_cache(entries: Dict[tuple, Tuple[int, int]], path: pathlib.Path = DEFAULT_CACHE) -> None:
    path = pathlib.Path(path)
    data = {}
    if path.exists():
        try:
            data = json.loads(path.read_text())
        except (OSError, ValueError):
            data = {}
    for (arch, n), (cs, cl) in entries.items():
        data[f"{arch}:{n}"] = {"chunk_small": int(cs), "chunk_large": int(cl)}
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
            k += 1
    return k
