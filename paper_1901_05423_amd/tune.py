"""Autotuner for the guide-table size, the build tile and the descent form.

The sampled indices do not depend on the number of guide cells m, nor on the
build tile; only speed does.  The paper leaves m to the user: whatever
memory can be spared, or a size that grows with n (Sec. 3).  More cells let more samples
finish in one cell record, but a larger table costs build bytes and cache
capacity.  Batches of many small distributions build faster in 1024-element
tiles, one large distribution in 2048-element ones.  `best_cell_ratio` and
`best_batched` time the candidates on the caller's own data and shape, and
remember the winner in a JSON cache keyed by the device architecture and the
size bucket (log2 of n and of S/n).

Environment: RTF_CELL_RATIO forces a ratio; RTF_TUNE_CACHE names the cache
file (default ~/.cache/rtforest/tune.json).
"""
from __future__ import annotations

import json
import math
import os

CANDIDATES = (0.125, 0.25, 0.5, 1.0, 2.0)


def cache_path() -> str:
    return os.environ.get("RTF_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "rtforest", "tune.json"))


def bucket_key(arch: str, op: str, n: int, samples: int) -> str:
    ln = int(round(math.log2(max(n, 1))))
    ls = int(round(math.log2(max(samples, 1) / max(n, 1)))) if samples else -99
    return f"{arch}|{op}|n2^{ln}|s/n2^{ls}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(entries: dict, path: str | None = None) -> bool:
    """Write the cache; an unwritable location only loses the cache."""
    path = path or cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(entries, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
        return True
    except OSError:
        return False


def forced_ratio():
    v = os.environ.get("RTF_CELL_RATIO")
    return float(v) if v else None


def device_arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _time_ms(fn, reps=5):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def best_cell_ratio(w, u, candidates=CANDIDATES, use_cache=True, reps=5, with_times=False):
    """Cell ratio m/n with the fastest build + sample for uint32 weights `w`
    (one distribution) and uniforms `u`, both device tensors.  With
    ``with_times`` also the measured ms per candidate ({} when the ratio came
    from the environment or the cache)."""
    forced = forced_ratio()
    if forced is not None:
        return (forced, {}) if with_times else forced
    from . import build, sample
    key = bucket_key(device_arch(), "single", w.numel(), u.numel())
    cache = load_cache() if use_cache else {}
    if key in cache:
        r = float(cache[key]["ratio"])
        return (r, {}) if with_times else r
    n = w.numel()
    times = {}
    for r in candidates:
        m = max(1, int(round(r * n)))
        holder = {}

        def step():
            holder["f"] = build(w, m)
            sample(holder["f"], u)

        times[r] = _time_ms(step, reps)
    best = min(times, key=times.get)
    if use_cache:
        cache[key] = {"ratio": best, "ms": {str(k): v for k, v in times.items()}}
        store_cache(cache)
    return (best, {str(k): v for k, v in times.items()}) if with_times else best


BATCH_CANDIDATES = tuple((r, c) for r in (0.125, 0.25, 0.5, 1.0) for c in (False, True))
TILES = (2048, 1024)


def best_tile(run, tiles=TILES, reps=5):
    """(tile, times): the build tile for which run(tile), a whole build +
    sample enqueued on the current stream, is fastest; times maps each tile
    to ms."""
    times = {int(tl): _time_ms(lambda: run(tl), reps) for tl in tiles}
    return min(times, key=times.get), {str(k): v for k, v in times.items()}


def best_batched(v, u, elem_off, sample_off, candidates=BATCH_CANDIDATES, use_cache=True,
                 reps=5, key_extra="", tiles=TILES):
    """(ratio, collapsed, tile, times) with the fastest quantise + build (+
    collapse) + sample of the batch: v float32 weights, u uint64 uniforms,
    elem_off and sample_off int64 device offsets (D+1).  The ratio and the
    descent form are chosen first with the default tile, then the tile for
    them.  times maps "ratio|collapsed|tile" to ms ({} when the choice came
    from the environment or the cache)."""
    forced = forced_ratio()
    if forced is not None:
        return forced, False, tiles[0], {}
    from . import cells_like
    from .plan import BatchedPlan
    D = elem_off.numel() - 1
    n, S = v.numel(), u.numel()
    key = bucket_key(device_arch(), f"batched|D2^{int(round(math.log2(max(D, 1))))}{key_extra}",
                     n, S)
    cache = load_cache() if use_cache else {}
    if key in cache:
        e = cache[key]
        return float(e["ratio"]), bool(e["collapsed"]), int(e.get("tile", tiles[0])), {}
    times = {}

    def run(r, c, tile):
        co = cells_like(elem_off, r)
        plan = BatchedPlan(elem_off, co, sample_off, n, int(co[-1].item()), S, collapsed=c,
                           tile=tile)
        times[f"{r}|{int(c)}|{tile}"] = _time_ms(lambda: plan.run(v, u), reps)
        del plan

    for r, c in candidates:
        run(r, c, tiles[0])
    best = min(times, key=times.get)
    r, c, _ = best.split("|")
    for tile in tiles[1:]:
        run(float(r), bool(int(c)), tile)
    best = min(times, key=times.get)
    r, c, tile = best.split("|")
    if use_cache:
        cache[key] = {"ratio": float(r), "collapsed": bool(int(c)), "tile": int(tile), "ms": times}
        store_cache(cache)
    return float(r), bool(int(c)), int(tile), times
