"""Autotuner for the merge-tile size and the segmented sort's base-case thresholds.

For a workload it times a grid of msn_tuning candidates on the GPU (median of
a few runs, HIP events on the current stream), requires every candidate to
produce exactly the bits of the default setting, and keeps the fastest.
Results are cached in a JSON file keyed by (GPU arch, library version,
operation, key type, pairs, leaf set, size bucket), so later calls of the same
shape reuse them.  Cache path: $MSN_AUTOTUNE_CACHE, else
~/.cache/msn/autotune.json.
"""
from __future__ import annotations

import json
import math
import os
import statistics
import threading

import torch

from . import _lib

_LOCK = threading.Lock()
CACHE_VERSION = 1


def cache_path() -> str:
    p = os.environ.get("MSN_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "msn", "autotune.json")


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        if data.get("version") == CACHE_VERSION:
            return data
    except (OSError, ValueError):
        pass
    return {"version": CACHE_VERSION, "entries": {}}


def _store_cache(path: str, data: dict):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(key: str, path: str | None = None):
    with _LOCK:
        return _load_cache(path or cache_path())["entries"].get(key)


def store(key: str, params: dict, path: str | None = None):
    path = path or cache_path()
    with _LOCK:
        data = _load_cache(path)
        data["entries"][key] = params
        _store_cache(path, data)


def size_bucket(n: int) -> int:
    """Sizes within a factor of two share a tuning (log2 bucket)."""
    return 0 if n <= 0 else int(math.log2(n))


def workload_key(op: str, dtype: int, pairs: bool, leaf: int, n: int, segments: int = 0,
                 arch: str | None = None) -> str:
    if arch is None:
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] \
            if torch.cuda.is_available() else "cpu"
    ver = _lib.lib().msn_version() if os.path.exists(_lib.LIB_PATH) else 0
    return (f"{arch}|v{ver}|{op}|dt{dtype}|pairs{int(pairs)}|leaf{leaf}|n2^{size_bucket(n)}"
            f"|s2^{size_bucket(segments)}")


def sort_candidates(leaf_keys: int = 8, integer_keys_only: bool = True) -> list[dict]:
    tiles = (1024, 2048, 4096) if integer_keys_only else (1024,)
    return [{"merge_tile": mt, "block_tile": bt * leaf_keys}
            for mt in (2048, 4096, 8192) for bt in tiles]


def segmented_candidates(leaf_keys: int, n_total: int, num_segments: int) -> list[dict]:
    """Grid over lane / wavefront / workgroup thresholds and grid size.

    Every candidate satisfies the C ABI's rules: 0 <= lane <= K <= ...,
    lane <= wave <= 128 K, wave <= block <= 1024 K.
    """
    k = leaf_keys
    out = []
    for lane in (1, k):
        for wave in (16 * k, 32 * k, 64 * k, 128 * k):
            for block in (256 * k, 512 * k, 1024 * k):
                if not (lane <= wave <= block):
                    continue
                for grid in (0, 1024):
                    out.append({"seg_lane_max": lane, "seg_wave_max": wave,
                                "seg_block_max": block, "seg_grid": grid})
    return out


def _time(fn, reps: int) -> float:
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def _same_bits(x: torch.Tensor, y: torch.Tensor) -> bool:
    return torch.equal(x.view(torch.int32), y.view(torch.int32))


def tune(run, candidates: list[dict], reps: int = 3):
    """Time run(tuning) for each candidate.  run returns a tuple of output
    tensors; every candidate's outputs must equal the default's bit for bit.
    Returns (best params, table of (params, ms))."""
    ref = [t.clone() for t in run(None)]
    torch.cuda.synchronize()
    table = []
    for cand in candidates:
        outs = run(cand)
        torch.cuda.synchronize()
        for r, o in zip(ref, outs):
            if not _same_bits(r, o):
                raise AssertionError(f"tuning candidate {cand} changed the result")
        ms = _time(lambda: run(cand), reps)
        table.append((cand, ms))
    best = min(table, key=lambda t: t[1])[0]
    return best, table


def tuned_sort_params(keys: torch.Tensor, *, pairs: bool, leaf, reps: int = 3,
                      force: bool = False) -> dict:
    """Cached or freshly tuned msn_tuning fields for a flat sort of `keys`."""
    from . import sort, sort_pairs

    dt = _lib.key_dtype(keys)
    lc = _lib.leaf_code(leaf)
    key = workload_key("sort", dt, pairs, lc, keys.numel())
    hit = None if force else lookup(key)
    if hit is not None:
        return hit

    def run(t):
        if pairs:
            return sort_pairs(keys, None, leaf=leaf, tuning=t)
        return (sort(keys, leaf=leaf, tuning=t),)

    k = _lib.group_keys(lc)
    best, _ = tune(run, sort_candidates(k, not pairs and dt != _lib.MSN_F32), reps)
    store(key, best)
    return best


def tuned_segmented_params(keys: torch.Tensor, offsets, *, num_segments: int, vals=None,
                           argsort=False, leaf="6To8", reps: int = 3,
                           force: bool = False) -> dict:
    """Cached or freshly tuned thresholds for a segmented sort of this shape."""
    from . import segmented_sort

    dt = _lib.key_dtype(keys)
    lc = _lib.leaf_code(leaf)
    pairs = argsort or vals is not None
    key = workload_key("segmented", dt, pairs, lc, keys.numel(), num_segments)
    hit = None if force else lookup(key)
    if hit is not None:
        return hit
    k = _lib.group_keys(lc)

    def run(t):
        out = segmented_sort(keys, offsets, vals, num_segments=num_segments, argsort=argsort,
                             leaf=leaf, tuning=t)
        return out if isinstance(out, tuple) else (out,)

    best, _ = tune(run, segmented_candidates(k, keys.numel(), num_segments), reps)
    store(key, best)
    return best
