"""Throughput of the network-leaf GPU merge sort on one MI355X.

Default workload: 2^28 uint32 keys, uniform random over the full range
(seed 0), msn_sort_keys with the 6-to-8 leaf set; sorted and nearly sorted
variants are timed too.  Prints ONE JSON line:
  value        whole-sort Gkeys/s (inputs resident in HBM when timing starts)
  roofline     the dominant kernel (the global merge pass) against HBM peak:
               algorithmic bytes per launch (8 B per key: one read, one write)
               over its average launch time, from HIP events recorded around
               each launch on the launching stream during the timed steps
  cpu_baseline the CPU oracle (Algorithm 1, 6-to-8, one thread) on a bounded
               sample of the same input

Other workloads (--workload pairs|segmented|rows|small|leaves|copy) print their own line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, 8 TB/s
METRIC = "Gkeys/s + % HBM roofline, 2^28 uint32 keys (random/sorted/nearly-sorted), 1 GPU"
T_RUN = 8192                    # run length of the reference binary schedule


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def reference_schedule_bytes(n: int, width: int) -> int:
    """Bytes per key of the binary merge-sort schedule: one read and one write
    per sweep, 1 + ceil(log2(n / 8192)) sweeps."""
    runs = -(-n // T_RUN)
    passes = max(0, int(np.ceil(np.log2(runs)))) if runs > 1 else 0
    return 2 * width * (1 + passes)


def kernel_source_hash(kernel_header: str) -> str:
    """First 16 hex digits of sha256(kernel header + device.hpp + internal.hpp)."""
    import hashlib

    csrc = os.path.join(ROOT, "paper_2503_05934_amd", "csrc")
    data = b"".join(open(os.path.join(csrc, f), "rb").read()
                    for f in (kernel_header, "device.hpp", "internal.hpp"))
    return hashlib.sha256(data).hexdigest()[:16]


def load_traffic(kernel_file: str, kernel_header: str):
    """Per-launch HBM bytes of a merge kernel from the committed rocprofv3 PMC
    summary, if it was taken on the current kernel source (the kernel's header
    + device.hpp + internal.hpp); None otherwise."""
    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256_16") != kernel_source_hash(kernel_header):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_steps(fn, steps: int, warmup: int):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall


def check_sorted_u32(out, inp) -> bool:
    import torch

    o = out.view(torch.int32) ^ torch.tensor(-2**31, dtype=torch.int32, device=out.device)
    ok = bool((o[1:] >= o[:-1]).all().item())
    s_in = inp.view(torch.int32).to(torch.int64).sum().item()
    s_out = out.view(torch.int32).to(torch.int64).sum().item()
    return ok and s_in == s_out


def cpu_baseline_start(keys_np: np.ndarray, sample_n: int):
    """Starts the CPU oracle on the first sample_n keys in two threads: the
    paper's Algorithm 1 with 6-to-8 networks, and the classical merge sort
    (its empty network set, Eq. 1's baseline).  Each sort is single-threaded;
    ctypes releases the GIL, so they run while the GPU workloads go on.
    Returns a function that waits and builds the cpu_baseline record."""
    import threading

    import oracle

    orc = oracle.load()
    sample = keys_np[:sample_n]
    times = {}

    def run(config):
        t0 = time.perf_counter()
        orc.sort(sample, dtype="u32", algo="ms", config=config)
        times[config] = time.perf_counter() - t0

    threads = [threading.Thread(target=run, args=(c,), daemon=True)
               for c in ("6To8", "Classical")]
    for t in threads:
        t.start()

    def finish():
        for t in threads:
            t.join()
        t1, t0 = times["6To8"], times["Classical"]
        whole = sample_n == keys_np.shape[0]
        what = ("the whole" if whole else f"the first 2^{int(np.log2(sample_n))} keys of the")
        return {
            "value": sample_n / t1 / 1e9,
            "unit": "Gkeys/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"{what} random 2^28 uint32 input; oracle Algorithm 1 with 6-to-8 "
                      f"networks, one thread, {t1:.2f} s; the classical merge sort ran at the "
                      f"same time on a second thread, {t0:.2f} s, while the GPU workloads ran",
            "classical": {"value": sample_n / t0 / 1e9, "seconds": t0},
            "eq1_speedup": t0 / t1,
            "host_cpu": _cpu_model(),
            "host_threads": os.cpu_count(),
        }

    return finish


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _graph_time(fn, steps, warmup):
    """fn captured once in a HIP graph and replayed: (ms per replay, wall s)."""
    import torch

    fn()
    torch.cuda.synchronize()
    gstream = torch.cuda.Stream()
    gstream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gstream):
        fn()
    ms, wall = time_steps(graph.replay, steps, warmup)
    del graph
    return ms, wall


def copy_ceiling(steps: int, warmup: int, words: int = 1 << 29):
    """The library's own 16-byte copy kernel (msn_copy_words) over 2 GiB:
    the rate a read-once write-once sweep reaches on this device."""
    import torch

    from paper_2503_05934_amd import _lib

    dev = torch.device("cuda:0")
    src = torch.arange(words, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    L = _lib.lib()

    def run():
        # the current stream: the capturing stream while a graph is recorded
        _lib.check("msn_copy_words", L.msn_copy_words(_lib.ptr(src), _lib.ptr(dst), words,
                                                      _lib.stream_handle(dev)))

    ms, _ = _graph_time(run, steps, warmup)
    if not torch.equal(src, dst):
        raise SystemExit("[bench] copy check failed")
    gbps = 8.0 * words / (ms / 1e3) / 1e9
    del src, dst
    return {"gbps": gbps, "frac_of_peak": gbps / HBM_PEAK_GBPS, "ms": ms,
            "bytes_per_launch": 8 * words,
            "kernel": "k_copy_words (msn_copy_words: 2 GiB read + 2 GiB written, 16-byte "
                      "accesses, graph replay)"}


def bench_keys(args):
    import torch

    import paper_2503_05934_amd as msn
    from paper_2503_05934_amd import _lib, workloads

    dev = torch.device("cuda:0")
    n = args.n
    leaf = args.leaf
    tuning = {k: v for k, v in (("merge_tile", args.merge_tile),
                                ("block_tile", args.block_tile),
                                ("merge_ways", args.merge_ways),
                                ("merge4_kpt", args.merge4_kpt)) if v}
    plan = msn.SortPlan(n, torch.uint32, dev, leaf=leaf, tuning=tuning or None)
    results = {}
    roof = None
    cpu_finish = None
    qws = None
    for dist in args.dists:
        log(f"[bench] generating {n} uint32 keys, {dist}")
        x_np = workloads.keys(n, dist, "u32", seed=0)
        if dist == "random" and not args.no_cpu:
            log(f"[bench] CPU oracle baseline on 2^{int(np.log2(args.cpu_sample))} keys "
                "(two threads, in the background)")
            cpu_finish = cpu_baseline_start(x_np, args.cpu_sample)
        x = torch.from_numpy(x_np).to(dev)
        del x_np
        steps = args.steps if dist == "random" else max(2, args.steps // 4)
        log(f"[bench] {dist}: warmup {args.warmup}, timing {steps} steps")
        stats = {}
        if dist == "random" and not args.graph_only:
            # eager steps with HIP events around every launch (per-kernel times)
            for _ in range(args.warmup):
                plan.run(x)
            torch.cuda.synchronize()
            _lib.timing_enable(64 * (steps + 1))
            ms_eager, wall = time_steps(lambda: plan.run(x), steps, 0)
            stats = _lib.timing_read()
            _lib.timing_disable()
        elif not args.graph_only:
            ms_eager, wall = time_steps(lambda: plan.run(x), steps, args.warmup)
        else:
            ms_eager = None
        # the same sort captured once in a HIP graph and replayed (no launch gaps)
        if args.eager:
            ms = ms_eager
        else:
            ms, wall = _graph_time(lambda: plan.run(x), steps, args.warmup)
        ok = check_sorted_u32(plan.out, x)
        if not ok:
            raise SystemExit(f"[bench] output check failed for {dist}")
        results[dist] = {"gkeys_per_s": n / (ms / 1e3) / 1e9, "ms_per_step": ms, "steps": steps,
                         "wall_s": wall, "eager_ms_per_step": ms_eager}
        log(f"[bench] {dist}: {ms:.3f} ms/step, {results[dist]['gkeys_per_s']:.2f} Gkeys/s")
        if dist == "random":
            # the dominant merge kernel: four-way passes if the plan used them
            mkind = max((k for k in ("merge", "merge4") if k in stats),
                        key=lambda k: stats[k]["total_ms"], default=None)
            m = stats.get(mkind) if mkind else None
            if m:
                avg_s = m["avg_ms"] / 1e3
                bytes_per_launch = 8.0 * n
                achieved = bytes_per_launch / avg_s / 1e9
                traffic = (load_traffic("k_merge4_2p28_u32_traffic.md", "merge4.hpp")
                           if mkind == "merge4" else
                           load_traffic("k_merge_keys_2p28_u32_traffic.md", "merge_keys.hpp"))
                roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                        "kernel": ("k_merge4 (four-way merge pass)" if mkind == "merge4"
                                   else "k_merge_keys (binary merge-path pass)"),
                        "avg_launch_ms": m["avg_ms"], "launches": m["launches"],
                        "algorithmic_bytes_per_launch": bytes_per_launch,
                        "timing": "HIP events around each launch of the timed eager steps"}
            results[dist]["kernels_ms_per_step"] = {
                k: v["total_ms"] / steps for k, v in stats.items()}
        if not args.no_quick and leaf != "classical":
            # the paper's Algorithm 2 on the same input: quick sort, network leaves
            if qws is None:
                qws = torch.empty(_lib.quick_workspace_bytes(n, _lib.MSN_U32), dtype=torch.uint8,
                                  device=dev)
            qout = torch.empty_like(x)
            qms, _ = _graph_time(lambda: msn.quick_sort(x, leaf=leaf, out=qout, workspace=qws),
                                 steps, args.warmup)
            if not torch.equal(qout, plan.out):
                raise SystemExit(f"[bench] quick sort disagrees with the merge sort ({dist})")
            results[dist]["quick"] = {"gkeys_per_s": n / (qms / 1e3) / 1e9, "ms_per_step": qms}
            log(f"[bench] {dist}: quick sort {qms:.3f} ms/step")
            del qout
        del x
    del qws
    head = results[args.dists[0]]
    sched = reference_schedule_bytes(n, 4)
    moved = 8 * (1 + plan_passes(n, leaf, plan))
    out = {
        "metric": METRIC,
        "value": head["gkeys_per_s"],
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"sort_keys: 2^{int(np.log2(n))} uint32 keys, uniform random "
                               f"over [0, 2^32), seed 0, {leaf} leaves",
                   "n": n, "leaf": leaf, "dist": args.dists[0],
                   "merge_tile": args.merge_tile or 8192,
                   "block_tile": args.block_tile or 2048 * _lib.GROUP_KEYS[leaf]},
        "roofline": roof,
        "hbm_schedule": {"bytes_per_key": sched,
                         "implied_gkeys_at_peak": HBM_PEAK_GBPS / sched,
                         "frac": head["gkeys_per_s"] / (HBM_PEAK_GBPS / sched)},
        "whole_sort": {"bytes_per_key_moved": moved,
                       "gbps": head["gkeys_per_s"] * moved,
                       "frac": head["gkeys_per_s"] * moved / HBM_PEAK_GBPS,
                       "how": "the sweeps this build runs (first sweep + global passes), "
                              "8 B per key each, over the whole sort's time"},
        "timing": "graph replay of one msn_sort_keys call per step" if not args.eager
                  else "eager msn_sort_keys call per step",
        "eager_ms_per_step": head["eager_ms_per_step"],
        "by_distribution": {d: {"gkeys_per_s": r["gkeys_per_s"], "ms_per_step": r["ms_per_step"],
                                "eager_ms_per_step": r["eager_ms_per_step"]}
                            for d, r in results.items()},
        "kernels_ms_per_step": results.get("random", {}).get("kernels_ms_per_step"),
    }
    if any("quick" in r for r in results.values()):
        out["quick_sort"] = {d: r["quick"] for d, r in results.items() if "quick" in r}
    if not args.no_copy:
        log("[bench] copy ceiling (msn_copy_words, 2 GiB)")
        out["copy_ceiling"] = copy_ceiling(args.steps, args.warmup)
        if roof:
            roof["frac_of_copy_ceiling"] = roof["achieved"] / out["copy_ceiling"]["gbps"]
    if not args.no_extras:
        out.update(side_workloads(args))
    if cpu_finish is not None:
        log("[bench] waiting for the CPU oracle baseline")
        out["cpu_baseline"] = cpu_finish()
    return out


def plan_passes(n: int, leaf: str, plan) -> int:
    """Global merge passes of the default plan: four-way while at least three
    runs remain, then binary (first-sweep runs of 2048 x leaf keys)."""
    from paper_2503_05934_amd import _lib

    runs = -(-n // (2048 * _lib.GROUP_KEYS[leaf]))
    p = 0
    while runs > 1:
        runs = -(-runs // (4 if runs >= 3 else 2))
        p += 1
    return p


def side_workloads(args):
    """The other workloads, condensed into keys of the default line."""
    import copy

    import torch

    extra = {}
    a = copy.copy(args)
    a.steps, a.warmup = max(4, args.steps // 2), 2
    for name, fn in (("pairs", bench_pairs), ("segmented", bench_segmented),
                     ("rows", bench_rows)):
        log(f"[bench] side workload: {name}")
        r = fn(a)
        keep = {k: r[k] for k in ("metric", "value", "unit", "ms_per_step", "roofline",
                                  "config", "per_array_baseline", "speedup_vs_per_array",
                                  "backward", "eager_ms_per_step", "kernels_ms_per_step")
                if k in r}
        extra[name] = keep
        torch.cuda.empty_cache()
    return extra


def _roof(stats, kind, bytes_per_launch_fn, peak=HBM_PEAK_GBPS):
    m = stats.get(kind)
    if not m:
        return None
    avg_s = m["avg_ms"] / 1e3
    per_launch = bytes_per_launch_fn(m)
    achieved = per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": peak, "unit": "GB/s",
            "frac": achieved / peak, "traffic": None, "kernel": kind,
            "avg_launch_ms": m["avg_ms"], "launches": m["launches"],
            "algorithmic_bytes_per_launch": per_launch}


def _timed_with_kernel_stats(fn, steps, warmup):
    import torch

    from paper_2503_05934_amd import _lib

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    _lib.timing_enable(256 * (steps + 1))
    ms, wall = time_steps(fn, steps, 0)
    stats = _lib.timing_read()
    _lib.timing_disable()
    return ms, wall, stats


def bench_pairs(args):
    """Stable key-value sort: 2^28 uint32 keys from [0, 2^16), payload = index."""
    import torch

    import paper_2503_05934_amd as msn
    from paper_2503_05934_amd import workloads

    dev = torch.device("cuda:0")
    n = args.n
    log(f"[bench] generating {n} pairs (keys < 2^16, payload = index)")
    k_np, v_np = workloads.pairs(n, seed=0)
    k = torch.from_numpy(k_np).to(dev)
    v = torch.from_numpy(v_np).to(dev)
    plan = msn.SortPlan(n, torch.uint32, dev, pairs=True, leaf=args.leaf)
    ms, wall, stats = _timed_with_kernel_stats(lambda: plan.run(k, v), args.steps, args.warmup)
    ko, vo = plan.out, plan.out_vals
    # stable and a permutation: keys non-decreasing, payload rising inside equal keys,
    # every index once, and keys_out[i] == keys_in[vals_out[i]]
    ki = ko.view(torch.int32).to(torch.int64)
    vi = vo.view(torch.int32).to(torch.int64)
    ok = bool((ki[1:] >= ki[:-1]).all())
    ok &= bool(((ki[1:] > ki[:-1]) | (vi[1:] > vi[:-1])).all())
    ok &= bool((torch.bincount(vi, minlength=n) == 1).all())
    ok &= bool(torch.equal(k.view(torch.int32)[vi], ko.view(torch.int32)))
    if not ok:
        raise SystemExit("[bench] pairs output check failed")
    # the dominant merge kernel: the four-way passes, unless the plan had none
    mkind = max((kk for kk in ("merge", "merge4_pairs") if kk in stats),
                key=lambda kk: stats[kk]["total_ms"], default="merge")
    pairs_roof = _roof(stats, mkind, lambda m: 16.0 * n)
    if pairs_roof and mkind == "merge4_pairs":
        pairs_roof["traffic"] = load_traffic("k_merge4_pairs_2p28_u32_traffic.md", "merge4.hpp")
        pairs_roof["kernel"] = "k_merge4_pairs (four-way key-value merge pass)"
    return {
        "metric": "Gkeys/s, 2^28 uint32 key-value pairs (keys < 2^16, payload = index), 1 GPU",
        "value": n / (ms / 1e3) / 1e9, "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"sort_pairs: 2^{int(np.log2(n))} uint32 keys uniform in "
                               "[0, 2^16), uint32 payload = index, stable", "n": n,
                   "leaf": args.leaf},
        "roofline": pairs_roof,
        "hbm_schedule": {"bytes_per_key": reference_schedule_bytes(n, 8),
                         "implied_gkeys_at_peak": HBM_PEAK_GBPS / reference_schedule_bytes(n, 8)},
        "kernels_ms_per_step": {kk: vv["total_ms"] / args.steps for kk, vv in stats.items()},
        "checked": "stable permutation (O(n) invariants on the GPU)",
    }


def bench_segmented(args):
    """100,000 int32 arrays, lengths log-uniform in [3, 65536], 30 % presorted,
    one graph-captured segmented sort vs one msn_sort_keys launch per array."""
    import ctypes

    import torch

    import paper_2503_05934_amd as msn
    from paper_2503_05934_amd import _lib, workloads

    dev = torch.device("cuda:0")
    S = args.segments
    log(f"[bench] generating {S} segments")
    x_np, off_np, _ = workloads.segments(S, seed=0)
    n = x_np.shape[0]
    x = torch.from_numpy(x_np).to(dev)
    off = torch.from_numpy(off_np).to(dev)
    tuning = None
    if not args.no_autotune:
        from paper_2503_05934_amd import autotune

        log("[bench] autotuning segmented thresholds")
        tuning = autotune.tuned_segmented_params(x, off, num_segments=S, leaf=args.leaf,
                                                 force=args.retune)
    out = torch.empty_like(x)
    ws = torch.empty(_lib.segmented_workspace_bytes(n, S, 1, False), dtype=torch.uint8,
                     device=dev)
    run = lambda: msn.segmented_sort(x, off, leaf=args.leaf, tuning=tuning, out_keys=out,
                                     workspace=ws)
    run()
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        run()
    ms, wall = time_steps(graph.replay, args.steps, args.warmup)
    ms_eager, _, stats = _timed_with_kernel_stats(run, args.steps, 1)
    # per-segment order check on the GPU: out non-decreasing except across segment starts
    o = out.to(torch.int64)
    starts = torch.zeros(n, dtype=torch.bool, device=dev)
    starts[off[:-1].to(torch.int64)[off[:-1].to(torch.int64) < n]] = True
    okd = (o[1:] >= o[:-1]) | starts[1:]
    ok = bool(okd.all()) and x.to(torch.int64).sum().item() == o.sum().item()
    if not ok:
        raise SystemExit("[bench] segmented output check failed")
    if args.no_per_array:
        base_ms = base_wall = None
    else:
        base_ms, base_wall = _per_array_baseline(x, off_np, out, args)
    # the dominant kernel: the block sort of every tile of the segments that
    # take the tiled path (longer than seg_block_max, at most 8 tiles)
    lens = (off_np[1:] - off_np[:-1]).astype(np.int64)
    kk_ = _lib.GROUP_KEYS[args.leaf]
    bmax = (tuning or {}).get("seg_block_max") or 1024 * kk_
    tiled = int(lens[(lens > bmax) & (lens <= 8 * 1024 * kk_)].sum())
    seg_roof = _roof(stats, "seg_tile_sort", lambda m: 8.0 * tiled) if tiled else None
    if seg_roof:
        seg_roof["kernel"] = "k_seg_tile_sort (every tile of the tiled segments, one launch)"
    return {
        "metric": "Gkeys/s, batched segmented sort: 100,000 int32 arrays, lengths log-uniform "
                  "in [3, 65536], 30% presorted, 1 GPU",
        "value": n / (ms / 1e3) / 1e9, "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": "segmented_sort, one hipGraph replay per step", "segments": S,
                   "keys": n, "leaf": args.leaf, "tuning": tuning},
        "eager_ms_per_step": ms_eager,
        "per_array_baseline": None if base_ms is None else {
            "ms": base_ms, "wall_s": base_wall, "gkeys_per_s": n / (base_ms / 1e3) / 1e9,
            "how": "one msn_sort_keys call per segment, eager, same GPU"},
        "speedup_vs_per_array": None if base_ms is None else base_ms / ms,
        "roofline": seg_roof,
        "kernels_ms_per_step": {kk: vv["total_ms"] / args.steps for kk, vv in stats.items()},
    }


def _per_array_baseline(x, off_np, out, args):
    """The batch sorted by one msn_sort_keys call per array (eager, same GPU);
    returns (GPU ms, wall s) and checks the result against the batched sort."""
    import ctypes

    import torch

    from paper_2503_05934_amd import _lib

    log("[bench] per-array baseline (one msn_sort_keys call per segment)")
    dev = x.device
    S = off_np.shape[0] - 1
    L = _lib.lib()
    wsb = _lib.sort_workspace_bytes(int((off_np[1:] - off_np[:-1]).max()), 1, False)
    ws2 = torch.empty(wsb, dtype=torch.uint8, device=dev)
    out2 = torch.empty_like(x)
    st = _lib.stream_handle(dev)
    base_in, base_out = x.data_ptr(), out2.data_ptr()
    offs = off_np.astype(np.int64)
    lc = _lib.leaf_code(args.leaf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for s_ in range(S):
        a, b = int(offs[s_]), int(offs[s_ + 1])
        rc = L.msn_sort_keys(ctypes.c_void_p(base_in + 4 * a), ctypes.c_void_p(base_out + 4 * a),
                             b - a, 1, lc, None, ctypes.c_void_p(ws2.data_ptr()), wsb, st)
        if rc:
            raise SystemExit(f"[bench] msn_sort_keys failed: {rc}")
    e1.record()
    torch.cuda.synchronize()
    base_ms = e0.elapsed_time(e1)
    base_wall = time.perf_counter() - t0
    if not torch.equal(out, out2):
        raise SystemExit("[bench] per-array baseline disagrees with the segmented sort")
    return base_ms, base_wall


def bench_rows(args):
    """4096 x 8192 fp32 rows: stable row sort (values + int32 perm) and the
    backward scatter, timed separately."""
    import torch

    import paper_2503_05934_amd as msn
    from paper_2503_05934_amd import workloads

    dev = torch.device("cuda:0")
    R, C = args.rows, args.cols
    log(f"[bench] generating {R}x{C} fp32 rows ({args.variant})")
    x_np, g_np, redraws = workloads.rows(R, C, variant=args.variant, seed=0)
    x = torch.from_numpy(x_np).to(dev)
    g = torch.from_numpy(g_np).to(dev)
    vals, perm = msn.sort_rows(x, leaf=args.leaf)
    fwd = lambda: msn.sort_rows(x, leaf=args.leaf)
    ms_f, _, st_f = _timed_with_kernel_stats(fwd, args.steps, args.warmup)
    out = torch.empty_like(g)
    bwd = lambda: msn.sort_backward(g, perm, out=out)
    ms_b, _, st_b = _timed_with_kernel_stats(bwd, args.steps, args.warmup)
    ne = R * C
    ok = bool(torch.equal(x.gather(1, perm.to(torch.int64)).view(torch.int32),
                          vals.view(torch.int32)))
    ok &= bool(torch.equal(out.gather(1, perm.to(torch.int64)), g))
    if not ok:
        raise SystemExit("[bench] rows output check failed")
    return {
        "metric": "Gelem/s, differentiable fp32 row sort 4096 x 8192 (forward values+perm, "
                  "backward scatter), 1 GPU",
        "value": ne / (ms_f / 1e3) / 1e9, "unit": "Gelem/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_f, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sort_rows + sort_backward, {R}x{C} fp32 Normal(0,1) "
                               f"{args.variant}", "rows": R, "cols": C, "redraws": redraws,
                   "leaf": args.leaf},
        "backward": {"ms": ms_b, "gelem_per_s": ne / (ms_b / 1e3) / 1e9,
                     "roofline": _roof(st_b, "backward", lambda m: 12.0 * ne)},
        "roofline": _roof(st_f, "segmented", lambda m: 12.0 * ne),
        "kernels_ms_per_step": {kk: vv["total_ms"] / args.steps for kk, vv in st_f.items()},
    }


def bench_small(args):
    """10,000 and 1,000,000 int32 keys (three distributions), both leaf sets;
    one graph replay per timed step.  These inputs fit in the 256 MB
    Infinity Cache, so the numbers are cache-resident."""
    import torch

    import paper_2503_05934_amd as msn
    from paper_2503_05934_amd import workloads

    dev = torch.device("cuda:0")
    table = {}
    for n, dists in ((10_000, ["random"]), (1_000_000, list(workloads.DISTRIBUTIONS))):
        for dist in dists:
            x = torch.from_numpy(workloads.keys(n, dist, "i32", seed=0)).to(dev)
            for leaf in ("6To8", "3To5"):
                plan = msn.SortPlan(n, torch.int32, dev, leaf=leaf)
                plan.run(x)
                torch.cuda.synchronize()
                s = torch.cuda.Stream()
                s.wait_stream(torch.cuda.current_stream())
                gph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(gph, stream=s):
                    plan.run(x)
                ms, _ = time_steps(gph.replay, max(args.steps, 20), args.warmup)
                table[f"n={n} {dist} {leaf}"] = {"us": ms * 1e3,
                                                 "gkeys_per_s": n / (ms / 1e3) / 1e9}
                log(f"[bench] n={n} {dist} {leaf}: {ms * 1e3:.1f} us")
    head = table["n=1000000 random 6To8"]
    return {
        "metric": "Gkeys/s, 1,000,000 int32 keys (and 10,000), 6-to-8 vs 3-to-5 leaves, 1 GPU",
        "value": head["gkeys_per_s"], "unit": "Gkeys/s", "n_gpus": 1,
        "steps": max(args.steps, 20), "warmup": args.warmup, "ms_per_step": head["us"] / 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": "sort_keys 1e6 int32 random (cache-resident), graph replay"},
        "table": table,
    }


def bench_leaves(args):
    """The paper's measurements (Figs. 1-3 for merge sort, 4-6 for quick sort)
    replayed on the GPU for every network set of Table 3: the speedup of each
    set over the same sort with no network at all (merges from single keys;
    for the quick sort, block-sort leaves that merge from single keys),
    Eq. 1: t_classical / t_set, over the paper's sizes (10,000 to 1,000,000
    int32 keys) and 2^28 uint32 keys, for random, sorted and nearly sorted
    inputs.  One graph replay per timed step; inputs up to 1,000,000 keys fit
    in the Infinity Cache, so those numbers are cache-resident."""
    import torch

    import paper_2503_05934_amd as msn
    from paper_2503_05934_amd import _lib, workloads

    dev = torch.device("cuda:0")
    sizes = [10_000, 25_000, 50_000, 100_000, 250_000, 500_000, 1_000_000, 1 << 28]
    sets = ["classical", "6To8", "3To5", "PowerOf2", "Even", "Odd", "3", "3To4", "3To8",
            "VarSort3", "VarSort4", "VarSort5"]
    table = {}
    for n in sizes:
        dtype, tdt = ("u32", torch.uint32) if n == 1 << 28 else ("i32", torch.int32)
        steps = max(args.steps, 20) if n < 1 << 28 else max(2, args.steps // 4)
        qws = torch.empty(_lib.quick_workspace_bytes(n, _lib.key_dtype(torch.empty(0, dtype=tdt))),
                          dtype=torch.uint8, device=dev)
        for dist in workloads.DISTRIBUTIONS:
            x = torch.from_numpy(workloads.keys(n, dist, dtype, seed=0)).to(dev)
            ms_row, qs_row = {}, {}
            ref = None
            for leaf in sets:
                plan = msn.SortPlan(n, tdt, dev, leaf=leaf)
                ms, _ = _graph_time(lambda: plan.run(x), steps, args.warmup)
                if ref is None:
                    ref = plan.out.clone()
                elif not torch.equal(plan.out, ref):
                    raise SystemExit(f"[bench] {leaf} merge sort output differs")
                ms_row[leaf] = {"us": ms * 1e3}
                del plan
                qout = torch.empty_like(x)
                qms, _ = _graph_time(lambda: msn.quick_sort(x, leaf=leaf, out=qout, workspace=qws),
                                     steps, args.warmup)
                if not torch.equal(qout, ref):
                    raise SystemExit(f"[bench] {leaf} quick sort output differs")
                qs_row[leaf] = {"us": qms * 1e3}
                del qout
            for row in (ms_row, qs_row):
                for leaf in sets:
                    row[leaf]["speedup"] = row["classical"]["us"] / row[leaf]["us"]
            table[f"n={n} {dist}"] = {"merge_sort": ms_row, "quick_sort": qs_row}
            log(f"[bench] n={n} {dist}: merge classical {ms_row['classical']['us']:.1f} us, "
                + " ".join(f"{l} x{ms_row[l]['speedup']:.2f}" for l in sets[1:])
                + f"; quick classical {qs_row['classical']['us']:.1f} us, "
                + " ".join(f"{l} x{qs_row[l]['speedup']:.2f}" for l in sets[1:]))
            del x
        del qws
    head = table[f"n={1 << 28} random"]["merge_sort"]
    return {
        "metric": "speedup of 6-to-8 network leaves over the network-free merge sort (Eq. 1), "
                  "2^28 uint32 keys random, 1 GPU",
        "value": head["6To8"]["speedup"], "unit": "x", "n_gpus": 1,
        "steps": max(2, args.steps // 4), "warmup": args.warmup,
        "ms_per_step": head["6To8"]["us"] / 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "sort_keys and quick sort under every Table 3 set and with no "
                               "networks; 10,000 to 1,000,000 int32 keys and 2^28 uint32 keys; "
                               "random, sorted, nearly sorted; graph replay"},
        "table": table,
    }


def bench_copy(args):
    """The library's own copy kernel (msn_copy_words) over n uint32 words:
    the achievable read+write bandwidth, and the kernel of known size that
    calibrates the HBM byte counters (FETCH_SIZE / WRITE_SIZE): every call
    reads and writes 4n bytes."""
    import torch

    from paper_2503_05934_amd import _lib

    dev = torch.device("cuda:0")
    n = args.n
    x = torch.arange(n, dtype=torch.int32, device=dev)
    y = torch.empty_like(x)
    L = _lib.lib()

    def run():
        _lib.check("msn_copy_words", L.msn_copy_words(_lib.ptr(x), _lib.ptr(y), n,
                                                      _lib.stream_handle(dev)))

    ms, _ = time_steps(run, args.steps, args.warmup)
    if not torch.equal(x, y):
        raise SystemExit("[bench] copy check failed")
    gbps = 8.0 * n / (ms / 1e3) / 1e9
    return {"metric": f"GB/s, msn_copy_words of {n} uint32 words (read + write)", "value": gbps,
            "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": f"msn_copy_words of {n} int32 words, eager", "n": n,
                       "calls": args.steps + args.warmup, "bytes_read": 4 * n,
                       "bytes_written": 4 * n},
            "frac_of_peak": gbps / HBM_PEAK_GBPS}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="keys",
                    choices=["keys", "pairs", "segmented", "rows", "small", "leaves", "copy"])
    ap.add_argument("--n", type=int, default=1 << 28)
    ap.add_argument("--leaf", default="6To8",
                    choices=["6To8", "3To5", "classical", "PowerOf2", "Even", "Odd", "3", "3To4",
                             "3To8", "VarSort3", "VarSort4", "VarSort5"])
    ap.add_argument("--merge-tile", type=int, default=0)
    ap.add_argument("--block-tile", type=int, default=0)
    ap.add_argument("--merge-ways", type=int, default=0)
    ap.add_argument("--merge4-kpt", type=int, default=0,
                    help="keys per thread of the four-way merge kernel (16 or 32)")
    ap.add_argument("--dists", default="random,sorted,nearly")
    ap.add_argument("--cpu-sample", type=int, default=1 << 28)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-quick", action="store_true", help="keys: skip the quick sort")
    ap.add_argument("--no-copy", action="store_true", help="keys: skip the copy ceiling")
    ap.add_argument("--no-extras", action="store_true",
                    help="keys: skip the pairs, segmented and rows workloads")
    ap.add_argument("--eager", action="store_true",
                    help="time eager calls instead of replays of a captured HIP graph")
    ap.add_argument("--segments", type=int, default=100_000)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-per-array", action="store_true",
                    help="segmented: skip the one-call-per-array comparison")
    ap.add_argument("--graph-only", action="store_true",
                    help="keys: time graph replays only (no eager per-kernel event pass)")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--rows", type=int, default=4096)
    ap.add_argument("--cols", type=int, default=8192)
    ap.add_argument("--variant", default="tiefree", choices=["tiefree", "ties"])
    args = ap.parse_args()
    args.dists = [d for d in args.dists.split(",") if d]
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(this build has no multi-GPU path)", file=sys.stderr)
        return 2
    fn = {"keys": bench_keys, "pairs": bench_pairs, "segmented": bench_segmented,
          "rows": bench_rows, "small": bench_small, "leaves": bench_leaves,
          "copy": bench_copy}[args.workload]
    out = fn(args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
