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

Other workloads (--workload pairs|segmented|rows) print their own line.
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
T_RUN = 8192                    # run length after the first sweep (6-to-8 leaves)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def reference_schedule_bytes(n: int, width: int) -> int:
    """Bytes per key of the binary merge-sort schedule: one read and one write
    per sweep, 1 + ceil(log2(n / 8192)) sweeps."""
    runs = -(-n // T_RUN)
    passes = max(0, int(np.ceil(np.log2(runs)))) if runs > 1 else 0
    return 2 * width * (1 + passes)


def load_traffic(kernel_file: str):
    """Per-launch HBM bytes of the merge kernel from committed rocprofv3 PMC
    summaries, if they were taken on the current kernel source."""
    import hashlib

    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2503_05934_amd", "csrc", "sort.hip")
    dev = os.path.join(ROOT, "paper_2503_05934_amd", "csrc", "device.hpp")
    h = hashlib.sha256(open(src, "rb").read() + open(dev, "rb").read()).hexdigest()[:16]
    if fields.get("source_sha256_16") != h:
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


def cpu_baseline(keys_np: np.ndarray, sample_n: int):
    import oracle

    orc = oracle.load()
    sample = keys_np[:sample_n]
    t0 = time.perf_counter()
    orc.sort(sample, dtype="u32", algo="ms", config="6To8")
    dt = time.perf_counter() - t0
    return {
        "value": sample_n / dt / 1e9,
        "unit": "Gkeys/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first 2^{int(np.log2(sample_n))} keys of the random 2^28 uint32 input; "
                  f"oracle Algorithm 1 with 6-to-8 networks, single thread, {dt:.2f} s",
        "host_cpu": _cpu_model(),
        "host_threads": os.cpu_count(),
    }


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_keys(args):
    import torch

    import paper_2503_05934_amd as msn
    from paper_2503_05934_amd import _lib, workloads

    dev = torch.device("cuda:0")
    n = args.n
    leaf = args.leaf
    plan = msn.SortPlan(n, torch.uint32, dev, leaf=leaf,
                        tuning={"merge_tile": args.merge_tile} if args.merge_tile else None)
    results = {}
    roof = None
    keys_random = None
    for dist in args.dists:
        log(f"[bench] generating {n} uint32 keys, {dist}")
        x_np = workloads.keys(n, dist, "u32", seed=0)
        if dist == "random":
            keys_random = x_np
        x = torch.from_numpy(x_np).to(dev)
        steps = args.steps if dist == "random" else max(2, args.steps // 4)
        log(f"[bench] {dist}: warmup {args.warmup}, timing {steps} steps")
        if dist == "random":
            _lib.timing_enable(64 * (steps + 1))
            # warmup first, then reset the events so only timed steps count
            for _ in range(args.warmup):
                plan.run(x)
            torch.cuda.synchronize()
            _lib.timing_enable(64 * (steps + 1))
            ms, wall = time_steps(lambda: plan.run(x), steps, 0)
            stats = _lib.timing_read()
            _lib.timing_disable()
        else:
            ms, wall = time_steps(lambda: plan.run(x), steps, args.warmup)
        ok = check_sorted_u32(plan.out, x)
        if not ok:
            raise SystemExit(f"[bench] output check failed for {dist}")
        results[dist] = {"gkeys_per_s": n / (ms / 1e3) / 1e9, "ms_per_step": ms, "steps": steps,
                         "wall_s": wall}
        log(f"[bench] {dist}: {ms:.3f} ms/step, {results[dist]['gkeys_per_s']:.2f} Gkeys/s")
        if dist == "random":
            m = stats.get("merge")
            if m:
                avg_s = m["avg_ms"] / 1e3
                bytes_per_launch = 8.0 * n
                achieved = bytes_per_launch / avg_s / 1e9
                traffic = load_traffic("k_merge_2p28_u32_traffic.md")
                roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                        "kernel": "k_merge (global merge-path pass)",
                        "avg_launch_ms": m["avg_ms"], "launches": m["launches"],
                        "algorithmic_bytes_per_launch": bytes_per_launch}
            results[dist]["kernels_ms_per_step"] = {
                k: v["total_ms"] / steps for k, v in stats.items()}
        del x
    head = results[args.dists[0]]
    sched = reference_schedule_bytes(n, 4)
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
                   "merge_tile": args.merge_tile or 8192},
        "roofline": roof,
        "hbm_schedule": {"bytes_per_key": sched,
                         "implied_gkeys_at_peak": HBM_PEAK_GBPS / sched,
                         "frac": head["gkeys_per_s"] / (HBM_PEAK_GBPS / sched)},
        "by_distribution": {d: {"gkeys_per_s": r["gkeys_per_s"], "ms_per_step": r["ms_per_step"]}
                            for d, r in results.items()},
        "kernels_ms_per_step": results.get("random", {}).get("kernels_ms_per_step"),
    }
    if not args.no_cpu and keys_random is not None:
        log(f"[bench] CPU oracle baseline on 2^{int(np.log2(args.cpu_sample))} keys")
        out["cpu_baseline"] = cpu_baseline(keys_random, args.cpu_sample)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="keys", choices=["keys"])
    ap.add_argument("--n", type=int, default=1 << 28)
    ap.add_argument("--leaf", default="6To8", choices=["6To8", "3To5"])
    ap.add_argument("--merge-tile", type=int, default=0)
    ap.add_argument("--dists", default="random,sorted,nearly")
    ap.add_argument("--cpu-sample", type=int, default=1 << 26)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    args.dists = [d for d in args.dists.split(",") if d]
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(this build has no multi-GPU path)", file=sys.stderr)
        return 2
    out = bench_keys(args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
