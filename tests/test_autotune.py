"""Autotuner: cache and candidate grid (CPU), tuned results exact (GPU)."""
import ctypes
import os

import numpy as np
import pytest

from paper_2503_05934_amd import autotune


def test_cache_round_trip(tmp_path, monkeypatch):
    path = str(tmp_path / "cache.json")
    monkeypatch.setenv("MSN_AUTOTUNE_CACHE", path)
    assert autotune.lookup("k") is None
    autotune.store("k", {"merge_tile": 4096})
    autotune.store("k2", {"seg_grid": 7})
    assert autotune.lookup("k") == {"merge_tile": 4096}
    assert autotune.lookup("k2") == {"seg_grid": 7}
    # a cache from another version is ignored
    with open(path, "w") as f:
        f.write('{"version": -1, "entries": {"k": {"merge_tile": 2048}}}')
    assert autotune.lookup("k") is None


def test_size_buckets_and_keys():
    assert autotune.size_bucket(1) == 0
    assert autotune.size_bucket(1 << 28) == 28
    assert autotune.size_bucket((1 << 28) + 5) == 28
    a = autotune.workload_key("sort", 0, False, 0, 1 << 20, arch="gfx950")
    b = autotune.workload_key("sort", 0, True, 0, 1 << 20, arch="gfx950")
    assert a != b and "gfx950" in a


@pytest.mark.parametrize("k", [8, 4])
def test_segmented_candidates_pass_abi_validation(k):
    """Every candidate is accepted by the library's host-side checks (the
    calls below are rejected later for the fake workspace size, never for
    the tuning)."""
    from paper_2503_05934_amd import _lib, build

    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    L = _lib.lib()
    leaf = 0 if k == 8 else 1
    cands = autotune.segmented_candidates(k, 1 << 20, 1000)
    assert len(cands) >= 8
    fake = ctypes.c_void_p(1 << 20)
    for c in cands:
        t = _lib.make_tuning(c)
        rc = L.msn_segmented_sort(fake, None, ctypes.c_void_p(3 << 20), None, fake, 10, 100, 1,
                                  leaf, 0, ctypes.byref(t), ctypes.c_void_p(9 << 20), 0, None)
        assert rc == -5, (c, rc)   # workspace too small: the tuning itself was accepted


@pytest.mark.gpu
def test_autotuned_segmented_sort_is_exact(tmp_path, monkeypatch):
    import torch

    import oracle
    import paper_2503_05934_amd as msn
    from paper_2503_05934_amd import workloads
    from gpu_util import gpu, host, say

    monkeypatch.setenv("MSN_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    x, off, _ = workloads.segments(300, seed=5, hi=30000)
    say(f"autotune segmented S=300 n={x.shape[0]}")
    y = host(msn.segmented_sort(gpu(x), gpu(off), tuning="auto"))
    assert np.array_equal(y, oracle.load().segmented_sort(x, off, dtype="i32"))
    assert autotune.lookup(autotune.workload_key("segmented", 1, False, 0, x.shape[0], 300))
    say("autotune flat sort")
    z = gpu(workloads.keys(300000, "random", "u32", seed=4))
    ref = host(msn.sort(z))
    assert np.array_equal(host(msn.sort(z, tuning="auto")), ref)
