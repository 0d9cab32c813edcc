"""Every network set of Table 3 as a GPU leaf configuration, against the
oracle run under the same configuration, element by element, through the C
ABI: the flat sorts (keys, stable pairs, argsort), the batched sort and the
quick sort.  The sorted output is the same under every set; what differs is
which networks run (the 8- or 4-key network, or two member networks and a
merge, and per-size networks for subarrays of at most one group)."""
import itertools

import numpy as np
import pytest

import oracle
import paper_2503_05934_amd as msn
from paper_2503_05934_amd import _lib, workloads
from gpu_util import bits, gpu, host, make_keys, say

pytestmark = pytest.mark.gpu

SETS = ["6To8", "3To5", "PowerOf2", "Even", "Odd", "3", "3To4", "3To8", "VarSort3", "VarSort4",
        "VarSort5"]
SIZES = [1, 2, 3, 5, 7, 8, 9, 17, 100, 1023, 4097, 8193, 16385, 70001, 300007]


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


def offsets_of(lengths):
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return off.astype(np.uint32)


@pytest.mark.parametrize("leaf", SETS)
def test_networks_exhaustive(leaf):
    """Every permutation and every 0-1 input of up to 8 keys, one segment
    each, through the lane path (the set's network for that size, or the
    group procedure), the wavefront path and the workgroup path."""
    segs = []
    for n in range(0, 9):
        segs += [np.array(p, dtype=np.int32) for p in itertools.permutations(range(n))]
        segs += [np.array(t, dtype=np.int32) for t in itertools.product([0, 1], repeat=n)]
    off = offsets_of(np.array([len(s) for s in segs]))
    x = np.concatenate(segs).astype(np.int32)
    ref = np.concatenate([np.sort(s) for s in segs]).astype(np.int32)
    refp = np.concatenate([np.argsort(s, kind="stable") for s in segs]).astype(np.int32)
    for tun in ({}, {"seg_lane_max": 1}, {"seg_lane_max": 1, "seg_wave_max": 1}):
        say(f"leaf set {leaf}: exhaustive networks, tuning {tun}")
        y = msn.segmented_sort(gpu(x), gpu(off), leaf=leaf, tuning=tun)
        assert np.array_equal(host(y), ref), tun
        _, po = msn.segmented_sort(gpu(x), gpu(off), argsort=True, leaf=leaf, tuning=tun)
        assert np.array_equal(host(po), refp), tun


@pytest.mark.parametrize("leaf", SETS)
def test_flat_sorts(orc, leaf):
    for i, n in enumerate(SIZES):
        for dtype in ("u32", "i32", "f32"):
            say(f"leaf set {leaf}: sort {dtype} n={n}")
            x = make_keys(n, dtype, seed=500 + i)
            got = host(msn.sort(gpu(x), leaf=leaf))
            # float keys are sorted stably (equal floats keep input order)
            ref = orc.sort(x, dtype=dtype, config=leaf, stable=dtype == "f32")
            assert np.array_equal(bits(got), bits(ref)), (dtype, n)
        say(f"leaf set {leaf}: sort_pairs / argsort n={n}")
        k = make_keys(n, "u32", seed=600 + i) % np.uint32(97)
        v = np.arange(n, dtype=np.uint32)[::-1].copy()
        ko, vo = msn.sort_pairs(gpu(k), gpu(v), leaf=leaf)
        rk, rv = orc.sort(k, vals=v, dtype="u32", config=leaf, stable=True)
        assert np.array_equal(host(ko), rk) and np.array_equal(host(vo), rv), n
        _, po = msn.sort_pairs(gpu(k), leaf=leaf)
        _, rp = orc.sort(k, dtype="u32", config=leaf, stable=True, want_perm=True)
        assert np.array_equal(host(po).view(np.uint32), rp), n
        say(f"leaf set {leaf}: quick sort n={n}")
        xi = make_keys(n, "i32", seed=700 + i)
        got = host(msn.quick_sort(gpu(xi), leaf=leaf))
        assert np.array_equal(got, orc.sort(xi, dtype="i32", algo="qs", config=leaf)), n


@pytest.mark.parametrize("leaf", SETS)
def test_large_and_presorted(orc, leaf):
    for dist in workloads.DISTRIBUTIONS:
        say(f"leaf set {leaf}: 1,000,000 int32 {dist}")
        x = workloads.keys(1_000_000, dist, "i32", seed=0)
        ref = orc.sort(x, dtype="i32", config=leaf)
        assert np.array_equal(host(msn.sort(gpu(x), leaf=leaf)), ref), dist
        assert np.array_equal(host(msn.quick_sort(gpu(x), leaf=leaf)), ref), dist


@pytest.mark.parametrize("leaf", SETS)
def test_segmented(orc, leaf):
    # lengths 0..20 (lane, wavefront classes), a few hundred to a few
    # thousand (wavefront, workgroup), and tiled and long segments
    rng = np.random.default_rng(41)
    lengths = np.concatenate([np.arange(0, 21), rng.integers(20, 3000, 60),
                              np.array([8191, 8193, 16384, 40000, 70000])])
    rng.shuffle(lengths)
    off = offsets_of(lengths)
    n = int(off[-1])
    for dtype in ("i32", "f32"):
        say(f"leaf set {leaf}: segmented {dtype} S={len(lengths)} n={n}")
        x = make_keys(n, dtype, seed=800)
        y = msn.segmented_sort(gpu(x), gpu(off), leaf=leaf)
        ref = orc.segmented_sort(x, off, dtype=dtype, config=leaf, stable=dtype == "f32")
        assert np.array_equal(bits(host(y)), bits(ref)), dtype
    xv = make_keys(n, "u32", seed=801) % np.uint32(50)
    v = np.arange(n, dtype=np.uint32)
    ko, vo = msn.segmented_sort(gpu(xv), gpu(off), gpu(v), leaf=leaf)
    rk, rv = orc.segmented_sort(xv, off, v, dtype="u32", config=leaf, stable=True)
    assert np.array_equal(host(ko), rk) and np.array_equal(host(vo), rv)


def test_group_sizes_match_the_library():
    # the binding's table of group sizes agrees with the codes the library
    # accepts for the segmented lane class (seg_lane_max may reach the group)
    for name, code in _lib.LEAVES.items():
        if name == "classical":
            continue
        g = _lib.group_keys(name)
        x = gpu(np.arange(64, dtype=np.int32)[::-1].copy())
        off = gpu(np.array([0, 64], dtype=np.uint32))
        msn.segmented_sort(x, off, leaf=name, tuning={"seg_lane_max": g})
        with pytest.raises(_lib.MsnError):
            msn.segmented_sort(x, off, leaf=name, tuning={"seg_lane_max": g + 1})
