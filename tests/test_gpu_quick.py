"""GPU quick sort with network leaves (Algorithm 2) against the oracle's
Algorithm 2, element by element, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_05934_amd as msn
from paper_2503_05934_amd import _lib, workloads
from gpu_util import BOUNDARY_SIZES, DEV, gpu, host, make_keys, say

pytestmark = pytest.mark.gpu

CONFIG = {"6To8": "6To8", "3To5": "3To5", "classical": "Classical"}


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("leaf", ["6To8", "3To5", "classical"])
@pytest.mark.parametrize("dtype", ["u32", "i32"])
def test_quick_boundary_sizes(orc, dtype, leaf):
    for i, n in enumerate(BOUNDARY_SIZES):
        say(f"quick_sort {dtype} {leaf} n={n}")
        x = make_keys(n, dtype, seed=100 + i)
        got = host(msn.quick_sort(gpu(x), leaf=leaf))
        ref = orc.sort(x, dtype=dtype, algo="qs", config=CONFIG[leaf])
        assert np.array_equal(got, ref), (dtype, leaf, n)


def _tricky(n, seed):
    """Inputs that stress the pivot rule and the three-way split."""
    rng = np.random.default_rng(seed)
    asc = np.arange(n, dtype=np.uint32)
    return {
        "equal": np.full(n, 7, dtype=np.uint32),
        "two values": rng.integers(0, 2, n, dtype=np.uint32),
        "four values": rng.integers(0, 4, n, dtype=np.uint32) * 1000,
        "ascending": asc,
        "descending": asc[::-1].copy(),
        "organ pipe": np.concatenate([asc[: n // 2], asc[: n - n // 2][::-1]]),
        "sawtooth": (asc % 1000).astype(np.uint32),
        "extremes": rng.choice(np.array([0, 1, 0xFFFFFFFE, 0xFFFFFFFF], np.uint32), n),
    }


@pytest.mark.parametrize("n", [8193, 100_003, 1_000_000])
def test_quick_tricky_inputs(orc, n):
    for name, x in _tricky(n, seed=n).items():
        say(f"quick_sort tricky {name} n={n}")
        got = host(msn.quick_sort(gpu(x)))
        assert np.array_equal(got, np.sort(x)), name
        if n <= 100_003 and name not in ("equal",):
            assert np.array_equal(got, orc.sort(x, dtype="u32", algo="ms")), name


@pytest.mark.parametrize("n", [1 << 23, (1 << 23) + 4097])
def test_quick_claim_sizes(orc, n):
    # sorts of at most 2^23 keys claim room per 8192-key chunk throughout;
    # larger ones per 65,536-key super-tile in their first rounds (the first
    # two, and while subarrays are longer than 2^21 keys) and per chunk after,
    # so the larger size here runs both kinds of round: on random keys and on
    # few distinct values (long runs of keys equal to the pivot)
    for dist, x in (("random", workloads.keys(n, "random", "u32", seed=n)),
                    ("four values", _tricky(n, seed=3)["four values"]),
                    ("organ pipe", _tricky(n, seed=3)["organ pipe"])):
        say(f"quick_sort claim sizes n={n} {dist}")
        got = host(msn.quick_sort(gpu(x)))
        assert np.array_equal(got, orc.sort(x, dtype="u32", algo="qs")), dist


@pytest.mark.parametrize("rounds", [1, 2, 3, 5])
def test_quick_merge_fallback_after_last_round(orc, rounds):
    # with few rounds, subarrays still longer than a tile go to the merge
    # fallback (one workgroup merge-sorts each)
    for n, dist in ((300_001, "random"), (1_000_000, "sorted"), (70_000, "nearly")):
        say(f"quick_sort rounds={rounds} n={n} {dist}")
        x = workloads.keys(n, dist, "i32", seed=rounds)
        got = host(msn.quick_sort(gpu(x), tuning={"quick_rounds": rounds}))
        assert np.array_equal(got, orc.sort(x, dtype="i32", algo="ms")), (rounds, n, dist)


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_quick_workloads(orc, dist, leaf):
    # the 10,000-key array and the 1,000,000-key arrays
    for n in (10_000, 1_000_000):
        say(f"quick_sort workload n={n} {dist} {leaf}")
        x = workloads.keys(n, dist, "i32", seed=0)
        got = host(msn.quick_sort(gpu(x), leaf=leaf))
        assert np.array_equal(got, orc.sort(x, dtype="i32", algo="qs", config=leaf)), (n, dist)


def test_quick_in_place_and_offset_views(orc):
    x = workloads.keys(500_001, "random", "u32", seed=5)
    ref = orc.sort(x, dtype="u32", algo="qs")
    t = gpu(x)
    msn.quick_sort(t, out=t)
    assert np.array_equal(host(t), ref)
    # views one element into a buffer: 4-byte aligned only
    buf = torch.zeros(500_003, dtype=torch.uint32, device=DEV)
    buf[1:500_002] = gpu(x)
    out = torch.zeros(500_003, dtype=torch.uint32, device=DEV)
    msn.quick_sort(buf[1:500_002], out=out[2:500_003])
    assert np.array_equal(host(out[2:500_003]), ref)


def test_quick_graph_replay(orc):
    # one call captured in a HIP graph, replayed with eager work between
    x = workloads.keys(2_000_003, "nearly", "u32", seed=9)
    ref = orc.sort(x, dtype="u32", algo="ms")
    src = gpu(x)
    out = torch.empty_like(src)
    ws = torch.empty(_lib.quick_workspace_bytes(src.numel(), _lib.MSN_U32), dtype=torch.uint8,
                     device=DEV)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        msn.quick_sort(src, out=out, workspace=ws)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        msn.quick_sort(src, out=out, workspace=ws)
    for rep in range(3):
        out.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out), ref), rep


def test_quick_rejects_float_keys_and_bad_rounds():
    x = torch.zeros(100, dtype=torch.float32, device=DEV)
    with pytest.raises(_lib.MsnError) as e:
        msn.quick_sort(x)
    assert e.value.status == -6
    y = torch.zeros(100, dtype=torch.int32, device=DEV)
    with pytest.raises(_lib.MsnError) as e:
        msn.quick_sort(y, tuning={"quick_rounds": 97})
    assert e.value.status == -4
