"""Segmented sort (binning, tile-sort, persistent and tile-merge launches) against the oracle, bit-exact."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import paper_2503_05934_amd as msn
from paper_2503_05934_amd import workloads
from gpu_util import bits, float_keys, gpu, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


def offsets_of(lengths):
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint32)


# every work class: empty, lane (<= 8), wave (<= 512), block (<= 8192), and
# the three big classes (<= 2x, <= 4x, > 4x of a block)
CLASS_LENGTHS = [0, 1, 2, 3, 5, 8, 9, 17, 100, 255, 256, 511, 512, 513, 2000, 4096, 8191, 8192,
                 8193, 12000, 16384, 16385, 30000, 32768, 32769, 65536, 0, 7, 0, 4, 3]


def mixed_lengths(seed, count=600):
    rng = np.random.default_rng(seed)
    lengths = np.floor(np.exp(rng.uniform(0, np.log(70000), count))).astype(np.int64)
    lengths[rng.random(count) < 0.1] = 0
    return np.concatenate([CLASS_LENGTHS, lengths])


def seg_keys(total, dtype, seed):
    if dtype == "f32":
        return float_keys(total, seed)
    rng = np.random.default_rng(seed)
    hi = 2**31 if dtype == "i32" else 2**32
    x = rng.integers(0, hi, total, dtype=np.int64)
    x[rng.random(total) < 0.3] = 12345  # ties
    return x.astype(np.int32 if dtype == "i32" else np.uint32)


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dtype", ["i32", "u32", "f32"])
def test_segmented_all_classes(orc, dtype, leaf):
    lengths = mixed_lengths(seed=len(dtype) + 3 * (leaf == "3To5"), count=120)
    off = offsets_of(lengths)
    x = seg_keys(int(off[-1]), dtype, seed=4)
    say(f"segmented keys dtype={dtype} leaf={leaf} S={len(lengths)} n={int(off[-1])}")
    y = msn.segmented_sort(gpu(x), gpu(off), leaf=leaf)
    ref = orc.segmented_sort(x, off, dtype=dtype, stable=True)
    assert np.array_equal(bits(host(y)), bits(ref))

    v = np.random.default_rng(8).integers(0, 2**32, x.shape[0], dtype=np.uint32)
    say(f"segmented pairs dtype={dtype} leaf={leaf}")
    ko, vo = msn.segmented_sort(gpu(x), gpu(off), gpu(v), leaf=leaf)
    rk, rv = orc.segmented_sort(x, off, vals=v, dtype=dtype, stable=True)
    assert np.array_equal(bits(host(ko)), bits(rk))
    assert np.array_equal(host(vo), rv)

    say(f"segmented argsort dtype={dtype} leaf={leaf}")
    ko, po = msn.segmented_sort(gpu(x), gpu(off), argsort=True, leaf=leaf)
    _, rp = orc.segmented_sort(x, off, dtype=dtype, stable=True, want_perm=True)
    assert np.array_equal(bits(host(ko)), bits(rk))
    assert np.array_equal(host(po).view(np.uint32), rp)


# Keys-only segments of three or four runs (runs of 2 x 1024 K keys after the
# tile sort) merge in one four-way pass; two-run segments in one binary pass.
FOUR_WAY_LENGTHS = {"6To8": [16385, 32768, 32769, 32770, 40000, 49151, 49152, 49153, 65535, 65536],
                    "3To5": [8193, 16384, 16385, 20000, 24576, 24577, 32767, 32768]}


def _four_way_keys(total, dist, dtype, seed):
    rng = np.random.default_rng(seed)
    hi = 2**31 if dtype == "i32" else 2**32
    if dist == "random":
        x = rng.integers(0, hi, total, dtype=np.int64)
    elif dist == "few":
        x = rng.integers(0, 3, total, dtype=np.int64) * (hi // 4)
    elif dist == "equal":
        x = np.full(total, hi // 2 + 1, dtype=np.int64)
    elif dist == "ascending":
        x = np.arange(total, dtype=np.int64) % hi
    else:  # descending, with the extremes
        x = (hi - 1 - np.arange(total, dtype=np.int64)) % hi
        x[:: 97] = 0
        x[1:: 89] = hi - 1
    return x.astype(np.int32 if dtype == "i32" else np.uint32)


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dtype", ["i32", "u32"])
def test_four_way_segments(orc, dtype, leaf):
    base = FOUR_WAY_LENGTHS[leaf]
    rng = np.random.default_rng(17)
    top = base[-1]
    lengths = np.concatenate([base, rng.integers(top // 2 + 1, top + 1, 40), [5, 0, 3000], base[::-1]])
    off = offsets_of(lengths)
    for i, dist in enumerate(("random", "few", "equal", "ascending", "descending")):
        x = _four_way_keys(int(off[-1]), dist, dtype, seed=30 + i)
        say(f"four-way segments {dtype} {leaf} {dist} S={len(lengths)} n={int(off[-1])}")
        y = msn.segmented_sort(gpu(x), gpu(off), leaf=leaf)
        ref = orc.segmented_sort(x, off, dtype=dtype, config=leaf)
        assert np.array_equal(host(y), ref), dist
    # equal-length rows of three and of four runs (no offsets array: the
    # host knows the pass plan)
    for rl in (base[3], base[-1]):
        x = _four_way_keys(rl * 7, "few", dtype, seed=rl)
        off_r = offsets_of(np.full(7, rl))
        say(f"four-way rows (offsets=None) {dtype} {leaf} 7 x {rl}")
        y = msn.segmented_sort(gpu(x), None, num_segments=7, leaf=leaf)
        assert np.array_equal(host(y), orc.segmented_sort(x, off_r, dtype=dtype, config=leaf)), rl


def test_segmented_batched_recipe(orc):
    # the batched workload's recipe (log-uniform 3..65536, 30 % presorted) at
    # 1,500 segments so the oracle finishes in seconds
    x, off, _ = workloads.segments(1500, seed=0)
    say(f"segmented recipe S=1500 n={x.shape[0]}")
    y = msn.segmented_sort(gpu(x), gpu(off))
    ref = orc.segmented_sort(x, off, dtype="i32", config="Classical")
    assert np.array_equal(host(y), ref)


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
def test_thresholds_do_not_change_bits(orc, leaf):
    k = 8 if leaf == "6To8" else 4
    lengths = mixed_lengths(seed=11, count=200)
    off = offsets_of(lengths)
    x = seg_keys(int(off[-1]), "i32", seed=12)
    ref = orc.segmented_sort(x, off, dtype="i32")
    for tun in ({}, {"seg_lane_max": 1}, {"seg_lane_max": 1, "seg_wave_max": 1},
                {"seg_lane_max": 1, "seg_wave_max": 1, "seg_block_max": 1},
                {"seg_wave_max": 64 * k, "seg_block_max": 1024 * k, "seg_grid": 3}):
        say(f"segmented thresholds leaf={leaf} tuning={tun}")
        y = msn.segmented_sort(gpu(x), gpu(off), leaf=leaf, tuning=tun)
        assert np.array_equal(host(y), ref), tun


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
def test_networks_exhaustive_on_gpu(leaf):
    """Every permutation and every 0-1 input of up to 8 keys, one segment
    each: on the lane path this is the leaf network alone (0-1 principle)."""
    segs = []
    for n in range(0, 9):
        segs += [np.array(p, dtype=np.int32) for p in itertools.permutations(range(n))]
        segs += [np.array(t, dtype=np.int32) for t in itertools.product([0, 1], repeat=n)]
    lengths = np.array([len(s) for s in segs])
    off = offsets_of(lengths)
    x = np.concatenate(segs).astype(np.int32)
    ref = np.concatenate([np.sort(s) for s in segs]).astype(np.int32)
    for tun in ({}, {"seg_lane_max": 1}, {"seg_lane_max": 1, "seg_wave_max": 1}):
        say(f"exhaustive networks leaf={leaf} tuning={tun} S={len(segs)}")
        y = msn.segmented_sort(gpu(x), gpu(off), leaf=leaf, tuning=tun)
        assert np.array_equal(host(y), ref), tun
        ko, po = msn.segmented_sort(gpu(x), gpu(off), argsort=True, leaf=leaf, tuning=tun)
        refp = np.concatenate([np.argsort(s, kind="stable") for s in segs]).astype(np.int32)
        assert np.array_equal(host(po), refp), tun


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
def test_equal_rows_without_offsets(orc, leaf):
    # one workgroup per row, tiled rows of two to five tiles (one to three
    # merge passes, their count known on the host), and rows past the tiled
    # limit
    for rows, cols in ((37, 3000), (9, 20000), (5, 70000)):
        x = seg_keys(rows * cols, "u32", seed=3 + cols)
        off = (np.arange(rows + 1) * cols).astype(np.uint32)
        say(f"segmented equal rows (offsets=None) leaf={leaf} rows={rows} cols={cols}")
        y = msn.segmented_sort(gpu(x), None, num_segments=rows, leaf=leaf)
        assert np.array_equal(host(y), orc.segmented_sort(x, off, dtype="u32", config=leaf))
        say(f"segmented equal rows argsort leaf={leaf} rows={rows} cols={cols}")
        yk, yp = msn.segmented_sort(gpu(x), None, num_segments=rows, leaf=leaf, argsort=True)
        rk, rp = orc.segmented_sort(x, off, dtype="u32", config=leaf, stable=True,
                                    want_perm=True)
        assert np.array_equal(host(yk), rk)
        assert np.array_equal(host(yp).view(np.uint32), rp)


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dtype", ["i32", "u32", "f32"])
def test_presorted_segments(orc, dtype, leaf):
    """Arrays that arrive sorted, or sorted but for one pair of keys at a
    thread edge (keys-per-thread apart), at a tile edge, or inside a thread,
    next to random arrays: keys-only integer tiles already in order are
    copied as they stand, every other tile is sorted."""
    kpt = 16 if leaf == "6To8" else 8
    tile = 512 * kpt
    lengths = np.concatenate([CLASS_LENGTHS, [tile * 3, tile * 8, tile * 2 + 5, 3 * kpt + 1],
                              mixed_lengths(seed=31, count=200)])
    off = offsets_of(lengths)
    x = seg_keys(int(off[-1]), dtype, seed=32)
    rng = np.random.default_rng(33)
    kinds = []
    for s in range(lengths.shape[0]):
        a, b = int(off[s]), int(off[s + 1])
        kind = ("random", "sorted", "thread", "tile", "inside")[s % 5]
        kinds.append(kind)
        if kind == "random" or b - a < 2:
            continue
        seg = orc.sort(x[a:b], dtype=dtype, stable=True)
        n = b - a
        if kind == "thread" and n > kpt:
            i = kpt * int(rng.integers(1, (n - 1) // kpt + 1))
            seg[i - 1], seg[i] = seg[i], seg[i - 1]
        elif kind == "tile" and n > tile:
            i = tile * int(rng.integers(1, (n - 1) // tile + 1))
            seg[i - 1], seg[i] = seg[i], seg[i - 1]
        elif kind == "inside" and n > 3:
            i = int(rng.integers(1, n - 1))
            seg[i - 1], seg[i] = seg[i], seg[i - 1]
        x[a:b] = seg
    ref = orc.segmented_sort(x, off, dtype=dtype, stable=True)
    # default classes, then every array of two keys or more through the tiled path
    for tun in (None, {"seg_lane_max": 1, "seg_wave_max": 1, "seg_block_max": 1}):
        say(f"segmented presorted dtype={dtype} leaf={leaf} segments={lengths.shape[0]} {tun}")
        y = msn.segmented_sort(gpu(x), gpu(off), leaf=leaf, tuning=tun)
        assert np.array_equal(bits(host(y)), bits(ref)), tun
    say("segmented presorted, in place")
    t = gpu(x)
    msn.segmented_sort(t, gpu(off), out_keys=t, leaf=leaf)
    assert np.array_equal(bits(host(t)), bits(ref))
    say("segmented presorted, argsort")
    _, p = msn.segmented_sort(gpu(x), gpu(off), argsort=True, leaf=leaf)
    _, rp = orc.segmented_sort(x, off, dtype=dtype, stable=True, want_perm=True)
    assert np.array_equal(host(p).view(np.uint32), rp)


def test_only_empty_and_tiny_segments(orc):
    lengths = np.array([0] * 50 + [1] * 50 + [0, 2, 0, 3])
    off = offsets_of(lengths)
    x = seg_keys(int(off[-1]), "i32", seed=1)
    say("segmented tiny segments")
    y = msn.segmented_sort(gpu(x), gpu(off))
    assert np.array_equal(host(y), orc.segmented_sort(x, off, dtype="i32"))


def test_segmented_in_place(orc):
    lengths = mixed_lengths(seed=5, count=80)
    off = offsets_of(lengths)
    x = seg_keys(int(off[-1]), "f32", seed=6)
    rk, rp = orc.segmented_sort(x, off, dtype="f32", stable=True, want_perm=True)
    t = gpu(x)
    say("segmented in place keys")
    msn.segmented_sort(t, gpu(off), out_keys=t)
    assert np.array_equal(bits(host(t)), bits(rk))
    t = gpu(x)
    v = gpu(np.arange(x.shape[0], dtype=np.uint32))
    say("segmented in place pairs")
    msn.segmented_sort(t, gpu(off), v, out_keys=t, out_vals=v)
    glob = np.concatenate([off[s] + rp[off[s]:off[s + 1]] for s in range(len(lengths))])
    assert np.array_equal(bits(host(t)), bits(rk))
    assert np.array_equal(host(v), glob.astype(np.uint32))


def test_hip_graph_replays_match_eager(orc):
    lengths = mixed_lengths(seed=9, count=150)
    off = offsets_of(lengths)
    x = seg_keys(int(off[-1]), "i32", seed=10)
    ref = orc.segmented_sort(x, off, dtype="i32")
    kin, offs = gpu(x), gpu(off)
    out = torch.empty_like(kin)
    n, S = x.shape[0], len(lengths)
    from paper_2503_05934_amd import _lib
    ws = torch.empty(_lib.segmented_workspace_bytes(n, S, 1, False), dtype=torch.uint8,
                     device=kin.device)
    say("segmented eager before capture")
    msn.segmented_sort(kin, offs, out_keys=out, workspace=ws)
    torch.cuda.synchronize()
    assert np.array_equal(host(out), ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    say("segmented graph capture")
    with torch.cuda.graph(g, stream=s):
        msn.segmented_sort(kin, offs, out_keys=out, workspace=ws)
    for r in range(4):
        out.zero_()
        ws.fill_(0xAB)
        torch.cuda.synchronize()
        say(f"graph replay {r}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out), ref), r


@pytest.mark.parametrize("debug_check", [False, True])
def test_invalid_offsets_set_status_and_leave_outputs(debug_check):
    """Offsets that break the CSR rules but stay inside the arrays (entries
    non-decreasing and at most n_total, so no access could leave the arrays
    even if the check were missing): the call reports the broken rule in its
    status word and writes nothing."""
    from paper_2503_05934_amd import _lib
    n = 1000
    x = seg_keys(n, "i32", seed=11)
    cases = [(np.array([0, 300, 700], np.uint32), _lib.MSN_SEG_BAD_LAST),
             (np.array([5, 300, 1000], np.uint32), _lib.MSN_SEG_BAD_FIRST),
             (np.array([0, 0, 999, 999], np.uint32), _lib.MSN_SEG_BAD_LAST)]
    for off, bit in cases:
        S = len(off) - 1
        ws = torch.empty(_lib.segmented_workspace_bytes(n, S, 1, False), dtype=torch.uint8,
                         device="cuda:0")
        ws.fill_(0xAB)
        out = torch.full((n,), 7, dtype=torch.int32, device="cuda:0")
        say(f"invalid offsets {off.tolist()} debug_check={debug_check}")
        msn.segmented_sort(gpu(x), gpu(off), out_keys=out, workspace=ws,
                           debug_check=debug_check)
        assert msn.segmented_status(ws, n, S) == bit
        assert bool((out == 7).all())
        # argsort: values untouched too
        wsp = torch.empty(_lib.segmented_workspace_bytes(n, S, 1, True), dtype=torch.uint8,
                          device="cuda:0")
        ov = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
        msn.segmented_sort(gpu(x), gpu(off), argsort=True, out_keys=out, out_vals=ov,
                           workspace=wsp, debug_check=debug_check)
        assert msn.segmented_status(wsp, n, S, pairs=True) == bit
        assert bool((out == 7).all()) and bool((ov == -1).all())


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_debug_check_on_valid_offsets(orc, dtype):
    from paper_2503_05934_amd import _lib
    lengths = mixed_lengths(seed=21, count=150)
    off = offsets_of(lengths)
    n, S = int(off[-1]), len(lengths)
    x = seg_keys(n, dtype, seed=22)
    ws = torch.empty(_lib.segmented_workspace_bytes(n, S, 2, False), dtype=torch.uint8,
                     device="cuda:0")
    ws.fill_(0xAB)
    say(f"segmented debug check on valid offsets dtype={dtype}")
    y = msn.segmented_sort(gpu(x), gpu(off), workspace=ws, debug_check=True)
    assert msn.segmented_status(ws, n, S) == 0
    assert np.array_equal(bits(host(y)), bits(orc.segmented_sort(x, off, dtype=dtype,
                                                                 stable=True)))
    ws.fill_(0xAB)
    y = msn.segmented_sort(gpu(x), gpu(off), workspace=ws)   # status cleared without the flag too
    assert msn.segmented_status(ws, n, S) == 0


def test_binding_rejects_mis_sized_buffers():
    """Every caller-supplied array is checked against n before the call: a
    short output, value or workspace array raises ValueError and nothing runs."""
    dev = "cuda:0"
    k = torch.arange(1000, dtype=torch.int32, device=dev)
    short = torch.empty(999, dtype=torch.int32, device=dev)
    wide = torch.empty(1000, dtype=torch.int64, device=dev)
    off = torch.tensor([0, 500, 1000], dtype=torch.int32, device=dev)
    cases = [
        lambda: msn.sort(k, out=short),
        lambda: msn.sort(k, out=wide),
        lambda: msn.sort(k, workspace=torch.empty(16, dtype=torch.uint8, device=dev)),
        lambda: msn.sort_pairs(k, short),
        lambda: msn.sort_pairs(k, out_keys=short),
        lambda: msn.sort_pairs(k, out_vals=short),
        lambda: msn.sort_pairs(k, k[::2].contiguous()),
        lambda: msn.segmented_sort(k, off, short),
        lambda: msn.segmented_sort(k, off, out_keys=short),
        lambda: msn.segmented_sort(k, off, argsort=True, out_vals=short),
        lambda: msn.segmented_sort(k, off, out_vals=short),
        lambda: msn.segmented_sort(k, off.cpu()),
        lambda: msn.sort_backward(k.float().view(10, 100), k.view(10, 100), out=short.float()),
        lambda: msn.SortPlan(1000, torch.int32, dev).run(short),
        lambda: msn.SortPlan(1000, torch.int32, dev, pairs=True).run(k, short),
        lambda: msn.SortPlan(1000, torch.int32, dev, pairs=True).run(k),
    ]
    for i, c in enumerate(cases):
        say(f"binding check case {i}")
        with pytest.raises(ValueError):
            c()
