"""Flat sorts on the GPU against the oracle, element by element (bit-exact)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_05934_amd as msn
from paper_2503_05934_amd import workloads
from gpu_util import BOUNDARY_SIZES, bits, gpu, host, make_keys, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dtype", ["u32", "i32", "f32"])
def test_sort_keys_boundary_sizes(orc, dtype, leaf):
    for n in BOUNDARY_SIZES:
        x = make_keys(n, dtype, seed=n)
        say(f"sort_keys dtype={dtype} leaf={leaf} n={n}")
        y = host(msn.sort(gpu(x), leaf=leaf))
        ref = orc.sort(x, dtype=dtype, stable=True, config=leaf)
        assert np.array_equal(bits(y), bits(ref)), (dtype, leaf, n)


def test_cfg1_10k_int32(orc):
    x = workloads.keys(10_000, "random", "i32", 0)
    say("sort_keys 10,000 int32 seed 0")
    y = host(msn.sort(gpu(x), leaf="6To8"))
    assert np.array_equal(y, orc.sort(x, dtype="i32", config="6To8"))


_CFG2 = {}


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_cfg2_1m_int32(orc, dist, leaf):
    x = workloads.keys(1_000_000, dist, "i32", 0)
    if dist not in _CFG2:
        _CFG2[dist] = orc.sort(x, dtype="i32", config="6To8")
    say(f"sort_keys 1e6 int32 dist={dist} leaf={leaf}")
    y = host(msn.sort(gpu(x), leaf=leaf))
    assert np.array_equal(y, _CFG2[dist])


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dtype", ["u32", "i32", "f32"])
def test_sort_pairs_stable(orc, dtype, leaf):
    rng = np.random.default_rng(21)
    for n in [1, 7, 9, 513, 8191, 8193, 40000, 262145]:
        if dtype == "f32":
            k = make_keys(n, "f32", seed=n)
        else:
            k = rng.integers(0, 64, n).astype(np.uint32 if dtype == "u32" else np.int32)
            if dtype == "i32":
                k -= 32
        v = rng.integers(0, 2**32, n, dtype=np.uint32)
        say(f"sort_pairs dtype={dtype} leaf={leaf} n={n}")
        ko, vo = msn.sort_pairs(gpu(k), gpu(v), leaf=leaf)
        rk, rv = orc.sort(k, vals=v, dtype=dtype, stable=True, config=leaf)
        assert np.array_equal(bits(host(ko)), bits(rk)), (dtype, n)
        assert np.array_equal(host(vo), rv), (dtype, n)
        say(f"argsort dtype={dtype} leaf={leaf} n={n}")
        ko, po = msn.sort_pairs(gpu(k), None, leaf=leaf)
        _, rp = orc.sort(k, dtype=dtype, stable=True, config=leaf, want_perm=True)
        assert np.array_equal(bits(host(ko)), bits(rk))
        assert np.array_equal(host(po).view(np.uint32), rp), (dtype, n)


def test_pairs_many_ties_payload_index(orc):
    n = (1 << 21) + 4097
    k, v = workloads.pairs(n, seed=3)
    say(f"sort_pairs keys<2^16 payload=index n={n}")
    ko, vo = msn.sort_pairs(gpu(k), gpu(v))
    rk, rv = orc.sort(k, vals=v, dtype="u32", stable=True)
    assert np.array_equal(host(ko), rk)
    assert np.array_equal(host(vo), rv)


@pytest.mark.parametrize("dtype", ["u32", "f32"])
def test_in_place(orc, dtype):
    for n in [5000, 8192 * 3 + 1, 100000]:
        x = make_keys(n, dtype, seed=7 + n)
        ref = orc.sort(x, dtype=dtype, stable=True)
        say(f"sort_keys in place dtype={dtype} n={n}")
        t = gpu(x)
        msn.sort(t, out=t)
        assert np.array_equal(bits(host(t)), bits(ref))
        say(f"sort_pairs in place dtype={dtype} n={n}")
        t = gpu(x)
        vals = gpu(np.arange(n, dtype=np.uint32))
        msn.sort_pairs(t, vals, out_keys=t, out_vals=vals)
        _, rp = orc.sort(x, dtype=dtype, stable=True, want_perm=True)
        assert np.array_equal(bits(host(t)), bits(ref))
        assert np.array_equal(host(vals), rp)


def test_merge_tiles_give_identical_bits(orc):
    n = 300007
    x = make_keys(n, "u32", seed=5)
    ref = orc.sort(x, dtype="u32")
    for mt in (2048, 4096, 8192):
        say(f"sort_keys merge_tile={mt}")
        y = host(msn.sort(gpu(x), tuning={"merge_tile": mt}))
        assert np.array_equal(y, ref), mt
        say(f"sort_pairs merge_tile={mt}")
        k, v = workloads.pairs(n, seed=9, key_hi=1000)
        ko, vo = msn.sort_pairs(gpu(k), gpu(v), tuning={"merge_tile": mt})
        rk, rv = orc.sort(k, vals=v, stable=True)
        assert np.array_equal(host(ko), rk) and np.array_equal(host(vo), rv), mt


@pytest.mark.parametrize("leaf,k", [("6To8", 8), ("3To5", 4)])
@pytest.mark.parametrize("dtype", ["u32", "i32"])
def test_block_tiles_give_identical_bits(orc, dtype, leaf, k):
    for n in (1, 4095, 8193, 16385, 32767, 32769, 65537, 300007):
        x = make_keys(n, dtype, seed=11 + n)
        ref = orc.sort(x, dtype=dtype)
        for bt in (1024 * k, 2048 * k, 4096 * k):
            say(f"sort_keys dtype={dtype} leaf={leaf} block_tile={bt} n={n}")
            y = host(msn.sort(gpu(x), leaf=leaf, tuning={"block_tile": bt}))
            assert np.array_equal(y, ref), (bt, n)


def _tricky_keys(n, kind, dtype, seed):
    rng = np.random.default_rng(seed)
    np_t = np.uint32 if dtype == "u32" else np.int32
    if kind == "random":
        return make_keys(n, dtype, seed)
    if kind == "few":        # four distinct values: every sample ties
        x = rng.integers(0, 4, n)
    elif kind == "equal":
        x = np.full(n, 3)
    elif kind == "clustered":  # half uniform, half inside a narrow band
        x = np.where(rng.random(n) < 0.5, rng.integers(0, 1 << 31, n),
                     (1 << 30) + rng.integers(0, 1000, n))
    elif kind == "sorted":
        x = np.sort(rng.integers(0, 1 << 20, n))
    elif kind == "reversed":
        x = np.sort(rng.integers(0, 1 << 20, n))[::-1]
    else:                    # extremes of the type mixed with ties
        lo, hi = (0, 2**32 - 1) if dtype == "u32" else (-2**31, 2**31 - 1)
        x = rng.choice(np.array([lo, hi, 0, 1, hi - 1], dtype=np.int64), n)
    return np.ascontiguousarray(x.astype(np.int64).astype(np_t) if dtype == "i32"
                                else x.astype(np.uint64).astype(np_t))


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dtype", ["u32", "i32"])
def test_four_way_passes_match_oracle_and_binary(orc, dtype, leaf):
    """Four-way passes (sampled splitters) against the oracle and against
    binary passes, on tie-heavy, sorted, reversed and extreme inputs, with
    groups that end in one, two or three runs."""
    t = 2048 * (8 if leaf == "6To8" else 4)   # default first-sweep run length
    runs_list = [3, 4, 5, 6, 7, 9, 17, 64 + 3]
    kinds = ["random", "few", "equal", "sorted", "reversed", "extremes"]
    for i, runs in enumerate(runs_list):
        n = runs * t - (i % 3) * 97
        for kind in kinds:
            x = _tricky_keys(n, kind, dtype, seed=100 * i + len(kind))
            ref = orc.sort(x, dtype=dtype)
            say(f"four-way dtype={dtype} leaf={leaf} n={n} kind={kind}")
            y4 = host(msn.sort(gpu(x), leaf=leaf, tuning={"merge_ways": 4}))
            assert np.array_equal(y4, ref), (n, kind, "4-way")
            y4w = host(msn.sort(gpu(x), leaf=leaf, tuning={"merge_ways": 4, "merge4_kpt": 32}))
            assert np.array_equal(y4w, ref), (n, kind, "4-way, 32 keys per thread")
            y2 = host(msn.sort(gpu(x), leaf=leaf, tuning={"merge_ways": 2}))
            assert np.array_equal(y2, ref), (n, kind, "2-way")
    # runs of 2^20 keys and more: boundary brackets wider than the LDS window
    for kind in ("clustered", "random"):
        n = 5 * (1 << 20) + 777
        x = _tricky_keys(n, kind, dtype, seed=11)
        say(f"four-way large groups dtype={dtype} leaf={leaf} n={n} kind={kind}")
        y4 = host(msn.sort(gpu(x), leaf=leaf, tuning={"merge_ways": 4}))
        assert np.array_equal(y4, orc.sort(x, dtype=dtype)), (n, kind)
    for bt_mult in (1024, 2048, 4096):
        k = 8 if leaf == "6To8" else 4
        n = 23 * bt_mult * k + 1234
        x = _tricky_keys(n, "few", dtype, seed=bt_mult)
        say(f"four-way block_tile={bt_mult * k} n={n}")
        y = host(msn.sort(gpu(x), leaf=leaf, tuning={"block_tile": bt_mult * k}))
        assert np.array_equal(y, orc.sort(x, dtype=dtype)), bt_mult


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dtype", ["u32", "i32"])
def test_four_way_pairs_stable(orc, dtype, leaf):
    """Four-way passes over key-value pairs against the oracle's stable sort
    and against binary passes: tie-heavy, sorted, reversed and extreme keys,
    explicit payloads and argsort, groups that end in one to three runs."""
    t = 1024 * (8 if leaf == "6To8" else 4)   # first-sweep run length of pairs
    runs_list = [3, 4, 5, 6, 7, 9, 17, 64 + 3]
    kinds = ["random", "few", "equal", "sorted", "reversed", "extremes"]
    rng = np.random.default_rng(5)
    for i, runs in enumerate(runs_list):
        n = runs * t - (i % 3) * 97
        for kind in kinds:
            k = _tricky_keys(n, kind, dtype, seed=300 * i + len(kind))
            v = rng.integers(0, 2**32, n, dtype=np.uint32)
            rk, rv = orc.sort(k, vals=v, dtype=dtype, stable=True, config=leaf)
            for ways in (4, 2):
                say(f"four-way pairs ways={ways} dtype={dtype} leaf={leaf} n={n} kind={kind}")
                ko, vo = msn.sort_pairs(gpu(k), gpu(v), leaf=leaf, tuning={"merge_ways": ways})
                assert np.array_equal(host(ko), rk), (n, kind, ways)
                assert np.array_equal(host(vo), rv), (n, kind, ways)
            say(f"four-way argsort dtype={dtype} leaf={leaf} n={n} kind={kind}")
            ko, po = msn.sort_pairs(gpu(k), None, leaf=leaf, tuning={"merge_ways": 4})
            _, rp = orc.sort(k, dtype=dtype, stable=True, config=leaf, want_perm=True)
            assert np.array_equal(host(ko), rk), (n, kind)
            assert np.array_equal(host(po).view(np.uint32), rp), (n, kind)
    # runs of 2^20 keys and more: boundary brackets wider than the LDS window
    for kind in ("clustered", "few"):
        n = 5 * (1 << 20) + 777
        k = _tricky_keys(n, kind, dtype, seed=13)
        v = np.arange(n, dtype=np.uint32)
        say(f"four-way pairs large groups dtype={dtype} leaf={leaf} n={n} kind={kind}")
        ko, vo = msn.sort_pairs(gpu(k), gpu(v), leaf=leaf)
        rk, rv = orc.sort(k, vals=v, dtype=dtype, stable=True, config=leaf)
        assert np.array_equal(host(ko), rk), (n, kind)
        assert np.array_equal(host(vo), rv), (n, kind)


def _presorted_variant(x, variant, t, rng):
    """Sorted keys x, then: "sorted" as is; "local": swaps inside first-sweep
    runs of length t, away from their ends (the runs come out of the first
    sweep in order); "edge": one swap across a run boundary; "last": the
    smallest key moved to the end (the two take every pass)."""
    x = x.copy()
    n = x.shape[0]
    if variant == "local":
        for _ in range(32):
            r = int(rng.integers(0, max(1, n // t)))
            lo, hi = r * t + 1, min(n, (r + 1) * t) - 1
            if hi - lo >= 2:
                i, j = rng.integers(lo, hi, 2)
                x[i], x[j] = x[j], x[i]
    elif variant == "edge":
        b = t * int(rng.integers(1, -(-n // t)))
        x[b - 1], x[b] = x[b], x[b - 1]
        if x[b - 1] == x[b]:
            x[b - 1], x[b] = x[0], x[-1]
    elif variant == "last":
        x = np.concatenate([x[1:], x[:1]])
    return x


@pytest.mark.parametrize("leaf", ["6To8", "3To5"])
@pytest.mark.parametrize("dtype", ["u32", "i32", "f32"])
def test_presorted_inputs(orc, dtype, leaf):
    """Inputs whose first-sweep runs already follow each other in order skip
    every global pass (the first sweep's result is copied to the output when
    it went to the workspace): keys, pairs and argsort under both pass plans,
    with odd and even pass counts, against inputs where a single pair of keys
    across a run boundary, or the last key, keeps the passes."""
    k = 8 if leaf == "6To8" else 4
    rng = np.random.default_rng(77)
    for runs in (2, 3, 5, 17, 65):
        for ways in (4, 2):
            for pairs in (False, True):
                t = (1024 if pairs or dtype == "f32" else 2048) * k  # first-sweep run
                n = runs * t - (runs % 3) * 51
                if dtype == "f32":
                    base = orc.sort(make_keys(n, "f32", seed=runs), dtype="f32", stable=True)
                else:
                    base = np.sort(_tricky_keys(n, "few" if runs % 2 else "random", dtype, runs))
                for variant in ("sorted", "local", "edge", "last"):
                    x = _presorted_variant(base, variant, t, rng)
                    tag = (dtype, leaf, n, ways, pairs, variant)
                    say(f"presorted {tag}")
                    tuning = {"merge_ways": ways}
                    if not pairs:
                        y = host(msn.sort(gpu(x), leaf=leaf, tuning=tuning))
                        ref = orc.sort(x, dtype=dtype, stable=True)
                        assert np.array_equal(bits(y), bits(ref)), tag
                        continue
                    v = rng.integers(0, 2**32, n, dtype=np.uint32)
                    ko, vo = msn.sort_pairs(gpu(x), gpu(v), leaf=leaf, tuning=tuning)
                    rk, rv = orc.sort(x, vals=v, dtype=dtype, stable=True)
                    assert np.array_equal(bits(host(ko)), bits(rk)), tag
                    assert np.array_equal(host(vo), rv), tag
                    _, po = msn.sort_pairs(gpu(x), None, leaf=leaf, tuning=tuning)
                    _, rp = orc.sort(x, dtype=dtype, stable=True, want_perm=True)
                    assert np.array_equal(host(po).view(np.uint32), rp), tag


@pytest.mark.parametrize("dtype", ["u32", "f32"])
def test_presorted_in_place_and_unaligned(orc, dtype):
    """The presorted path's copy when the output is the input (odd pass
    counts: the first sweep writes the workspace) and on views offset by one
    element (4-byte aligned only)."""
    for runs in (2, 3, 4, 5, 17):
        t = 2048 * 8 if dtype == "u32" else 1024 * 8
        n = runs * t - 7
        x = orc.sort(make_keys(n + 1, dtype, seed=runs), dtype=dtype, stable=True)
        ref = x[1:]
        say(f"presorted in place dtype={dtype} n={n}")
        buf = gpu(x[1:].copy())
        msn.sort(buf, out=buf)
        assert np.array_equal(bits(host(buf)), bits(ref)), (runs, "in place")
        say(f"presorted unaligned dtype={dtype} n={n}")
        view = gpu(x)[1:]
        y = host(msn.sort(view))
        assert np.array_equal(bits(y), bits(ref)), (runs, "unaligned")
        ko, po = msn.sort_pairs(view)
        assert np.array_equal(bits(host(ko)), bits(ref)), (runs, "argsort keys")
        assert np.array_equal(host(po), np.arange(n, dtype=np.int32)), (runs, "argsort")


@pytest.mark.parametrize("dtype", ["u32", "i32", "f32"])
def test_classical_leaf(orc, dtype):
    """No networks at all (merges from runs of one key: the classical merge
    sort the paper measures against): keys, pairs and argsort against the
    oracle's merge sort with the empty network set, over the first-sweep tile
    shapes and both pass plans; the segmented sort refuses this leaf."""
    rng = np.random.default_rng(41)
    sizes = [0, 1, 2, 3, 7, 16, 17, 1023, 1025, 8191, 8193, 16385, 100003, 262145, 1_000_000]
    for n in sizes:
        x = make_keys(n, dtype, seed=n + 3)
        ref = orc.sort(x, dtype=dtype, stable=True, config=0)
        tunings = [None] if dtype == "f32" else [None, {"block_tile": 8192},
                                                 {"block_tile": 32768}, {"merge_ways": 2}]
        for t in tunings:
            say(f"classical sort_keys dtype={dtype} n={n} tuning={t}")
            y = host(msn.sort(gpu(x), leaf="classical", tuning=t))
            assert np.array_equal(bits(y), bits(ref)), (n, t)
        v = rng.integers(0, 2**32, n, dtype=np.uint32)
        say(f"classical sort_pairs dtype={dtype} n={n}")
        ko, vo = msn.sort_pairs(gpu(x), gpu(v), leaf="classical")
        rk, rv = orc.sort(x, vals=v, dtype=dtype, stable=True, config=0)
        assert np.array_equal(bits(host(ko)), bits(rk)), n
        assert np.array_equal(host(vo), rv), n
        _, po = msn.sort_pairs(gpu(x), None, leaf="classical")
        _, rp = orc.sort(x, dtype=dtype, stable=True, config=0, want_perm=True)
        assert np.array_equal(host(po).view(np.uint32), rp), n
    if dtype != "f32":
        for dist in ("sorted", "nearly"):
            x = workloads.keys(1_000_000, dist, dtype, 5)
            say(f"classical sort_keys dtype={dtype} 1e6 {dist}")
            y = host(msn.sort(gpu(x), leaf="classical"))
            assert np.array_equal(y, orc.sort(x, dtype=dtype, config=0)), dist
    off = gpu(np.array([0, 5, 9], dtype=np.uint32))
    with pytest.raises(msn.MsnError):
        msn.segmented_sort(gpu(make_keys(9, dtype, seed=1)), off, leaf="classical")


def test_unaligned_views(orc):
    # offsets by one element: 4-byte aligned, not 16-byte aligned
    n = 50001
    x = make_keys(n + 1, "i32", seed=1)
    t = gpu(x)[1:]
    say("sort_keys on a view offset by one element")
    y = host(msn.sort(t))
    assert np.array_equal(y, orc.sort(x[1:], dtype="i32"))


def test_sort_is_deterministic():
    x = gpu(make_keys(1 << 20, "f32", seed=2))
    say("sort_pairs f32 twice")
    a = msn.sort_pairs(x)
    b = msn.sort_pairs(x)
    assert torch.equal(a[0].view(torch.int32), b[0].view(torch.int32))
    assert torch.equal(a[1], b[1])


@pytest.mark.parametrize("pairs", [False, True])
def test_flat_sort_graph_replay(orc, pairs):
    # the benchmark's launch configuration: one call captured in a HIP graph,
    # replayed several times with eager work and synchronisations between
    n = 3_000_017
    x = workloads.keys(n, "random", "u32", seed=31)
    v = np.arange(n, dtype=np.uint32)[::-1].copy()
    if pairs:
        rk, rv = orc.sort(x, vals=v, dtype="u32", stable=True)
    else:
        rk = orc.sort(x, dtype="u32")
    plan = msn.SortPlan(n, torch.uint32, "cuda:0", pairs=pairs)
    xs, vs = gpu(x), gpu(v)
    run = (lambda: plan.run(xs, vs)) if pairs else (lambda: plan.run(xs))
    run()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        run()
    for rep in range(3):
        plan.out.fill_(0)
        if pairs:
            plan.out_vals.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"flat graph replay {rep} pairs={pairs}")
        assert np.array_equal(host(plan.out), rk), rep
        if pairs:
            assert np.array_equal(host(plan.out_vals), rv), rep


def test_packed_composite_edges(orc):
    # Stable tiles of 8192 pairs whose keys all fit 19 bits sort 32-bit
    # (key << 13 | position) composites.  Key 2^19 - 1 at tile position 8191
    # makes the composite all ones, the value that pads short tiles; a single
    # key of 2^19 must keep its tile on 64-bit composites.
    tile = 8192
    rng = np.random.default_rng(77)
    n = 4 * tile + 123
    k = rng.integers(0, 1 << 19, n, dtype=np.uint32)
    top = (1 << 19) - 1
    k[tile - 1] = top                       # tile 0: the all-ones composite
    k[tile + 4000] = 1 << 19                # tile 1: one key too wide to pack
    k[2 * tile: 3 * tile: 7] = top          # tile 2: many ties at the top key ...
    k[3 * tile - 1] = top                   # ... and the all-ones composite
    k[3 * tile + 50] = top                  # the short last tile also holds it
    k[-1] = top
    v = rng.integers(0, 2**32, n, dtype=np.uint32)
    rk, rv = orc.sort(k, vals=v, dtype="u32", stable=True)
    for dtype in ("u32", "i32"):
        kk = k if dtype == "u32" else k.view(np.int32)
        rkk = rk if dtype == "u32" else rk.view(np.int32)
        ko, vo = msn.sort_pairs(gpu(kk), gpu(v))
        assert np.array_equal(host(ko), rkk), dtype
        assert np.array_equal(host(vo), rv), dtype
        ko, po = msn.sort_pairs(gpu(kk))
        _, rp = orc.sort(kk, dtype=dtype, stable=True, want_perm=True)
        assert np.array_equal(host(po).view(np.uint32), rp), dtype


def test_packed_and_wide_tiles_across_flag_windows(orc):
    # The stable first sweep sorts packable tiles in one launch and flags the
    # others for a second, which scans the flags 64 tiles at a time: wide
    # tiles at both ends of a window, in later windows, and the ragged last
    # tile; argsort (positions as payload) takes the same two launches.
    tile = 8192
    rng = np.random.default_rng(91)
    ntiles = 150
    n = (ntiles - 1) * tile + 77
    k = rng.integers(0, 1 << 16, n, dtype=np.uint32)
    for t in (0, 63, 64, 100, 127, 128, ntiles - 1):
        lo = t * tile
        k[lo + (rng.integers(0, min(tile, n - lo)))] = np.uint32(rng.integers(1 << 19, 2**32))
    v = rng.integers(0, 2**32, n, dtype=np.uint32)
    say(f"packed and wide tiles: n={n}")
    rk, rv = orc.sort(k, vals=v, dtype="u32", stable=True)
    ko, vo = msn.sort_pairs(gpu(k), gpu(v))
    assert np.array_equal(host(ko), rk) and np.array_equal(host(vo), rv)
    _, po = msn.sort_pairs(gpu(k))
    _, rp = orc.sort(k, dtype="u32", stable=True, want_perm=True)
    assert np.array_equal(host(po).view(np.uint32), rp)
    # every tile wide, and every tile packed
    for kk in (rng.integers(0, 2**32, n, dtype=np.uint32), k & np.uint32(0xffff)):
        rk, rv = orc.sort(kk, vals=v, dtype="u32", stable=True)
        ko, vo = msn.sort_pairs(gpu(kk), gpu(v))
        assert np.array_equal(host(ko), rk) and np.array_equal(host(vo), rv)


def _cpu_corank(a, b, d):
    """Elements of a among the first d outputs of the stable merge of a and b
    (a first on equal keys): the merge itself, step by step."""
    i = j = 0
    for _ in range(d):
        if j >= len(b) or (i < len(a) and not b[j] < a[i]):
            i += 1
        else:
            j += 1
    return i


@pytest.mark.parametrize("dtype", ["u32", "i32", "f32"])
def test_merge_path_split_matches_cpu(dtype):
    from paper_2503_05934_amd import _lib

    rng = np.random.default_rng(5)
    cases = [(0, 0), (0, 5), (5, 0), (1, 1), (7, 300), (300, 7), (257, 256), (1000, 1000)]
    for la, lb in cases:
        for hi in (3, 1000, 2**31):  # heavy ties, some ties, distinct
            a = np.sort(make_keys(la, dtype, seed=la * 7 + lb)[:la] if dtype == "f32"
                        else rng.integers(0, min(hi, 2**31), la).astype(NPT[dtype]))
            b = np.sort(make_keys(lb, dtype, seed=lb * 11 + la)[:lb] if dtype == "f32"
                        else rng.integers(0, min(hi, 2**31), lb).astype(NPT[dtype]))
            if dtype == "f32":  # order by the float rule: NaNs last, -0 == +0
                a = np.sort(a)
                b = np.sort(b)
            diags = np.arange(-1, la + lb + 2, dtype=np.int32)
            out = torch.empty(len(diags), dtype=torch.int32, device="cuda:0")
            ag, bg, dg = gpu(a), gpu(b), gpu(diags)
            L = _lib.lib()
            rc = L.msn_merge_path_split(_lib.ptr(ag) if la else None, la,
                                        _lib.ptr(bg) if lb else None, lb, _lib.ptr(dg),
                                        _lib.ptr(out), len(diags), {"u32": 0, "i32": 1, "f32": 2}[dtype],
                                        _lib.stream_handle(out.device))
            assert rc == 0
            got = host(out)
            # the float order: -0 == +0, every NaN above +inf and all NaNs equal
            ka = [(1, 0.0) if np.isnan(v) else (0, v) for v in a.tolist()]
            kb = [(1, 0.0) if np.isnan(v) else (0, v) for v in b.tolist()]
            want = [-1] + [_cpu_corank(ka, kb, d) for d in range(la + lb + 1)] + [-1]
            assert got.tolist() == want, (dtype, la, lb, hi)
            if dtype == "f32":
                break


NPT = {"u32": np.uint32, "i32": np.int32}
