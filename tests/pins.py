"""Pins for the CPU oracle: checks against facts that do not come from it.

Each ``pin_*`` function takes an :class:`oracle.Oracle` and raises
AssertionError on any disagreement.  The sources of truth are
  * the paper's printed tables and its worked 6-to-8 example (golden files),
  * textbook facts about sorting networks (0-1 principle, optimal sizes,
    Batcher's closed forms),
  * brute force over every input of tiny sizes,
  * numpy / torch library sorts (stable) as independent implementations,
  * calculus (finite differences) for the backward.
``test_oracle.py`` runs them on the real oracle; ``test_oracle_plants.py``
runs them on copies of the oracle with planted mistakes and expects failures.
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

ALL_CONFIGS = ["PowerOf2", "Even", "Odd", "3", "3To4", "3To5", "3To8", "6To8",
               "VarSort3", "VarSort4", "VarSort5", "Classical"]


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


# --------------------------------------------------------------- networks ---

def pin_network_zero_one(orc):
    """0-1 principle: a comparator network sorts every input iff it sorts all
    2^n zero-one inputs (Knuth, TAOCP 3, Sec. 5.3.4)."""
    for n in range(1, 9):
        ins = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.uint32).reshape(-1, n)
        out, _ = orc.apply_network(n, ins)
        assert np.array_equal(out, np.sort(ins, axis=1)), f"n={n} fails a 0-1 input"


def pin_network_permutations(orc):
    """Every permutation of 0..n-1 comes out as 0..n-1 (n <= 8)."""
    for n in range(1, 9):
        ins = np.array(list(itertools.permutations(range(n))), dtype=np.uint32)
        out, perm = orc.apply_network(n, ins)
        assert (out == np.arange(n, dtype=np.uint32)).all(), f"n={n}"
        # perm says where each output came from
        assert np.array_equal(np.take_along_axis(ins, perm.astype(np.int64), 1), out)


def pin_network_sizes(orc):
    """Comparator counts equal the proven minimum for n <= 8 (golden table),
    and the 8-network has Batcher's depth k(k+1)/2 = 6."""
    for n_s, c_s in _golden_rows("optimal_networks.txt"):
        n, c = int(n_s), int(c_s)
        net = orc.network(n)
        assert len(net) == c, f"n={n}: {len(net)} comparators, minimum is {c}"
        assert all(0 <= i < j < max(n, 1) for i, j in net)
    k = 3
    net = orc.network(8)
    assert len(net) == (k * k - k + 4) * 2 ** (k - 2) - 1
    depth = [0] * 8
    for i, j in net:
        d = max(depth[i], depth[j]) + 1
        depth[i] = depth[j] = d
    assert max(depth) == k * (k + 1) // 2


def pin_network_stability(orc):
    """With (key, position) comparison every tie pattern over {0,1,2}^n leaves
    equal keys in input order; with keys alone n >= 3 networks are unstable."""
    for n in range(2, 9):
        ins = np.array(list(itertools.product([0, 1, 2], repeat=n)), dtype=np.uint32)
        out, perm = orc.apply_network(n, ins, stable=True)
        assert np.array_equal(out, np.sort(ins, axis=1))
        ref = np.argsort(ins, axis=1, kind="stable")
        assert np.array_equal(perm, ref.astype(np.uint32)), f"n={n} unstable"
        if n >= 3:
            _, p2 = orc.apply_network(n, ins, stable=False)
            assert not np.array_equal(p2, ref.astype(np.uint32))


# ----------------------------------------------------------- configurations --

def pin_table3(orc):
    """The oracle's configuration sets equal Table 3."""
    for row in _golden_rows("table3_configs.txt"):
        name, sizes = row[0], [int(s) for s in row[1:]]
        assert orc.config_mask(name) == sum(1 << s for s in sizes), name


def pin_alg1_leaves(orc):
    """Leaf sizes Algorithm 1 reaches, worked by hand from its definition."""
    for row in _golden_rows("alg1_leaves.txt"):
        n, cfg, hist = int(row[0]), row[1], [int(v) for v in row[2:]]
        assert list(orc.leaf_histogram(n, cfg)) == hist, f"n={n} {cfg}"


# -------------------------------------------------------------- whole sorts --

def _arrays(rng):
    """Small arrays of every shape that tends to break sorts."""
    out = []
    for n in list(range(0, 40)) + [63, 64, 65, 127, 128, 129, 257, 1000, 2049]:
        out.append(rng.integers(0, 2**32, n, dtype=np.uint32))
        out.append(np.sort(rng.integers(0, 2**32, n, dtype=np.uint32)))
        out.append(np.sort(rng.integers(0, 2**32, n, dtype=np.uint32))[::-1].copy())
        out.append(np.full(n, 7, dtype=np.uint32))
        out.append(rng.integers(0, 2, n, dtype=np.uint32))
        out.append(rng.integers(0, 5, n, dtype=np.uint32))
    return out


def pin_sorts_vs_numpy(orc):
    """Algorithms 1 and 2 under every Table 3 configuration agree with numpy's
    stable sort: keys, payload and original positions."""
    rng = np.random.default_rng(1234)
    arrays = _arrays(rng)
    for algo in ("ms", "qs"):
        for cfg in ALL_CONFIGS:
            for a in arrays:
                k, v, p = orc.sort(a, vals=(a * 3 + 1).astype(np.uint32), algo=algo,
                                   config=cfg, stable=True, want_perm=True)
                ref = np.argsort(a, kind="stable")
                assert np.array_equal(k, a[ref]), (algo, cfg, a.shape)
                assert np.array_equal(p, ref.astype(np.uint32)), (algo, cfg, a.shape)
                assert np.array_equal(v, (a[ref] * 3 + 1).astype(np.uint32))
                kk = orc.sort(a, algo=algo, config=cfg, stable=False)
                assert np.array_equal(kk, np.sort(a)), (algo, cfg, "keys-only")
    # The classical merge sort is stable on keys alone: Merge takes the left
    # run's element on ties, so no position tie-break is needed.
    for a in arrays:
        _, p = orc.sort(a, algo="ms", config="Classical", stable=False, want_perm=True)
        assert np.array_equal(p, np.argsort(a, kind="stable").astype(np.uint32)), a.shape


def pin_sorts_brute_force(orc):
    """Every permutation (n <= 7) and every {0,1,2}^n (n <= 8) input, as one
    batch of segments, under both algorithms and the paper's main configs."""
    segs = []
    for n in range(0, 8):
        segs += [np.array(p, dtype=np.uint32) for p in itertools.permutations(range(n))]
    for n in range(0, 9):
        segs += [np.array(t, dtype=np.uint32) for t in itertools.product([0, 1, 2], repeat=n)]
    lens = np.array([len(s) for s in segs])
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint32)
    flat = np.concatenate(segs).astype(np.uint32)
    expect_k = np.concatenate([np.sort(s) for s in segs]).astype(np.uint32)
    expect_p = np.concatenate([np.argsort(s, kind="stable") for s in segs]).astype(np.uint32)
    for algo in ("ms", "qs"):
        for cfg in ("Classical", "6To8", "3To5", "3To8", "VarSort4", "PowerOf2"):
            k, p = orc.segmented_sort(flat, off, algo=algo, config=cfg, stable=True,
                                      want_perm=True)
            assert np.array_equal(k, expect_k), (algo, cfg)
            assert np.array_equal(p, expect_p), (algo, cfg)


def pin_dtype_orders(orc):
    """int32 is signed, uint32 unsigned, float32 is IEEE '<' with -0 == +0
    tied and NaNs (any payload) after +inf, tied: the same order as
    torch.sort(stable=True) and numpy's stable sort."""
    import torch

    rng = np.random.default_rng(7)
    i32 = rng.integers(-2**31, 2**31, 3000, dtype=np.int64).astype(np.int32)
    i32[:4] = [-2**31, 2**31 - 1, -1, 0]
    for algo in ("ms", "qs"):
        k = orc.sort(i32, dtype="i32", algo=algo, stable=True)
        assert np.array_equal(k, np.sort(i32)), algo
        u = i32.view(np.uint32)
        k = orc.sort(u, dtype="u32", algo=algo, stable=True)
        assert np.array_equal(k, np.sort(u)), algo

    specials = np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45, 3.0, -3.0],
                        dtype=np.float32)
    nan_bits = np.array([0x7fc00000, 0xffc00000, 0x7f800001, 0x7fbfffff], dtype=np.uint32)
    base = rng.standard_normal(2000).astype(np.float32)
    base = np.round(base * 8) / 8                       # many ties, and -0.0
    x = np.concatenate([base, specials, nan_bits.view(np.float32), specials]).astype(np.float32)
    x = x[rng.permutation(x.shape[0])]
    tv, ti = torch.sort(torch.from_numpy(x.copy()), stable=True)
    for algo in ("ms", "qs"):
        for cfg in ("Classical", "6To8", "3To5"):
            k, p = orc.sort(x, dtype="f32", algo=algo, config=cfg, stable=True, want_perm=True)
            assert np.array_equal(p.astype(np.int64), ti.numpy()), (algo, cfg)
            assert np.array_equal(k.view(np.uint32), x[ti.numpy()].view(np.uint32))
    # closed form for a few values: (-inf, -3, -0 / +0 in input order, 3, +inf, NaN, NaN)
    y = np.array([np.nan, 3.0, 0.0, -np.inf, -0.0, np.inf, -3.0, -np.nan], dtype=np.float32)
    _, p = orc.sort(y, dtype="f32", stable=True, want_perm=True)
    assert list(p) == [3, 6, 2, 4, 1, 5, 0, 7]


def pin_segmented(orc):
    """Per-segment results equal per-array numpy sorts; empty segments pass."""
    rng = np.random.default_rng(99)
    lens = rng.integers(0, 40, 300)
    lens[::17] = 0
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint32)
    x = rng.integers(-50, 50, int(off[-1])).astype(np.int32)
    for algo in ("ms", "qs"):
        k, p = orc.segmented_sort(x, off, dtype="i32", algo=algo, stable=True, want_perm=True)
        for s in range(300):
            a, b = off[s], off[s + 1]
            ref = np.argsort(x[a:b], kind="stable")
            assert np.array_equal(k[a:b], x[a:b][ref]), (algo, s)
            assert np.array_equal(p[a:b], ref.astype(np.uint32)), (algo, s)


def pin_row_argsort(orc):
    """Row argsort equals torch's stable sort per row, values as bit copies."""
    import torch

    g = torch.Generator().manual_seed(5)
    x = torch.round(torch.randn(12, 300, generator=g) * 16) / 16
    v, p = orc.row_argsort(x.numpy())
    tv, ti = torch.sort(x, dim=1, stable=True)
    assert np.array_equal(p, ti.numpy().astype(np.int32))
    assert np.array_equal(v.view(np.uint32), tv.numpy().view(np.uint32))


# ------------------------------------------------------------------ backward --

def pin_backward(orc):
    """The gather backward against calculus: for L(x) = <g, sort(x)> on
    tie-free rows, central finite differences in fp64 give dL/dx_j, which must
    equal grad_in[j]; also grad_in is a permutation of grad_out and
    <grad_in, x> == <grad_out, sort(x)> (fp64)."""
    rng = np.random.default_rng(3)
    rows, cols = 6, 64
    x = rng.standard_normal((rows, cols)).astype(np.float32)
    g = rng.standard_normal((rows, cols)).astype(np.float32)
    vals, perm = orc.row_argsort(x)
    gi = orc.gather_backward(g, perm)
    for r in range(rows):
        assert np.array_equal(np.sort(gi[r]), np.sort(g[r]))
        lhs = math.fsum((gi[r].astype(np.float64) * x[r].astype(np.float64)).tolist())
        rhs = math.fsum((g[r].astype(np.float64) * vals[r].astype(np.float64)).tolist())
        assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))

    def loss(xr, gr):
        return math.fsum((np.sort(xr) * gr).tolist())

    x64 = x.astype(np.float64)
    g64 = g.astype(np.float64)
    for r in range(rows):
        s = np.sort(x64[r])
        gaps = np.diff(s)
        for j in range(0, cols, 5):
            pos = int(np.searchsorted(s, x64[r, j]))
            lo = gaps[pos - 1] if pos > 0 else np.inf
            hi = gaps[pos] if pos < cols - 1 else np.inf
            gap = min(lo, hi)
            if gap < 1e-6:
                continue
            h = gap / 4
            xp = x64[r].copy()
            xm = x64[r].copy()
            xp[j] += h
            xm[j] -= h
            fd = (loss(xp, g64[r]) - loss(xm, g64[r])) / (2 * h)
            assert abs(fd - gi[r, j]) <= 1e-5 * max(1.0, abs(fd)), (r, j, fd, gi[r, j])


def pin_rank_bounds(orc):
    """Rank bounds equal numpy's searchsorted on the sorted keys."""
    rng = np.random.default_rng(11)
    for dtype, x in (("u32", rng.integers(0, 50, 5000, dtype=np.uint32)),
                     ("i32", rng.integers(-50, 50, 5000).astype(np.int32)),
                     ("f32", (np.round(rng.standard_normal(5000) * 4) / 4).astype(np.float32))):
        s = np.sort(x)
        for v in list(x[:40]) + [s[0], s[-1]]:
            lt, le = orc.rank_bounds(x, v, dtype=dtype)
            assert lt == int(np.searchsorted(s, v, side="left")), (dtype, v)
            assert le == int(np.searchsorted(s, v, side="right")), (dtype, v)


ALL_PINS = [
    pin_network_zero_one,
    pin_network_permutations,
    pin_network_sizes,
    pin_network_stability,
    pin_table3,
    pin_alg1_leaves,
    pin_sorts_vs_numpy,
    pin_sorts_brute_force,
    pin_dtype_orders,
    pin_segmented,
    pin_row_argsort,
    pin_backward,
    pin_rank_bounds,
]
