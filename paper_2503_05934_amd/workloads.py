"""Seeded synthetic inputs with the shapes of the paper's workloads.

The paper sorts random, sorted and nearly sorted arrays of 10,000 to 1,000,000
keys (Sec. 3, Table 2); it names no dataset.  These generators produce those
three distributions, at the sizes used here for measurement, plus the batched
(many uneven arrays) and row-wise fp32 inputs.  Every input is a pure function
of its seed.  Nothing in this module sorts with the method under test: the
"sorted" inputs use numpy's own sort to build the data.

Recipes
-------
* keys(n, dist, dtype, seed): uniform random integers over [0, 2^31) for int32
  and over [0, 2^32) for uint32 (or ``[0, hi)`` when ``hi`` is given); "sorted"
  is numpy's ascending sort of that draw; "nearly" is the sorted array after
  floor(n/100) sequential swaps of positions (i_t, j_t), both drawn uniformly
  from [0, n) with the same generator.
* segments(S, ...): lengths floor(exp(U(ln lo, ln(hi+1)))) clipped to [lo, hi],
  CSR uint32 offsets, uniform int32 keys in [0, 2^31), and a random 30 % of the
  segments sorted ascending in place.
* rows(...): Normal(0, 1) float32 rows from torch's CPU generator; "tiefree"
  redraws any row that holds an exact duplicate; "ties" rounds to multiples of
  1/64 (which also yields -0.0); grad_out is Normal(0, 1) from seed + 1.
"""
from __future__ import annotations

import numpy as np

DISTRIBUTIONS = ("random", "sorted", "nearly")


def keys(n: int, dist: str = "random", dtype: str = "u32", seed: int = 0, hi: int | None = None):
    """One array of n keys of the given distribution ("random", "sorted", "nearly")."""
    if dist not in DISTRIBUTIONS:
        raise ValueError(f"unknown distribution {dist!r}")
    rng = np.random.default_rng(seed)
    if dtype == "u32":
        x = rng.integers(0, 2**32 if hi is None else hi, n, dtype=np.uint32)
    elif dtype == "i32":
        x = rng.integers(0, 2**31 if hi is None else hi, n, dtype=np.int32)
    else:
        raise ValueError(f"keys() draws integer keys, not {dtype!r}")
    if dist == "random":
        return x
    x = np.sort(x)
    if dist == "nearly":
        m = n // 100
        i = rng.integers(0, n, m)
        j = rng.integers(0, n, m)
        for a, b in zip(i.tolist(), j.tolist()):
            x[a], x[b] = x[b], x[a]
    return x


def pairs(n: int, seed: int = 0, key_hi: int = 2**16):
    """Keys drawn from [0, key_hi) (many ties) with payload = original index."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, key_hi, n, dtype=np.uint32)
    return k, np.arange(n, dtype=np.uint32)


def segment_lengths(num_segments: int, seed: int = 0, lo: int = 3, hi: int = 65536):
    rng = np.random.default_rng(seed)
    u = rng.uniform(np.log(lo), np.log(hi + 1), num_segments)
    return np.clip(np.floor(np.exp(u)), lo, hi).astype(np.int64), rng


def segments(num_segments: int = 100_000, seed: int = 0, lo: int = 3, hi: int = 65536,
             presorted_frac: float = 0.3):
    """Batched input: (keys int32, offsets uint32[S+1], presorted bool[S])."""
    lengths, rng = segment_lengths(num_segments, seed, lo, hi)
    offsets = np.zeros(num_segments + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    if offsets[-1] >= 2**32:
        raise ValueError("total length does not fit uint32 offsets")
    total = int(offsets[-1])
    k = rng.integers(0, 2**31, total, dtype=np.int32)
    presorted = rng.random(num_segments) < presorted_frac
    for s in np.nonzero(presorted)[0].tolist():
        a, b = int(offsets[s]), int(offsets[s + 1])
        k[a:b].sort()
    return k, offsets.astype(np.uint32), presorted


def rows(num_rows: int = 4096, cols: int = 8192, variant: str = "tiefree", seed: int = 0):
    """fp32 rows ~ Normal(0,1): (x [R, C] float32 numpy, grad_out [R, C], redraws).

    ``variant`` is "tiefree" (rows with an exact duplicate are redrawn; the
    number of redraws is returned) or "ties" (values rounded to 1/64).
    """
    import torch

    g = torch.Generator().manual_seed(seed)
    x = torch.randn(num_rows, cols, generator=g)
    redraws = 0
    if variant == "tiefree":
        while True:
            s, _ = torch.sort(x, dim=1)
            dup = (s[:, 1:] == s[:, :-1]).any(dim=1)
            bad = torch.nonzero(dup).flatten()
            if bad.numel() == 0:
                break
            redraws += int(bad.numel())
            x[bad] = torch.randn(int(bad.numel()), cols, generator=g)
    elif variant == "ties":
        x = torch.round(x * 64) / 64
    else:
        raise ValueError(f"unknown rows variant {variant!r}")
    gg = torch.Generator().manual_seed(seed + 1)
    grad = torch.randn(num_rows, cols, generator=gg)
    return x.numpy(), grad.numpy(), redraws
