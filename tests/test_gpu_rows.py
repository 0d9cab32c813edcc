"""Row-wise fp32 sort (DiffSort forward) and the backward scatter, exact."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2503_05934_amd as msn
from paper_2503_05934_amd import workloads
from gpu_util import bits, gpu, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("variant", ["tiefree", "ties"])
def test_rows_forward_and_backward(orc, variant):
    x, g, redraws = workloads.rows(64, 8192, variant=variant, seed=0)
    say(f"sort_rows 64x8192 {variant} (redraws {redraws})")
    vals, perm = msn.sort_rows(gpu(x))
    rv, rp = orc.row_argsort(x)
    assert np.array_equal(bits(host(vals)), bits(rv))
    assert np.array_equal(host(perm), rp)
    say("sort_backward 64x8192")
    gi = host(msn.sort_backward(gpu(g), perm))
    assert np.array_equal(bits(gi), bits(orc.gather_backward(g, rp)))


@pytest.mark.parametrize("cols", [1, 3, 7, 8, 9, 100, 513, 4097, 8192, 8193, 20000, 40000])
def test_rows_odd_shapes(orc, cols):
    rows = 5
    rng = np.random.default_rng(cols)
    x = (np.round(rng.standard_normal((rows, cols)) * 16) / 16).astype(np.float32)
    g = rng.standard_normal((rows, cols)).astype(np.float32)
    say(f"sort_rows {rows}x{cols}")
    vals, perm = msn.sort_rows(gpu(x))
    rv, rp = orc.row_argsort(x)
    assert np.array_equal(bits(host(vals)), bits(rv))
    assert np.array_equal(host(perm), rp)
    say(f"sort_backward {rows}x{cols}")
    gi = host(msn.sort_backward(gpu(g), perm))
    assert np.array_equal(bits(gi), bits(orc.gather_backward(g, rp)))


def test_diffsort_autograd_and_finite_differences(orc):
    x, g, _ = workloads.rows(8, 512, variant="tiefree", seed=4)
    xt = gpu(x).requires_grad_(True)
    say("DiffSort forward/backward 8x512")
    y, perm = msn.DiffSort.apply(xt)
    assert not perm.requires_grad
    (y * gpu(g)).sum().backward()
    gi = host(xt.grad)
    assert np.array_equal(bits(gi), bits(orc.gather_backward(g, host(perm))))
    # central differences in fp64 on the CPU for L(x) = <g, sort(x)>
    x64, g64 = x.astype(np.float64), g.astype(np.float64)
    for r in range(x.shape[0]):
        s = np.sort(x64[r])
        gaps = np.diff(s)
        for j in range(0, x.shape[1], 37):
            pos = int(np.searchsorted(s, x64[r, j]))
            lo = gaps[pos - 1] if pos > 0 else np.inf
            hi = gaps[pos] if pos < len(gaps) else np.inf
            gap = min(lo, hi)
            if gap < 1e-6:
                continue
            h = gap / 4
            xp, xm = x64[r].copy(), x64[r].copy()
            xp[j] += h
            xm[j] -= h
            fd = (math.fsum(np.sort(xp) * g64[r]) - math.fsum(np.sort(xm) * g64[r])) / (2 * h)
            assert abs(fd - gi[r, j]) <= 1e-5 * max(1.0, abs(fd)), (r, j)


def test_backward_skips_out_of_range_indices():
    g = torch.arange(8, dtype=torch.float32, device="cuda:0").view(1, 8)
    p = torch.tensor([[7, 6, 5, 4, 3, 2, 1, 99]], dtype=torch.int32, device="cuda:0")
    say("sort_backward with an out-of-range index")
    gi = host(msn.sort_backward(g, p))
    assert list(gi[0, 1:]) == [6, 5, 4, 3, 2, 1, 0]


def test_backward_tall_narrow_rows(orc):
    """More rows than one workgroup per row can launch (2^24 + 1 rows of 4
    columns: 2^32 + 256 threads at 256 per row): the row loop covers them."""
    rows, cols = (1 << 24) + 1, 4
    rng = np.random.default_rng(5)
    g = rng.standard_normal((rows, cols)).astype(np.float32)
    p = np.argsort(rng.random((rows, cols)), axis=1).astype(np.int32)
    say(f"sort_backward {rows}x{cols}")
    gi = host(msn.sort_backward(gpu(g), gpu(p)))
    assert np.array_equal(bits(gi), bits(orc.gather_backward(g, p)))
