"""msn_sort_keys_noalloc through the C ABI: the same bits as msn_sort_keys,
call after call on the library's one scratch array per device."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import DEV, gpu, host, make_keys, say
from paper_2503_05934_amd import _lib

pytestmark = pytest.mark.gpu

DT = {"u32": _lib.MSN_U32, "i32": _lib.MSN_I32, "f32": _lib.MSN_F32}


def with_workspace(x, dtype, leaf):
    """msn_sort_keys with a workspace from torch: the entry point the
    allocation-free call must match."""
    L = _lib.lib()
    out = torch.empty_like(x)
    ws = torch.empty(_lib.sort_workspace_bytes(x.numel(), DT[dtype], False), dtype=torch.uint8,
                     device=DEV)
    _lib.check("msn_sort_keys", L.msn_sort_keys(
        _lib.ptr(x), _lib.ptr(out), x.numel(), DT[dtype], leaf, None, _lib.ptr(ws), ws.numel(),
        _lib.stream_handle(x.device)))
    return out


def without_workspace(x, dtype, leaf, out=None):
    L = _lib.lib()
    out = torch.empty_like(x) if out is None else out
    _lib.check("msn_sort_keys_noalloc", L.msn_sort_keys_noalloc(
        _lib.ptr(x), _lib.ptr(out), x.numel(), DT[dtype], leaf, None,
        _lib.stream_handle(x.device)))
    return out


@pytest.mark.parametrize("dtype,leaf", [("u32", 0), ("i32", 1), ("f32", 0), ("i32", 2)])
def test_noalloc_matches_workspace_call_twice(dtype, leaf):
    # a large call, then a smaller one on the scratch the first left behind
    for n, seed, dist in ((_lib.MSN_NOALLOC_MAX_KEYS - 5, 11, "random"),
                          (300_001, 12, "random"), (70_001, 13, "sorted")):
        if dtype == "f32" and dist == "sorted":
            dist = "random"
        say(f"noalloc {dtype} leaf {leaf} n={n} {dist}")
        x = gpu(make_keys(n, dtype, seed, dist))
        ref = with_workspace(x, dtype, leaf)
        got = without_workspace(x, dtype, leaf)
        torch.cuda.synchronize()
        assert np.array_equal(host(got).view(np.uint32), host(ref).view(np.uint32)), (dtype, n)


def test_noalloc_maximum_size_and_in_place():
    n = _lib.MSN_NOALLOC_MAX_KEYS
    say(f"noalloc maximum n={n}, in place")
    x = gpu(make_keys(n, "u32", 21))
    ref = with_workspace(x, "u32", 0)
    without_workspace(x, "u32", 0, out=x)
    torch.cuda.synchronize()
    assert np.array_equal(host(x), host(ref))
    y = gpu(make_keys(1000, "u32", 22))
    ref = with_workspace(y, "u32", 0)
    assert np.array_equal(host(without_workspace(y, "u32", 0)), host(ref))


def test_noalloc_rejects_beyond_maximum_before_launch():
    L = _lib.lib()
    n = _lib.MSN_NOALLOC_MAX_KEYS + 1
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: the size check comes first
    assert L.msn_sort_keys_noalloc(fake, ctypes.c_void_p(1 << 30), n, 0, 0, None, None) == -2
    assert L.msn_sort_keys_noalloc(None, None, 0, 0, 0, None, None) == 0
