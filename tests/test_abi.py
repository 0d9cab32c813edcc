"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msn.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2503_05934_amd import _lib, build

    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msn_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_entry_points():
    names = declared_functions()
    for fn in ("msn_sort_keys", "msn_sort_pairs", "msn_segmented_sort", "msn_sort_backward"):
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_status_strings(lib):
    assert lib.msn_version() >= 10000
    for code in (0, -1, -2, -3, -4, -5, -6, 1):
        assert lib.msn_status_string(code)


FAKE = ctypes.c_void_p(1 << 20)         # never dereferenced: every call below is rejected
FAKE2 = ctypes.c_void_p(3 << 20)
ODD = ctypes.c_void_p((1 << 20) + 2)    # not 4-byte aligned


def keys(lib, kin=FAKE, kout=FAKE2, n=100, dtype=0, leaf=0, tuning=None, ws=FAKE, wsb=1 << 30):
    return lib.msn_sort_keys(kin, kout, n, dtype, leaf, tuning, ws, wsb, None)


def test_sort_keys_argument_errors(lib):
    assert keys(lib, dtype=7) == -3
    assert keys(lib, leaf=12) == -4
    assert keys(lib, leaf=-1) == -4
    assert keys(lib, n=-1) == -2
    assert keys(lib, n=1 << 31) == -2
    assert keys(lib, kin=None) == -1
    assert keys(lib, kout=None) == -1
    assert keys(lib, ws=None) == -5
    assert keys(lib, wsb=16) == -5
    assert keys(lib, kin=ODD) == -6
    # partial overlap of input and output
    assert keys(lib, kin=FAKE, kout=ctypes.c_void_p((1 << 20) + 64), n=100) == -2
    from paper_2503_05934_amd import _lib
    bad = _lib.Tuning(merge_tile=1000)
    assert keys(lib, tuning=ctypes.byref(bad)) == -4
    # nothing to do: n == 0 needs no pointers
    assert lib.msn_sort_keys(None, None, 0, 0, 0, None, None, 0, None) == 0


def test_sort_pairs_argument_errors(lib):
    f = lib.msn_sort_pairs
    assert f(FAKE, None, FAKE2, None, 10, 0, 0, None, FAKE, 1 << 30, None) == -1  # vals_out
    assert f(FAKE, None, FAKE2, FAKE2, 10, 0, 0, None, FAKE, 1 << 30, None) == -2  # keys_out == vals_out
    assert f(FAKE, None, FAKE2, ctypes.c_void_p(5 << 20), 10, 2, 0, None, FAKE, 8, None) == -5


def test_segmented_argument_errors(lib):
    f = lib.msn_segmented_sort
    off = FAKE

    def call(kin=FAKE, vin=None, kout=FAKE2, vout=None, offsets=off, S=10, n=100, dtype=1,
             leaf=0, flags=0, tuning=None, ws=ctypes.c_void_p(9 << 20), wsb=1 << 30):
        return f(kin, vin, kout, vout, offsets, S, n, dtype, leaf, flags, tuning, ws, wsb, None)

    assert call(S=-1) == -2
    assert call(S=0, n=5) == -2
    assert call(S=0, n=0) == 0
    assert call(offsets=None, S=7, n=100) == -2          # rows must divide n
    assert call(flags=4) == -4
    assert call(flags=1, vin=FAKE) == -4                  # argsort takes no vals_in
    assert call(flags=1) == -1                            # argsort needs vals_out
    assert call(vout=ctypes.c_void_p(7 << 20)) == -4      # vals_out without vals_in or argsort
    assert call(dtype=5) == -3
    assert call(leaf=12) == -4
    assert call(leaf=2) == -6                             # no network: flat sorts only
    assert call(wsb=0) == -5
    from paper_2503_05934_amd import _lib
    for bad in (dict(seg_lane_max=9), dict(seg_wave_max=10000), dict(seg_block_max=9000),
                dict(seg_lane_max=8, seg_wave_max=4), dict(seg_grid=-1)):
        t = _lib.make_tuning(bad)
        assert call(tuning=ctypes.byref(t)) == -4, bad


def test_backward_argument_errors(lib):
    f = lib.msn_sort_backward
    assert f(FAKE, FAKE2, ctypes.c_void_p(5 << 20), -1, 4, None) == -2
    assert f(None, FAKE2, ctypes.c_void_p(5 << 20), 2, 4, None) == -1
    assert f(FAKE, FAKE2, FAKE, 2, 4, None) == -2                     # grad_in == grad_out
    assert f(FAKE, FAKE2, ctypes.c_void_p((1 << 20) + 8), 2, 4, None) == -2
    assert f(None, None, None, 0, 5, None) == 0


def test_workspace_queries(lib):
    from paper_2503_05934_amd import _lib
    a = _lib.sort_workspace_bytes(1 << 20, 0, False)
    b = _lib.sort_workspace_bytes(1 << 20, 0, True)
    assert a >= 4 << 20 and b >= 8 << 20 and b > a
    s = _lib.segmented_workspace_bytes(1000, 10, 2, True)
    assert s >= 8000
    out = ctypes.c_size_t()
    assert lib.msn_sort_workspace_bytes(-5, 0, 0, ctypes.byref(out)) == -2
    assert lib.msn_sort_workspace_bytes(5, 9, 0, ctypes.byref(out)) == -3


def test_values_may_not_overlap_the_other_array(lib):
    # a key array and a value array never share words, in-place calls included
    f = lib.msn_sort_pairs
    V = ctypes.c_void_p(5 << 20)
    assert f(FAKE, None, FAKE2, FAKE, 10, 0, 0, None, ctypes.c_void_p(9 << 20), 1 << 30, None) == -2
    assert f(FAKE, FAKE2, FAKE2, V, 10, 0, 0, None, ctypes.c_void_p(9 << 20), 1 << 30, None) == -2
    assert f(FAKE, V, FAKE, ctypes.c_void_p((5 << 20) + 8), 10, 0, 0, None,
             ctypes.c_void_p(9 << 20), 1 << 30, None) == -2          # vals partly in place
    g = lib.msn_segmented_sort
    ws = ctypes.c_void_p(9 << 20)
    # offsets inside the key output
    assert g(FAKE, None, FAKE2, None, ctypes.c_void_p((3 << 20) + 40), 10, 100, 1, 0, 0, None,
             ws, 1 << 30, None) == -2
    # keys_in overlapping vals_out
    assert g(FAKE, None, FAKE2, FAKE, ctypes.c_void_p(7 << 20), 10, 100, 1, 0, 1, None,
             ws, 1 << 30, None) == -2
    # offsets (11 words) ending just before the key output, which is longer: no overlap,
    # so validation passes and the call goes on to launch (rc 100 without a GPU)
    if not _gpu_present():
        assert g(FAKE, None, FAKE2, None, ctypes.c_void_p((3 << 20) - 44), 10, 100, 1, 0, 0,
                 None, ws, 1 << 30, None) > 0


def _gpu_present():
    import torch
    return torch.cuda.is_available()


def test_workspace_query_names_agree(lib):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    for n, pairs in ((0, 0), (1000, 0), (1 << 20, 1), ((1 << 31) - 1, 1)):
        assert lib.msn_sort_keys_workspace_bytes(n, 0, pairs, ctypes.byref(a)) == 0
        assert lib.msn_sort_workspace_bytes(n, 0, pairs, ctypes.byref(b)) == 0
        assert a.value == b.value


def test_segmented_status_offset(lib):
    from paper_2503_05934_amd import _lib
    for n, S, pairs in ((100, 10, False), (651_672_148, 100_000, False), (33_554_432, 4096, True)):
        off = _lib.segmented_status_offset(n, S, pairs)
        ws = _lib.segmented_workspace_bytes(n, S, 0, pairs)
        assert off % 4 == 0 and off + 4 <= ws
    out = ctypes.c_size_t()
    assert lib.msn_segmented_status_offset(-1, 3, 0, ctypes.byref(out)) == -2
    assert lib.msn_segmented_status_offset(3, 3, 0, None) == -1


def test_segmented_accepts_debug_check_flag(lib):
    f = lib.msn_segmented_sort
    # MSN_ARGSORT | MSN_DEBUG_CHECK is a valid flag set (rejected later for the NULL workspace)
    assert f(FAKE, None, FAKE2, ctypes.c_void_p(7 << 20), FAKE, 10, 100, 1, 0, 3, None, None, 0,
             None) == -5
    assert f(FAKE, None, FAKE2, None, FAKE, 10, 100, 1, 0, 2 | 4, None, None, 0, None) == -4


def test_every_leaf_set_passes_validation(lib):
    # each Table 3 code is accepted: with a zero-length array the call returns
    # before anything could be launched
    for code in range(12):
        assert lib.msn_sort_keys(None, None, 0, 0, code, None, None, 0, None) == 0, code
        assert lib.msn_sort_pairs(None, None, None, None, 0, 0, code, None, None, 0, None) == 0
        assert lib.msn_quick_sort_keys(None, None, 0, 0, code, None, None, 0, None) == 0
    for code in (12, 13, 100):
        assert lib.msn_sort_keys(None, None, 0, 0, code, None, None, 0, None) == -4
