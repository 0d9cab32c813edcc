"""ctypes binding of libmsn.so (include/msn.h).

Argument marshalling only: every step of every sort runs in the library's
HIP kernels.  If the library is missing or cannot be loaded, every call raises
RuntimeError; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsn.so")

# include/msn.h constants
MSN_U32, MSN_I32, MSN_F32 = 0, 1, 2
MSN_LEAF_6TO8, MSN_LEAF_3TO5, MSN_LEAF_NONE = 0, 1, 2
MSN_LEAF_POW2, MSN_LEAF_EVEN, MSN_LEAF_ODD, MSN_LEAF_3, MSN_LEAF_3TO4, MSN_LEAF_3TO8 = 3, 4, 5, 6, 7, 8
MSN_LEAF_VARSORT3, MSN_LEAF_VARSORT4, MSN_LEAF_VARSORT5 = 9, 10, 11
MSN_ARGSORT = 1
MSN_DEBUG_CHECK = 2
MSN_SEG_BAD_FIRST, MSN_SEG_BAD_ORDER, MSN_SEG_BAD_LAST, MSN_SEG_BAD_RESULT = 1, 2, 4, 8
MSN_NOALLOC_MAX_KEYS = 4194304

# Table 3's names (and "classical" for the empty set)
LEAVES = {"6To8": MSN_LEAF_6TO8, "3To5": MSN_LEAF_3TO5, "classical": MSN_LEAF_NONE,
          "PowerOf2": MSN_LEAF_POW2, "Even": MSN_LEAF_EVEN, "Odd": MSN_LEAF_ODD, "3": MSN_LEAF_3,
          "3To4": MSN_LEAF_3TO4, "3To8": MSN_LEAF_3TO8, "VarSort3": MSN_LEAF_VARSORT3,
          "VarSort4": MSN_LEAF_VARSORT4, "VarSort5": MSN_LEAF_VARSORT5}
# keys of a lane's group under each set (8 or 4): the tile shapes follow it
GROUP_KEYS = {"6To8": 8, "3To5": 4, "classical": 8, "PowerOf2": 8, "Even": 8, "Odd": 8, "3": 4,
              "3To4": 4, "3To8": 8, "VarSort3": 4, "VarSort4": 4, "VarSort5": 8}
_DTYPES = {torch.uint32: MSN_U32, torch.int32: MSN_I32, torch.float32: MSN_F32}


class MsnError(RuntimeError):
    """A libmsn call returned a non-zero status."""

    def __init__(self, fn: str, status: int, text: str):
        super().__init__(f"{fn} failed with status {status}: {text}")
        self.status = status


class Tuning(ctypes.Structure):
    """msn_tuning: zero fields mean "default"."""

    _fields_ = [
        ("merge_tile", ctypes.c_int32),
        ("seg_lane_max", ctypes.c_int32),
        ("seg_wave_max", ctypes.c_int32),
        ("seg_block_max", ctypes.c_int32),
        ("seg_grid", ctypes.c_int32),
        ("block_tile", ctypes.c_int32),
        ("merge_ways", ctypes.c_int32),
        ("merge4_kpt", ctypes.c_int32),
        ("quick_rounds", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def make_tuning(params: dict | None) -> Tuning | None:
    if not params:
        return None
    t = Tuning()
    for k, v in params.items():
        setattr(t, k, int(v))
    return t


_lib = None


def lib():
    """The loaded library (loads it on first use, raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -m paper_2503_05934_amd.build` "
            "(needs hipcc with gfx950 support)")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint
    SZ = ctypes.POINTER(ctypes.c_size_t)
    L.msn_version.argtypes = []
    L.msn_version.restype = I
    L.msn_status_string.argtypes = [I]
    L.msn_status_string.restype = ctypes.c_char_p
    L.msn_sort_workspace_bytes.argtypes = [I64, I, I, SZ]
    L.msn_sort_workspace_bytes.restype = I
    L.msn_sort_keys_workspace_bytes.argtypes = [I64, I, I, SZ]
    L.msn_sort_keys_workspace_bytes.restype = I
    L.msn_segmented_status_offset.argtypes = [I64, I64, I, SZ]
    L.msn_segmented_status_offset.restype = I
    L.msn_sort_keys.argtypes = [P, P, I64, I, I, P, P, ctypes.c_size_t, P]
    L.msn_sort_keys.restype = I
    L.msn_sort_keys_noalloc.argtypes = [P, P, I64, I, I, P, P]
    L.msn_sort_keys_noalloc.restype = I
    L.msn_quick_sort_workspace_bytes.argtypes = [I64, I, SZ]
    L.msn_quick_sort_workspace_bytes.restype = I
    L.msn_quick_sort_keys.argtypes = [P, P, I64, I, I, P, P, ctypes.c_size_t, P]
    L.msn_quick_sort_keys.restype = I
    L.msn_sort_pairs.argtypes = [P, P, P, P, I64, I, I, P, P, ctypes.c_size_t, P]
    L.msn_sort_pairs.restype = I
    L.msn_segmented_sort_workspace_bytes.argtypes = [I64, I64, I, I, SZ]
    L.msn_segmented_sort_workspace_bytes.restype = I
    L.msn_segmented_sort.argtypes = [P, P, P, P, P, I64, I64, I, I, U, P, P, ctypes.c_size_t, P]
    L.msn_segmented_sort.restype = I
    L.msn_merge_path_split.argtypes = [P, I64, P, I64, P, P, I64, I, P]
    L.msn_merge_path_split.restype = I
    L.msn_copy_words.argtypes = [P, P, I64, P]
    L.msn_copy_words.restype = I
    L.msn_sort_backward.argtypes = [P, P, P, I64, I64, P]
    L.msn_sort_backward.restype = I
    _lib = L
    return L


def check(fn: str, status: int):
    if status != 0:
        raise MsnError(fn, status, lib().msn_status_string(status).decode())


def status_string(status: int) -> str:
    return lib().msn_status_string(status).decode()


def key_dtype(t: torch.Tensor) -> int:
    try:
        return _DTYPES[t.dtype]
    except KeyError:
        raise TypeError(f"keys must be uint32, int32 or float32, not {t.dtype}") from None


def leaf_code(leaf) -> int:
    if isinstance(leaf, int):
        return leaf
    try:
        return LEAVES[leaf]
    except KeyError:
        raise ValueError(f"leaf must be one of {sorted(LEAVES)}, not {leaf!r}") from None


def group_keys(leaf) -> int:
    """Keys of a lane's group (8 or 4) under a leaf set given by name or code."""
    code = leaf_code(leaf)
    for name, c in LEAVES.items():
        if c == code:
            return GROUP_KEYS[name]
    raise ValueError(f"unknown leaf code {leaf!r}")


def ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def stream_handle(device: torch.device, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def sort_workspace_bytes(n: int, dtype: int, pairs: bool) -> int:
    out = ctypes.c_size_t(0)
    check("msn_sort_keys_workspace_bytes",
          lib().msn_sort_keys_workspace_bytes(n, dtype, int(pairs), ctypes.byref(out)))
    return out.value


def quick_workspace_bytes(n: int, dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check("msn_quick_sort_workspace_bytes",
          lib().msn_quick_sort_workspace_bytes(n, dtype, ctypes.byref(out)))
    return out.value


def segmented_status_offset(n_total: int, num_segments: int, pairs: bool) -> int:
    out = ctypes.c_size_t(0)
    check("msn_segmented_status_offset",
          lib().msn_segmented_status_offset(n_total, num_segments, int(pairs), ctypes.byref(out)))
    return out.value


def segmented_workspace_bytes(n_total: int, num_segments: int, dtype: int, pairs: bool) -> int:
    out = ctypes.c_size_t(0)
    check("msn_segmented_sort_workspace_bytes",
          lib().msn_segmented_sort_workspace_bytes(n_total, num_segments, dtype, int(pairs),
                                                   ctypes.byref(out)))
    return out.value


class KernelStats(ctypes.Structure):
    """msn_kernel_stats."""

    _fields_ = [
        ("kind", ctypes.c_char * 24),
        ("launches", ctypes.c_int64),
        ("elements", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
    ]


def timing_enable(max_launches: int):
    L = lib()
    L.msn_timing_enable.argtypes = [ctypes.c_int]
    L.msn_timing_enable.restype = ctypes.c_int
    check("msn_timing_enable", L.msn_timing_enable(max_launches))


def timing_read() -> dict:
    """Per kernel kind: {"launches", "elements", "total_ms", "avg_ms"} (waits for the events)."""
    L = lib()
    L.msn_timing_read.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.msn_timing_read.restype = ctypes.c_int
    cap = 512
    arr = (KernelStats * cap)()
    count = ctypes.c_int(0)
    check("msn_timing_read", L.msn_timing_read(ctypes.cast(arr, ctypes.c_void_p), cap,
                                               ctypes.byref(count)))
    out = {}
    for i in range(min(count.value, cap)):
        s = arr[i]
        out[s.kind.decode()] = {"launches": s.launches, "elements": s.elements,
                                "total_ms": s.total_ms,
                                "avg_ms": s.total_ms / max(s.launches, 1)}
    return out


def timing_disable():
    L = lib()
    L.msn_timing_disable.argtypes = []
    L.msn_timing_disable.restype = ctypes.c_int
    check("msn_timing_disable", L.msn_timing_disable())
