"""CPU oracle for the network-leaf merge sort: test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the library under ``paper_2503_05934_amd`` never imports it.  The
arithmetic lives in ``oracle.c`` (plain C, single-threaded); this module only
builds it with gcc and marshals numpy arrays through ctypes.

Functions follow the paper (arXiv 2503.05934):
  * :func:`sort` with ``algo="ms"``: Algorithm 1 (merge sort with network base cases); the
    empty network set gives the classical merge sort of Eq. 1's baseline.
  * :func:`sort` with ``algo="qs"``: Algorithm 2 (quick sort with network base cases).
  * :func:`config_mask`: the network sets of Table 3.
  * :func:`network`: the fixed 2..8-input networks used as base cases.
  * :func:`segmented_sort`, :func:`row_argsort`: the above per segment / row.
  * :func:`gather_backward`: gradient of a sort through its permutation
    (a definition; the paper has no gradients).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

DTYPES = {"u32": 0, "i32": 1, "f32": 2}
ALGOS = {"ms": 0, "qs": 1}
_NP_OF = {"u32": np.uint32, "i32": np.int32, "f32": np.float32}


def build(src: str = _SRC, out: str = _LIB_PATH, extra=()) -> str:
    """Compile the oracle with gcc into a shared library and return its path."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", *extra, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class Oracle:
    """ctypes view of one compiled oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        U32 = ctypes.c_uint32
        lib.orc_network.argtypes = [I, P]
        lib.orc_network.restype = I
        lib.orc_apply_network_batch.argtypes = [I, I, I, P, P, I64]
        lib.orc_apply_network_batch.restype = I
        lib.orc_config_mask.argtypes = [ctypes.c_char_p]
        lib.orc_config_mask.restype = I64
        lib.orc_sort.argtypes = [I, I, U32, I, P, P, P, I64]
        lib.orc_sort.restype = I
        lib.orc_segmented_sort.argtypes = [I, I, U32, I, P, P, P, P, I64]
        lib.orc_segmented_sort.restype = I
        lib.orc_alg1_leaf_histogram.argtypes = [I64, U32, P]
        lib.orc_alg1_leaf_histogram.restype = I
        lib.orc_gather_backward.argtypes = [P, P, P, I64, I64]
        lib.orc_gather_backward.restype = I
        lib.orc_rank_bounds.argtypes = [I, P, I64, U32, P, P]
        lib.orc_rank_bounds.restype = I
        self.lib = lib

    # -- networks ---------------------------------------------------------
    def network(self, n: int) -> list[tuple[int, int]]:
        """Comparators (i, j), i < j, of the oracle's n-input network."""
        buf = np.zeros(64, dtype=np.int32)
        cnt = self.lib.orc_network(n, buf.ctypes.data)
        if cnt < 0:
            raise ValueError(f"no network for n={n}")
        return [(int(buf[2 * c]), int(buf[2 * c + 1])) for c in range(cnt)]

    def apply_network(self, n: int, tuples: np.ndarray, dtype: str = "u32", stable: bool = False):
        """Run the n-network over each row of ``tuples`` ([count, n]).

        Returns (sorted rows, perm) where perm[t, i] is the row-local position
        the i-th output of row t came from.
        """
        keys = np.ascontiguousarray(tuples, dtype=_NP_OF[dtype]).copy().view(np.uint32)
        count = keys.shape[0] if keys.ndim == 2 else 0
        perm = np.zeros_like(keys, dtype=np.uint32)
        rc = self.lib.orc_apply_network_batch(n, DTYPES[dtype], int(stable), keys.ctypes.data,
                                              perm.ctypes.data, count)
        if rc:
            raise ValueError(f"orc_apply_network_batch rc={rc}")
        return keys.view(_NP_OF[dtype]), perm

    # -- configurations -----------------------------------------------------
    def config_mask(self, name: str) -> int:
        m = self.lib.orc_config_mask(name.encode())
        if m < 0:
            raise KeyError(name)
        return int(m)

    # -- sorts --------------------------------------------------------------
    def sort(self, keys, vals=None, *, dtype="u32", algo="ms", config="6To8", stable=False,
             want_perm=False):
        """Sort a 1-D array with Algorithm 1 ("ms") or Algorithm 2 ("qs").

        Returns sorted keys, plus the permuted vals if given, plus the
        original position of each output if ``want_perm``.
        """
        k = np.ascontiguousarray(keys, dtype=_NP_OF[dtype]).copy()
        v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
        p = np.zeros(k.shape[0], dtype=np.uint32) if want_perm else None
        mask = config if isinstance(config, int) else self.config_mask(config)
        rc = self.lib.orc_sort(ALGOS[algo], DTYPES[dtype], mask, int(stable), k.ctypes.data,
                               None if v is None else v.ctypes.data,
                               None if p is None else p.ctypes.data, k.shape[0])
        if rc:
            raise ValueError(f"orc_sort rc={rc}")
        out = [k]
        if v is not None:
            out.append(v)
        if p is not None:
            out.append(p)
        return out[0] if len(out) == 1 else tuple(out)

    def segmented_sort(self, keys, offsets, vals=None, *, dtype="u32", algo="ms",
                       config="6To8", stable=False, want_perm=False):
        """Sort each CSR segment keys[offsets[s]:offsets[s+1]] independently.

        ``want_perm`` returns the segment-local original position of each
        output element.
        """
        k = np.ascontiguousarray(keys, dtype=_NP_OF[dtype]).copy()
        off = np.ascontiguousarray(offsets, dtype=np.uint32)
        v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
        p = np.zeros(k.shape[0], dtype=np.uint32) if want_perm else None
        mask = config if isinstance(config, int) else self.config_mask(config)
        rc = self.lib.orc_segmented_sort(ALGOS[algo], DTYPES[dtype], mask, int(stable),
                                         k.ctypes.data, None if v is None else v.ctypes.data,
                                         None if p is None else p.ctypes.data, off.ctypes.data,
                                         off.shape[0] - 1)
        if rc:
            raise ValueError(f"orc_segmented_sort rc={rc}")
        out = [k]
        if v is not None:
            out.append(v)
        if p is not None:
            out.append(p)
        return out[0] if len(out) == 1 else tuple(out)

    def row_argsort(self, x, *, config="6To8", algo="ms"):
        """Stable ascending sort of each row of a 2-D float32 array.

        Returns (values, perm) with values[r, i] == x[r, perm[r, i]] (bit copies).
        """
        x = np.ascontiguousarray(x, dtype=np.float32)
        rows, cols = x.shape
        off = (np.arange(rows + 1, dtype=np.int64) * cols).astype(np.uint32)
        vals, perm = self.segmented_sort(x.reshape(-1), off, dtype="f32", algo=algo,
                                         config=config, stable=True, want_perm=True)
        return vals.reshape(rows, cols), perm.astype(np.int32).reshape(rows, cols)

    def leaf_histogram(self, n: int, config="6To8") -> np.ndarray:
        """Elements that Algorithm 1 hands to a network of each size 0..8."""
        hist = np.zeros(9, dtype=np.int64)
        mask = config if isinstance(config, int) else self.config_mask(config)
        rc = self.lib.orc_alg1_leaf_histogram(n, mask, hist.ctypes.data)
        if rc:
            raise ValueError(f"orc_alg1_leaf_histogram rc={rc}")
        return hist

    def rank_bounds(self, keys, value, *, dtype="u32"):
        """(number of keys before ``value``, number not after it) in dtype order."""
        k = np.ascontiguousarray(keys, dtype=_NP_OF[dtype]).view(np.uint32)
        v = int(np.asarray(value, dtype=_NP_OF[dtype]).view(np.uint32))
        lt = np.zeros(1, dtype=np.int64)
        le = np.zeros(1, dtype=np.int64)
        rc = self.lib.orc_rank_bounds(DTYPES[dtype], k.ctypes.data, k.shape[0], v,
                                      lt.ctypes.data, le.ctypes.data)
        if rc:
            raise ValueError(f"orc_rank_bounds rc={rc}")
        return int(lt[0]), int(le[0])

    def gather_backward(self, grad_out, perm):
        """grad_in[r, perm[r, i]] = grad_out[r, i] for a batch of rows."""
        g = np.ascontiguousarray(grad_out, dtype=np.float32)
        p = np.ascontiguousarray(perm, dtype=np.int32)
        if g.shape != p.shape or g.ndim != 2:
            raise ValueError("grad_out and perm must be 2-D and of one shape")
        out = np.zeros_like(g)
        rc = self.lib.orc_gather_backward(g.ctypes.data, p.ctypes.data, out.ctypes.data,
                                          g.shape[0], g.shape[1])
        if rc:
            raise ValueError(f"orc_gather_backward rc={rc}")
        return out


_default: Oracle | None = None


def load() -> Oracle:
    """The oracle built from ``oracle.c`` (compiled on first use if absent or stale)."""
    global _default
    if _default is None:
        if (not os.path.exists(_LIB_PATH)
                or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        _default = Oracle(_LIB_PATH)
    return _default
