"""Network-leaf GPU merge sort for AMD MI355X (gfx950).

The method of Aly, Jensen, ElAarag (ACMSE 2025, arXiv 2503.05934, Sec. 3,
Algorithm 1): merge sort whose base cases are fixed sorting networks, the
6-to-8 configuration of Table 3 by default.  The work runs in the HIP kernels
of ``libmsn.so`` (C ABI in ``include/msn.h``); these functions only allocate
outputs and workspace with torch and pass pointers and the current stream.

    sort(keys)                        ascending sort of 1-D uint32/int32/float32
    quick_sort(keys)                  the same by quick sort (Algorithm 2), integer keys
    sort_pairs(keys, vals=None)       stable key-value sort / argsort
    segmented_sort(keys, offsets)     many arrays in one persistent launch
    sort_rows(x)                      stable row-wise sort -> (values, perm)
    sort_backward(grad_out, perm)     grad_in[r, perm[r, i]] = grad_out[r, i]
    DiffSort.apply(x)                 autograd sort over the last dim
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import LEAVES, MsnError, Tuning, make_tuning

__all__ = [
    "sort", "quick_sort", "sort_pairs", "segmented_sort", "segmented_status", "sort_rows",
    "sort_backward",
    "DiffSort", "MsnError", "Tuning", "LEAVES", "version", "SortPlan",
]


def version() -> int:
    return _lib.lib().msn_version()


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _check_keys(keys: torch.Tensor, ndim: int = 1):
    if not isinstance(keys, torch.Tensor) or not keys.is_cuda:
        raise ValueError("keys must be a GPU tensor")
    if keys.dim() != ndim or not keys.is_contiguous():
        raise ValueError(f"keys must be a contiguous {ndim}-D tensor")
    return _lib.key_dtype(keys)


def _check_buf(t, n: int, name: str, device, optional: bool = True):
    """A caller-supplied array the library reads or writes n 32-bit words of:
    it must hold exactly n contiguous 4-byte elements on the keys' device
    (the C ABI sees only a pointer, so a short array would be overrun)."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, not {t.device}")
    if t.numel() != n or t.element_size() != 4 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous tensor of {n} 32-bit elements "
                         f"(got {t.numel()} x {t.element_size()} bytes, "
                         f"contiguous={t.is_contiguous()})")
    return t


def _check_workspace(ws, need: int, device):
    if ws is None:
        return None
    if not isinstance(ws, torch.Tensor) or ws.device != device or not ws.is_contiguous():
        raise ValueError(f"workspace must be a contiguous tensor on {device}")
    if ws.numel() * ws.element_size() < need:
        raise ValueError(f"workspace holds {ws.numel() * ws.element_size()} bytes, "
                         f"{need} needed")
    return ws


def _tuning_ptr(tuning):
    t = tuning if isinstance(tuning, Tuning) or tuning is None else make_tuning(tuning)
    return t, (None if t is None else _lib.ctypes.byref(t))


def sort(keys: torch.Tensor, *, leaf="6To8", tuning=None, out: torch.Tensor | None = None,
         workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Ascending sort of a 1-D uint32/int32/float32 GPU tensor.

    tuning: None (defaults), a dict of msn_tuning fields, or "auto" (the
    autotuner's cached or freshly measured choice for this shape).
    """
    dt = _check_keys(keys)
    n = keys.numel()
    if tuning == "auto":
        from . import autotune
        tuning = autotune.tuned_sort_params(keys, pairs=False, leaf=leaf)
    out = torch.empty_like(keys) if out is None else _check_buf(out, n, "out", keys.device)
    ws_bytes = _lib.sort_workspace_bytes(n, dt, False)
    ws = (_workspace(ws_bytes, keys.device) if workspace is None
          else _check_workspace(workspace, ws_bytes, keys.device))
    t, tp = _tuning_ptr(tuning)
    _lib.check("msn_sort_keys", _lib.lib().msn_sort_keys(
        _lib.ptr(keys), _lib.ptr(out), n, dt, _lib.leaf_code(leaf), tp, _lib.ptr(ws),
        ws.numel() * ws.element_size(), _lib.stream_handle(keys.device, stream)))
    return out


def quick_sort(keys: torch.Tensor, *, leaf="6To8", tuning=None, out: torch.Tensor | None = None,
               workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Ascending sort of a 1-D uint32/int32 GPU tensor by the quick sort with
    network leaves (the paper's Algorithm 2); the same result as sort()."""
    dt = _check_keys(keys)
    n = keys.numel()
    out = torch.empty_like(keys) if out is None else _check_buf(out, n, "out", keys.device)
    ws_bytes = _lib.quick_workspace_bytes(n, dt)
    ws = (_workspace(ws_bytes, keys.device) if workspace is None
          else _check_workspace(workspace, ws_bytes, keys.device))
    t, tp = _tuning_ptr(tuning)
    _lib.check("msn_quick_sort_keys", _lib.lib().msn_quick_sort_keys(
        _lib.ptr(keys), _lib.ptr(out), n, dt, _lib.leaf_code(leaf), tp, _lib.ptr(ws),
        ws.numel() * ws.element_size(), _lib.stream_handle(keys.device, stream)))
    return out


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor | None = None, *, leaf="6To8",
               tuning=None, out_keys=None, out_vals=None, workspace=None, stream=None):
    """Stable key-value sort.  vals=None returns the argsort (int32 indices)."""
    dt = _check_keys(keys)
    n = keys.numel()
    if tuning == "auto":
        from . import autotune
        tuning = autotune.tuned_sort_params(keys, pairs=True, leaf=leaf)
    _check_buf(vals, n, "vals", keys.device)
    ok = (torch.empty_like(keys) if out_keys is None
          else _check_buf(out_keys, n, "out_keys", keys.device))
    ov = (torch.empty(n, dtype=torch.int32, device=keys.device) if vals is None
          else torch.empty_like(vals)) if out_vals is None else _check_buf(
              out_vals, n, "out_vals", keys.device)
    ws_bytes = _lib.sort_workspace_bytes(n, dt, True)
    ws = (_workspace(ws_bytes, keys.device) if workspace is None
          else _check_workspace(workspace, ws_bytes, keys.device))
    t, tp = _tuning_ptr(tuning)
    _lib.check("msn_sort_pairs", _lib.lib().msn_sort_pairs(
        _lib.ptr(keys), _lib.ptr(vals), _lib.ptr(ok), _lib.ptr(ov), n, dt, _lib.leaf_code(leaf),
        tp, _lib.ptr(ws), ws.numel() * ws.element_size(),
        _lib.stream_handle(keys.device, stream)))
    return ok, ov


def segmented_sort(keys: torch.Tensor, offsets: torch.Tensor | None = None,
                   vals: torch.Tensor | None = None, *, num_segments: int | None = None,
                   argsort: bool = False, leaf="6To8", tuning=None, out_keys=None,
                   out_vals=None, workspace=None, stream=None, debug_check: bool = False):
    """Sort every CSR segment keys[offsets[s]:offsets[s+1]] independently.

    offsets: uint32/int32 GPU tensor of num_segments + 1 entries, or None with
    ``num_segments`` for equal-length rows.  Returns keys, or (keys, vals) when
    vals is given or argsort=True (segment-local int32 indices).
    debug_check: validate the offsets on the device first (MSN_DEBUG_CHECK);
    a bad array leaves the outputs untouched and is reported by
    :func:`segmented_status` on the same workspace.
    """
    dt = _check_keys(keys)
    n = keys.numel()
    if offsets is not None:
        if (not isinstance(offsets, torch.Tensor) or offsets.element_size() != 4
                or not offsets.is_contiguous() or offsets.device != keys.device
                or offsets.numel() < 1):
            raise ValueError("offsets must be a non-empty contiguous 32-bit tensor on the "
                             "keys' device")
        num_segments = offsets.numel() - 1
    elif num_segments is None:
        raise ValueError("give offsets or num_segments")
    if argsort and vals is not None:
        raise ValueError("argsort takes no vals")
    if tuning == "auto":
        from . import autotune
        tuning = autotune.tuned_segmented_params(keys, offsets, num_segments=num_segments,
                                                 vals=vals, argsort=argsort, leaf=leaf)
    pairs = argsort or vals is not None
    _check_buf(vals, n, "vals", keys.device)
    ok = (torch.empty_like(keys) if out_keys is None
          else _check_buf(out_keys, n, "out_keys", keys.device))
    ov = None
    if pairs:
        ov = _check_buf(out_vals, n, "out_vals", keys.device) if out_vals is not None else (
            torch.empty(n, dtype=torch.int32, device=keys.device) if vals is None
            else torch.empty_like(vals))
    elif out_vals is not None:
        raise ValueError("out_vals needs vals or argsort=True")
    ws_bytes = _lib.segmented_workspace_bytes(n, num_segments, dt, pairs)
    ws = (_workspace(ws_bytes, keys.device) if workspace is None
          else _check_workspace(workspace, ws_bytes, keys.device))
    t, tp = _tuning_ptr(tuning)
    flags = (_lib.MSN_ARGSORT if argsort else 0) | (_lib.MSN_DEBUG_CHECK if debug_check else 0)
    _lib.check("msn_segmented_sort", _lib.lib().msn_segmented_sort(
        _lib.ptr(keys), _lib.ptr(vals), _lib.ptr(ok), _lib.ptr(ov), _lib.ptr(offsets),
        num_segments, n, dt, _lib.leaf_code(leaf), flags, tp, _lib.ptr(ws),
        ws.numel() * ws.element_size(), _lib.stream_handle(keys.device, stream)))
    return (ok, ov) if pairs else ok


def segmented_status(workspace: torch.Tensor, n_total: int, num_segments: int,
                     pairs: bool = False) -> int:
    """The status word a segmented_sort call left in ``workspace``: 0 when the
    offsets were valid, else MSN_SEG_BAD_* bits (see include/msn.h).  Waits for
    the device."""
    off = _lib.segmented_status_offset(n_total, num_segments, pairs)
    word = workspace.view(torch.uint8)[off:off + 4]
    return int(word.view(torch.int32).item()) & 0xffffffff


def sort_rows(x: torch.Tensor, *, leaf="6To8", tuning=None, stream=None):
    """Stable ascending sort of every row of a 2-D float32 (or int) tensor.

    Returns (values, perm) with values[r, i] == x[r, perm[r, i]] bit for bit.
    """
    if x.dim() != 2 or not x.is_contiguous():
        raise ValueError("x must be a contiguous 2-D tensor")
    rows, cols = x.shape
    v, p = segmented_sort(x.reshape(-1), None, num_segments=rows, argsort=True, leaf=leaf,
                          tuning=tuning, stream=stream)
    return v.view(rows, cols), p.view(rows, cols)


def sort_backward(grad_out: torch.Tensor, perm: torch.Tensor, *, out=None, stream=None):
    """grad_in[r, perm[r, i]] = grad_out[r, i] for 2-D float32 grad_out, int32 perm."""
    if grad_out.dtype != torch.float32 or perm.dtype != torch.int32:
        raise TypeError("grad_out must be float32 and perm int32")
    if grad_out.shape != perm.shape or grad_out.dim() != 2:
        raise ValueError("grad_out and perm must be 2-D and of one shape")
    if not grad_out.is_cuda or perm.device != grad_out.device:
        raise ValueError("grad_out and perm must be on one GPU")
    g = grad_out.contiguous()
    p = perm.contiguous()
    rows, cols = g.shape
    if out is None:
        gi = torch.empty_like(g)
    else:
        _check_buf(out, rows * cols, "out", g.device)
        if out.dtype != torch.float32:
            raise TypeError("out must be float32")
        gi = out
    _lib.check("msn_sort_backward", _lib.lib().msn_sort_backward(
        _lib.ptr(g), _lib.ptr(p), _lib.ptr(gi), rows, cols,
        _lib.stream_handle(g.device, stream)))
    return gi


class DiffSort(torch.autograd.Function):
    """y, perm = DiffSort.apply(x): stable sort along the last dim of a 2-D
    float32 tensor.  dL/dx[r, perm[r, i]] = dL/dy[r, i]; perm is not
    differentiable."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, leaf="6To8"):
        values, perm = sort_rows(x.contiguous(), leaf=leaf)
        ctx.save_for_backward(perm)
        ctx.mark_non_differentiable(perm)
        return values, perm

    @staticmethod
    def backward(ctx, grad_values, grad_perm):
        (perm,) = ctx.saved_tensors
        if grad_values is None:
            return None, None
        return sort_backward(grad_values.float(), perm), None


class SortPlan:
    """Preallocated output + workspace for repeated flat sorts of one size.

    ``run(keys)`` enqueues msn_sort_keys/msn_sort_pairs with no allocation,
    which is what benchmarks and graph capture want.
    """

    def __init__(self, n: int, dtype: torch.dtype, device, *, pairs=False, argsort=False,
                 leaf="6To8", tuning=None):
        self.n = n
        self.dt = {torch.uint32: 0, torch.int32: 1, torch.float32: 2}[dtype]
        self.pairs = pairs or argsort
        self.argsort = argsort
        self.leaf = _lib.leaf_code(leaf)
        self.tuning, self._tp = _tuning_ptr(tuning)
        self.out = torch.empty(n, dtype=dtype, device=device)
        self.out_vals = torch.empty(n, dtype=torch.int32, device=device) if self.pairs else None
        self.ws = _workspace(_lib.sort_workspace_bytes(n, self.dt, self.pairs), device)

    def run(self, keys: torch.Tensor, vals: torch.Tensor | None = None, stream=None):
        if (not isinstance(keys, torch.Tensor) or keys.dtype != self.out.dtype
                or keys.dim() != 1):
            raise ValueError(f"keys must be a 1-D {self.out.dtype} tensor")
        _check_buf(keys, self.n, "keys", self.out.device)
        if self.pairs and not self.argsort:
            _check_buf(vals, self.n, "vals", self.out.device, optional=False)
        st = _lib.stream_handle(keys.device, stream)
        if self.pairs:
            rc = _lib.lib().msn_sort_pairs(
                _lib.ptr(keys), None if self.argsort else _lib.ptr(vals), _lib.ptr(self.out),
                _lib.ptr(self.out_vals), self.n, self.dt, self.leaf, self._tp,
                _lib.ptr(self.ws), self.ws.numel(), st)
            _lib.check("msn_sort_pairs", rc)
            return self.out, self.out_vals
        rc = _lib.lib().msn_sort_keys(_lib.ptr(keys), _lib.ptr(self.out), self.n, self.dt,
                                      self.leaf, self._tp, _lib.ptr(self.ws), self.ws.numel(), st)
        _lib.check("msn_sort_keys", rc)
        return self.out
