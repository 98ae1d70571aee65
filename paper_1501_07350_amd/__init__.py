"""offt -- MI355X-native 3-D complex-to-complex FFT (Python binding).

Python side of the C ABI in include/offt.h.  torch supplies device memory
and streams only; the transform runs in the library's HIP kernels.

    plan = Plan((Na, Nb, Nc), dtype=torch.complex128, batch=1)
    y = plan.forward(x)            # x: contiguous cuda tensor (batch?, Na, Nb, Nc)
    z = plan.backward(y)           # unnormalised unless normalize_inverse=True

With layout="cba" the forward output and the backward input are in reversed
axis order, (batch?, Nc, Nb, Na), as the paper's transform finishes.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (BACKWARD, C2C_F32, C2C_F64, COMM_METHODS, FORWARD, MANY_LEVELS, MANY_LEVELS_GRAPH,
                   MANY_LEVELS_GROUPED_GRAPH, MANY_PERSISTENT,
                   MANY_PERSISTENT_GRAPH, MANY_SEPARATE_HEURISTIC, MANY_SEPARATE_TUNED, MANY_SYNC, MANY_SYNC_GRAPH,
                   LAYOUT_NATURAL, LAYOUT_REVERSED, MAX_AXIS, OfftError,
                   TUNE_EXHAUSTIVE, TUNE_FORCED, TUNE_LEARNED, TUNE_NONE)

__all__ = ["Plan", "ManyPlan", "DistPlan", "OfftError", "twiddles", "default_plan_string", "plan_string", "plan_string_nd", "pass_bytes",
           "decomp_start", "transpose_count", "transpose_volume", "FORWARD", "BACKWARD", "MAX_AXIS"]

_LAYOUT = {"natural": LAYOUT_NATURAL, "abc": LAYOUT_NATURAL, "cba": LAYOUT_REVERSED,
           "reversed": LAYOUT_REVERSED}


def _layout_code(layout) -> int:
    if layout not in _LAYOUT:
        raise ValueError(f"layout must be one of {sorted(_LAYOUT)}")
    return _LAYOUT[layout]

_TUNE = {"none": TUNE_NONE, "exhaustive": TUNE_EXHAUSTIVE, "learned": TUNE_LEARNED,
         "forced": TUNE_FORCED}


def _dtype_code(dtype) -> int:
    if dtype == torch.complex128:
        return C2C_F64
    if dtype == torch.complex64:
        return C2C_F32
    raise ValueError("dtype must be torch.complex128 or torch.complex64")


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _make_opts(tune="none", reps=2, normalize_inverse=False, forced_plan=None, cache_path=None,
               weights_path=None, stream=None, tune_inplace=False, use_graph=False, layout="natural"):
    o = _lib.default_opts()
    if tune not in _TUNE:
        raise ValueError(f"tune must be one of {sorted(_TUNE)}")
    o.tune = _TUNE[tune]
    o.reps = int(reps)
    o.normalize_inverse = 1 if normalize_inverse else 0
    keep = []
    for field, val in (("forced_plan", forced_plan), ("cache_path", cache_path),
                       ("weights_path", weights_path)):
        if val is not None:
            b = str(val).encode()
            keep.append(b)
            setattr(o, field, b)
    o.stream = ctypes.c_void_p(stream) if stream else None
    o.tune_inplace = 1 if tune_inplace else 0
    o.use_graph = 1 if use_graph else 0
    o.layout = _layout_code(layout)
    return o, keep


class Plan:
    """Plan for `batch` grids of `shape` = (Na, Nb, Nc).  use_graph: forward
    and backward replay a HIP graph of the pass kernels (captured by the first
    call, updated when buffers or direction change).  layout="cba": forward
    output and backward input are (batch?, Nc, Nb, Na), Y[c, b, a] = X[a, b, c].
    `shape` may have 1 to 5 axes (row-major, last axis fastest); up to three
    are the three-dimensional plan of the shape padded with unit axes."""

    def __init__(self, shape, dtype=torch.complex128, batch: int = 1, tune: str = "none",
                 normalize_inverse: bool = False, forced_plan: str | None = None,
                 cache_path: str | None = None, weights_path: str | None = None, reps: int = 2,
                 tune_inplace: bool = False, use_graph: bool = False, layout: str = "natural"):
        lib = _lib.load()
        if not 1 <= len(shape) <= _lib.MAX_DIMS:
            raise ValueError(f"shape must have 1 to {_lib.MAX_DIMS} axes")
        self.shape = tuple(int(s) for s in shape)
        self.dtype = dtype
        self.batch = int(batch)
        self.normalize_inverse = bool(normalize_inverse)
        self.reversed = _layout_code(layout) == LAYOUT_REVERSED
        code = _dtype_code(dtype)
        stream = _stream_handle() if torch.cuda.is_available() else None
        opts, keep = _make_opts(tune, reps, normalize_inverse, forced_plan, cache_path, weights_path,
                                stream, tune_inplace, use_graph, layout)
        if len(self.shape) == 3:
            h = lib.offt_plan_ex(self.shape[0], self.shape[1], self.shape[2], code, self.batch,
                                 ctypes.byref(opts))
        else:
            dims = (ctypes.c_int64 * len(self.shape))(*self.shape)
            h = lib.offt_plan_nd(len(self.shape), dims, code, self.batch, ctypes.byref(opts))
        del keep
        if not h:
            raise OfftError(_lib.last_error(), f"offt_plan{self.shape}")
        self._h = h

    @property
    def spectral_shape(self):
        """Grid shape of the forward output and backward input."""
        return self.shape[::-1] if self.reversed else self.shape

    def _check_tensor(self, x: torch.Tensor, name: str, shape):
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise ValueError(f"{name} must be a CUDA (HIP) tensor")
        if x.dtype != self.dtype:
            raise ValueError(f"{name} has dtype {x.dtype}, plan expects {self.dtype}")
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        n = self.batch
        for v in shape:
            n *= v
        if x.numel() != n or tuple(x.shape[-len(shape):]) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(x.shape)}, plan expects "
                             f"{(self.batch,) + tuple(shape) if self.batch > 1 else tuple(shape)}")

    def _run(self, fn, x, out, in_shape, out_shape, *extra):
        self._check_tensor(x, "x", in_shape)
        if out is None:
            out = torch.empty(x.shape[:-len(out_shape)] + tuple(out_shape), dtype=x.dtype, device=x.device)
        else:
            self._check_tensor(out, "out", out_shape)
        _lib.check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), *extra,
                      ctypes.c_void_p(_stream_handle())), "exec")
        return out

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._run(_lib.load().offt_exec_fwd, x, out, self.shape, self.spectral_shape)

    def backward(self, x: torch.Tensor, out: torch.Tensor | None = None,
                 normalize: bool | None = None) -> torch.Tensor:
        """Backward transform; normalize=True divides by the grid's point
        count, False does not, None (default) follows the plan's
        normalize_inverse."""
        norm = -1 if normalize is None else (1 if normalize else 0)
        return self._run(_lib.load().offt_exec_bwd_norm, x, out, self.spectral_shape, self.shape,
                         ctypes.c_int(norm))

    def exec_ptr(self, direction: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
        """Raw-pointer execution (no tensor checks) for benchmarking loops."""
        lib = _lib.load()
        fn = lib.offt_exec_fwd if direction == FORWARD else lib.offt_exec_bwd
        _lib.check(fn(self._h, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                      ctypes.c_void_p(stream)), "exec")

    def npasses(self) -> int:
        return _lib.check(_lib.load().offt_plan_passes(self._h), "plan_passes")

    def exec_pass(self, i: int, direction: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
        """Launch only axis pass i (plan order); passes 0..n-1 in order equal exec."""
        _lib.check(_lib.load().offt_exec_pass(self._h, int(i), int(direction), ctypes.c_void_p(in_ptr),
                                              ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream)),
                   "exec_pass")

    def exec_range(self, first: int, count: int, direction: int, in_ptr: int, out_ptr: int,
                   stream: int = 0) -> None:
        """Launch passes first..first+count-1 as exec does (a slab schedule's
        passes interleaved slab by slab)."""
        _lib.check(_lib.load().offt_exec_range(self._h, int(first), int(count), int(direction),
                                               ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                                               ctypes.c_void_p(stream)), "exec_range")

    def _schedule_field(self, key: str) -> int:
        for field in self.describe().split("|")[0].split(";"):
            if field.startswith(key + "="):
                return int(field[len(key) + 1:])
        return 0

    def slab(self) -> int:
        """Planes per slab of the plan's slab schedule, or 0."""
        return self._schedule_field("slab")

    def col(self) -> int:
        """Columns per block of the plan's column-block schedule, or 0."""
        return self._schedule_field("col")

    def pass_groups(self):
        """Passes as exec launches them: each on its own, except that the
        passes after the first of a slab or column-block schedule run
        interleaved block by block (launch such a group with exec_range)."""
        n = self.npasses()
        if (self.slab() or self.col()) and n > 1:
            return [[0], list(range(1, n))]
        return [[i] for i in range(n)]

    def copy_pass(self, i: int, in_ptr: int, out_ptr: int, stream: int = 0) -> None:
        """The copy of pass i's memory accesses (its measured ceiling)."""
        _lib.check(_lib.load().offt_copy_pass(self._h, int(i), ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                                              ctypes.c_void_p(stream)), "copy_pass")

    def describe(self) -> str:
        lib = _lib.load()
        n = _lib.check(lib.offt_plan_describe(self._h, None, 0), "describe")
        buf = ctypes.create_string_buffer(n + 1)
        lib.offt_plan_describe(self._h, buf, n + 1)
        return buf.value.decode()

    def workspace_bytes(self) -> int:
        return _lib.check(_lib.load().offt_workspace_bytes(self._h), "workspace_bytes")

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.load().offt_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ManyPlan:
    """Plan for an uneven batch: grid i has shape dims[i]; grids are packed
    back to back in one buffer, grid i at element offset offset(i)."""

    def __init__(self, dims, dtype=torch.complex64, tune: str = "none",
                 normalize_inverse: bool = False, cache_path: str | None = None, reps: int = 2):
        lib = _lib.load()
        self.dims = [tuple(int(v) for v in d) for d in dims]
        if not self.dims or any(len(d) != 3 for d in self.dims):
            raise ValueError("dims must be a non-empty list of (Na, Nb, Nc)")
        self.dtype = dtype
        code = _dtype_code(dtype)
        flat = (ctypes.c_int64 * (3 * len(self.dims)))(*[v for d in self.dims for v in d])
        stream = _stream_handle() if torch.cuda.is_available() else None
        opts, keep = _make_opts(tune, reps, normalize_inverse, None, cache_path, None, stream)
        h = lib.offt_plan_many(len(self.dims), flat, code, ctypes.byref(opts))
        del keep
        if not h:
            raise OfftError(_lib.last_error(), "offt_plan_many")
        self._h = h
        self.offsets = [_lib.check(lib.offt_many_offset(h, i)) for i in range(len(self.dims) + 1)]
        self.total = self.offsets[-1]

    def pack(self, grids) -> torch.Tensor:
        buf = torch.zeros(self.total, dtype=self.dtype, device=grids[0].device)
        for i, g in enumerate(grids):
            n = g.numel()
            buf[self.offsets[i]:self.offsets[i] + n] = g.reshape(-1)
        return buf

    def unpack(self, buf):
        out = []
        for i, d in enumerate(self.dims):
            n = d[0] * d[1] * d[2]
            out.append(buf[self.offsets[i]:self.offsets[i] + n].view(d))
        return out

    def execute(self, x: torch.Tensor, out: torch.Tensor | None = None, direction: int = FORWARD,
                use_graph: int = 1) -> torch.Tensor:
        if not x.is_cuda or x.dtype != self.dtype or not x.is_contiguous() or x.numel() < self.total:
            raise ValueError("x must be a contiguous CUDA tensor holding the packed grids")
        if out is None:
            out = torch.empty_like(x)
        lib = _lib.load()
        _lib.check(lib.offt_exec_many(self._h, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), int(direction), int(use_graph),
                                      ctypes.c_void_p(_stream_handle())), "exec_many")
        return out

    def _default(self, fn, x, out):
        if not x.is_cuda or x.dtype != self.dtype or not x.is_contiguous() or x.numel() < self.total:
            raise ValueError("x must be a contiguous CUDA tensor holding the packed grids")
        if out is None:
            out = torch.empty_like(x)
        _lib.check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                      ctypes.c_void_p(_stream_handle())), "exec_many")
        return out

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Forward transform of every grid in the default launch form (level
        kernels from a graph when every axis is at most 160 long, else
        separate launches)."""
        return self._default(_lib.load().offt_exec_many_fwd, x, out)

    def backward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        return self._default(_lib.load().offt_exec_many_bwd, x, out)

    def exec_ptr(self, in_ptr: int, out_ptr: int, direction: int = FORWARD, use_graph: int = 1,
                 stream: int = 0) -> None:
        _lib.check(_lib.load().offt_exec_many(self._h, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                                              int(direction), int(use_graph), ctypes.c_void_p(stream)),
                   "exec_many")

    def status(self) -> int:
        """0, or the error code of a persistent run whose dependency wait timed out
        (synchronise the stream first)."""
        return _lib.load().offt_many_status(self._h)

    def describe(self) -> str:
        lib = _lib.load()
        n = _lib.check(lib.offt_plan_describe(self._h, None, 0), "describe")
        buf = ctypes.create_string_buffer(n + 1)
        lib.offt_plan_describe(self._h, buf, n + 1)
        return buf.value.decode()

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.load().offt_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DistPlan:
    """The paper's distributed flow over `nprocs` virtual processes on one GPU
    (include/offt.h, offt_plan_dist).  forward(x) takes a (Na, Nb, Nc) grid
    and returns the transform in cba order, shape (Nc, Nb, Na), as the
    paper's transform finishes; backward(y) the reverse.  method: one of
    COMM_METHODS (User-select) or "auto" (every method timed at plan time,
    the fastest kept)."""

    def __init__(self, shape, nprocs: int, dtype=torch.complex128, method="auto", block_size: int = 32,
                 normalize_inverse: bool = False, reps: int = 2):
        lib = _lib.load()
        self.shape = tuple(int(v) for v in shape)
        if len(self.shape) != 3:
            raise ValueError("shape must be (Na, Nb, Nc)")
        self.dtype = dtype
        self.nprocs = int(nprocs)
        if method == "auto":
            code_m = _lib.COMM_AUTO
        elif method in _lib.COMM_METHODS:
            code_m = _lib.COMM_METHODS.index(method)
        elif isinstance(method, int):
            code_m = method
        else:
            raise ValueError(f"method must be 'auto' or one of {_lib.COMM_METHODS}")
        stream = _stream_handle() if torch.cuda.is_available() else None
        opts, keep = _make_opts("none", reps, normalize_inverse, None, None, None, stream)
        h = lib.offt_plan_dist(*self.shape, _dtype_code(dtype), self.nprocs, int(code_m), int(block_size),
                               ctypes.byref(opts))
        del keep
        if not h:
            raise OfftError(_lib.last_error(), "offt_plan_dist")
        self._h = h

    @property
    def method(self) -> str:
        return _lib.COMM_METHODS[_lib.check(_lib.load().offt_dist_method(self._h), "dist_method")]

    def method_times(self):
        """{method: ms} measured at plan time (empty when the method was given)."""
        ms = (ctypes.c_float * 6)()
        _lib.check(_lib.load().offt_dist_method_times(self._h, ms), "dist_method_times")
        return {m: float(v) for m, v in zip(_lib.COMM_METHODS, ms) if v >= 0}

    def counts(self, step: int, direction: int = FORWARD):
        """counts[p][q]: elements process p sends to q in transpose `step`."""
        lib = _lib.load()
        return [[_lib.check(lib.offt_dist_count(self._h, int(direction), int(step), p, q), "dist_count")
                 for q in range(self.nprocs)] for p in range(self.nprocs)]

    def block(self, order: str, proc: int):
        """[start, end) of process proc's block in order 'abc', 'cab' or 'cba'."""
        end = ctypes.c_int64()
        o = {"abc": _lib.ORDER_ABC, "cab": _lib.ORDER_CAB, "cba": _lib.ORDER_CBA}[order]
        start = _lib.check(_lib.load().offt_dist_block(self._h, o, int(proc), ctypes.byref(end)), "dist_block")
        return start, end.value

    def _check(self, x, shape):
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != self.dtype or not x.is_contiguous():
            raise ValueError(f"expected a contiguous CUDA tensor of dtype {self.dtype}")
        if x.numel() != self.shape[0] * self.shape[1] * self.shape[2]:
            raise ValueError(f"expected {shape}")

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check(x, self.shape)
        out = torch.empty(self.shape[::-1], dtype=x.dtype, device=x.device) if out is None else out
        self._check(out, self.shape[::-1])
        _lib.check(_lib.load().offt_exec_fwd(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(_stream_handle())), "exec")
        return out

    def backward(self, y: torch.Tensor, out: torch.Tensor | None = None,
                 normalize: bool | None = None) -> torch.Tensor:
        self._check(y, self.shape[::-1])
        out = torch.empty(self.shape, dtype=y.dtype, device=y.device) if out is None else out
        self._check(out, self.shape)
        norm = -1 if normalize is None else (1 if normalize else 0)
        _lib.check(_lib.load().offt_exec_bwd_norm(self._h, ctypes.c_void_p(y.data_ptr()),
                                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_int(norm),
                                                  ctypes.c_void_p(_stream_handle())), "exec")
        return out

    def exec_steps(self, x: torch.Tensor, steps: int, direction: int = FORWARD, method=None) -> torch.Tensor:
        """The first `steps` steps of the flow; returns the flat array of the
        processes' local arrays after that step, in process order."""
        self._check(x, self.shape)
        out = torch.empty(x.numel(), dtype=x.dtype, device=x.device)
        m = _lib.COMM_AUTO if method is None else (_lib.COMM_METHODS.index(method) if isinstance(method, str)
                                                  else int(method))
        _lib.check(_lib.load().offt_dist_exec_steps(self._h, int(direction), int(steps), m,
                                                    ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                                    ctypes.c_void_p(_stream_handle())), "dist_exec_steps")
        return out

    def exec_ptr(self, direction: int, in_ptr: int, out_ptr: int, stream: int = 0, method=None,
                 steps: int = 5) -> None:
        """Raw-pointer execution of the first `steps` steps (no tensor checks),
        with `method` (None: the plan's) -- for benchmarking loops."""
        m = _lib.COMM_AUTO if method is None else (_lib.COMM_METHODS.index(method) if isinstance(method, str)
                                                  else int(method))
        _lib.check(_lib.load().offt_dist_exec_steps(self._h, int(direction), int(steps), m, ctypes.c_void_p(in_ptr),
                                                    ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream)), "exec")

    def describe(self) -> str:
        lib = _lib.load()
        n = _lib.check(lib.offt_plan_describe(self._h, None, 0), "describe")
        buf = ctypes.create_string_buffer(n + 1)
        lib.offt_plan_describe(self._h, buf, n + 1)
        return buf.value.decode()

    def workspace_bytes(self) -> int:
        return _lib.check(_lib.load().offt_workspace_bytes(self._h), "workspace_bytes")

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.load().offt_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_string(shape, dtype=torch.complex128, layout: str = "natural", plan: str | None = None) -> str:
    """Heuristic plan string of `layout` for a grid shape, or `plan` checked
    and in canonical form (no device needed)."""
    lib = _lib.load()
    code = _dtype_code(dtype)
    lay = _layout_code(layout)
    p = plan.encode() if plan is not None else None
    n = _lib.check(lib.offt_plan_string(shape[0], shape[1], shape[2], code, lay, p, None, 0), "plan string")
    buf = ctypes.create_string_buffer(n + 1)
    lib.offt_plan_string(shape[0], shape[1], shape[2], code, lay, p, buf, n + 1)
    return buf.value.decode()


def plan_string_nd(shape, dtype=torch.complex128, plan: str | None = None) -> str:
    """Heuristic plan string of a 4- or 5-axis grid, or `plan` checked and in
    canonical form (no device needed)."""
    lib = _lib.load()
    code = _dtype_code(dtype)
    dims = (ctypes.c_int64 * len(shape))(*[int(v) for v in shape])
    p = plan.encode() if plan is not None else None
    n = _lib.check(lib.offt_plan_string_nd(len(shape), dims, code, p, None, 0), "plan string")
    buf = ctypes.create_string_buffer(n + 1)
    lib.offt_plan_string_nd(len(shape), dims, code, p, buf, n + 1)
    return buf.value.decode()


def default_plan_string(shape, dtype=torch.complex128) -> str:
    """Heuristic plan string of a grid shape (no device needed)."""
    lib = _lib.load()
    code = _dtype_code(dtype)
    n = _lib.check(lib.offt_default_plan_string(shape[0], shape[1], shape[2], code, None, 0), "plan string")
    buf = ctypes.create_string_buffer(n + 1)
    lib.offt_default_plan_string(shape[0], shape[1], shape[2], code, buf, n + 1)
    return buf.value.decode()


def twiddles(n: int, dtype=torch.complex128):
    """Device-generated forward twiddle table W_n^m, m < n, copied to the host."""
    import numpy as np
    code = _dtype_code(dtype)
    out = np.empty(n, dtype=np.complex128 if code == C2C_F64 else np.complex64)
    _lib.check(_lib.load().offt_twiddles(n, code, out.ctypes.data_as(ctypes.c_void_p)), "twiddles")
    return out


# ---- byte and volume accounting (host only) ---------------------------------
def pass_bytes(shape, dtype=torch.complex128, batch: int = 1) -> int:
    """HBM bytes one axis pass moves (every element read and written once)."""
    a, b, c = shape
    return _lib.check(_lib.load().offt_pass_bytes(a, b, c, _dtype_code(dtype), batch), "pass_bytes")


def decomp_start(n1: int, n2: int, n3: int, np_: int, myid: int) -> int:
    """First linear index of process myid's block (Sec. 2, Eq. 2)."""
    return _lib.check(_lib.load().offt_decomp_start(n1, n2, n3, np_, myid), "decomp_start")


def transpose_count(n1: int, n2: int, n3: int, np_: int, step: int, src: int, dst: int) -> int:
    """Elements src holds before transpose `step` (0: abc -> cab, 1: cab -> cba)
    and dst holds after it."""
    return _lib.check(_lib.load().offt_transpose_count(n1, n2, n3, np_, step, src, dst), "transpose_count")


def transpose_volume(n1: int, n2: int, n3: int, np_: int, step: int) -> int:
    """Elements that leave their process in transpose `step`."""
    return _lib.check(_lib.load().offt_transpose_volume(n1, n2, n3, np_, step), "transpose_volume")
