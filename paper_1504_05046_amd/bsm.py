"""Python binding of the bsm C ABI (argument marshalling only).

Every step of the multiply runs in libbsm.so; torch only provides device memory and the
stream.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bsm.h")

FP64, FP32, BF16X3 = 0, 1, 2
SCHED_FLOPS, SCHED_MLP = 0, 1
OUT_F64, OUT_F32 = 0, 1
REAL, COMPLEX = 0, 1
ORDER_DEFAULT, ORDER_INTERLEAVE, ORDER_LOCALITY, ORDER_LPT, ORDER_PATCH = 0, 1, 2, 3, 4

OK, E_INVALID, E_MISMATCH, E_NOMEM, E_HIP, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_MISMATCH", -3: "E_NOMEM", -4: "E_HIP",
          -5: "E_UNSUPPORTED", -6: "E_STATE"}


class BsmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("sched", ctypes.c_int32),
                ("k_window", ctypes.c_int64), ("record_timings", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("out", ctypes.c_int32), ("order", ctypes.c_int32),
                ("patch_rows", ctypes.c_int32), ("patch_cols", ctypes.c_int32),
                ("device_klists", ctypes.c_int32), ("trans_a", ctypes.c_int32),
                ("trans_b", ctypes.c_int32), ("elem", ctypes.c_int32), ("k_split", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("K", ctypes.c_int64), ("N", ctypes.c_int64),
                ("a_blocks", ctypes.c_int64), ("b_blocks", ctypes.c_int64),
                ("c_blocks", ctypes.c_int64), ("a_elems", ctypes.c_int64),
                ("b_elems", ctypes.c_int64), ("c_elems", ctypes.c_int64),
                ("triples", ctypes.c_int64), ("tasks", ctypes.c_int64),
                ("useful_flops", ctypes.c_double), ("workspace_bytes", ctypes.c_int64),
                ("k_windows", ctypes.c_int64), ("tile", ctypes.c_int32),
                ("out", ctypes.c_int32), ("device_klists", ctypes.c_int32),
                ("elem", ctypes.c_int32), ("k_split", ctypes.c_int32)]


class LrInfo(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("K", ctypes.c_int64), ("N", ctypes.c_int64),
                ("a_blocks", ctypes.c_int64), ("factored_blocks", ctypes.c_int64),
                ("a_elems", ctypes.c_int64), ("b_elems", ctypes.c_int64),
                ("c_blocks", ctypes.c_int64), ("c_elems", ctypes.c_int64),
                ("tasks", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("useful_flops", ctypes.c_double), ("dense_flops", ctypes.c_double)]


class TensorDesc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("modes", ctypes.c_void_p), ("nblocks", ctypes.c_void_p),
                ("sizes", ctypes.c_void_p), ("bits", ctypes.c_void_p)]


class TcInfo(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("K", ctypes.c_int64), ("N", ctypes.c_int64),
                ("a_blocks", ctypes.c_int64), ("b_blocks", ctypes.c_int64),
                ("c_blocks", ctypes.c_int64), ("a_elems", ctypes.c_int64),
                ("b_elems", ctypes.c_int64), ("c_elems", ctypes.c_int64),
                ("tasks", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("useful_flops", ctypes.c_double), ("permute_a", ctypes.c_int32),
                ("permute_b", ctypes.c_int32), ("permute_c", ctypes.c_int32)]


_lib: Optional[ctypes.CDLL] = None
_p = ctypes.c_void_p
_i64 = ctypes.c_int64


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1504_05046_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    L.bsm_last_error.restype = ctypes.c_char_p
    L.bsm_options_default.argtypes = [ctypes.POINTER(Options)]
    L.bsm_options_default.restype = None
    L.bsm_concurrent_iterations.restype = _i64
    L.bsm_concurrent_iterations.argtypes = [_i64, _i64, _i64]
    L.bsm_tile_variants.restype = ctypes.c_int32
    L.bsm_tile_variants.argtypes = [_p, _p, ctypes.c_int32]
    L.bsm_bf16_tile_variants.restype = ctypes.c_int32
    L.bsm_bf16_tile_variants.argtypes = [_p, _p, ctypes.c_int32]
    L.bsm_plan_create.argtypes = [ctypes.POINTER(_p), _i64, _p, _i64, _p, _i64, _p, _p, _p,
                                  ctypes.POINTER(Options)]
    L.bsm_plan_query.argtypes = [_p, ctypes.POINTER(PlanInfo)]
    L.bsm_plan_c_shape.argtypes = [_p, _p]
    L.bsm_plan_c_offsets.argtypes = [_p, _p]
    L.bsm_execute.argtypes = [_p, ctypes.c_double, _p, _p, _p, ctypes.c_int, _p]
    L.bsm_execute_complex.argtypes = [_p, ctypes.c_double, ctypes.c_double, _p, _p, _p,
                                      ctypes.c_int, _p]
    L.bsm_execute_static.argtypes = [_p, ctypes.c_double, _p, _p, _p, ctypes.c_int, _p]
    L.bsm_plan_verify.argtypes = [_p, _p]
    L.bsm_plan_tile_classes.argtypes = [_p, _p, ctypes.c_int32]
    L.bsm_plan_set_tile_classes.argtypes = [_p, _p]
    L.bsm_batch_tile_classes.argtypes = [_p, _p, ctypes.c_int32]
    L.bsm_plan_debug_skip_task.argtypes = [_p, _i64]
    L.bsm_batch_verify.argtypes = [_p, _p]
    L.bsm_plan_destroy.argtypes = [_p]
    L.bsm_plan_timings.argtypes = [_p, _p, _p, _i64, _p]
    L.bsm_plan_features.argtypes = [_p, _p, _i64]
    L.bsm_plan_set_costs.argtypes = [_p, _p, _i64]
    L.bsm_autotune.argtypes = [_p, _p, _p, _p, _p, _p]
    L.bsm_batch_create.argtypes = [ctypes.POINTER(_p), _p, _i64]
    L.bsm_batch_query.argtypes = [_p, _p, _p, _p]
    L.bsm_batch_execute.argtypes = [_p, _p, _p, _p, _p, ctypes.c_int, _p]
    L.bsm_batch_timings.argtypes = [_p, _p, _p, _i64, _p]
    L.bsm_batch_set_costs.argtypes = [_p, _p, _i64]
    L.bsm_batch_autotune.argtypes = [_p, _p, _p, _p, _p, _p]
    L.bsm_batch_destroy.argtypes = [_p]
    L.bsm_costmodel_create.argtypes = [ctypes.POINTER(_p), ctypes.c_uint64]
    L.bsm_costmodel_param_count.restype = _i64
    L.bsm_costmodel_param_count.argtypes = []
    L.bsm_costmodel_params.argtypes = [_p, _p, _i64, _p]
    L.bsm_costmodel_set_params.argtypes = [_p, _p, _i64, _p]
    L.bsm_costmodel_train.argtypes = [_p, _p, _p, _i64, _i64, _i64, ctypes.c_float, _p, _p]
    L.bsm_costmodel_predict.argtypes = [_p, _p, _i64, _p, _p]
    L.bsm_costmodel_save.argtypes = [_p, ctypes.c_char_p]
    L.bsm_costmodel_load.argtypes = [ctypes.POINTER(_p), ctypes.c_char_p]
    L.bsm_costmodel_destroy.argtypes = [_p]
    L.bsm_plan_set_costmodel.argtypes = [_p, _p, _p]
    L.bsm_batch_set_costmodel.argtypes = [_p, _p, _p]
    L.bsm_mlp_forward.argtypes = [_p, _p, _i64, _p, _p]
    L.bsm_mlp_loss_grad.argtypes = [_p, _p, _p, _i64, _p, _p, _p]
    L.bsm_adam_step.argtypes = [_p, _p, _p, _p, _i64, _i64, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, _p]
    L.bsm_lr_plan_create.argtypes = [ctypes.POINTER(_p), _i64, _p, _i64, _p, _i64, _p, _p, _p,
                                     _p, ctypes.POINTER(Options)]
    L.bsm_lr_plan_query.argtypes = [_p, ctypes.POINTER(LrInfo)]
    L.bsm_lr_plan_c_offsets.argtypes = [_p, _p]
    L.bsm_lr_execute.argtypes = [_p, ctypes.c_double, _p, _p, _p, ctypes.c_int, _p]
    L.bsm_lr_plan_verify.argtypes = [_p, _p]
    L.bsm_lr_plan_destroy.argtypes = [_p]
    L.bsm_tc_plan_create.argtypes = [ctypes.POINTER(_p), ctypes.POINTER(TensorDesc),
                                     ctypes.POINTER(TensorDesc), ctypes.c_int32, _p,
                                     ctypes.POINTER(Options)]
    L.bsm_tc_plan_query.argtypes = [_p, ctypes.POINTER(TcInfo)]
    L.bsm_tc_plan_c_shape.argtypes = [_p, _p]
    L.bsm_tc_execute.argtypes = [_p, ctypes.c_double, _p, _p, _p, ctypes.c_int, _p]
    L.bsm_tc_plan_verify.argtypes = [_p, _p]
    L.bsm_tc_plan_destroy.argtypes = [_p]
    for name in ("bsm_tc_plan_create", "bsm_tc_plan_query", "bsm_tc_plan_c_shape",
                 "bsm_tc_execute", "bsm_tc_plan_verify", "bsm_tc_plan_destroy"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("bsm_lr_plan_create", "bsm_lr_plan_query", "bsm_lr_plan_c_offsets",
                 "bsm_lr_execute", "bsm_lr_plan_verify", "bsm_lr_plan_destroy",
                 "bsm_execute_complex"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("bsm_plan_create", "bsm_plan_query", "bsm_plan_c_shape", "bsm_plan_c_offsets",
                 "bsm_execute", "bsm_execute_static", "bsm_plan_verify", "bsm_plan_tile_classes",
                 "bsm_plan_set_tile_classes", "bsm_batch_tile_classes", "bsm_plan_debug_skip_task", "bsm_batch_verify",
                 "bsm_plan_destroy", "bsm_plan_timings", "bsm_plan_features",
                 "bsm_plan_set_costs", "bsm_autotune", "bsm_batch_create", "bsm_batch_query",
                 "bsm_batch_execute", "bsm_batch_timings", "bsm_batch_set_costs",
                 "bsm_batch_autotune", "bsm_batch_destroy", "bsm_costmodel_create",
                 "bsm_costmodel_params", "bsm_costmodel_set_params", "bsm_costmodel_train",
                 "bsm_costmodel_predict", "bsm_costmodel_save", "bsm_costmodel_load",
                 "bsm_costmodel_destroy", "bsm_plan_set_costmodel", "bsm_batch_set_costmodel",
                 "bsm_mlp_forward", "bsm_mlp_loss_grad", "bsm_adam_step"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def declared_symbols() -> list:
    """Names of the functions include/bsm.h declares."""
    import re
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(bsm_[a-z0-9_]+)\s*\(", text)))


def _check(code: int):
    if code != OK:
        raise BsmError(code, load().bsm_last_error().decode())


def _arr(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def options(precision=FP64, sched=SCHED_FLOPS, k_window=0, record_timings=0, tile=0,
            use_graph=0, out=OUT_F64, order=ORDER_DEFAULT, patch=(0, 0), device_klists=0,
            tune_cache=None, trans_a=0, trans_b=0, elem=0, k_split=0) -> Options:
    o = Options()
    load().bsm_options_default(ctypes.byref(o))
    o.precision, o.sched, o.k_window, o.record_timings, o.tile = precision, sched, k_window, record_timings, tile
    o.use_graph, o.out, o.order = use_graph, out, order
    o.patch_rows, o.patch_cols = int(patch[0]), int(patch[1])
    o.device_klists = int(device_klists)
    o.trans_a, o.trans_b, o.elem, o.k_split = int(trans_a), int(trans_b), int(elem), int(k_split)
    o.tune_cache = tune_cache.encode() if tune_cache else None
    return o


def concurrent_iterations(p_row: int, p_col: int, K: int) -> int:
    return int(load().bsm_concurrent_iterations(p_row, p_col, K))


def tile_variants(precision=FP64):
    """[(tm, tn)] of every tile variant of a precision form (option tile = index + 1)."""
    L = load()
    fn = L.bsm_bf16_tile_variants if precision == BF16X3 else L.bsm_tile_variants
    n = int(fn(None, None, 0))
    tm = np.zeros(n, np.int32)
    tn = np.zeros(n, np.int32)
    fn(tm.ctypes.data, tn.ctypes.data, n)
    return list(zip(tm.tolist(), tn.tolist()))


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t) -> int:
    if t is None:
        return 0
    return t.data_ptr()


def _check_operands(info, A, B, C):
    """Device buffers handed to the library must hold the plan's element counts and be
    contiguous device tensors of the right type: FP64 (complex128) A and B, C in the plan's output
    type (the C ABI only sees the pointers)."""
    bufs = (("A", A, info.a_elems), ("B", B, info.b_elems), ("C", C, info.c_elems))
    for name, t, need in bufs:
        if need > 0 and t is None:
            raise ValueError(f"{name} is required ({need} elements)")
        if need > 0 and t.numel() < need:
            raise ValueError(f"{name} holds {t.numel()} elements, the plan needs {need}")
    used = [(name, t) for name, t, need in bufs if need > 0 and t is not None]
    for name, t in used:
        f32 = name == "C" and info.out == OUT_F32
        if info.elem == COMPLEX:
            want = "torch.complex64" if f32 else "torch.complex128"
        else:
            want = "torch.float32" if f32 else "torch.float64"
        if getattr(t, "dtype", None) is not None and str(t.dtype) != want:
            raise ValueError(f"{name} must be {want[6:]}, got {t.dtype}")
    for name, t in used:
        if hasattr(t, "is_contiguous") and not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    for name, t in used:
        if hasattr(t, "is_cuda") and not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")


class Plan:
    """A planned block-sparse product (host planning happens in the constructor)."""

    def __init__(self, rows, inner, cols, a_bits, b_bits, opts: Optional[Options] = None, **kw):
        L = load()
        self._rows = _arr(rows, np.int64)
        self._inner = _arr(inner, np.int64)
        self._cols = _arr(cols, np.int64)
        self._a = _arr(a_bits, np.uint64)
        self._b = _arr(b_bits, np.uint64)
        o = opts if opts is not None else options(**kw)
        self._opts = o  # keeps the tune-cache string alive for the call
        # shapes as stored: op(A) = A^T is given as K x M, op(B) = B^T as N x K
        M, K, N = self._rows.size, self._inner.size, self._cols.size
        ar, ac = (K, M) if o.trans_a else (M, K)
        br, bc = (N, K) if o.trans_b else (K, N)
        for name, bits, r, c in (("a_bits", self._a, ar, ac), ("b_bits", self._b, br, bc)):
            if bits.size < r * ((c + 63) // 64):
                raise ValueError(f"{name}: {bits.size} words, the {r} x {c} shape needs "
                                 f"{r * ((c + 63) // 64)}")
        h = _p()
        _check(L.bsm_plan_create(ctypes.byref(h), self._rows.size, self._rows.ctypes.data,
                                 self._inner.size, self._inner.ctypes.data, self._cols.size,
                                 self._cols.ctypes.data, self._a.ctypes.data, self._b.ctypes.data,
                                 ctypes.byref(o)))
        self._h = h

    @classmethod
    def from_problem(cls, p, **kw) -> "Plan":
        return cls(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), **kw)

    @property
    def handle(self):
        return self._h

    def info(self) -> PlanInfo:
        i = PlanInfo()
        _check(load().bsm_plan_query(self._h, ctypes.byref(i)))
        return i

    def c_shape(self) -> np.ndarray:
        out = np.zeros(self._rows.size * ((self._cols.size + 63) // 64), dtype=np.uint64)
        _check(load().bsm_plan_c_shape(self._h, out.ctypes.data))
        return out

    def c_offsets(self) -> np.ndarray:
        out = np.zeros(self._rows.size * self._cols.size, dtype=np.int64)
        _check(load().bsm_plan_c_offsets(self._h, out.ctypes.data))
        return out.reshape(self._rows.size, self._cols.size)

    def execute(self, A, B, C, alpha: float = 1.0, accumulate: bool = False, stream=None):
        """C = alpha*A*B (+C); A, B are FP64 device tensors holding the packed tiles, C a device
        tensor of the plan's output type."""
        info = self.info()
        _check_operands(info, A, B, C)
        if info.elem == COMPLEX:
            a = complex(alpha)
            _check(load().bsm_execute_complex(self._h, a.real, a.imag, _dev_ptr(A), _dev_ptr(B),
                                              _dev_ptr(C), int(bool(accumulate)),
                                              _stream_handle(stream)))
            return
        _check(load().bsm_execute(self._h, float(alpha), _dev_ptr(A), _dev_ptr(B), _dev_ptr(C),
                                  int(bool(accumulate)), _stream_handle(stream)))

    def execute_static(self, A, B, C, alpha: float = 1.0, accumulate: bool = False, stream=None):
        """As execute, with every device buffer the library needs taken from its static scratch
        (no allocation; calls that overlap on one GPU race)."""
        _check_operands(self.info(), A, B, C)
        _check(load().bsm_execute_static(self._h, float(alpha), _dev_ptr(A), _dev_ptr(B),
                                         _dev_ptr(C), int(bool(accumulate)), _stream_handle(stream)))

    def verify(self, stream=None):
        """Wait for the stream; raise BsmError(E_STATE) unless every task ran once per launch."""
        _check(load().bsm_plan_verify(self._h, _stream_handle(stream)))

    def debug_skip_task(self, task: int):
        """Fault injection for tests: later launches leave task `task` out (-1 = none)."""
        _check(load().bsm_plan_debug_skip_task(self._h, int(task)))

    def timings(self, stream=None):
        """(features[tasks, 5], seconds[tasks]) of the last timed execute."""
        n = self.info().tasks
        f = np.zeros((n, 5), dtype=np.float32)
        t = np.zeros(n, dtype=np.float32)
        _check(load().bsm_plan_timings(self._h, f.ctypes.data, t.ctypes.data, n, _stream_handle(stream)))
        return f, t

    def features(self) -> np.ndarray:
        n = self.info().tasks
        f = np.zeros((n, 5), dtype=np.float32)
        _check(load().bsm_plan_features(self._h, f.ctypes.data, n))
        return f

    def set_costs(self, costs):
        c = _arr(costs, np.float32)
        _check(load().bsm_plan_set_costs(self._h, c.ctypes.data, c.size))

    def autotune(self, A, B, C, stream=None) -> int:
        _check_operands(self.info(), A, B, C)
        chosen = ctypes.c_int32(0)
        _check(load().bsm_autotune(self._h, _dev_ptr(A), _dev_ptr(B), _dev_ptr(C),
                                   _stream_handle(stream), ctypes.byref(chosen)))
        return int(chosen.value)

    def set_costmodel(self, model: "CostModel", stream=None):
        _check(load().bsm_plan_set_costmodel(self._h, model.handle, _stream_handle(stream)))

    def tile_classes(self):
        """Tile variant (id + 1) of each of the four C-block size classes."""
        out = np.zeros(4, np.int32)
        _check(load().bsm_plan_tile_classes(self._h, out.ctypes.data, 4))
        return out.tolist()

    def set_tile_classes(self, variants):
        v = _arr(variants, np.int32)
        if v.size != 4:
            raise ValueError("one tile variant per size class (4)")
        _check(load().bsm_plan_set_tile_classes(self._h, v.ctypes.data))

    def close(self):
        if getattr(self, "_h", None):
            _check(load().bsm_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LowRankPlan:
    """C = alpha A B (+ C) with a block-rank-sparse A: a_ranks[q] is the rank of the q-th present
    block of A (row-major block order), 0 = dense; factored blocks are stored as U (r x rho) then
    V (s x rho), A_ik = U V^T."""

    def __init__(self, rows, inner, cols, a_bits, a_ranks, b_bits, opts: Optional[Options] = None,
                 **kw):
        L = load()
        self._rows = _arr(rows, np.int64)
        self._inner = _arr(inner, np.int64)
        self._cols = _arr(cols, np.int64)
        self._a = _arr(a_bits, np.uint64)
        self._r = _arr(a_ranks, np.int32)
        self._b = _arr(b_bits, np.uint64)
        M, K, N = self._rows.size, self._inner.size, self._cols.size
        for name, bits, r, c in (("a_bits", self._a, M, K), ("b_bits", self._b, K, N)):
            if bits.size < r * ((c + 63) // 64):
                raise ValueError(f"{name}: {bits.size} words, the {r} x {c} shape needs "
                                 f"{r * ((c + 63) // 64)}")
        o = opts if opts is not None else options(**kw)
        self._opts = o
        present = int(sum(bin(int(w)).count("1") for w in self._a))
        if self._r.size < present:
            raise ValueError(f"a_ranks: {self._r.size} entries, A has {present} present blocks")
        h = _p()
        _check(L.bsm_lr_plan_create(ctypes.byref(h), M, self._rows.ctypes.data, K,
                                    self._inner.ctypes.data, N, self._cols.ctypes.data,
                                    self._a.ctypes.data, self._r.ctypes.data, self._b.ctypes.data,
                                    ctypes.byref(o)))
        self._h = h

    def info(self) -> LrInfo:
        i = LrInfo()
        _check(load().bsm_lr_plan_query(self._h, ctypes.byref(i)))
        return i

    def c_offsets(self) -> np.ndarray:
        out = np.zeros(self._rows.size * self._cols.size, dtype=np.int64)
        _check(load().bsm_lr_plan_c_offsets(self._h, out.ctypes.data))
        return out.reshape(self._rows.size, self._cols.size)

    def execute(self, A, B, C, alpha: float = 1.0, accumulate: bool = False, stream=None):
        i = self.info()
        for name, t, need, dt in (("A", A, i.a_elems, "torch.float64"), ("B", B, i.b_elems, "torch.float64"),
                                  ("C", C, i.c_elems, None)):
            if need > 0 and (t is None or t.numel() < need):
                raise ValueError(f"{name} must hold {need} elements")
            if need > 0 and dt and str(t.dtype) != dt:
                raise ValueError(f"{name} must be {dt[6:]}")
            if need > 0 and hasattr(t, "is_contiguous") and not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
        _check(load().bsm_lr_execute(self._h, float(alpha), _dev_ptr(A), _dev_ptr(B), _dev_ptr(C),
                                     int(bool(accumulate)), _stream_handle(stream)))

    def verify(self, stream=None):
        _check(load().bsm_lr_plan_verify(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _check(load().bsm_lr_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Contraction:
    """C = alpha contract(A, B) (+ C) of block-sparse tensors.  Each operand is given as
    (labels, tilings, bits): one label and one block-size vector per mode, and the block shape in
    the library's word layout over the flattened (row-major) block grid."""

    def __init__(self, a, b, c_modes, opts: Optional[Options] = None, **kw):
        L = load()
        self._keep = []

        def desc(labels, tilings, bits):
            modes = _arr(labels, np.int32)
            nb = _arr([len(t) for t in tilings], np.int64)
            sizes = _arr(np.concatenate([np.asarray(t, np.int64) for t in tilings])
                         if len(tilings) else [], np.int64)
            grid = int(np.prod(nb)) if nb.size else 1
            bw = _arr(bits, np.uint64)
            if bw.size < (grid + 63) // 64:
                raise ValueError(f"bits: {bw.size} words, a grid of {grid} blocks needs {(grid + 63) // 64}")
            self._keep += [modes, nb, sizes, bw]
            return TensorDesc(int(modes.size), modes.ctypes.data, nb.ctypes.data,
                              sizes.ctypes.data if sizes.size else None, bw.ctypes.data if bw.size else None)

        da, db = desc(*a), desc(*b)
        cm = _arr(c_modes, np.int32)
        self._keep.append(cm)
        self._c_grid = int(np.prod([len(a[1][list(a[0]).index(m)]) if m in list(a[0])
                                    else len(b[1][list(b[0]).index(m)]) for m in c_modes])) \
            if len(c_modes) else 1
        o = opts if opts is not None else options(**kw)
        self._opts = o
        h = _p()
        _check(L.bsm_tc_plan_create(ctypes.byref(h), ctypes.byref(da), ctypes.byref(db),
                                    int(cm.size), cm.ctypes.data if cm.size else None,
                                    ctypes.byref(o)))
        self._h = h

    def info(self) -> TcInfo:
        i = TcInfo()
        _check(load().bsm_tc_plan_query(self._h, ctypes.byref(i)))
        return i

    def c_shape(self) -> np.ndarray:
        out = np.zeros(max(1, (self._c_grid + 63) // 64), dtype=np.uint64)
        _check(load().bsm_tc_plan_c_shape(self._h, out.ctypes.data))
        return out

    def execute(self, A, B, C, alpha: float = 1.0, accumulate: bool = False, stream=None):
        i = self.info()
        cdt = "torch.float32" if self._opts.out == OUT_F32 else "torch.float64"
        for name, t, need, dt in (("A", A, i.a_elems, "torch.float64"),
                                  ("B", B, i.b_elems, "torch.float64"), ("C", C, i.c_elems, cdt)):
            if need > 0 and (t is None or t.numel() < need):
                raise ValueError(f"{name} must hold {need} elements")
            if need > 0 and str(t.dtype) != dt:
                raise ValueError(f"{name} must be {dt[6:]}")
            if need > 0 and hasattr(t, "is_contiguous") and not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
        _check(load().bsm_tc_execute(self._h, float(alpha), _dev_ptr(A), _dev_ptr(B), _dev_ptr(C),
                                     int(bool(accumulate)), _stream_handle(stream)))

    def verify(self, stream=None):
        _check(load().bsm_tc_plan_verify(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _check(load().bsm_tc_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr_array(xs):
    arr = (ctypes.c_void_p * len(xs))()
    for q, x in enumerate(xs):
        arr[q] = _dev_ptr(x) if x is not None else 0
    return arr


class Batch:
    """Many independent products executed as one graph-captured launch."""

    def __init__(self, plans):
        self._plans = list(plans)  # keep the member plans alive
        hs = (ctypes.c_void_p * len(self._plans))(*[p.handle.value for p in self._plans])
        h = _p()
        _check(load().bsm_batch_create(ctypes.byref(h), hs, len(self._plans)))
        self._h = h

    def query(self):
        t = ctypes.c_int64(0)
        f = ctypes.c_double(0)
        v = ctypes.c_int32(0)
        _check(load().bsm_batch_query(self._h, ctypes.byref(t), ctypes.byref(f), ctypes.byref(v)))
        return int(t.value), float(f.value), int(v.value)

    def execute(self, As, Bs, Cs, alphas=None, accumulate=False, stream=None):
        n = len(self._plans)
        if not (len(As) == len(Bs) == len(Cs) == n):
            raise ValueError("one A, B and C per member plan")
        for p, A, B, C in zip(self._plans, As, Bs, Cs):
            _check_operands(p.info(), A, B, C)
        al = None
        if alphas is not None:
            al = np.ascontiguousarray(np.asarray(alphas, dtype=np.float64))
        _check(load().bsm_batch_execute(self._h, al.ctypes.data if al is not None else None,
                                        _ptr_array(As), _ptr_array(Bs), _ptr_array(Cs),
                                        int(bool(accumulate)), _stream_handle(stream)))

    def verify(self, stream=None):
        _check(load().bsm_batch_verify(self._h, _stream_handle(stream)))

    def timings(self, stream=None):
        n = self.query()[0]
        f = np.zeros((n, 5), dtype=np.float32)
        t = np.zeros(n, dtype=np.float32)
        _check(load().bsm_batch_timings(self._h, f.ctypes.data, t.ctypes.data, n, _stream_handle(stream)))
        return f, t

    def set_costs(self, costs):
        c = _arr(costs, np.float32)
        _check(load().bsm_batch_set_costs(self._h, c.ctypes.data, c.size))

    def autotune(self, As, Bs, Cs, stream=None) -> int:
        for p, A, B, C in zip(self._plans, As, Bs, Cs):
            _check_operands(p.info(), A, B, C)
        chosen = ctypes.c_int32(0)
        _check(load().bsm_batch_autotune(self._h, _ptr_array(As), _ptr_array(Bs), _ptr_array(Cs),
                                         _stream_handle(stream), ctypes.byref(chosen)))
        return int(chosen.value)

    def set_costmodel(self, model: "CostModel", stream=None):
        _check(load().bsm_batch_set_costmodel(self._h, model.handle, _stream_handle(stream)))

    def tile_classes(self):
        out = np.zeros(4, np.int32)
        _check(load().bsm_batch_tile_classes(self._h, out.ctypes.data, 4))
        return out.tolist()

    def close(self):
        if getattr(self, "_h", None):
            _check(load().bsm_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_IN, MLP_HIDDEN = 5, 32


def mlp_param_count() -> int:
    return int(load().bsm_costmodel_param_count())


class CostModel:
    """The learned task cost model (parameters and Adam state live on the device)."""

    def __init__(self, seed: int = 0, _handle=None):
        if _handle is not None:
            self._h = _handle
        else:
            h = _p()
            _check(load().bsm_costmodel_create(ctypes.byref(h), int(seed)))
            self._h = h

    @property
    def handle(self):
        return self._h

    @classmethod
    def load_file(cls, path: str) -> "CostModel":
        h = _p()
        _check(load().bsm_costmodel_load(ctypes.byref(h), path.encode()))
        return cls(_handle=h)

    def save(self, path: str):
        _check(load().bsm_costmodel_save(self._h, path.encode()))

    def params(self):
        n = mlp_param_count()
        p = np.zeros(n, dtype=np.float32)
        norm = np.zeros(12, dtype=np.float32)
        _check(load().bsm_costmodel_params(self._h, p.ctypes.data, n, norm.ctypes.data))
        return p, norm

    def set_params(self, params=None, norm=None):
        p = _arr(params, np.float32) if params is not None else None
        nm = _arr(norm, np.float32) if norm is not None else None
        _check(load().bsm_costmodel_set_params(self._h, p.ctypes.data if p is not None else None,
                                               p.size if p is not None else 0,
                                               nm.ctypes.data if nm is not None else None))

    def train(self, features, log_seconds, epochs=200, batch=1024, lr=3e-3, stream=None) -> float:
        f = _arr(features, np.float32).reshape(-1, MLP_IN)
        t = _arr(log_seconds, np.float32).reshape(-1)
        loss = ctypes.c_float(0)
        _check(load().bsm_costmodel_train(self._h, f.ctypes.data, t.ctypes.data, t.size, epochs,
                                          batch, lr, ctypes.byref(loss), _stream_handle(stream)))
        return float(loss.value)

    def predict(self, features, stream=None) -> np.ndarray:
        f = _arr(features, np.float32).reshape(-1, MLP_IN)
        out = np.zeros(f.shape[0], dtype=np.float32)
        _check(load().bsm_costmodel_predict(self._h, f.ctypes.data, f.shape[0], out.ctypes.data,
                                            _stream_handle(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            _check(load().bsm_costmodel_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward(d_params, d_x, d_y, stream=None):
    _check(load().bsm_mlp_forward(_dev_ptr(d_params), _dev_ptr(d_x), d_x.shape[0], _dev_ptr(d_y),
                                  _stream_handle(stream)))


def mlp_loss_grad(d_params, d_x, d_t, d_grad, d_loss=None, stream=None):
    _check(load().bsm_mlp_loss_grad(_dev_ptr(d_params), _dev_ptr(d_x), _dev_ptr(d_t), d_x.shape[0],
                                    _dev_ptr(d_grad), _dev_ptr(d_loss), _stream_handle(stream)))


def adam_step(d_params, d_grad, d_m, d_v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load().bsm_adam_step(_dev_ptr(d_params), _dev_ptr(d_grad), _dev_ptr(d_m), _dev_ptr(d_v),
                                d_params.numel(), int(step), lr, beta1, beta2, eps,
                                _stream_handle(stream)))
