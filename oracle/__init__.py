"""CPU reference (the oracle) for the block-sparse product and the task cost model.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline leg are the
only callers.  The GPU library never imports, links or runs anything here, and nothing here
imports the GPU library.  The arithmetic lives in plain C (``bsmm_ref.c``, ``mlp_ref.c``), built
with gcc at -O2 with floating-point contraction off; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "bsmm_ref.c"), os.path.join(_HERE, "mlp_ref.c")]
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build_library() -> str:
    """Compile the oracle (always; a few seconds)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
           "-std=c11", "-Wall", "-o", LIB_PATH + ".tmp"] + _SRC + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_library()
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_words.restype = _i64
        L.oracle_words.argtypes = [_i64]
        L.oracle_shape_product.argtypes = [_i64, _i64, _i64, _p, _p, _p]
        L.oracle_block_offsets.restype = _i64
        L.oracle_block_offsets.argtypes = [_i64, _i64, _p, _p, _p, _p]
        L.oracle_useful_flops.restype = ctypes.c_double
        L.oracle_useful_flops.argtypes = [_i64, _i64, _i64, _p, _p, _p, _p, _p]
        L.oracle_bsmm.argtypes = [_i64, _i64, _i64, _p, _p, _p, _p, _p, _p, _p, ctypes.c_double,
                                  ctypes.c_int, _p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_bsmm_blocks.argtypes = [_i64, _i64, _i64, _p, _p, _p, _p, _p, _p, _p,
                                         ctypes.c_double, _i64, _p, _p, _p, _p, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int]
        L.oracle_zbsmm.argtypes = [_i64, _i64, _i64, _p, _p, _p, _p, _p, _p, _p, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, _p, ctypes.c_int, ctypes.c_int]
        L.oracle_zbsmm_blocks.argtypes = [_i64, _i64, _i64, _p, _p, _p, _p, _p, _p, _p, _i64, _p,
                                          _p, _p, _p, ctypes.c_int, ctypes.c_int]
        L.oracle_lr_expand.argtypes = [_i64, _i64, _p, _p, _p, _p, _p, _p]
        L.oracle_concurrent_iterations.restype = _i64
        L.oracle_concurrent_iterations.argtypes = [_i64, _i64, _i64]
        L.oracle_memory_overhead.restype = ctypes.c_double
        L.oracle_memory_overhead.argtypes = [ctypes.c_double] * 7
        L.oracle_mlp_param_count.restype = _i64
        L.oracle_mlp_param_count.argtypes = [_i64, _i64, _i64]
        L.oracle_mlp_forward.argtypes = [_i64, _i64, _i64, _p, _i64, _p, _p]
        L.oracle_mlp_loss_grad.restype = ctypes.c_double
        L.oracle_mlp_loss_grad.argtypes = [_i64, _i64, _i64, _p, _i64, _p, _p, _p]
        L.oracle_adam_step.argtypes = [_i64, _p, _p, _p, _p, _i64, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _c64(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def set_threads(n: int) -> int:
    """Sets the OpenMP threads of later oracle calls (timing only); returns the previous count."""
    return int(lib().oracle_set_threads(int(n)))


# ---- block-sparse product ---------------------------------------------------------------------
def shape_product(M: int, K: int, N: int, a_bits, b_bits) -> np.ndarray:
    a = _c64(a_bits, np.uint64)
    b = _c64(b_bits, np.uint64)
    c = np.zeros(M * lib().oracle_words(N), dtype=np.uint64)
    lib().oracle_shape_product(M, K, N, _ptr(a), _ptr(b), _ptr(c))
    return c


def block_offsets(rsz, csz, bits) -> Tuple[np.ndarray, int]:
    r = _c64(rsz, np.int64)
    c = _c64(csz, np.int64)
    w = _c64(bits, np.uint64)
    off = np.empty(r.size * c.size, dtype=np.int64)
    total = lib().oracle_block_offsets(r.size, c.size, _ptr(r), _ptr(c), _ptr(w), _ptr(off))
    return off.reshape(r.size, c.size), int(total)


def useful_flops(rows, inner, cols, a_bits, b_bits) -> float:
    r, s, t = (_c64(x, np.int64) for x in (rows, inner, cols))
    a = _c64(a_bits, np.uint64)
    b = _c64(b_bits, np.uint64)
    return lib().oracle_useful_flops(r.size, s.size, t.size, _ptr(r), _ptr(s), _ptr(t), _ptr(a), _ptr(b))


def product_shape(M: int, K: int, N: int, a_bits, b_bits, trans_a: bool = False,
                  trans_b: bool = False) -> np.ndarray:
    """C-shape of op(A) op(B) from the stored shapes (a transposed operand's bitmap is stored
    transposed: K x M for A, N x K for B)."""
    if not trans_a and not trans_b:
        return shape_product(M, K, N, a_bits, b_bits)
    from itertools import product as _prod
    wa = lib().oracle_words(M if trans_a else K)
    wb = lib().oracle_words(K if trans_b else N)
    a = _c64(a_bits, np.uint64)
    b = _c64(b_bits, np.uint64)
    bit = lambda w, words, x, y: bool((int(w[x * words + y // 64]) >> (y % 64)) & 1)
    la = np.zeros((M, K), bool)
    lb = np.zeros((K, N), bool)
    for i, k in _prod(range(M), range(K)):
        la[i, k] = bit(a, wa, k, i) if trans_a else bit(a, wa, i, k)
    for k, j in _prod(range(K), range(N)):
        lb[k, j] = bit(b, wb, j, k) if trans_b else bit(b, wb, k, j)
    wn = lib().oracle_words(N)
    out = np.zeros(M * wn, dtype=np.uint64)
    for i in range(M):
        for j in range(N):
            if np.any(la[i] & lb[:, j]):
                out[i * wn + j // 64] |= np.uint64(1) << np.uint64(j % 64)
    return out


def bsmm(rows, inner, cols, a_bits, b_bits, A, B, alpha: float = 1.0,
         C: Optional[np.ndarray] = None, extended: bool = False, trans_a: bool = False,
         trans_b: bool = False) -> np.ndarray:
    """Packed C = alpha*op(A)*op(B) (+ C when C is given).  Returns a new array."""
    r, s, t = (_c64(x, np.int64) for x in (rows, inner, cols))
    a = _c64(a_bits, np.uint64)
    b = _c64(b_bits, np.uint64)
    Ad = _c64(A, np.float64)
    Bd = Ad if B is A else _c64(B, np.float64)
    c_bits = product_shape(r.size, s.size, t.size, a, b, trans_a, trans_b)
    _, total = block_offsets(r, t, c_bits)
    if C is None:
        out = np.zeros(total, dtype=np.float64)
        acc = 0
    else:
        out = _c64(C, np.float64).copy()
        if out.size != total:
            raise ValueError("C has the wrong size")
        acc = 1
    st = lib().oracle_bsmm(r.size, s.size, t.size, _ptr(r), _ptr(s), _ptr(t), _ptr(a), _ptr(b),
                           _ptr(Ad), _ptr(Bd), float(alpha), acc, _ptr(out), int(extended),
                           int(bool(trans_a)), int(bool(trans_b)))
    if st != 0:
        raise MemoryError("oracle_bsmm failed")
    return out


def bsmm_blocks(rows, inner, cols, a_bits, b_bits, A, B, sel: Sequence[Tuple[int, int]],
                alpha: float = 1.0, extended: bool = False, trans_a: bool = False,
                trans_b: bool = False):
    """Selected C blocks: returns (list of 2-D arrays, list of presence flags)."""
    r, s, t = (_c64(x, np.int64) for x in (rows, inner, cols))
    a = _c64(a_bits, np.uint64)
    b = _c64(b_bits, np.uint64)
    Ad = _c64(A, np.float64)
    Bd = Ad if B is A else _c64(B, np.float64)
    si = _c64([q[0] for q in sel], np.int64)
    sj = _c64([q[1] for q in sel], np.int64)
    sizes = [int(r[i]) * int(t[j]) for i, j in sel]
    out = np.zeros(max(1, sum(sizes)), dtype=np.float64)
    present = np.zeros(max(1, len(sel)), dtype=np.int32)
    st = lib().oracle_bsmm_blocks(r.size, s.size, t.size, _ptr(r), _ptr(s), _ptr(t), _ptr(a),
                                  _ptr(b), _ptr(Ad), _ptr(Bd), float(alpha), len(sel), _ptr(si),
                                  _ptr(sj), _ptr(out), _ptr(present), int(extended),
                                  int(bool(trans_a)), int(bool(trans_b)))
    if st != 0:
        raise ValueError("oracle_bsmm_blocks failed")
    blocks, pos = [], 0
    for (i, j), n in zip(sel, sizes):
        blocks.append(out[pos:pos + n].reshape(int(r[i]), int(t[j])).copy())
        pos += n
    return blocks, [bool(x) for x in present[:len(sel)]]


def _ops(op):
    """'N' / 'T' / 'C' (or 0 / 1 / 2, or a bool for the transpose) -> 0 / 1 / 2."""
    return {"N": 0, "T": 1, "C": 2}[op] if isinstance(op, str) else int(op)


def zbsmm(rows, inner, cols, a_bits, b_bits, A, B, alpha: complex = 1.0,
          C: Optional[np.ndarray] = None, op_a="N", op_b="N") -> np.ndarray:
    """Packed complex C = alpha*op(A)*op(B) (+ C when C is given); op is 'N', 'T' (transpose) or
    'C' (adjoint); A, B, C are complex128 arrays of the packed blocks.  Returns a new array."""
    r, s, t = (_c64(x, np.int64) for x in (rows, inner, cols))
    a = _c64(a_bits, np.uint64)
    b = _c64(b_bits, np.uint64)
    oa, ob = _ops(op_a), _ops(op_b)
    Ad = _c64(A, np.complex128)
    Bd = Ad if B is A else _c64(B, np.complex128)
    c_bits = product_shape(r.size, s.size, t.size, a, b, oa != 0, ob != 0)
    _, total = block_offsets(r, t, c_bits)
    out = np.zeros(total, np.complex128) if C is None else _c64(C, np.complex128).copy()
    if out.size != total:
        raise ValueError("C has the wrong size")
    al = complex(alpha)
    st = lib().oracle_zbsmm(r.size, s.size, t.size, _ptr(r), _ptr(s), _ptr(t), _ptr(a), _ptr(b),
                            _ptr(Ad), _ptr(Bd), al.real, al.imag, int(C is not None), _ptr(out),
                            oa, ob)
    if st != 0:
        raise MemoryError("oracle_zbsmm failed")
    return out


def zbsmm_blocks(rows, inner, cols, a_bits, b_bits, A, B, sel: Sequence[Tuple[int, int]],
                 op_a="N", op_b="N"):
    """Selected complex C blocks (alpha = 1): (list of 2-D complex arrays, presence flags)."""
    r, s, t = (_c64(x, np.int64) for x in (rows, inner, cols))
    a = _c64(a_bits, np.uint64)
    b = _c64(b_bits, np.uint64)
    Ad = _c64(A, np.complex128)
    Bd = Ad if B is A else _c64(B, np.complex128)
    si = _c64([q[0] for q in sel], np.int64)
    sj = _c64([q[1] for q in sel], np.int64)
    sizes = [int(r[i]) * int(t[j]) for i, j in sel]
    out = np.zeros(max(1, sum(sizes)), dtype=np.complex128)
    present = np.zeros(max(1, len(sel)), dtype=np.int32)
    st = lib().oracle_zbsmm_blocks(r.size, s.size, t.size, _ptr(r), _ptr(s), _ptr(t), _ptr(a),
                                   _ptr(b), _ptr(Ad), _ptr(Bd), len(sel), _ptr(si), _ptr(sj),
                                   _ptr(out), _ptr(present), _ops(op_a), _ops(op_b))
    if st != 0:
        raise ValueError("oracle_zbsmm_blocks failed")
    blocks, pos = [], 0
    for (i, j), n in zip(sel, sizes):
        blocks.append(out[pos:pos + n].reshape(int(r[i]), int(t[j])).copy())
        pos += n
    return blocks, [bool(x) for x in present[:len(sel)]]


def lr_expand(rows, inner, a_bits, ranks, A_lr) -> np.ndarray:
    """Dense packed A from a block-rank-sparse packed A (factored blocks U V^T multiplied out)."""
    r, s = _c64(rows, np.int64), _c64(inner, np.int64)
    a = _c64(a_bits, np.uint64)
    rk = _c64(ranks, np.int32)
    src = _c64(A_lr, np.float64)
    M, K = r.size, s.size
    w = (K + 63) // 64
    total = 0
    for i in range(M):
        for k in range(K):
            if (int(a[i * w + k // 64]) >> (k % 64)) & 1:
                total += int(r[i]) * int(s[k])
    out = np.zeros(max(1, total), dtype=np.float64)
    if lib().oracle_lr_expand(M, K, _ptr(r), _ptr(s), _ptr(a), _ptr(rk), _ptr(src), _ptr(out)) != 0:
        raise ValueError("negative rank")
    return out[:total]


def concurrent_iterations(prow: int, pcol: int, K: int) -> int:
    return int(lib().oracle_concurrent_iterations(prow, pcol, K))


def memory_overhead(M, N, m, n, k, prow, pcol) -> float:
    return float(lib().oracle_memory_overhead(M, N, m, n, k, prow, pcol))


# ---- cost-model network ----------------------------------------------------------------------
def mlp_param_count(F: int, H1: int, H2: int) -> int:
    return int(lib().oracle_mlp_param_count(F, H1, H2))


def mlp_forward(F, H1, H2, params, X) -> np.ndarray:
    p = _c64(params, np.float64)
    x = _c64(X, np.float64)
    B = x.shape[0]
    y = np.empty(B, dtype=np.float64)
    lib().oracle_mlp_forward(F, H1, H2, _ptr(p), B, _ptr(x), _ptr(y))
    return y


def mlp_loss_grad(F, H1, H2, params, X, T):
    p = _c64(params, np.float64)
    x = _c64(X, np.float64)
    t = _c64(T, np.float64)
    g = np.empty(p.size, dtype=np.float64)
    loss = lib().oracle_mlp_loss_grad(F, H1, H2, _ptr(p), x.shape[0], _ptr(x), _ptr(t), _ptr(g))
    return float(loss), g


def adam_step(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In place on params, m, v (all float64 contiguous)."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().oracle_adam_step(params.size, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step),
                           lr, beta1, beta2, eps)
