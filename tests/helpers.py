"""Test-side helpers: dense views of packed block-sparse data, error measures.

Written independently of both the oracle and the GPU library (plain Python/numpy loops)."""
import numpy as np


def packed_offsets(rsz, csz, mask):
    """dict (i, j) -> element offset of each present block, row-major block order."""
    off, pos = {}, 0
    for i in range(len(rsz)):
        for j in range(len(csz)):
            if mask[i][j]:
                off[(i, j)] = pos
                pos += int(rsz[i]) * int(csz[j])
    return off, pos


def to_dense(rsz, csz, mask, data):
    rsz = [int(x) for x in rsz]
    csz = [int(x) for x in csz]
    ro = np.concatenate([[0], np.cumsum(rsz)]).astype(int)
    co = np.concatenate([[0], np.cumsum(csz)]).astype(int)
    D = np.zeros((ro[-1], co[-1]), dtype=np.asarray(data).dtype)
    off, _ = packed_offsets(rsz, csz, mask)
    for (i, j), o in off.items():
        D[ro[i]:ro[i + 1], co[j]:co[j + 1]] = np.asarray(data[o:o + rsz[i] * csz[j]]).reshape(rsz[i], csz[j])
    return D


def from_dense(rsz, csz, mask, D):
    rsz = [int(x) for x in rsz]
    csz = [int(x) for x in csz]
    ro = np.concatenate([[0], np.cumsum(rsz)]).astype(int)
    co = np.concatenate([[0], np.cumsum(csz)]).astype(int)
    off, total = packed_offsets(rsz, csz, mask)
    out = np.zeros(total, dtype=D.dtype)
    for (i, j), o in off.items():
        out[o:o + rsz[i] * csz[j]] = D[ro[i]:ro[i + 1], co[j]:co[j + 1]].reshape(-1)
    return out


def rel_fro(x, ref):
    """Relative Frobenius error; absolute when the reference is zero."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm(x - ref)
    n = np.linalg.norm(ref)
    return float(d / n) if n > 0 else float(d)


def higham_gamma(n):
    u = 2.0 ** -53
    return n * u / (1 - n * u)
