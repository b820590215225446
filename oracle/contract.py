"""CPU reference for block-sparse tensor contraction -- TEST INFRASTRUCTURE ONLY (same rules as the
rest of this package: the GPU library never uses it, it never uses the GPU library).

The paper's title calls the block-sparse matrix product a step towards block-sparse tensor
computing (Sec. 1 and the conclusion): a contraction of two block-sparse tensors is a product of
their block-sparse matricizations.  This module computes the contraction directly from its
definition, block by block:

  a tensor of order d has a tiling per mode (block sizes) and a block shape (which block tuples
  are present); its present blocks are packed in row-major order over the block grid (last mode
  fastest), each block dense and row-major over its modes.  Modes carry labels; a label shared by
  A and B and absent from C is contracted, a label of C comes from exactly one of A and B.

  C-shape: C block c is present iff some contracted block tuple t has A(c_A, t) and B(c_B, t)
  present.  Values: C_c = alpha * sum over such t, in lexicographic order of t, of the
  contraction of the two dense blocks over the contracted modes (+ C_c when accumulating).

numpy's tensordot is the block-level contraction step (a library primitive); everything else is
plain Python over block tuples.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


class Tensor:
    """A block-sparse tensor: labels, per-mode tilings, present block tuples and packed data."""

    def __init__(self, modes: Sequence[int], tilings: Sequence[Sequence[int]],
                 present: np.ndarray, data: np.ndarray):
        self.modes = [int(m) for m in modes]
        self.tilings = [np.asarray(t, dtype=np.int64) for t in tilings]
        self.present = np.asarray(present, dtype=bool)   # boolean array over the block grid
        self.data = np.asarray(data, dtype=np.float64)
        assert self.present.shape == tuple(len(t) for t in self.tilings)

    def blocks(self) -> Dict[Tuple[int, ...], np.ndarray]:
        """Present block tuple -> dense block (a view into data), in packed order."""
        out, pos = {}, 0
        for idx in zip(*np.nonzero(self.present)):
            idx = tuple(int(v) for v in idx)
            shape = tuple(int(self.tilings[m][idx[m]]) for m in range(len(idx)))
            n = int(np.prod(shape, dtype=np.int64))
            out[idx] = self.data[pos:pos + n].reshape(shape)
            pos += n
        assert pos == self.data.size, (pos, self.data.size)
        return out


def contract(A: Tensor, B: Tensor, c_modes: Sequence[int], alpha: float = 1.0,
             C: Optional[Tuple[np.ndarray, np.ndarray]] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Returns (C's block shape as a boolean grid array, C's packed data)."""
    c_modes = [int(m) for m in c_modes]
    contracted = [m for m in A.modes if m in B.modes and m not in c_modes]
    where = {}
    for m in c_modes:
        if m in A.modes:
            where[m] = ("A", A.modes.index(m))
        else:
            where[m] = ("B", B.modes.index(m))
    c_tilings = [A.tilings[where[m][1]] if where[m][0] == "A" else B.tilings[where[m][1]]
                 for m in c_modes]
    ab, bb = A.blocks(), B.blocks()
    grid = tuple(len(t) for t in c_tilings)
    t_ranges = [range(len(A.tilings[A.modes.index(m)])) for m in contracted]
    c_present = np.zeros(grid, dtype=bool)
    results = {}
    for cidx in itertools.product(*[range(n) for n in grid]):
        acc = None
        for t in itertools.product(*t_ranges):
            a_idx = tuple(cidx[c_modes.index(m)] if m in c_modes else t[contracted.index(m)]
                          for m in A.modes)
            b_idx = tuple(cidx[c_modes.index(m)] if m in c_modes else t[contracted.index(m)]
                          for m in B.modes)
            if a_idx not in ab or b_idx not in bb:
                continue
            # contract the dense blocks over the contracted modes; the result's modes are A's
            # free modes then B's free modes, each in its operand's order
            part = np.tensordot(ab[a_idx], bb[b_idx],
                                axes=([A.modes.index(m) for m in contracted],
                                      [B.modes.index(m) for m in contracted]))
            acc = part if acc is None else acc + part
        if acc is None:
            continue
        order = [m for m in A.modes if m in c_modes] + [m for m in B.modes if m in c_modes]
        acc = np.transpose(acc, [order.index(m) for m in c_modes])
        c_present[cidx] = True
        results[cidx] = alpha * acc
    parts = []
    prev = C[1] if C is not None else None
    pos = 0
    for cidx in np.ndindex(*c_present.shape):   # row-major; also the scalar (order-0) C
        if not c_present[cidx]:
            continue
        blk = results[cidx].reshape(-1)
        if prev is not None:
            blk = blk + prev[pos:pos + blk.size]
        parts.append(blk)
        pos += blk.size
    if C is not None and pos != prev.size:
        raise ValueError("C has the wrong size")
    return c_present, (np.concatenate(parts) if parts else np.zeros(0))


def contract_blocks(A: Tensor, B: Tensor, c_modes: Sequence[int],
                    sel: Sequence[Tuple[int, ...]]) -> List[Optional[np.ndarray]]:
    """Selected C blocks (alpha = 1), each from the same definition as `contract`; None for a
    block outside C's shape."""
    c_modes = [int(m) for m in c_modes]
    contracted = [m for m in A.modes if m in B.modes and m not in c_modes]
    ab, bb = A.blocks(), B.blocks()
    t_ranges = [range(len(A.tilings[A.modes.index(m)])) for m in contracted]
    order = [m for m in A.modes if m in c_modes] + [m for m in B.modes if m in c_modes]
    out = []
    for cidx in sel:
        acc = None
        for t in itertools.product(*t_ranges):
            a_idx = tuple(cidx[c_modes.index(m)] if m in c_modes else t[contracted.index(m)]
                          for m in A.modes)
            b_idx = tuple(cidx[c_modes.index(m)] if m in c_modes else t[contracted.index(m)]
                          for m in B.modes)
            if a_idx not in ab or b_idx not in bb:
                continue
            part = np.tensordot(ab[a_idx], bb[b_idx],
                                axes=([A.modes.index(m) for m in contracted],
                                      [B.modes.index(m) for m in contracted]))
            acc = part if acc is None else acc + part
        out.append(None if acc is None else np.transpose(acc, [order.index(m) for m in c_modes]))
    return out


def densify(T: Tensor) -> np.ndarray:
    """The zero-filled dense tensor (modes in T's order)."""
    offs = [np.concatenate([[0], np.cumsum(t)]) for t in T.tilings]
    D = np.zeros(tuple(int(o[-1]) for o in offs))
    for idx, blk in T.blocks().items():
        sl = tuple(slice(int(offs[m][idx[m]]), int(offs[m][idx[m] + 1])) for m in range(len(idx)))
        D[sl] = blk
    return D


def pack(c_present: np.ndarray, tilings: Sequence[np.ndarray], D: np.ndarray) -> np.ndarray:
    """Packed data of the present blocks of a dense tensor D (inverse of densify)."""
    offs = [np.concatenate([[0], np.cumsum(t)]) for t in tilings]
    parts = []
    for idx in np.ndindex(*c_present.shape):
        if not c_present[idx]:
            continue
        sl = tuple(slice(int(offs[m][idx[m]]), int(offs[m][idx[m] + 1])) for m in range(len(idx)))
        parts.append(D[sl].reshape(-1))
    return np.concatenate(parts) if parts else np.zeros(0)
