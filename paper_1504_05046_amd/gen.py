"""Seeded synthetic inputs for block-sparse products (shared by the tests and the benchmark).

This module only *draws* inputs; it holds none of the multiply's arithmetic.  A problem is
described the way the library consumes it:

* three tilings (vectors of block sizes): ``rows`` (M blocks of C and A), ``inner`` (K blocks
  shared by A's columns and B's rows) and ``cols`` (N blocks of C and B) -- the problem-given,
  possibly nonuniform blocking of the matrix dimensions (paper Sec. 3.2: the matrices are cut
  into many more blocks than processes, of sizes the problem chooses);
* two block-shape masks ``a_mask`` (M x K) and ``b_mask`` (K x N) saying which blocks are present
  (block sparsity, paper Sec. 1);
* the present blocks' values, packed: blocks in row-major block order (i, then k), each block
  row-major with leading dimension equal to its column count.

Every block's values come from its own counter-addressed numpy stream
``SeedSequence(entropy=seed, spawn_key=(VALUES, matrix, i, k))`` so that any block can be
regenerated on its own -- except in ``decay_cloud``, whose 6.9 million blocks (at full size) come
from one stream per block row.

Workloads (sizes and distributions), one function each:

* ``uniform_1024``      N=1024, 16x16 blocks of 64, Bernoulli(0.5) per A and B block, U[-1,1].
* ``nonuniform_16384``  N=16384, sizes U{32..256} (last adjusted), Bernoulli(0.3), N(0,1).
* ``batch64``           64 independent products, N in {1024,2048,4096,8192}, sizes U{16..192},
                        density U[0.1,0.9] per product, N(0,1).
* ``precision_32768``   N=32768, sizes U{64..256}, Bernoulli(0.4), N(0,1)*10^U(-4,0) per block.
* ``decay_cloud``       4000 points in a 60-unit cube, block size per point from {10,25,40,60},
                        block (i,j) present iff exp(-r_ij/2) > 1e-8, values N(0,1)*exp(-r_ij/2);
                        C = A*A.
* ``paper_dense``       the paper's dense square experiment shape (Sec. 4.1): uniform blocks, or
                        the add-one-row-at-a-time nonuniform blocking with the same block count.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# spawn-key tags, so that the streams for tilings, shapes and values never coincide
_TILING, _SHAPE, _VALUES, _SCALE, _POINTS = 1, 2, 3, 4, 5
MAT_A, MAT_B = 0, 1
_IMAG_A, _IMAG_B = 2, 3  # streams of the imaginary parts of complex operands
_FACTORS = 6             # streams of the factors of low-rank blocks
_TENSOR = 7              # streams of block-sparse tensors


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(entropy=int(seed), spawn_key=tuple(int(k) for k in key)))


# --------------------------------------------------------------------------------------------
# tilings
# --------------------------------------------------------------------------------------------
def tiling_uniform(n: int, b: int) -> np.ndarray:
    """n split into blocks of b (the last one smaller if b does not divide n)."""
    q, r = divmod(n, b)
    sizes = [b] * q + ([r] if r else [])
    return np.asarray(sizes, dtype=np.int64)


def tiling_random(n: int, lo: int, hi: int, rng: np.random.Generator) -> np.ndarray:
    """Block sizes drawn uniformly from the integers lo..hi until the rest fits in one block;
    the last block takes the remainder (so it may be smaller than lo)."""
    sizes: List[int] = []
    rest = n
    while rest > hi:
        s = int(rng.integers(lo, hi + 1))
        sizes.append(s)
        rest -= s
    if rest > 0:
        sizes.append(rest)
    return np.asarray(sizes, dtype=np.int64)


def tiling_add_one(n: int, nblocks: int, rng: np.random.Generator) -> np.ndarray:
    """The paper's nonuniform blocking (Sec. 4.1): start from nblocks empty blocks and add one
    row to a uniformly chosen block until the sizes sum to n.  Blocks that stay empty are
    dropped (a block needs at least one row)."""
    counts = rng.multinomial(n, [1.0 / nblocks] * nblocks)
    return np.asarray([c for c in counts if c > 0], dtype=np.int64)


# --------------------------------------------------------------------------------------------
# problems
# --------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """One block-sparse product C = alpha * A * B (+ C)."""
    name: str
    rows: np.ndarray      # int64[M]
    inner: np.ndarray     # int64[K]
    cols: np.ndarray      # int64[N]
    a_mask: np.ndarray    # bool[M, K]
    b_mask: np.ndarray    # bool[K, N]
    a_data: np.ndarray    # float64, packed present blocks of A
    b_data: np.ndarray    # float64, packed present blocks of B (same object as a_data when aliased)
    b_is_a: bool = False  # C = A * A

    @property
    def M(self) -> int:
        return int(self.rows.shape[0])

    @property
    def K(self) -> int:
        return int(self.inner.shape[0])

    @property
    def N(self) -> int:
        return int(self.cols.shape[0])

    def a_bits(self) -> np.ndarray:
        return pack_bits(self.a_mask)

    def b_bits(self) -> np.ndarray:
        return pack_bits(self.b_mask)


def pack_bits(mask: np.ndarray) -> np.ndarray:
    """Block-shape bitmap in the library's word layout: bit (i, j) is bit j % 64 of word
    i * ceil(cols / 64) + j // 64; padding bits are zero."""
    mask = np.asarray(mask, dtype=bool)
    r, c = mask.shape
    w = (c + 63) // 64
    padded = np.zeros((r, w * 64), dtype=bool)
    padded[:, :c] = mask
    bits = np.packbits(padded.reshape(r, w, 8, 8)[:, :, :, ::-1], axis=-1).reshape(r, w, 8)
    # packbits gives big-endian bit order inside a byte; bytes are little-endian in the word
    return bits.view("<u8").reshape(r * w).astype(np.uint64) if r * w else np.zeros(0, np.uint64)


def unpack_bits(words: np.ndarray, r: int, c: int) -> np.ndarray:
    w = (c + 63) // 64
    if r * w == 0:
        return np.zeros((r, c), dtype=bool)
    b = np.asarray(words, dtype="<u8").reshape(r, w).view(np.uint8).reshape(r, w, 8)
    bits = np.unpackbits(b, axis=-1).reshape(r, w, 8, 8)[:, :, :, ::-1].reshape(r, w * 64)
    return bits[:, :c].astype(bool)


def stored_transpose(rsz, csz, mask, data) -> Tuple[np.ndarray, np.ndarray]:
    """Storage of X^T for a packed block matrix X (rsz x csz tiling): bitmap of mask^T and each
    present block transposed, packed in the transposed matrix's row-major block order.  Used to
    hand a product an operand that it reads as op(X) = X^T."""
    rsz = np.asarray(rsz, dtype=np.int64)
    csz = np.asarray(csz, dtype=np.int64)
    mask = np.asarray(mask, dtype=bool)
    data = np.asarray(data)
    offs = np.concatenate([[0], np.cumsum(rsz[np.nonzero(mask)[0]] * csz[np.nonzero(mask)[1]])])
    where = {(int(i), int(j)): int(offs[n]) for n, (i, j) in enumerate(zip(*np.nonzero(mask)))}
    out = np.empty(int(offs[-1]), dtype=data.dtype if data.size else np.float64)
    pos = 0
    mt = mask.T
    for j, i in zip(*np.nonzero(mt)):
        h, w = int(rsz[i]), int(csz[j])
        o = where[(int(i), int(j))]
        out[pos:pos + h * w] = data[o:o + h * w].reshape(h, w).T.reshape(-1)
        pos += h * w
    return pack_bits(mt), out


def imag_parts(p: Problem, seed: int, draw=None) -> Tuple[np.ndarray, np.ndarray]:
    """Complex operands of the same block structure: A and B with p's values as real parts and
    independent seeded draws (same shapes, same distribution as `draw`, N(0,1) by default) as
    imaginary parts, packed like p's buffers (complex128)."""
    draw = draw or _normal
    ia = _fill_blocks(seed, _IMAG_A, p.a_mask, p.rows, p.inner, draw)
    ib = ia if p.b_is_a else _fill_blocks(seed, _IMAG_B, p.b_mask, p.inner, p.cols, draw)
    za = p.a_data + 1j * ia
    zb = za if p.b_is_a else p.b_data + 1j * ib
    return za, zb


def low_rank_operand(p: Problem, seed: int, rank_fn, draw=None) -> Tuple[np.ndarray, np.ndarray]:
    """Block-rank-sparse A with p's block shape: for every present block (row-major block order)
    rank_fn(i, k, r_i, s_k) gives its rank rho; rho = 0 keeps p's dense block, otherwise the block
    is stored as factors U (r_i x rho) then V (s_k x rho), drawn from the block's own stream
    (N(0,1) / sqrt(rho) by default).  Returns (ranks int32, packed data)."""
    def _scaled(rng, i, k, h, w):
        return rng.standard_normal((h, w)) / np.sqrt(w)
    draw = draw or _scaled
    ranks, parts, pos = [], [], 0
    for i, k in zip(*np.nonzero(p.a_mask)):
        h, d = int(p.rows[i]), int(p.inner[k])
        rho = int(rank_fn(int(i), int(k), h, d))
        if rho == 0:
            parts.append(p.a_data[pos:pos + h * d])
        else:
            rng = _rng(seed, _FACTORS, int(i), int(k))
            parts.append(draw(rng, int(i), int(k), h, rho).reshape(-1))
            parts.append(draw(rng, int(i), int(k), d, rho).reshape(-1))
        ranks.append(rho)
        pos += h * d
    data = np.concatenate(parts) if parts else np.zeros(0)
    return np.asarray(ranks, dtype=np.int32), data


def block_rank_8192(seed: int = 6000):
    """Block-rank-sparse workload: N=8192 with the nonuniform tilings (sizes U{32..256}), A with
    every block present, blocks whose centres lie within 512 rows of the diagonal dense and the
    others of rank U{4..16}; B Bernoulli(0.3), N(0,1).  Returns (problem with A's dense shape,
    ranks, A's block-rank-sparse data)."""
    rows = tiling_random(8192, 32, 256, _rng(seed, _TILING, 0))
    inner = tiling_random(8192, 32, 256, _rng(seed, _TILING, 1))
    cols = tiling_random(8192, 32, 256, _rng(seed, _TILING, 2))
    a_mask = np.ones((rows.size, inner.size), dtype=bool)
    b_mask = _rng(seed, _SHAPE).random((inner.size, cols.size)) < 0.3
    p = make_problem("block_rank_8192", seed, rows, inner, cols, a_mask, b_mask)
    rc = np.cumsum(rows) - rows / 2.0
    ic = np.cumsum(inner) - inner / 2.0
    pick = _rng(seed, _SHAPE, 1)
    table = pick.integers(4, 17, (rows.size, inner.size))
    ranks, data = low_rank_operand(
        p, seed, lambda i, k, h, d: 0 if abs(rc[i] - ic[k]) < 512 else int(table[i, k]))
    return p, ranks, data


def block_sparse_tensor(seed: int, tilings: Sequence[Sequence[int]], density: float,
                        draw=None) -> Tuple[np.ndarray, np.ndarray]:
    """A block-sparse tensor with the given per-mode tilings: each block tuple present with
    probability `density` (at least one present), values N(0,1) (or draw(rng, shape)), one stream
    per block.  Returns (present: bool array over the block grid, data packed in row-major block
    order, each block row-major over its modes)."""
    tilings = [np.asarray(t, dtype=np.int64) for t in tilings]
    grid = tuple(len(t) for t in tilings)
    present = _rng(seed, _TENSOR, 0).random(grid) < density
    if present.size and not present.any():
        present.flat[0] = True
    parts = []
    for idx in zip(*np.nonzero(present)):
        shape = tuple(int(tilings[m][int(idx[m])]) for m in range(len(idx)))
        rng = _rng(seed, _TENSOR, 1, *[int(v) for v in idx])
        blk = draw(rng, shape) if draw else rng.standard_normal(shape)
        parts.append(np.asarray(blk, dtype=np.float64).reshape(-1))
    return present, (np.concatenate(parts) if parts else np.zeros(0))


def ladder_tensors(seed: int = 7000):
    """The coupled-cluster particle-particle ladder shape, C[i,j,a,b] = sum_{c,d} T[i,j,c,d]
    V[a,b,c,d]: 48 occupied indices in blocks U{8..24}, 192 virtual indices in blocks U{16..48}
    (one tiling per index space, shared by its modes), T with block density 0.5, V (stored with
    the contracted modes last, as integrals usually are) with block density 0.3, N(0,1) values.
    Returns (occupied tiling, virtual tiling, (T present, T data), (V present, V data))."""
    occ = tiling_random(48, 8, 24, _rng(seed, _TILING, 0))
    vir = tiling_random(192, 16, 48, _rng(seed, _TILING, 1))
    T = block_sparse_tensor(seed * 10 + 1, [occ, occ, vir, vir], 0.5)
    V = block_sparse_tensor(seed * 10 + 2, [vir, vir, vir, vir], 0.3)
    return occ, vir, T, V


def tensor_bits(present: np.ndarray) -> np.ndarray:
    """Block shape of a tensor in the library's word layout: bit q = the block with flattened
    (row-major) index q."""
    flat = np.asarray(present, dtype=bool).reshape(1, -1)
    return pack_bits(flat) if flat.size else np.zeros(0, np.uint64)


def _fill_blocks(seed: int, mat: int, mask: np.ndarray, rsz: np.ndarray, csz: np.ndarray,
                 draw) -> np.ndarray:
    """Concatenate the present blocks in row-major block order; draw(rng, i, j, h, w) -> values."""
    total = int(sum(int(rsz[i]) * int(csz[j]) for i, j in zip(*np.nonzero(mask))))
    out = np.empty(total, dtype=np.float64)
    pos = 0
    for i, j in zip(*np.nonzero(mask)):
        h, w = int(rsz[i]), int(csz[j])
        out[pos:pos + h * w] = draw(_rng(seed, _VALUES, mat, i, j), int(i), int(j), h, w).reshape(-1)
        pos += h * w
    return out


def block_values(p: Problem, seed: int, mat: int, i: int, j: int, draw) -> np.ndarray:
    """Regenerate one block on its own (same stream as the packed buffer)."""
    rsz, csz = (p.rows, p.inner) if mat == MAT_A else (p.inner, p.cols)
    return draw(_rng(seed, _VALUES, mat, i, j), i, j, int(rsz[i]), int(csz[j]))


def _normal(rng, i, j, h, w):
    return rng.standard_normal((h, w))


def _uniform_pm1(rng, i, j, h, w):
    return rng.uniform(-1.0, 1.0, (h, w))


def make_problem(name: str, seed: int, rows, inner, cols, a_mask, b_mask, draw=_normal,
                 b_is_a: bool = False) -> Problem:
    rows = np.asarray(rows, dtype=np.int64)
    inner = np.asarray(inner, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    a_mask = np.asarray(a_mask, dtype=bool)
    b_mask = np.asarray(b_mask, dtype=bool)
    a = _fill_blocks(seed, MAT_A, a_mask, rows, inner, draw)
    b = a if b_is_a else _fill_blocks(seed, MAT_B, b_mask, inner, cols, draw)
    return Problem(name, rows, inner, cols, a_mask, b_mask, a, b, b_is_a)


def random_problem(seed: int, M: int, K: int, N: int, lo: int, hi: int, pa: float, pb: float,
                   draw=_normal, name: str = "random") -> Problem:
    """Small random problem: M x K x N blocks with sizes U{lo..hi}, Bernoulli masks."""
    t = _rng(seed, _TILING)
    rows = t.integers(lo, hi + 1, M)
    inner = t.integers(lo, hi + 1, K)
    cols = t.integers(lo, hi + 1, N)
    s = _rng(seed, _SHAPE)
    a_mask = s.random((M, K)) < pa
    b_mask = s.random((K, N)) < pb
    return make_problem(name, seed, rows, inner, cols, a_mask, b_mask, draw)


def integer_problem(seed: int, M: int, K: int, N: int, lo: int, hi: int, pa: float, pb: float,
                    vmax: int = 8) -> Problem:
    """Random problem with integer values in [-vmax, vmax]: exact in bf16 and fp32, so every
    precision form must reproduce the FP64 result bit for bit while partial sums stay < 2^24."""
    def draw(rng, i, j, h, w):
        return rng.integers(-vmax, vmax + 1, (h, w)).astype(np.float64)
    return random_problem(seed, M, K, N, lo, hi, pa, pb, draw, name="integer")


# ---- the five workloads -----------------------------------------------------------------------
def uniform_1024(seed: int = 1000) -> Problem:
    rows = tiling_uniform(1024, 64)
    s = _rng(seed, _SHAPE)
    a_mask = s.random((16, 16)) < 0.5
    b_mask = s.random((16, 16)) < 0.5
    return make_problem("uniform_1024", seed, rows, rows, rows, a_mask, b_mask, _uniform_pm1)


def nonuniform(seed: int, n: int, lo: int, hi: int, density: float, draw=_normal,
               name: Optional[str] = None) -> Problem:
    rows = tiling_random(n, lo, hi, _rng(seed, _TILING, 0))
    inner = tiling_random(n, lo, hi, _rng(seed, _TILING, 1))
    cols = tiling_random(n, lo, hi, _rng(seed, _TILING, 2))
    s = _rng(seed, _SHAPE)
    a_mask = s.random((rows.size, inner.size)) < density
    b_mask = s.random((inner.size, cols.size)) < density
    return make_problem(name or f"nonuniform_{n}", seed, rows, inner, cols, a_mask, b_mask, draw)


def nonuniform_16384(seed: int = 2000) -> Problem:
    return nonuniform(seed, 16384, 32, 256, 0.3, name="nonuniform_16384")


def batch64(seed: int = 3000, count: int = 64, sizes: Sequence[int] = (1024, 2048, 4096, 8192)) -> List[Problem]:
    out = []
    for b in range(count):
        ps = seed * 1000 + b
        c = _rng(ps, _SHAPE, 99)
        n = int(sizes[int(c.integers(0, len(sizes)))])
        dens = float(c.uniform(0.1, 0.9))
        out.append(nonuniform(ps, n, 16, 192, dens, name=f"batch{b}_{n}_{dens:.2f}"))
    return out


def _scaled_normal(seed: int):
    def draw(rng, i, j, h, w):
        # one continuous factor 10^U(-4,0) per block, drawn from the block's own stream
        f = 10.0 ** rng.uniform(-4.0, 0.0)
        return rng.standard_normal((h, w)) * f
    return draw


def precision_32768(seed: int = 4000, n: int = 32768) -> Problem:
    return nonuniform(seed, n, 64, 256, 0.4, draw=_scaled_normal(seed), name=f"precision_{n}")


def decay_cloud(seed: int = 5000, npts: int = 4000, box: float = 60.0,
                sizes: Sequence[int] = (10, 25, 40, 60), cutoff: float = 1e-8,
                threads: Optional[int] = None) -> Problem:
    """Distance-decay structure: points uniform in a cube, a block size per point; block (i, j)
    is present iff exp(-r_ij / 2) > cutoff, with values N(0,1) * exp(-r_ij / 2); C = A * A.

    At the full size (4000 points, 63 GB of values) one stream per block *row* is used: row i's
    present blocks are drawn, in column order, from SeedSequence(seed, (VALUES, A, i)) in one call
    and each block is then scaled; rows are filled by a thread pool."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    p = _rng(seed, _POINTS)
    pts = p.uniform(0.0, box, (npts, 3))
    bs = np.asarray(sizes, dtype=np.int64)[p.integers(0, len(sizes), npts)]
    rmax = -2.0 * math.log(cutoff)
    mask = np.zeros((npts, npts), dtype=bool)
    for i0 in range(0, npts, 256):
        d = np.sqrt(((pts[i0:i0 + 256, None, :] - pts[None, :, :]) ** 2).sum(axis=2))
        mask[i0:i0 + 256] = d < rmax
    row_elems = bs * (mask.astype(np.int64) @ bs)
    off = np.concatenate([[0], np.cumsum(row_elems)])
    out = np.empty(int(off[-1]), dtype=np.float64)

    def fill(i):
        js = np.nonzero(mask[i])[0]
        seg = out[off[i]:off[i + 1]]
        _rng(seed, _VALUES, MAT_A, i).standard_normal(out=seg)
        r = np.sqrt(((pts[js] - pts[i]) ** 2).sum(axis=1))
        seg *= np.repeat(np.exp(-0.5 * r), bs[i] * bs[js])

    workers = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(fill, range(npts)))
    return Problem(f"decay_cloud_{npts}", bs, bs, bs, mask, mask, out, out, b_is_a=True)


def paper_dense(seed: int, n: int, block: int, nonuniform_blocks: bool) -> Problem:
    if nonuniform_blocks:
        nb = n // block
        rows = tiling_add_one(n, nb, _rng(seed, _TILING, 0))
        inner = tiling_add_one(n, nb, _rng(seed, _TILING, 1))
        cols = tiling_add_one(n, nb, _rng(seed, _TILING, 2))
    else:
        rows = inner = cols = tiling_uniform(n, block)
    a_mask = np.ones((rows.size, inner.size), dtype=bool)
    b_mask = np.ones((inner.size, cols.size), dtype=bool)
    return make_problem(f"paper_dense_{n}_{'nonuni' if nonuniform_blocks else 'uni'}", seed,
                        rows, inner, cols, a_mask, b_mask)
