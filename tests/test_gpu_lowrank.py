"""Block-rank-sparse A (factored blocks U V^T) on the GPU, through the C ABI, against the oracle
(which multiplies the factors out and takes the ordinary product).

Gates: FP64 relative Frobenius error <= 1e-12 and every element inside 4 gamma_{n + rho_max}
(|U||V|^T)|B| (the GPU sums V^T B first, the oracle U V^T first); FP32 form 1e-5, split-bf16 1e-6;
integer factors bit-exact; all-dense ranks give the ordinary plan's bits."""
import sys

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import bsm, gen
from tests.helpers import higham_gamma, rel_fro

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = torch.device("cuda:0")
GATE = {bsm.FP64: 1e-12, bsm.FP32: 1e-5, bsm.BF16X3: 1e-6}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(p, ranks, data, alpha=1.0, C0=None, **kw):
    plan = bsm.LowRankPlan(p.rows, p.inner, p.cols, p.a_bits(), ranks, p.b_bits(), **kw)
    info = plan.info()
    A = torch.from_numpy(data).to(DEV)
    B = torch.from_numpy(p.b_data).to(DEV)
    C = (torch.full((max(1, info.c_elems),), float("nan"), dtype=torch.float64, device=DEV)
         if C0 is None else torch.from_numpy(C0.copy()).to(DEV))
    plan.execute(A, B, C, alpha=alpha, accumulate=C0 is not None)
    torch.cuda.synchronize()
    plan.verify()
    return C.cpu().numpy()[:info.c_elems], plan


def reference(p, ranks, data, alpha=1.0, C0=None):
    dense = oracle.lr_expand(p.rows, p.inner, p.a_bits(), ranks, data)
    return oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), dense, p.b_data, alpha, C=C0)


def check(p, ranks, data, precision=bsm.FP64, alpha=1.0, C0=None, **kw):
    _say(f"[lowrank] {p.name} M={p.M} K={p.K} N={p.N} factored={int((ranks > 0).sum())} "
         f"precision={precision} {kw}")
    got, plan = run(p, ranks, data, alpha=alpha, C0=C0, precision=precision, **kw)
    ref = reference(p, ranks, data, alpha, C0)
    assert got.shape == ref.shape and np.all(np.isfinite(got))
    assert rel_fro(got, ref) <= GATE[precision]
    if precision == bsm.FP64:
        absA = oracle.lr_expand(p.rows, p.inner, p.a_bits(), ranks, np.abs(data))
        absab = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), absA,
                            np.abs(p.b_data), abs(alpha))
        n = int(p.inner.sum()) + int(max(ranks.max(initial=0), 1))
        assert np.all(np.abs(got - ref) <= 4 * higham_gamma(n) * absab + 1e-300)
    return got, ref, plan


def _ragged(seed):
    rng = np.random.default_rng(seed)
    sizes = np.array([1, 17, 33, 64, 65, 129, 200])
    rows, inner, cols = rng.permutation(sizes), rng.permutation(sizes), rng.permutation(sizes)[:5]
    a_mask = rng.random((7, 7)) < 0.7
    b_mask = rng.random((7, 5)) < 0.6
    a_mask[0, 0] = b_mask[0, 0] = True
    return gen.make_problem(f"lrragged{seed}", seed, rows, inner, cols, a_mask, b_mask)


@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32, bsm.BF16X3])
def test_low_rank_mixed_ranks(precision):
    """Dense and factored blocks mixed, ranks 1..20 (some above a block's own size)."""
    p = _ragged(6100 + precision)
    ranks, data = gen.low_rank_operand(p, 6101, lambda i, k, h, d: 0 if (i + k) % 3 == 0 else 1 + (i * 7 + k) % 20)
    check(p, ranks, data, precision, alpha=-0.75)


def test_low_rank_integer_factors_bit_exact():
    p = gen.integer_problem(6200, 6, 7, 5, 1, 120, 0.7, 0.6)
    draw = lambda g, i, k, h, w: g.integers(-3, 4, (h, w)).astype(float)
    ranks, data = gen.low_rank_operand(p, 6201, lambda i, k, h, d: (i + 2 * k) % 5, draw=draw)
    for precision in (bsm.FP64, bsm.FP32, bsm.BF16X3):
        got, ref, _ = check(p, ranks, data, precision)
        assert np.array_equal(got, ref)


def test_low_rank_all_dense_is_the_ordinary_product():
    p = _ragged(6300)
    ranks = np.zeros(int(p.a_mask.sum()), np.int32)
    got, _ = run(p, ranks, p.a_data)
    plan = bsm.Plan.from_problem(p)
    C = torch.zeros(plan.info().c_elems, dtype=torch.float64, device=DEV)
    plan.execute(torch.from_numpy(p.a_data).to(DEV), torch.from_numpy(p.b_data).to(DEV), C)
    assert np.array_equal(got, C.cpu().numpy())


def test_low_rank_all_factored_accumulate_and_windows():
    p = _ragged(6400)
    ranks, data = gen.low_rank_operand(p, 6401, lambda i, k, h, d: 1 + (i + k) % 8)
    C0 = np.random.default_rng(3).standard_normal(reference(p, ranks, data).size)
    outs = []
    for kw in ({}, {"k_window": 2}, {"use_graph": 1}):
        got, _, _ = check(p, ranks, data, alpha=1.5, C0=C0, **kw)
        outs.append(got)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_low_rank_empty_and_degenerate():
    """No factored block, no present A block, an empty inner dimension: no fault, empty or
    ordinary results."""
    p = gen.make_problem("emptyA", 1, [5, 9], [3, 4], [7], np.zeros((2, 2), bool),
                         np.ones((2, 1), bool))
    got, plan = run(p, np.zeros(0, np.int32), p.a_data)
    assert plan.info().c_elems == 0
    q = gen.make_problem("one", 2, [5], [3], [7], np.ones((1, 1), bool), np.zeros((1, 1), bool))
    ranks, data = gen.low_rank_operand(q, 3, lambda i, k, h, d: 2)
    got, plan = run(q, ranks, data)
    assert plan.info().c_elems == 0


def test_block_rank_8192_sampled():
    """The block-rank-sparse workload the benchmark times (N=8192, band of dense blocks, ranks
    4..16 elsewhere): sampled C blocks against the oracle."""
    p, ranks, data = gen.block_rank_8192()
    _say(f"[lowrank 8192] factored {int((ranks > 0).sum())} of {ranks.size}")
    got, plan = run(p, ranks, data)
    dense = oracle.lr_expand(p.rows, p.inner, p.a_bits(), ranks, data)
    off = plan.c_offsets()
    present = np.argwhere(off >= 0)
    rng = np.random.default_rng(13)
    sel = [tuple(int(v) for v in present[q]) for q in rng.choice(len(present), 24, replace=False)]
    blocks, pres = oracle.bsmm_blocks(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), dense,
                                      p.b_data, sel)
    num = den = 0.0
    for (i, j), blk, pr in zip(sel, blocks, pres):
        assert pr
        g = got[int(off[i, j]):int(off[i, j]) + blk.size].reshape(blk.shape)
        num += float(np.sum((g - blk) ** 2))
        den += float(np.sum(blk ** 2))
    assert (num / den) ** 0.5 <= 1e-12
