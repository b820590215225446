"""Transposed operands C = alpha op(A) op(B) on the GPU, through the C ABI, against the oracle
(which reads the stored transposed blocks itself).

Gates: the same as for the untransposed product in each form (FP64: relative Frobenius error
<= 1e-12 and every element inside twice the Higham bound; FP32: 1e-5; split-bf16: 1e-6), plus:
the transposition is pure data movement, so a transposed product gives exactly the bits of the
same product handed over untransposed."""
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
TRANS = [(1, 0), (0, 1), (1, 1)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def stored(p: gen.Problem, ta: int, tb: int):
    """(a_bits, a_data, b_bits, b_data) as the caller hands them over for op(A) op(B)."""
    a_bits, a_data = (gen.stored_transpose(p.rows, p.inner, p.a_mask, p.a_data) if ta
                      else (p.a_bits(), p.a_data))
    b_bits, b_data = (gen.stored_transpose(p.inner, p.cols, p.b_mask, p.b_data) if tb
                      else (p.b_bits(), p.b_data))
    return a_bits, a_data, b_bits, b_data


def run(p, a_bits, a_data, b_bits, b_data, alpha=1.0, C0=None, static=False, alias=False, **kw):
    plan = bsm.Plan(p.rows, p.inner, p.cols, a_bits, b_bits, **kw)
    info = plan.info()
    A = torch.from_numpy(a_data).to(DEV)
    B = A if alias else torch.from_numpy(b_data).to(DEV)
    C = (torch.full((max(1, info.c_elems),), float("nan"), dtype=torch.float64, device=DEV)
         if C0 is None else torch.from_numpy(C0.copy()).to(DEV))
    (plan.execute_static if static else plan.execute)(A, B, C, alpha=alpha,
                                                       accumulate=C0 is not None)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:info.c_elems], plan


def check(p, ta, tb, precision, alpha=1.0, **kw):
    _say(f"[trans] {p.name} M={p.M} K={p.K} N={p.N} ta={ta} tb={tb} precision={precision} {kw}")
    a_bits, a_data, b_bits, b_data = stored(p, ta, tb)
    got, plan = run(p, a_bits, a_data, b_bits, b_data, alpha=alpha, precision=precision,
                    trans_a=ta, trans_b=tb, **kw)
    plan.verify()
    ref = oracle.bsmm(p.rows, p.inner, p.cols, a_bits, b_bits, a_data, b_data, alpha,
                      trans_a=bool(ta), trans_b=bool(tb))
    assert got.shape == ref.shape and np.all(np.isfinite(got))
    err = rel_fro(got, ref)
    assert err <= GATE[precision], err
    if precision == bsm.FP64:
        absab = oracle.bsmm(p.rows, p.inner, p.cols, a_bits, b_bits, np.abs(a_data),
                            np.abs(b_data), abs(alpha), trans_a=bool(ta), trans_b=bool(tb))
        assert np.all(np.abs(got - ref) <= 2 * higham_gamma(int(p.inner.sum())) * absab + 1e-300)
    # the same product handed over untransposed: the same bits
    plain, _ = run(p, p.a_bits(), p.a_data, p.b_bits(), p.b_data, alpha=alpha,
                   precision=precision, **kw)
    assert np.array_equal(got, plain)
    return got


def _ragged(seed):
    rng = np.random.default_rng(seed)
    sizes = np.array([1, 17, 33, 64, 65, 129, 200])
    rows, inner, cols = rng.permutation(sizes), rng.permutation(sizes), rng.permutation(sizes)[:5]
    a_mask = rng.random((7, 7)) < 0.6
    b_mask = rng.random((7, 5)) < 0.6
    a_mask[0, 0] = b_mask[0, 0] = True
    return gen.make_problem(f"ragged{seed}", seed, rows, inner, cols, a_mask, b_mask)


@pytest.mark.parametrize("ta,tb", TRANS)
@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32, bsm.BF16X3])
def test_transposed_ragged(precision, ta, tb):
    check(_ragged(3100 + 4 * precision + 2 * ta + tb), ta, tb, precision, alpha=-1.25)


@pytest.mark.parametrize("ta,tb", TRANS)
def test_transposed_integer_inputs_bit_exact(ta, tb):
    p = gen.integer_problem(3200 + 2 * ta + tb, 6, 7, 5, 1, 200, 0.6, 0.6)
    for precision in (bsm.FP64, bsm.FP32, bsm.BF16X3):
        got = check(p, ta, tb, precision)
        a_bits, a_data, b_bits, b_data = stored(p, ta, tb)
        assert np.array_equal(got, oracle.bsmm(p.rows, p.inner, p.cols, a_bits, b_bits, a_data,
                                               b_data, trans_a=bool(ta), trans_b=bool(tb)))


@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32, bsm.BF16X3])
def test_gram_products_from_one_buffer(precision):
    """X^T X and X X^T with both operands the same device buffer X (3 x 5 blocks): the Gram
    products of Sec. 2.1's transposed variants; the FP32 form must not share one converted copy
    between the transposed and the plain operand."""
    rng = np.random.default_rng(33)
    xr, xc = np.array([40, 7, 90]), np.array([16, 130, 1, 65, 33])
    mask = rng.random((3, 5)) < 0.7
    mask[:, 0] = True
    x = gen.make_problem("X", 34, xr, xc, xc, mask, np.ones((5, 5), bool))
    X, xbits = x.a_data, x.a_bits()
    for ta, tb, rows, inner, cols in ((1, 0, xc, xr, xc), (0, 1, xr, xc, xr)):
        _say(f"[gram] ta={ta} tb={tb} precision={precision}")
        p = gen.Problem("gram", rows, inner, cols, np.zeros((len(rows), len(inner)), bool),
                        np.zeros((len(inner), len(cols)), bool), X, X)
        got, plan = run(p, xbits, X, xbits, X, alias=True, precision=precision, trans_a=ta,
                        trans_b=tb)
        plan.verify()
        ref = oracle.bsmm(rows, inner, cols, xbits, xbits, X, X, trans_a=bool(ta),
                          trans_b=bool(tb))
        assert rel_fro(got, ref) <= GATE[precision]
        # symmetric result: C = C^T blockwise (the kernel's sums run in the same order for (i, j)
        # and (j, i) only up to rounding, so compare to the gate)
        cm = gen.unpack_bits(plan.c_shape(), len(rows), len(cols))
        assert np.array_equal(cm, cm.T)


@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32])
def test_transposed_static_entry_point(precision):
    """The allocation-free entry point stages a transposed operand in its static scratch."""
    p = _ragged(3300 + precision)
    a_bits, a_data, b_bits, b_data = stored(p, 1, 1)
    got, _ = run(p, a_bits, a_data, b_bits, b_data, static=True, precision=precision, trans_a=1,
                 trans_b=1)
    want, _ = run(p, a_bits, a_data, b_bits, b_data, precision=precision, trans_a=1, trans_b=1)
    assert np.array_equal(got, want)


def test_transposed_accumulate_windows_and_device_klists():
    p = _ragged(3400)
    a_bits, a_data, b_bits, b_data = stored(p, 0, 1)
    C0 = np.random.default_rng(5).standard_normal(
        oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data).size)
    ref = oracle.bsmm(p.rows, p.inner, p.cols, a_bits, b_bits, a_data, b_data, 0.5, C=C0,
                      trans_b=True)
    outs = []
    for kw in ({}, {"k_window": 2}, {"device_klists": 1}):
        got, plan = run(p, a_bits, a_data, b_bits, b_data, alpha=0.5, C0=C0, trans_b=1, **kw)
        plan.verify()
        assert rel_fro(got, ref) <= 1e-12
        outs.append(got)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_transposed_members_in_a_batch():
    """A batch of a transposed and a plain product: each member stages its own operands."""
    p1, p2 = _ragged(3500), _ragged(3501)
    s1 = stored(p1, 1, 0)
    plans = [bsm.Plan(p1.rows, p1.inner, p1.cols, s1[0], s1[2], trans_a=1),
             bsm.Plan.from_problem(p2)]
    batch = bsm.Batch(plans)
    As = [torch.from_numpy(s1[1]).to(DEV), torch.from_numpy(p2.a_data).to(DEV)]
    Bs = [torch.from_numpy(s1[3]).to(DEV), torch.from_numpy(p2.b_data).to(DEV)]
    Cs = [torch.zeros(max(1, pl.info().c_elems), dtype=torch.float64, device=DEV) for pl in plans]
    batch.execute(As, Bs, Cs, alphas=[2.0, -1.0])
    batch.verify()
    torch.cuda.synchronize()
    r1 = oracle.bsmm(p1.rows, p1.inner, p1.cols, s1[0], s1[2], s1[1], s1[3], 2.0, trans_a=True)
    r2 = oracle.bsmm(p2.rows, p2.inner, p2.cols, p2.a_bits(), p2.b_bits(), p2.a_data, p2.b_data,
                     -1.0)
    assert rel_fro(Cs[0].cpu().numpy()[:r1.size], r1) <= 1e-12
    assert rel_fro(Cs[1].cpu().numpy()[:r2.size], r2) <= 1e-12


def test_transposed_empty_and_degenerate():
    """No present blocks in the stored A^T, and an empty inner dimension: C is empty, no fault."""
    p = gen.make_problem("emptyA", 1, [5, 9], [3, 4, 2], [7], np.zeros((2, 3), bool),
                         np.ones((3, 1), bool))
    a_bits, a_data, b_bits, b_data = stored(p, 1, 1)
    got, plan = run(p, a_bits, a_data, b_bits, b_data, trans_a=1, trans_b=1)
    assert plan.info().c_elems == 0 and plan.info().tasks == 0
    q = gen.make_problem("noK", 2, [5, 9], [], [7, 3], np.zeros((2, 0), bool),
                         np.zeros((0, 2), bool))
    a_bits, a_data, b_bits, b_data = stored(q, 1, 0)
    got, plan = run(q, a_bits, a_data, b_bits, b_data, trans_a=1)
    assert plan.info().c_elems == 0


def test_nonuniform_16384_transposed_b_sampled():
    """The 16384-row nonuniform workload with B handed over transposed, in the launch setup the
    benchmark times: sampled C blocks against the oracle, and the whole C against the untransposed
    run bit for bit."""
    p = gen.nonuniform_16384()
    _say(f"[trans 16384] M={p.M} K={p.K} N={p.N}")
    b_bits, b_data = gen.stored_transpose(p.inner, p.cols, p.b_mask, p.b_data)
    got, plan = run(p, p.a_bits(), p.a_data, b_bits, b_data, trans_b=1)
    plan.verify()
    plain, _ = run(p, p.a_bits(), p.a_data, p.b_bits(), p.b_data)
    assert np.array_equal(got, plain)
    off = plan.c_offsets()
    present = np.argwhere(off >= 0)
    rng = np.random.default_rng(9)
    sel = [tuple(int(v) for v in present[q]) for q in rng.choice(len(present), 24, replace=False)]
    blocks, pres = oracle.bsmm_blocks(p.rows, p.inner, p.cols, p.a_bits(), b_bits, p.a_data,
                                      b_data, sel, trans_b=True)
    num = den = 0.0
    for (i, j), blk, pr in zip(sel, blocks, pres):
        assert pr
        o = int(off[i, j])
        g = got[o:o + blk.size].reshape(blk.shape)
        num += float(np.sum((g - blk) ** 2))
        den += float(np.sum(blk ** 2))
    assert (num / den) ** 0.5 <= 1e-12
