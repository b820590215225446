"""Block-sparse tensor contraction on the GPU (permutation passes + the block-sparse product),
through the C ABI, against the oracle's contraction.

Gates: FP64 relative Frobenius error <= 1e-12 and every element inside 2 gamma_n |A||B| (n = the
contracted length); FP32 form 1e-5, split-bf16 1e-6; integer values bit-exact in every form."""
import sys

import numpy as np
import pytest

from oracle import contract as tc
from paper_1504_05046_amd import bsm, gen
from tests.helpers import higham_gamma, rel_fro

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = torch.device("cuda:0")
GATE = {bsm.FP64: 1e-12, bsm.FP32: 1e-5, bsm.BF16X3: 1e-6}

CASES = [
    ([0, 2], [2, 1], [0, 1]),
    ([0, 3, 2], [2, 1, 3], [1, 0]),
    ([0, 2, 3, 1], [3, 4, 2], [4, 0, 1]),
    ([0, 4], [4, 1, 2, 3], [0, 1, 2, 3]),
    ([2, 0, 4, 1], [3, 4, 2], [0, 3, 1]),
    ([0, 1, 2], [2, 1, 0], []),   # full contraction to a scalar
]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem(case, seed, lo=1, hi=40, density=0.6, draw=None):
    am, bm, cm = CASES[case]
    rng = np.random.default_rng(seed)
    til = {m: rng.integers(lo, hi + 1, int(rng.integers(1, 4))) for m in set(am) | set(bm)}
    pa, da = gen.block_sparse_tensor(seed + 1, [til[m] for m in am], density, draw)
    pb, db = gen.block_sparse_tensor(seed + 2, [til[m] for m in bm], density, draw)
    A = tc.Tensor(am, [til[m] for m in am], pa, da)
    B = tc.Tensor(bm, [til[m] for m in bm], pb, db)
    return A, B, cm, til


def run(A, B, cm, alpha=1.0, C0=None, out=bsm.OUT_F64, **kw):
    plan = bsm.Contraction((A.modes, A.tilings, gen.tensor_bits(A.present)),
                           (B.modes, B.tilings, gen.tensor_bits(B.present)), cm, out=out, **kw)
    info = plan.info()
    dt = torch.float32 if out == bsm.OUT_F32 else torch.float64
    dA = torch.from_numpy(A.data).to(DEV)
    dB = torch.from_numpy(B.data).to(DEV)
    dC = (torch.full((max(1, info.c_elems),), float("nan"), dtype=dt, device=DEV) if C0 is None
          else torch.from_numpy(C0.astype(np.float32 if out == bsm.OUT_F32 else np.float64)).to(DEV))
    plan.execute(dA, dB, dC, alpha=alpha, accumulate=C0 is not None)
    torch.cuda.synchronize()
    plan.verify()
    return dC.cpu().numpy()[:info.c_elems], plan


def check(A, B, cm, til, precision=bsm.FP64, alpha=1.0, C0=None, **kw):
    _say(f"[contract] A{A.modes} B{B.modes} -> C{cm} precision={precision} {kw}")
    got, plan = run(A, B, cm, alpha=alpha, C0=C0, precision=precision, **kw)
    shape, ref = tc.contract(A, B, cm, alpha=alpha,
                             C=None if C0 is None else (None, C0))
    assert np.array_equal(plan.c_shape()[:max(1, (shape.size + 63) // 64)], gen.tensor_bits(shape))
    assert got.shape == ref.shape and np.all(np.isfinite(got))
    assert rel_fro(got, ref) <= GATE[precision]
    if precision == bsm.FP64:
        absA = tc.Tensor(A.modes, A.tilings, A.present, np.abs(A.data))
        absB = tc.Tensor(B.modes, B.tilings, B.present, np.abs(B.data))
        _, absab = tc.contract(absA, absB, cm, alpha=abs(alpha))
        n = int(np.prod([til[m].sum() for m in A.modes if m in B.modes and m not in cm]))
        assert np.all(np.abs(got - ref) <= 2 * higham_gamma(max(n, 1)) * absab + 1e-300)
    return got, ref, plan


@pytest.mark.parametrize("case", range(len(CASES)))
def test_contractions_fp64(case):
    A, B, cm, til = _problem(case, 8000 + 10 * case)
    check(A, B, cm, til, alpha=-0.5)


@pytest.mark.parametrize("precision", [bsm.FP32, bsm.BF16X3])
def test_contraction_precision_forms(precision):
    A, B, cm, til = _problem(2, 8100 + precision)
    check(A, B, cm, til, precision=precision)


def test_contraction_integer_values_bit_exact_and_fp32_output():
    draw = lambda g, shape: g.integers(-5, 6, shape).astype(float)
    A, B, cm, til = _problem(4, 8200, hi=24, draw=draw)
    for precision in (bsm.FP64, bsm.FP32, bsm.BF16X3):
        got, ref, _ = check(A, B, cm, til, precision=precision)
        assert np.array_equal(got, ref)
    # FP32 C through the permutation pass, accumulating
    _, ref = tc.contract(A, B, cm, alpha=2.0)
    C0 = np.random.default_rng(3).integers(-50, 50, ref.size).astype(np.float32)
    got, _ = run(A, B, cm, alpha=2.0, C0=C0, out=bsm.OUT_F32)
    assert got.dtype == np.float32 and np.array_equal(got, (ref + C0).astype(np.float32))


def test_contraction_accumulate_graph_and_windows():
    A, B, cm, til = _problem(1, 8300)
    _, ref = tc.contract(A, B, cm)
    C0 = np.random.default_rng(4).standard_normal(ref.size)
    outs = [check(A, B, cm, til, alpha=1.5, C0=C0, **kw)[0]
            for kw in ({}, {"use_graph": 1}, {"k_window": 2})]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_contraction_empty_operand():
    am, bm, cm = CASES[1]
    til = {0: np.array([3, 4]), 1: np.array([5]), 2: np.array([2, 2]), 3: np.array([6])}
    A = tc.Tensor(am, [til[m] for m in am], np.zeros((2, 1, 2), bool), np.zeros(0))
    pb, db = gen.block_sparse_tensor(5, [til[m] for m in bm], 1.0)
    B = tc.Tensor(bm, [til[m] for m in bm], pb, db)
    got, plan = run(A, B, cm)
    assert plan.info().c_elems == 0


def test_ladder_contraction_sampled():
    """The coupled-cluster ladder shape the benchmark times (T[i,j,c,d] V[a,b,c,d] -> C[i,j,a,b],
    V permuted into matrix order): sampled C blocks against the oracle."""
    occ, vir, (pt, dt_), (pv, dv) = gen.ladder_tensors()
    T = tc.Tensor([0, 1, 2, 3], [occ, occ, vir, vir], pt, dt_)
    V = tc.Tensor([4, 5, 2, 3], [vir, vir, vir, vir], pv, dv)
    cm = [0, 1, 4, 5]
    _say(f"[ladder] T blocks {int(pt.sum())}, V blocks {int(pv.sum())}")
    got, plan = run(T, V, cm)
    info = plan.info()
    assert (info.permute_a, info.permute_b, info.permute_c) == (0, 1, 0)
    cshape = gen.unpack_bits(plan.c_shape(), 1, len(occ) ** 2 * len(vir) ** 2).reshape(
        len(occ), len(occ), len(vir), len(vir))
    present = [tuple(int(v) for v in idx) for idx in zip(*np.nonzero(cshape))]
    sizes = [int(occ[i] * occ[j] * vir[a] * vir[b]) for i, j, a, b in present]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    rng = np.random.default_rng(17)
    pick = rng.choice(len(present), 12, replace=False)
    blocks = tc.contract_blocks(T, V, cm, [present[q] for q in pick])
    num = den = 0.0
    for q, blk in zip(pick, blocks):
        assert blk is not None
        g = got[offs[q]:offs[q + 1]].reshape(blk.shape)
        num += float(np.sum((g - blk) ** 2))
        den += float(np.sum(blk ** 2))
    assert (num / den) ** 0.5 <= 1e-12
