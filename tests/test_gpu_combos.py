"""Option combinations on one ragged product, against the oracle: precision form x element type x
transposed/adjoint operands x reduction variant x k-windows x output type x accumulation.  Each
feature is tested on its own elsewhere; this file checks that they compose.

Gates: relative Frobenius error (over real and imaginary parts for complex elements) <= 1e-12 for
FP64, 1e-5 for FP32, 1e-6 for split-bf16, plus the FP32 rounding of C (2^-24 relative) for FP32
output."""
import itertools
import sys

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import bsm, gen
from tests.helpers import rel_fro

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = torch.device("cuda:0")
GATE = {bsm.FP64: 1e-12, bsm.FP32: 1e-5, bsm.BF16X3: 1e-6}
OPS = ("N", "T", "C")


def _problem():
    rng = np.random.default_rng(12000)
    sizes = np.array([3, 17, 40, 64, 65, 130])
    rows, inner, cols = rng.permutation(sizes), rng.permutation(sizes), rng.permutation(sizes)[:4]
    a_mask = rng.random((6, 6)) < 0.6
    b_mask = rng.random((6, 4)) < 0.6
    a_mask[0, 0] = b_mask[0, 0] = True
    return gen.make_problem("combo", 12000, rows, inner, cols, a_mask, b_mask)


P = _problem()
ZA, ZB = gen.imag_parts(P, 12001)

CASES = []
for precision, cplx, (oa, ob), ks, kw, out, acc in itertools.product(
        (bsm.FP64, bsm.FP32, bsm.BF16X3), (False, True), (("N", "N"), ("T", "N"), ("N", "C"), ("C", "T")),
        (0, 3), (0, 2), (bsm.OUT_F64, bsm.OUT_F32), (False, True)):
    if ks and kw:
        continue                      # the reduction variant needs all k-iterations at once
    if not cplx and "C" in (oa, ob):
        oa, ob = oa.replace("C", "T"), ob.replace("C", "T")
    CASES.append((precision, cplx, oa, ob, ks, kw, out, acc))
# keep the suite quick: every precision x element x ops pair, with the other options rotated
_seen, SELECTED = set(), []
for n, c in enumerate(CASES):
    key = c[:4] + (n % 5,)
    if key[:4] not in _seen or n % 7 == 0:
        _seen.add(key[:4])
        SELECTED.append(c)


def _stored(x, op, rsz, csz, mask):
    if op == "N":
        return gen.pack_bits(mask), x
    return gen.stored_transpose(rsz, csz, mask, x if op == "T" else x.conj())


@pytest.mark.parametrize("precision,cplx,oa,ob,ks,kw,out,acc", SELECTED)
def test_combination(precision, cplx, oa, ob, ks, kw, out, acc):
    print(f"[combo] precision={precision} complex={cplx} op=({oa},{ob}) k_split={ks} "
          f"k_window={kw} out={out} accumulate={acc}", flush=True)
    sys.stdout.flush()
    p = P
    a = ZA if cplx else P.a_data
    b = ZB if cplx else P.b_data
    a_bits, a_st = _stored(a, oa, p.rows, p.inner, p.a_mask)
    b_bits, b_st = _stored(b, ob, p.inner, p.cols, p.b_mask)
    tr = {"N": 0, "T": 1, "C": 2}
    plan = bsm.Plan(p.rows, p.inner, p.cols, a_bits, b_bits, precision=precision,
                    elem=bsm.COMPLEX if cplx else bsm.REAL, trans_a=tr[oa], trans_b=tr[ob],
                    k_split=ks, k_window=kw, out=out)
    info = plan.info()
    alpha = (0.75 - 0.5j) if cplx else -0.75
    n = info.c_elems
    rng = np.random.default_rng(5)
    C0 = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    if cplx:
        ref = oracle.zbsmm(p.rows, p.inner, p.cols, a_bits, b_bits, a_st, b_st, alpha,
                           C=C0 if acc else None, op_a=oa, op_b=ob)
        dt = torch.complex64 if out == bsm.OUT_F32 else torch.complex128
    else:
        ref = oracle.bsmm(p.rows, p.inner, p.cols, a_bits, b_bits, a_st, b_st, alpha,
                          C=C0 if acc else None, trans_a=oa != "N", trans_b=ob != "N")
        dt = torch.float32 if out == bsm.OUT_F32 else torch.float64
    A = torch.from_numpy(np.ascontiguousarray(a_st)).to(DEV)
    B = torch.from_numpy(np.ascontiguousarray(b_st)).to(DEV)
    if acc:
        C = torch.from_numpy(C0).to(dt).to(DEV)
    else:
        C = torch.full((max(1, n),), float("nan"), dtype=dt, device=DEV)
    plan.execute(A, B, C, alpha=alpha, accumulate=acc)
    torch.cuda.synchronize()
    plan.verify()
    got = C.cpu().numpy()[:n].astype(np.complex128 if cplx else np.float64)
    assert np.all(np.isfinite(got))
    g = np.concatenate([got.real, got.imag]) if cplx else got
    r = np.concatenate([ref.real, ref.imag]) if cplx else ref
    tol = GATE[precision] + (2.0 ** -24 if out == bsm.OUT_F32 else 0.0) * 2
    if acc and out == bsm.OUT_F32:
        tol += 2.0 ** -23   # the previous C itself was rounded to FP32 on the way in
    assert rel_fro(g, r) <= tol
    plan.close()
