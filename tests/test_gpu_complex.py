"""Complex elements on the GPU (the real embedding of the operands, the real tile kernels, the
complex epilogue), through the C ABI, against the complex oracle.

Gates: FP64 relative Frobenius error <= 1e-12 and every real and imaginary part inside
4 gamma_{2n+4} (|alpha| (|A|_1 |B|_1) + |C0|_1) with |X|_1 = |Re X| + |Im X| (each part of a C
element is a real dot product of length 2n); FP32 form 1e-5; split-bf16 form 1e-6; Gaussian-integer
inputs bit-exact in every form."""
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
OPS = {"N": 0, "T": 1, "C": 2}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _stored(rsz, csz, mask, z, op):
    """(bits, packed complex data) of an operand the product reads as op(X) = z's matrix under op."""
    if op == "N":
        return gen.pack_bits(mask), z
    return gen.stored_transpose(rsz, csz, mask, z if op == "T" else z.conj())


def run(p, a_bits, za, b_bits, zb, alpha=1.0, C0=None, alias=False, out=bsm.OUT_F64, **kw):
    plan = bsm.Plan(p.rows, p.inner, p.cols, a_bits, b_bits, elem=bsm.COMPLEX, out=out, **kw)
    info = plan.info()
    assert info.elem == bsm.COMPLEX
    ct = torch.complex64 if out == bsm.OUT_F32 else torch.complex128
    A = torch.from_numpy(np.ascontiguousarray(za)).to(DEV)
    B = A if alias else torch.from_numpy(np.ascontiguousarray(zb)).to(DEV)
    C = (torch.full((max(1, info.c_elems),), complex("nan+nanj"), dtype=ct, device=DEV)
         if C0 is None else torch.from_numpy(C0.astype(np.complex64 if out == bsm.OUT_F32
                                                       else np.complex128)).to(DEV))
    plan.execute(A, B, C, alpha=alpha, accumulate=C0 is not None)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:info.c_elems], plan


def _bound(p, a_bits, za, b_bits, zb, alpha, C0, oa, ob):
    mag = lambda z: np.abs(z.real) + np.abs(z.imag)
    ab = oracle.bsmm(p.rows, p.inner, p.cols, a_bits, b_bits, mag(za), mag(zb),
                     trans_a=oa != "N", trans_b=ob != "N")
    extra = mag(C0) if C0 is not None else 0.0
    return 4 * higham_gamma(2 * int(p.inner.sum()) + 4) * (abs(alpha) * ab + extra) + 1e-300


def check(p, za, zb, oa="N", ob="N", precision=bsm.FP64, alpha=1.0, C0=None, **kw):
    _say(f"[complex] {p.name} M={p.M} K={p.K} N={p.N} op=({oa},{ob}) precision={precision} {kw}")
    a_bits, a_st = _stored(p.rows, p.inner, p.a_mask, za, oa)
    b_bits, b_st = _stored(p.inner, p.cols, p.b_mask, zb, ob)
    got, plan = run(p, a_bits, a_st, b_bits, b_st, alpha=alpha, C0=C0, precision=precision,
                    trans_a=OPS[oa], trans_b=OPS[ob], **kw)
    plan.verify()
    ref = oracle.zbsmm(p.rows, p.inner, p.cols, a_bits, b_bits, a_st, b_st, alpha, C=C0,
                       op_a=oa, op_b=ob)
    assert got.shape == ref.shape and np.all(np.isfinite(got))
    assert rel_fro(np.concatenate([got.real, got.imag]),
                   np.concatenate([ref.real, ref.imag])) <= GATE[precision]
    if precision == bsm.FP64:
        bound = _bound(p, a_bits, a_st, b_bits, b_st, alpha, C0, oa, ob)
        assert np.all(np.abs(got.real - ref.real) <= bound)
        assert np.all(np.abs(got.imag - ref.imag) <= bound)
    return got, ref


def _ragged(seed, lo=1):
    rng = np.random.default_rng(seed)
    sizes = np.array([lo, 17, 33, 64, 65, 129, 200])
    rows, inner, cols = rng.permutation(sizes), rng.permutation(sizes), rng.permutation(sizes)[:5]
    a_mask = rng.random((7, 7)) < 0.6
    b_mask = rng.random((7, 5)) < 0.6
    a_mask[0, 0] = b_mask[0, 0] = True
    return gen.make_problem(f"zragged{seed}", seed, rows, inner, cols, a_mask, b_mask)


@pytest.mark.parametrize("oa,ob", [("N", "N"), ("T", "N"), ("N", "C"), ("C", "T"), ("C", "C")])
def test_complex_ragged_ops(oa, ob):
    p = _ragged(5100 + 3 * OPS[oa] + OPS[ob])
    za, zb = gen.imag_parts(p, 5101)
    C0 = None
    if (oa, ob) == ("C", "T"):
        n = oracle.zbsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), za, zb).size
        C0 = np.random.default_rng(2).standard_normal(n) + 1j * np.random.default_rng(3).standard_normal(n)
    check(p, za, zb, oa, ob, alpha=0.5 - 2.0j, C0=C0)


@pytest.mark.parametrize("precision", [bsm.FP32, bsm.BF16X3])
def test_complex_precision_forms(precision):
    p = gen.random_problem(5200 + precision, 6, 7, 5, 1, 200, 0.5, 0.5)
    za, zb = gen.imag_parts(p, 5201)
    check(p, za, zb, "N", "C", precision=precision, alpha=1j)


@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32, bsm.BF16X3])
def test_complex_gaussian_integers_bit_exact(precision):
    """Gaussian integers in [-8, 8] + i[-8, 8]: exact in every form (sums stay below 2^24)."""
    p = gen.integer_problem(5300 + precision, 5, 6, 5, 1, 120, 0.6, 0.6)
    rng = np.random.default_rng(5301)
    za = p.a_data + 1j * rng.integers(-8, 9, p.a_data.size)
    zb = p.b_data + 1j * rng.integers(-8, 9, p.b_data.size)
    for oa, ob in (("N", "N"), ("C", "T")):
        got, ref = check(p, za, zb, oa, ob, precision=precision, alpha=-1j)
        assert np.array_equal(got, ref)


def test_complex_fp32_output_and_accumulate():
    p = gen.integer_problem(5400, 5, 6, 5, 1, 100, 0.6, 0.6)
    rng = np.random.default_rng(5401)
    za = p.a_data + 1j * rng.integers(-8, 9, p.a_data.size)
    zb = p.b_data + 1j * rng.integers(-8, 9, p.b_data.size)
    ref = oracle.zbsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), za, zb, 2.0 + 1j)
    got, _ = run(p, p.a_bits(), za, p.b_bits(), zb, alpha=2.0 + 1j, out=bsm.OUT_F32)
    assert got.dtype == np.complex64 and np.array_equal(got, ref.astype(np.complex64))
    C0 = (rng.integers(-50, 50, ref.size) + 1j * rng.integers(-50, 50, ref.size)).astype(np.complex64)
    got, _ = run(p, p.a_bits(), za, p.b_bits(), zb, alpha=2.0 + 1j, C0=C0, out=bsm.OUT_F32,
                 k_window=2)
    assert np.array_equal(got, (ref + C0.astype(np.complex128)).astype(np.complex64))


def test_complex_real_inputs_match_the_real_product():
    """Zero imaginary parts: the real part agrees with the real plan's product (the embedding adds
    exact zero terms), the imaginary part is zero."""
    p = _ragged(5500)
    got, _ = run(p, p.a_bits(), p.a_data + 0j, p.b_bits(), p.b_data + 0j)
    plan = bsm.Plan.from_problem(p)
    C = torch.zeros(plan.info().c_elems, dtype=torch.float64, device=DEV)
    plan.execute(torch.from_numpy(p.a_data).to(DEV), torch.from_numpy(p.b_data).to(DEV), C)
    real = C.cpu().numpy()
    _say(f"[complex] real part bitwise equal to the real product: {np.array_equal(got.real, real)}")
    assert rel_fro(got.real, real) <= 1e-15
    assert np.all(got.imag == 0)


def test_complex_hermitian_gram_from_one_buffer():
    """X^H X from one device buffer X: Hermitian C (C_ji = C_ij^H to rounding), real diagonal
    blocks' diagonals, and the oracle's values."""
    rng = np.random.default_rng(56)
    xr, xc = np.array([40, 7, 90]), np.array([16, 130, 1, 65, 33])
    mask = rng.random((3, 5)) < 0.7
    mask[:, 0] = True
    x = gen.make_problem("X", 57, xr, xc, xc, mask, np.ones((5, 5), bool))
    zx, _ = gen.imag_parts(x, 58)
    xbits = x.a_bits()
    p = gen.Problem("gram", xc, xr, xc, np.zeros((5, 3), bool), np.zeros((3, 5), bool), zx, zx)
    got, plan = run(p, xbits, zx, xbits, zx, alias=True, trans_a=2)
    ref = oracle.zbsmm(xc, xr, xc, xbits, xbits, zx, zx, op_a="C")
    assert rel_fro(np.concatenate([got.real, got.imag]), np.concatenate([ref.real, ref.imag])) <= 1e-12
    off = plan.c_offsets()
    for i in range(5):
        for j in range(5):
            if off[i, j] >= 0:
                a = got[off[i, j]:off[i, j] + xc[i] * xc[j]].reshape(xc[i], xc[j])
                b = got[off[j, i]:off[j, i] + xc[j] * xc[i]].reshape(xc[j], xc[i])
                assert np.allclose(a, b.conj().T, rtol=1e-12, atol=1e-12)


def test_complex_graph_replay_and_autotune():
    p = _ragged(5600)
    za, zb = gen.imag_parts(p, 5601)
    plan = bsm.Plan.from_problem(p, elem=bsm.COMPLEX, use_graph=1)
    info = plan.info()
    A = torch.from_numpy(za).to(DEV)
    B = torch.from_numpy(zb).to(DEV)
    C = torch.zeros(info.c_elems, dtype=torch.complex128, device=DEV)
    plan.autotune(A, B, C)
    outs = []
    for _ in range(3):
        plan.execute(A, B, C, alpha=1.5 - 0.5j)
        torch.cuda.synchronize()
        outs.append(C.cpu().numpy().copy())
    plan.verify()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    ref = oracle.zbsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), za, zb, 1.5 - 0.5j)
    assert rel_fro(np.concatenate([outs[0].real, outs[0].imag]),
                   np.concatenate([ref.real, ref.imag])) <= 1e-12


def test_complex_nonuniform_16384_sampled():
    """The 16384-row nonuniform workload with complex N(0,1) parts, B read as its adjoint, in the
    launch setup the benchmark times: sampled C blocks against the oracle."""
    p = gen.nonuniform_16384()
    za, zb = gen.imag_parts(p, 16384)
    b_bits, b_st = gen.stored_transpose(p.inner, p.cols, p.b_mask, zb.conj())
    _say(f"[complex 16384] M={p.M} K={p.K} N={p.N}")
    got, plan = run(p, p.a_bits(), za, b_bits, b_st, trans_b=2)
    plan.verify()
    off = plan.c_offsets()
    present = np.argwhere(off >= 0)
    rng = np.random.default_rng(11)
    sel = [tuple(int(v) for v in present[q]) for q in rng.choice(len(present), 16, replace=False)]
    blocks, pres = oracle.zbsmm_blocks(p.rows, p.inner, p.cols, p.a_bits(), b_bits, za, b_st, sel,
                                       op_b="C")
    num = den = 0.0
    for (i, j), blk, pr in zip(sel, blocks, pres):
        assert pr
        g = got[int(off[i, j]):int(off[i, j]) + blk.size].reshape(blk.shape)
        num += float(np.sum(np.abs(g - blk) ** 2))
        den += float(np.sum(np.abs(blk) ** 2))
    assert (num / den) ** 0.5 <= 1e-12
