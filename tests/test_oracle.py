"""Pins for the CPU oracle (no GPU): each test checks it against something other than itself --
a library routine, an exact special case, a brute-force count, a closed form or the paper's
equations -- so that a dropped term, a wrong sign or index or a transposed operand fails."""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import gen
from tests.helpers import from_dense, higham_gamma, packed_offsets, to_dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense_product_check(p: gen.Problem, alpha=1.0):
    """Oracle vs numpy's matmul of the zero-filled dense matrices (elementwise Higham bound)."""
    A = to_dense(p.rows, p.inner, p.a_mask, p.a_data)
    B = to_dense(p.inner, p.cols, p.b_mask, p.b_data)
    c_mask = (p.a_mask.astype(np.int64) @ p.b_mask.astype(np.int64)) > 0
    ref = alpha * (A @ B)
    bound = 2 * higham_gamma(max(1, int(p.inner.sum()))) * (np.abs(A) @ np.abs(B)) * abs(alpha) + 1e-300
    got = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data, alpha)
    got_dense = to_dense(p.rows, p.cols, c_mask, got)
    assert got.size == packed_offsets(p.rows, p.cols, c_mask)[1]
    assert np.all(np.abs(got_dense - ref) <= bound)
    # blocks outside the C-shape are zero in the dense product too
    assert np.all(ref[got_dense == 0] == 0) or np.all(np.abs(ref - got_dense) <= bound)


@pytest.mark.parametrize("seed", range(12))
def test_matches_numpy_dense(seed):
    rng = np.random.default_rng(seed)
    M, K, N = (int(x) for x in rng.integers(1, 6, 3))
    p = gen.random_problem(seed, M, K, N, 1, 8, float(rng.uniform(0.2, 1.0)), float(rng.uniform(0.2, 1.0)))
    _dense_product_check(p, alpha=float(rng.choice([1.0, -0.75, 3.0])))


def test_matches_numpy_dense_ragged_sizes():
    # block sizes that are not multiples of any tile: 1, 3, 15, 17, 31, 33
    rows = [1, 17, 33]
    inner = [3, 31, 15, 1]
    cols = [17, 1, 33]
    rng = np.random.default_rng(5)
    a_mask = rng.random((3, 4)) < 0.7
    b_mask = rng.random((4, 3)) < 0.7
    p = gen.make_problem("ragged", 5, rows, inner, cols, a_mask, b_mask)
    _dense_product_check(p)


def _stored(rsz, csz, mask, D, trans):
    """Packed storage of an operand whose product-side view is the dense D (rsz x csz blocks):
    as is, or as the transposed block matrix when trans."""
    if trans:
        return gen.pack_bits(mask.T), from_dense(csz, rsz, mask.T, D.T)
    return gen.pack_bits(mask), from_dense(rsz, csz, mask, D)


@pytest.mark.parametrize("ta,tb", [(False, True), (True, False), (True, True)])
@pytest.mark.parametrize("seed", range(4))
def test_transposed_operands_match_numpy(seed, ta, tb):
    """C = op(A) op(B) with an operand stored as the transposed block matrix: numpy's product of
    the dense transposes, elementwise within Higham's bound, and C's shape is the boolean product
    of the logical shapes."""
    p = gen.random_problem(100 + seed, 4, 5, 3, 1, 9, 0.6, 0.6)
    A = to_dense(p.rows, p.inner, p.a_mask, p.a_data)
    B = to_dense(p.inner, p.cols, p.b_mask, p.b_data)
    a_bits, a_st = _stored(p.rows, p.inner, p.a_mask, A, ta)
    b_bits, b_st = _stored(p.inner, p.cols, p.b_mask, B, tb)
    c_mask = (p.a_mask.astype(np.int64) @ p.b_mask.astype(np.int64)) > 0
    got = oracle.bsmm(p.rows, p.inner, p.cols, a_bits, b_bits, a_st, b_st, -1.5, trans_a=ta,
                      trans_b=tb)
    c_bits = oracle.product_shape(p.M, p.K, p.N, a_bits, b_bits, ta, tb)
    assert np.array_equal(gen.unpack_bits(c_bits, p.M, p.N), c_mask)
    ref = -1.5 * (A @ B)
    bound = 2 * higham_gamma(int(p.inner.sum())) * 1.5 * (np.abs(A) @ np.abs(B)) + 1e-300
    assert got.size == packed_offsets(p.rows, p.cols, c_mask)[1]
    assert np.all(np.abs(to_dense(p.rows, p.cols, c_mask, got) - ref) <= bound)
    # selected blocks follow the same reading
    sel = [(i, j) for i in range(p.M) for j in range(p.N)][::3]
    out, present = oracle.bsmm_blocks(p.rows, p.inner, p.cols, a_bits, b_bits, a_st, b_st, sel,
                                      -1.5, trans_a=ta, trans_b=tb)
    ro = np.concatenate([[0], np.cumsum(p.rows)])
    co = np.concatenate([[0], np.cumsum(p.cols)])
    for n, (i, j) in enumerate(sel):
        assert bool(present[n]) == bool(c_mask[i, j])
        blk = ref[ro[i]:ro[i + 1], co[j]:co[j + 1]]
        assert np.allclose(out[n].reshape(blk.shape), blk, rtol=1e-13, atol=1e-13)


def test_transposed_product_identity_bitwise():
    """(AB)^T = B^T A^T: the oracle multiplying the stored B and A as transposed operands gives the
    transpose of C = AB bit for bit (same products, same summation order)."""
    p = gen.random_problem(7, 4, 6, 5, 1, 12, 0.5, 0.7)
    c = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    ct = oracle.bsmm(p.cols, p.inner, p.rows, p.b_bits(), p.a_bits(), p.b_data, p.a_data,
                     trans_a=True, trans_b=True)
    c_mask = (p.a_mask.astype(np.int64) @ p.b_mask.astype(np.int64)) > 0
    D = to_dense(p.rows, p.cols, c_mask, c)
    Dt = to_dense(p.cols, p.rows, c_mask.T, ct)
    assert np.array_equal(D.T, Dt)


def test_gen_stored_transpose_matches_dense_transpose():
    p = gen.random_problem(9, 3, 4, 2, 1, 7, 0.7, 0.7)
    bits, data = gen.stored_transpose(p.rows, p.inner, p.a_mask, p.a_data)
    A = to_dense(p.rows, p.inner, p.a_mask, p.a_data)
    assert np.array_equal(bits, gen.pack_bits(p.a_mask.T))
    assert np.array_equal(data, from_dense(p.inner, p.rows, p.a_mask.T, A.T))


def test_shape_product_exhaustive_2x2x2():
    """All 2^4 x 2^4 pairs of 2x2 block shapes: C-shape is the boolean product (numpy), bit-exact,
    and the values agree with the dense product."""
    sizes = [2, 3]
    for abits in range(16):
        for bbits in range(16):
            a_mask = np.array([[(abits >> (2 * i + k)) & 1 for k in range(2)] for i in range(2)], bool)
            b_mask = np.array([[(bbits >> (2 * k + j)) & 1 for j in range(2)] for k in range(2)], bool)
            c_ref = (a_mask.astype(int) @ b_mask.astype(int)) > 0
            c = oracle.shape_product(2, 2, 2, gen.pack_bits(a_mask), gen.pack_bits(b_mask))
            assert np.array_equal(gen.unpack_bits(c, 2, 2), c_ref)
            p = gen.make_problem("x", abits * 16 + bbits, sizes, sizes, sizes, a_mask, b_mask)
            _dense_product_check(p)


def test_shape_product_random_wide():
    """Shapes wider than one 64-bit word (bitmap row padding) vs numpy's boolean product."""
    rng = np.random.default_rng(3)
    for M, K, N in [(5, 70, 130), (64, 64, 64), (1, 129, 1), (3, 1, 65)]:
        a = rng.random((M, K)) < 0.1
        b = rng.random((K, N)) < 0.1
        c = oracle.shape_product(M, K, N, gen.pack_bits(a), gen.pack_bits(b))
        assert np.array_equal(gen.unpack_bits(c, M, N), (a.astype(int) @ b.astype(int)) > 0)
        # padding bits stay zero
        full = np.asarray(c, dtype=np.uint64).reshape(M, -1)
        if N % 64:
            assert np.all((full[:, -1] >> np.uint64(N % 64)) == 0)


def test_identity_blocks_give_b_bitwise():
    """A = block-diagonal identity (row tiling = inner tiling) => C = B exactly, and C's shape is
    B's shape."""
    rng = np.random.default_rng(11)
    inner = np.array([4, 1, 7, 3, 5])
    cols = np.array([2, 6, 3])
    a_mask = np.eye(5, dtype=bool)
    b_mask = rng.random((5, 3)) < 0.6
    b_mask[0, 0] = True
    p = gen.make_problem("id", 11, inner, inner, cols, a_mask, b_mask)
    # overwrite A's packed data with identity blocks
    a = np.concatenate([np.eye(int(s)).reshape(-1) for s in inner])
    c = oracle.bsmm(inner, inner, cols, p.a_bits(), p.b_bits(), a, p.b_data)
    c_bits = oracle.shape_product(5, 5, 3, p.a_bits(), p.b_bits())
    assert np.array_equal(gen.unpack_bits(c_bits, 5, 3), b_mask)
    assert np.array_equal(c, p.b_data)


def test_permutation_blocks_bitwise():
    """A = a block permutation (equal-size blocks) with an element permutation inside each block
    => C is B with its rows permuted, exactly."""
    rng = np.random.default_rng(12)
    nb, bs = 6, 5
    sizes = np.full(nb, bs)
    cols = np.array([3, 4, 2, 7])
    perm = rng.permutation(nb)
    a_mask = np.zeros((nb, nb), bool)
    a_blocks = []
    for i in range(nb):
        a_mask[i, perm[i]] = True
    inner_perm = [rng.permutation(bs) for _ in range(nb)]
    for i in range(nb):
        P = np.zeros((bs, bs))
        P[np.arange(bs), inner_perm[i]] = 1.0
        a_blocks.append(P.reshape(-1))
    a = np.concatenate(a_blocks)
    b_mask = rng.random((nb, 4)) < 0.7
    p = gen.make_problem("perm", 12, sizes, sizes, cols, a_mask, b_mask)
    c = oracle.bsmm(sizes, sizes, cols, gen.pack_bits(a_mask), p.b_bits(), a, p.b_data)
    Bd = to_dense(sizes, cols, b_mask, p.b_data)
    rows_src = np.concatenate([perm[i] * bs + inner_perm[i] for i in range(nb)])
    Cd = Bd[rows_src]
    c_mask = b_mask[perm]
    assert np.array_equal(c, from_dense(sizes, cols, c_mask, Cd))


def test_integer_inputs_exact():
    """Integer values: the FP64 sum is exact, so it equals numpy's int64 product exactly."""
    p = gen.integer_problem(21, 4, 5, 3, 1, 19, 0.6, 0.6)
    A = to_dense(p.rows, p.inner, p.a_mask, p.a_data).astype(np.int64)
    B = to_dense(p.inner, p.cols, p.b_mask, p.b_data).astype(np.int64)
    c_mask = (p.a_mask.astype(int) @ p.b_mask.astype(int)) > 0
    ref = from_dense(p.rows, p.cols, c_mask, (A @ B).astype(np.float64))
    got = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    assert np.array_equal(got, ref)


def test_alpha_power_of_two_and_accumulate():
    p = gen.random_problem(31, 3, 4, 3, 2, 9, 0.6, 0.6)
    args = (p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    c1 = oracle.bsmm(*args)
    assert np.array_equal(oracle.bsmm(*args, alpha=0.25), 0.25 * c1)
    assert np.array_equal(oracle.bsmm(*args, alpha=-8.0), -8.0 * c1)
    # C <- AB + C applied to C = AB gives exactly 2 AB
    assert np.array_equal(oracle.bsmm(*args, C=c1), 2.0 * c1)
    # and accumulation adds alpha*AB to an arbitrary C elementwise
    c0 = np.random.default_rng(0).standard_normal(c1.size)
    assert np.array_equal(oracle.bsmm(*args, alpha=0.5, C=c0), 0.5 * c1 + c0)


def test_aliased_a_times_a():
    rows = np.array([3, 5, 2, 4])
    rng = np.random.default_rng(4)
    mask = rng.random((4, 4)) < 0.6
    np.fill_diagonal(mask, True)
    p = gen.make_problem("alias", 4, rows, rows, rows, mask, mask, b_is_a=True)
    assert p.b_data is p.a_data
    _dense_product_check(p)


def test_selected_blocks_match_full_product():
    p = gen.random_problem(41, 5, 4, 6, 1, 12, 0.5, 0.5)
    args = (p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    full = oracle.bsmm(*args, alpha=1.5)
    c_bits = oracle.shape_product(p.M, p.K, p.N, p.a_bits(), p.b_bits())
    c_mask = gen.unpack_bits(c_bits, p.M, p.N)
    off, _ = packed_offsets(p.rows, p.cols, c_mask)
    sel = [(i, j) for i in range(p.M) for j in range(p.N)]
    blocks, present = oracle.bsmm_blocks(*args, sel, alpha=1.5)
    for (i, j), blk, pr in zip(sel, blocks, present):
        assert pr == bool(c_mask[i, j])
        if pr:
            o = off[(i, j)]
            assert np.array_equal(blk.reshape(-1), full[o:o + blk.size])
        else:
            assert not np.any(blk)


def test_extended_accumulator_vs_exact_rationals():
    """Long-double accumulation agrees with exact rational arithmetic to within an FP64 ulp or two,
    and the FP64 accumulation to within its Higham bound."""
    p = gen.random_problem(51, 2, 3, 2, 2, 6, 1.0, 1.0)
    args = (p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    ext = oracle.bsmm(*args, extended=True)
    dbl = oracle.bsmm(*args)
    A = to_dense(p.rows, p.inner, p.a_mask, p.a_data)
    B = to_dense(p.inner, p.cols, p.b_mask, p.b_data)
    n = A.shape[1]
    exact = np.array([[float(sum(Fraction(A[r, k]) * Fraction(B[k, c]) for k in range(n)))
                       for c in range(B.shape[1])] for r in range(A.shape[0])])
    c_mask = np.ones((p.M, p.N), bool)
    ref = from_dense(p.rows, p.cols, c_mask, exact)
    absab = from_dense(p.rows, p.cols, c_mask, np.abs(A) @ np.abs(B))
    assert np.all(np.abs(ext - ref) <= 2 * np.spacing(np.abs(ref)) + 1e-300)
    assert np.all(np.abs(dbl - ref) <= higham_gamma(n) * absab)


def test_useful_flops_closed_form():
    """2 * sum over present triples of r_i s_k t_j = 2 r^T ((Ahat * s) Bhat) t, a matrix
    expression evaluated by numpy (brute force is the oracle's triple loop)."""
    for seed in range(5):
        p = gen.random_problem(60 + seed, 7, 9, 5, 1, 30, 0.4, 0.5)
        f = oracle.useful_flops(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits())
        Ah = p.a_mask.astype(np.int64)
        Bh = p.b_mask.astype(np.int64)
        closed = 2 * int(p.rows @ ((Ah * p.inner[None, :]) @ Bh) @ p.cols)
        assert f == closed


def test_block_offsets_layout():
    rows = [2, 3]
    cols = [4, 1, 2]
    mask = np.array([[1, 0, 1], [1, 1, 0]], bool)
    off, total = oracle.block_offsets(rows, cols, gen.pack_bits(mask))
    # row-major block order: (0,0) 8 elems, (0,2) 4, (1,0) 12, (1,1) 3
    assert total == 8 + 4 + 12 + 3
    assert off.tolist() == [[0, -1, 8], [12, 24, -1]]


# ---- the paper's closed forms ------------------------------------------------------------------
def test_eq1_concurrent_iterations_golden():
    with open(os.path.join(GOLDEN, "eq1_concurrent_iterations.txt")) as f:
        rows = [list(map(int, ln.split())) for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) >= 10
    for prow, pcol, K, want in rows:
        assert oracle.concurrent_iterations(prow, pcol, K) == want, (prow, pcol, K)


def test_eq2_memory_overhead_vs_cyclic_count():
    """Eq. 2 against a brute-force count: distribute an M x N block grid (uniform blocks m x n,
    inner blocks k) cyclically over a P_row x P_col grid; in one SUMMA iteration every process
    holds its rows' A(*,k) blocks, its columns' B(k,*) blocks and its local C blocks.  The average
    over processes equals the closed form exactly (also when the grid does not divide M, N)."""
    for (M, N, m, n, k, prow, pcol) in [(8, 8, 4, 4, 3, 2, 2), (7, 5, 3, 2, 6, 3, 2),
                                        (16, 12, 5, 7, 2, 4, 3), (3, 3, 1, 1, 1, 1, 1),
                                        (10, 9, 2, 3, 4, 5, 4)]:
        total = 0
        for p in range(prow):
            for q in range(pcol):
                my_rows = sum(1 for i in range(M) if i % prow == p)
                my_cols = sum(1 for j in range(N) if j % pcol == q)
                total += my_rows * m * k + k * my_cols * n + my_rows * my_cols * m * n
        avg = Fraction(total, prow * pcol)
        got = oracle.memory_overhead(M, N, m, n, k, prow, pcol)
        assert abs(got - float(avg)) <= 1e-12 * float(avg)


# ---- cost-model network ------------------------------------------------------------------------
F, H1, H2 = 5, 32, 32


def _rand_params(seed, F=F, H1=H1, H2=H2):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(oracle.mlp_param_count(F, H1, H2)) * 0.3


def test_mlp_param_count():
    assert oracle.mlp_param_count(5, 32, 32) == 32 * 5 + 32 + 32 * 32 + 32 + 32 + 1


def test_mlp_forward_exact_network():
    """A network built to return x_2 exactly: h1 = (relu(x_2), relu(-x_2), 0...),
    h2 = h1 (identity block), y = h2_0 - h2_1.  A transposed weight or a wrong offset in the
    parameter layout breaks it."""
    Fi, A1, A2 = 5, 4, 3
    p = np.zeros(oracle.mlp_param_count(Fi, A1, A2))
    W1 = np.zeros((A1, Fi)); W1[0, 2] = 1.0; W1[1, 2] = -1.0; W1[3, 0] = 0.0
    b1 = np.zeros(A1)
    W2 = np.zeros((A2, A1)); W2[0, 0] = 1.0; W2[1, 1] = 1.0
    b2 = np.zeros(A2)
    w3 = np.array([1.0, -1.0, 0.0])
    b3 = np.array([0.25])
    p[:] = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, b3])
    X = np.random.default_rng(0).standard_normal((50, Fi))
    y = oracle.mlp_forward(Fi, A1, A2, p, X)
    assert np.array_equal(y, X[:, 2] + 0.25)


def test_mlp_forward_exact_network_negative_layer2():
    """A network whose second layer has pre-activations of both signs and one that is always
    negative: z2 = (x_2, -x_2, -|x_2| - 1), so y = relu(x_2) + relu(-x_2) + 7 * 0 + 0.25 =
    |x_2| + 0.25 exactly.  Dropping either ReLU, or applying the first layer's activation where
    the second one belongs, changes y."""
    Fi, A1, A2 = 5, 4, 3
    W1 = np.zeros((A1, Fi)); W1[0, 2] = 1.0; W1[1, 2] = -1.0
    b1 = np.zeros(A1)
    W2 = np.zeros((A2, A1))
    W2[0, :2] = [1.0, -1.0]
    W2[1, :2] = [-1.0, 1.0]
    W2[2, :2] = [-1.0, -1.0]
    b2 = np.array([0.0, 0.0, -1.0])
    w3 = np.array([1.0, 1.0, 7.0])
    b3 = np.array([0.25])
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, b3])
    assert p.size == oracle.mlp_param_count(Fi, A1, A2)
    X = np.random.default_rng(1).standard_normal((64, Fi))
    X[0, 2] = 0.0
    y = oracle.mlp_forward(Fi, A1, A2, p, X)
    assert np.array_equal(y, np.abs(X[:, 2]) + 0.25)


def test_mlp_gradient_vs_central_differences():
    rng = np.random.default_rng(7)
    params = _rand_params(7)
    X = rng.standard_normal((64, F))
    T = rng.standard_normal(64)
    loss, g = oracle.mlp_loss_grad(F, H1, H2, params, X, T)
    y = oracle.mlp_forward(F, H1, H2, params, X)
    assert abs(loss - np.mean((y - T) ** 2)) <= 1e-12 * loss
    h = 1e-6
    idx = rng.choice(params.size, 120, replace=False)
    for q in idx:
        pp = params.copy(); pp[q] += h
        pm = params.copy(); pm[q] -= h
        fd = (oracle.mlp_loss_grad(F, H1, H2, pp, X, T)[0] - oracle.mlp_loss_grad(F, H1, H2, pm, X, T)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(g[q])), (q, fd, g[q])


def test_adam_closed_form_constant_gradient():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2, so every step
    moves a parameter by lr * g / (|g| + eps)."""
    P = 7
    g = np.array([1.0, -2.0, 0.5, 3.0, -0.125, 1e-3, 0.0])
    p = np.zeros(P); m = np.zeros(P); v = np.zeros(P)
    lr, eps = 0.01, 1e-8
    for step in range(1, 6):
        before = p.copy()
        oracle.adam_step(p, g.copy(), m, v, step, lr=lr, eps=eps)
        assert np.allclose(before - p, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)


def _adam_exact(p0, grads, lr, b1, b2, eps):
    """Adam (Kingma & Ba 2015) from its update rule, with the moments and their bias corrections
    in exact rational arithmetic and only the square root and the final division in 60-digit
    decimal arithmetic."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    b1, b2 = Fraction(b1), Fraction(b2)
    m = Fraction(0)
    v = Fraction(0)
    p = Decimal(p0)
    out = []
    for n, g in enumerate(grads, start=1):
        g = Fraction(g)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mhat = m / (1 - b1 ** n)
        vhat = v / (1 - b2 ** n)
        num = Decimal(mhat.numerator) / Decimal(mhat.denominator)
        den = (Decimal(vhat.numerator) / Decimal(vhat.denominator)).sqrt() + Decimal(eps)
        p = p - Decimal(lr) * num / den
        out.append((float(p), float(m), float(v)))
    return out


def test_adam_varying_gradients_vs_exact_rationals():
    """Three Adam steps with a different gradient at every step and the usual beta1 = 0.9,
    beta2 = 0.999: parameters and both moments after each step agree with the update rule evaluated
    exactly.  Gradients that change sign and size make the first and second moments and their
    bias corrections distinguishable, so exchanging beta1 and beta2 anywhere fails."""
    lr, b1, b2, eps = 0.05, 0.9, 0.999, 1e-8
    steps = [np.array([1.0, -2.0, 0.5, 3.0]),
             np.array([-0.25, 4.0, 0.5, -1.0]),
             np.array([2.0, -0.5, -3.0, 0.125])]
    p0 = np.array([0.5, -1.0, 2.0, 0.0])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    want = [_adam_exact(p0[q], [s[q] for s in steps], lr, b1, b2, eps) for q in range(4)]
    for n, g in enumerate(steps, start=1):
        oracle.adam_step(p, g.copy(), m, v, n, lr=lr, beta1=b1, beta2=b2, eps=eps)
        for q in range(4):
            wp, wm, wv = want[q][n - 1]
            assert abs(p[q] - wp) <= 1e-13 * max(1.0, abs(wp)), (n, q, p[q], wp)
            assert abs(m[q] - wm) <= 1e-14 * max(1e-300, abs(wm)) + 1e-300, (n, q)
            assert abs(v[q] - wv) <= 1e-14 * max(1e-300, abs(wv)) + 1e-300, (n, q)
    # after three steps the moments are not the constant-gradient ones
    assert not np.allclose(v, m * m)


def test_adam_decreases_loss():
    rng = np.random.default_rng(9)
    params = _rand_params(9)
    X = rng.standard_normal((256, F))
    T = np.sin(X[:, 0]) + 0.5 * X[:, 1]
    m = np.zeros_like(params); v = np.zeros_like(params)
    first = oracle.mlp_loss_grad(F, H1, H2, params, X, T)[0]
    for step in range(1, 301):
        loss, g = oracle.mlp_loss_grad(F, H1, H2, params, X, T)
        oracle.adam_step(params, g, m, v, step, lr=3e-3)
    assert loss < 0.2 * first


# ---- complex elements ------------------------------------------------------------------------
def _zdense(rsz, csz, mask, z):
    return to_dense(rsz, csz, mask, z.real) + 1j * to_dense(rsz, csz, mask, z.imag)


def _zstored(rsz, csz, mask, D, op):
    """Packed storage of an operand whose product-side view is D under op ('N', 'T', 'C')."""
    if op == "N":
        return gen.pack_bits(mask), from_dense(rsz, csz, mask, D.real) + 1j * from_dense(rsz, csz, mask, D.imag)
    S = D.T if op == "T" else D.conj().T
    return gen.pack_bits(mask.T), from_dense(csz, rsz, mask.T, S.real) + 1j * from_dense(csz, rsz, mask.T, S.imag)


@pytest.mark.parametrize("op_a,op_b", [("N", "N"), ("T", "N"), ("N", "C"), ("C", "T"), ("C", "C")])
def test_complex_matches_numpy_dense(op_a, op_b):
    """Complex C = alpha op(A) op(B) + C against numpy's complex product of the dense matrices,
    elementwise within a Higham-type bound (each real output is a real dot product of length 2n
    over the real and imaginary parts)."""
    p = gen.random_problem(410, 4, 5, 3, 1, 11, 0.6, 0.6)
    za, zb = gen.imag_parts(p, 411)
    A, B = _zdense(p.rows, p.inner, p.a_mask, za), _zdense(p.inner, p.cols, p.b_mask, zb)
    a_bits, a_st = _zstored(p.rows, p.inner, p.a_mask, A, op_a)
    b_bits, b_st = _zstored(p.inner, p.cols, p.b_mask, B, op_b)
    c_mask = (p.a_mask.astype(np.int64) @ p.b_mask.astype(np.int64)) > 0
    C0 = np.random.default_rng(4).standard_normal((2, packed_offsets(p.rows, p.cols, c_mask)[1]))
    C0 = C0[0] + 1j * C0[1]
    alpha = 0.75 - 1.5j
    got = oracle.zbsmm(p.rows, p.inner, p.cols, a_bits, b_bits, a_st, b_st, alpha, C=C0,
                       op_a=op_a, op_b=op_b)
    ref = alpha * (A @ B) + _zdense(p.rows, p.cols, c_mask, C0)
    n = int(p.inner.sum())
    mag = lambda X: np.abs(X.real) + np.abs(X.imag)
    bound = 4 * higham_gamma(2 * n + 4) * (mag(np.array([alpha]))[0] * (mag(A) @ mag(B)) +
                                           mag(_zdense(p.rows, p.cols, c_mask, C0))) + 1e-300
    diff = _zdense(p.rows, p.cols, c_mask, got) - ref
    assert np.all(np.abs(diff.real) <= bound) and np.all(np.abs(diff.imag) <= bound)


def test_complex_real_inputs_reduce_to_the_real_product():
    """Zero imaginary parts: the real part is the real oracle's product bit for bit (every
    dropped term is an exact zero) and the imaginary part is zero."""
    p = gen.random_problem(420, 5, 4, 6, 1, 20, 0.6, 0.6)
    got = oracle.zbsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data + 0j,
                       p.b_data + 0j, 2.0)
    real = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data, 2.0)
    assert np.array_equal(got.real, real) and np.all(got.imag == 0)


def test_complex_gaussian_integers_exact():
    """Gaussian-integer blocks: every partial sum is an integer below 2^53, so the product equals
    numpy's exactly."""
    p = gen.integer_problem(430, 4, 6, 5, 1, 30, 0.6, 0.6)
    rng = np.random.default_rng(431)
    za = p.a_data + 1j * rng.integers(-8, 9, p.a_data.size)
    zb = p.b_data + 1j * rng.integers(-8, 9, p.b_data.size)
    got = oracle.zbsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), za, zb, 1j)
    A, B = _zdense(p.rows, p.inner, p.a_mask, za), _zdense(p.inner, p.cols, p.b_mask, zb)
    c_mask = (p.a_mask.astype(np.int64) @ p.b_mask.astype(np.int64)) > 0
    assert np.array_equal(_zdense(p.rows, p.cols, c_mask, got), 1j * (A @ B))


def test_complex_adjoint_identity_bitwise():
    """(AB)^H = B^H A^H: multiplying the stored B and A as adjoint operands gives the conjugate
    transpose of C = AB bit for bit (the same products, negated, summed in the same order)."""
    p = gen.random_problem(440, 4, 5, 3, 1, 12, 0.6, 0.7)
    za, zb = gen.imag_parts(p, 441)
    c = oracle.zbsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), za, zb)
    ch = oracle.zbsmm(p.cols, p.inner, p.rows, p.b_bits(), p.a_bits(), zb, za, op_a="C", op_b="C")
    c_mask = (p.a_mask.astype(np.int64) @ p.b_mask.astype(np.int64)) > 0
    D = _zdense(p.rows, p.cols, c_mask, c)
    Dh = _zdense(p.cols, p.rows, c_mask.T, ch)
    assert np.array_equal(D.conj().T, Dh)


def test_complex_selected_blocks_match_full_product():
    p = gen.random_problem(450, 5, 4, 5, 1, 16, 0.6, 0.6)
    za, zb = gen.imag_parts(p, 451)
    zt_bits, zt = gen.stored_transpose(p.inner, p.cols, p.b_mask, zb.conj())
    full = oracle.zbsmm(p.rows, p.inner, p.cols, p.a_bits(), zt_bits, za, zt, op_b="C")
    c_mask = (p.a_mask.astype(np.int64) @ p.b_mask.astype(np.int64)) > 0
    off, _ = packed_offsets(p.rows, p.cols, c_mask)
    sel = [(i, j) for i in range(p.M) for j in range(p.N)]
    blocks, pres = oracle.zbsmm_blocks(p.rows, p.inner, p.cols, p.a_bits(), zt_bits, za, zt, sel,
                                       op_b="C")
    for (i, j), blk, pr in zip(sel, blocks, pres):
        assert pr == bool(c_mask[i, j])
        if pr:
            o = off[(i, j)]
            assert np.array_equal(full[o:o + blk.size], blk.reshape(-1))
    # adjoint of the stored conj-transpose is B itself: same result as the plain product
    plain = oracle.zbsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), za, zb)
    assert np.array_equal(full, plain)


# ---- block-rank-sparse operands --------------------------------------------------------------
def _factors_of(p, ranks, data):
    """(i, k, U, V) of every factored block and (i, k, block) of every dense one, from the packed
    block-rank-sparse buffer (test-side walk of the layout)."""
    pos, fac, dense = 0, [], []
    for q, (i, k) in enumerate(zip(*np.nonzero(p.a_mask))):
        h, d, rho = int(p.rows[i]), int(p.inner[k]), int(ranks[q])
        if rho == 0:
            dense.append((i, k, data[pos:pos + h * d].reshape(h, d)))
            pos += h * d
        else:
            U = data[pos:pos + h * rho].reshape(h, rho)
            V = data[pos + h * rho:pos + (h + d) * rho].reshape(d, rho)
            fac.append((i, k, U, V))
            pos += (h + d) * rho
    assert pos == data.size
    return fac, dense


def test_low_rank_expansion_matches_numpy():
    """Factored blocks multiply out to numpy's U @ V^T (inside gamma_rho |U||V|^T), rank-1 blocks to
    numpy's outer product bit for bit, dense blocks pass through bit for bit."""
    p = gen.random_problem(460, 5, 6, 3, 1, 40, 0.8, 0.5)
    ranks, data = gen.low_rank_operand(p, 461, lambda i, k, h, d: (i + k) % 4)
    full = oracle.lr_expand(p.rows, p.inner, p.a_bits(), ranks, data)
    D = to_dense(p.rows, p.inner, p.a_mask, full)
    ro = np.concatenate([[0], np.cumsum(p.rows)])
    so = np.concatenate([[0], np.cumsum(p.inner)])
    fac, dense = _factors_of(p, ranks, data)
    assert fac and dense
    for i, k, U, V in fac:
        blk = D[ro[i]:ro[i + 1], so[k]:so[k + 1]]
        if U.shape[1] == 1:
            assert np.array_equal(blk, np.outer(U[:, 0], V[:, 0]))
        bound = 2 * higham_gamma(U.shape[1]) * (np.abs(U) @ np.abs(V).T) + 1e-300
        assert np.all(np.abs(blk - U @ V.T) <= bound)
    for i, k, B in dense:
        assert np.array_equal(D[ro[i]:ro[i + 1], so[k]:so[k + 1]], B)


def test_low_rank_integer_factors_exact_and_errors():
    p = gen.integer_problem(470, 4, 5, 3, 1, 30, 0.9, 0.6)
    ranks, data = gen.low_rank_operand(p, 472, lambda i, k, h, d: 3 if (i + 2 * k) % 3 else 0,
                                       draw=lambda g, i, k, h, w: g.integers(-4, 5, (h, w)).astype(float))
    full = oracle.lr_expand(p.rows, p.inner, p.a_bits(), ranks, data)
    fac, _ = _factors_of(p, ranks, data)
    D = to_dense(p.rows, p.inner, p.a_mask, full)
    ro = np.concatenate([[0], np.cumsum(p.rows)])
    so = np.concatenate([[0], np.cumsum(p.inner)])
    for i, k, U, V in fac:
        assert np.array_equal(D[ro[i]:ro[i + 1], so[k]:so[k + 1]],
                              (U.astype(np.int64) @ V.T.astype(np.int64)).astype(float))
    bad = ranks.copy()
    bad[0] = -1
    with pytest.raises(ValueError):
        oracle.lr_expand(p.rows, p.inner, p.a_bits(), bad, data)



# ---- block-sparse tensor contraction ----------------------------------------------------------
from oracle import contract as tc  # noqa: E402

_LETTERS = "abcdefghij"


def _tensor(seed, modes, tilings, density, draw=None):
    present, data = gen.block_sparse_tensor(seed, tilings, density, draw)
    return tc.Tensor(modes, tilings, present, data)


def _einsum(A, B, c_modes, Da, Db):
    spec = ("".join(_LETTERS[m] for m in A.modes) + "," + "".join(_LETTERS[m] for m in B.modes)
            + "->" + "".join(_LETTERS[m] for m in c_modes))
    return np.einsum(spec, Da, Db)


CONTRACTIONS = [
    # (A modes, B modes, C modes): matrix product, C order interleaving A and B modes, two
    # contracted modes in different orders, order-4 result
    ([0, 2], [2, 1], [0, 1]),
    ([0, 3, 2], [2, 1, 3], [1, 0]),
    ([0, 2, 3, 1], [3, 4, 2], [4, 0, 1]),
    ([0, 4], [4, 1, 2, 3], [0, 1, 2, 3]),
    ([2, 0, 4, 1], [3, 4, 2], [0, 3, 1]),
]


def _tilings(rng, labels):
    return {m: rng.integers(1, 6, int(rng.integers(1, 4))) for m in labels}


@pytest.mark.parametrize("case", range(len(CONTRACTIONS)))
def test_contraction_matches_numpy_einsum(case):
    """Against numpy's einsum of the zero-filled dense tensors: C-shape from the boolean
    contraction of the block shapes (exact), values inside the Higham bound of the contracted
    length."""
    am, bm, cm = CONTRACTIONS[case]
    rng = np.random.default_rng(900 + case)
    til = _tilings(rng, set(am) | set(bm))
    A = _tensor(910 + case, am, [til[m] for m in am], 0.6)
    B = _tensor(920 + case, bm, [til[m] for m in bm], 0.6)
    shape, data = tc.contract(A, B, cm, alpha=-1.25)
    mask = _einsum(A, B, cm, A.present.astype(np.int64), B.present.astype(np.int64)) > 0
    assert np.array_equal(shape, mask)
    ref = -1.25 * _einsum(A, B, cm, tc.densify(A), tc.densify(B))
    absref = 1.25 * _einsum(A, B, cm, np.abs(tc.densify(A)), np.abs(tc.densify(B)))
    n = int(np.prod([til[m].sum() for m in am if m in bm and m not in cm]))
    c_til = [til[m] for m in cm]
    got = tc.densify(tc.Tensor(cm, c_til, shape, data))
    assert np.all(np.abs(got - ref) <= 2 * higham_gamma(max(n, 1)) * absref + 1e-300)
    # absent C blocks are zero in the dense contraction too
    assert np.array_equal(tc.pack(shape, c_til, ref).size, data.size)


def test_contraction_order2_is_the_block_sparse_matrix_product():
    """Modes (i,k), (k,j) -> (i,j): the C-shape is the block-sparse matrix oracle's bit for bit and
    the values agree inside the Higham bound."""
    p = gen.random_problem(930, 4, 5, 3, 1, 9, 0.6, 0.6)
    A = tc.Tensor([0, 2], [p.rows, p.inner], p.a_mask, p.a_data)
    B = tc.Tensor([2, 1], [p.inner, p.cols], p.b_mask, p.b_data)
    shape, data = tc.contract(A, B, [0, 1])
    c_bits = oracle.shape_product(p.M, p.K, p.N, p.a_bits(), p.b_bits())
    assert np.array_equal(shape, gen.unpack_bits(c_bits, p.M, p.N))
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    assert data.shape == ref.shape
    assert np.allclose(data, ref, rtol=1e-13, atol=1e-13)


def test_contraction_brute_force_tiny():
    """Element-level brute force (pure Python loops over every index) on a tiny order-3 x order-3
    contraction with an accumulated C."""
    am, bm, cm = [0, 2, 3], [3, 1, 2], [1, 0]
    til = {0: np.array([2, 1]), 1: np.array([1, 2]), 2: np.array([2, 1]), 3: np.array([1, 2])}
    A = _tensor(940, am, [til[m] for m in am], 0.7)
    B = _tensor(941, bm, [til[m] for m in bm], 0.7)
    shape, first = tc.contract(A, B, cm)
    C0 = np.random.default_rng(942).standard_normal(first.size)
    shape2, data = tc.contract(A, B, cm, alpha=2.0, C=(shape, C0))
    Da, Db = tc.densify(A), tc.densify(B)
    dims = {m: int(til[m].sum()) for m in til}
    ref = np.zeros((dims[1], dims[0]))
    for x1 in range(dims[1]):
        for x0 in range(dims[0]):
            s = 0.0
            for x2 in range(dims[2]):
                for x3 in range(dims[3]):
                    s += Da[x0, x2, x3] * Db[x3, x1, x2]
            ref[x1, x0] = s
    want = 2.0 * tc.pack(shape, [til[1], til[0]], ref) + C0
    assert np.allclose(data, want, rtol=1e-14, atol=1e-14)


def test_contraction_integer_values_exact():
    am, bm, cm = CONTRACTIONS[2]
    rng = np.random.default_rng(950)
    til = _tilings(rng, set(am) | set(bm))
    draw = lambda g, shape: g.integers(-6, 7, shape).astype(float)
    A = _tensor(951, am, [til[m] for m in am], 0.7, draw)
    B = _tensor(952, bm, [til[m] for m in bm], 0.7, draw)
    shape, data = tc.contract(A, B, cm)
    ref = _einsum(A, B, cm, tc.densify(A).astype(np.int64), tc.densify(B).astype(np.int64))
    assert np.array_equal(data, tc.pack(shape, [til[m] for m in cm], ref).astype(float))


def test_contraction_selected_blocks_match_full():
    am, bm, cm = CONTRACTIONS[4]
    rng = np.random.default_rng(960)
    til = _tilings(rng, set(am) | set(bm))
    A = _tensor(961, am, [til[m] for m in am], 0.6)
    B = _tensor(962, bm, [til[m] for m in bm], 0.6)
    shape, data = tc.contract(A, B, cm)
    full = tc.Tensor(cm, [til[m] for m in cm], shape, data).blocks()
    sel = [tuple(int(v) for v in idx) for idx in np.ndindex(*shape.shape)]
    for idx, blk in zip(sel, tc.contract_blocks(A, B, cm, sel)):
        if blk is None:
            assert idx not in full
        else:
            assert np.array_equal(blk, full[idx])


def test_contraction_to_a_scalar():
    """All modes contracted: C is one number, the sum over present block pairs of their elementwise
    products (numpy einsum of the dense tensors)."""
    til = {0: np.array([3, 1]), 1: np.array([2]), 2: np.array([4, 2])}
    A = _tensor(970, [0, 1, 2], [til[0], til[1], til[2]], 0.7)
    B = _tensor(971, [2, 1, 0], [til[2], til[1], til[0]], 0.7)
    shape, data = tc.contract(A, B, [])
    ref = np.einsum("abc,cba->", tc.densify(A), tc.densify(B))
    assert shape.shape == () and data.size == (1 if shape else 0)
    if shape:
        assert abs(data[0] - ref) <= 1e-12 * max(1.0, abs(ref))
