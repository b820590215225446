"""FP64 GPU path vs the CPU oracle, through the C ABI.

Gates: relative Frobenius error <= 1e-12 per product, every element inside twice the Higham bound
gamma_n |A||B| (n = the C block's summed inner size), bit-exact C-shape, and bit-exact values for
integer inputs and for identity blocks."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import bsm, gen
from tests.helpers import higham_gamma, rel_fro

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(p: gen.Problem, alpha=1.0, C0=None, plan=None, **kw):
    plan = plan or bsm.Plan.from_problem(p, **kw)
    info = plan.info()
    dev = torch.device("cuda:0")
    A = torch.from_numpy(p.a_data).to(dev)
    B = A if p.b_is_a else torch.from_numpy(p.b_data).to(dev)
    if C0 is None:
        C = torch.full((max(1, info.c_elems),), float("nan"), dtype=torch.float64, device=dev)
    else:
        C = torch.from_numpy(C0.copy()).to(dev)
    plan.execute(A, B, C, alpha=alpha, accumulate=C0 is not None)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:info.c_elems], plan


def _abs_bound(p: gen.Problem, alpha=1.0):
    """Elementwise 2 gamma_n |alpha| |A||B| with n = the total inner dimension (an upper bound on
    every C block's summed inner size)."""
    absab = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), np.abs(p.a_data),
                        np.abs(p.b_data), abs(alpha))
    return 2 * higham_gamma(max(1, int(p.inner.sum()))) * absab


def check(p: gen.Problem, alpha=1.0, **kw):
    _say(f"[fp64] {p.name} M={p.M} K={p.K} N={p.N} kw={kw}")
    got, plan = run_gpu(p, alpha=alpha, **kw)
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data, alpha)
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got))
    err = rel_fro(got, ref)
    assert err <= 1e-12, err
    assert np.all(np.abs(got - ref) <= _abs_bound(p, alpha) + 1e-300)
    return got, ref, plan


def test_uniform_1024_full():
    check(gen.uniform_1024())


@pytest.mark.parametrize("sizes", [
    [1, 3, 15], [16, 17, 31], [33, 63, 64], [65, 127, 128], [129, 255, 256], [1, 256, 17, 100],
])
def test_ragged_block_sizes(sizes):
    rng = np.random.default_rng(len(sizes) * 100 + sizes[0])
    rows = rng.permutation(sizes)
    inner = rng.permutation(sizes)
    cols = rng.permutation(sizes)
    a_mask = rng.random((len(rows), len(inner))) < 0.7
    b_mask = rng.random((len(inner), len(cols))) < 0.7
    a_mask[0, 0] = b_mask[0, 0] = True
    p = gen.make_problem(f"ragged{sizes}", 7, rows, inner, cols, a_mask, b_mask)
    check(p)


@pytest.mark.parametrize("seed", range(4))
def test_random_nonuniform(seed):
    check(gen.random_problem(100 + seed, 9, 11, 8, 1, 200, 0.35, 0.4))


def test_paper_dense_blockings():
    """The paper's dense square product at N = 1536: uniform blocks of 256, and the add-one-row
    blocking of the same mean (Sec. 4.1), whose blocks above 256 rows are cut into three
    sub-tiles per side; FP64 to the FP64 gates, the FP32 and split-bf16 forms to theirs."""
    uni = gen.paper_dense(8100, 1536, 256, False)
    assert set(uni.rows.tolist()) == {256}
    check(uni)
    p = gen.paper_dense(8100, 1536, 256, True)
    assert p.rows.sum() == p.inner.sum() == p.cols.sum() == 1536
    assert p.rows.max() > 256 and p.cols.max() > 256      # three-way cuts on both sides
    _, ref, _ = check(p)
    for precision, gate in ((bsm.FP32, 1e-5), (bsm.BF16X3, 1e-6)):
        got, _ = run_gpu(p, precision=precision)
        assert rel_fro(got, ref) <= gate


@pytest.mark.parametrize("tile", range(1, len(bsm.tile_variants()) + 1))
def test_every_tile_variant(tile):
    check(gen.random_problem(200 + tile, 6, 7, 6, 1, 300, 0.5, 0.5), tile=tile)
    p = gen.integer_problem(250 + tile, 5, 6, 5, 1, 200, 0.6, 0.6)
    got, _ = run_gpu(p, tile=tile)
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("order,patch", [(bsm.ORDER_LOCALITY, (0, 0)), (bsm.ORDER_LPT, (0, 0)),
                                         (bsm.ORDER_INTERLEAVE, (0, 0)), (bsm.ORDER_PATCH, (0, 0)),
                                         (bsm.ORDER_PATCH, (3, 2))])
def test_task_orders_bitwise_identical(order, patch):
    p = gen.random_problem(300, 8, 8, 8, 20, 200, 0.5, 0.5)
    a, _ = run_gpu(p)
    b, plan = run_gpu(p, order=order, patch=patch)
    plan.verify()
    assert np.array_equal(a, b)


def test_integer_inputs_bit_exact():
    p = gen.integer_problem(400, 7, 9, 6, 1, 150, 0.6, 0.6)
    got, _ = run_gpu(p)
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    assert np.array_equal(got, ref)


def test_identity_blocks_give_b():
    rng = np.random.default_rng(5)
    inner = np.array([40, 17, 130, 64, 1])
    cols = np.array([33, 128, 7])
    a_mask = np.eye(5, dtype=bool)
    b_mask = rng.random((5, 3)) < 0.6
    b_mask[2, 1] = True
    p = gen.make_problem("id", 5, inner, inner, cols, a_mask, b_mask)
    p.a_data = np.concatenate([np.eye(int(s)).reshape(-1) for s in inner])
    got, _ = run_gpu(p)
    assert np.array_equal(got, p.b_data)


def test_alpha_and_accumulate():
    p = gen.random_problem(500, 5, 6, 5, 10, 140, 0.6, 0.6)
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    c1, plan = run_gpu(p)
    c2, _ = run_gpu(p, alpha=0.25, plan=plan)
    assert np.array_equal(c2, 0.25 * c1)
    C0 = np.random.default_rng(1).standard_normal(c1.size)
    c3, _ = run_gpu(p, alpha=-1.5, C0=C0, plan=plan)
    ref3 = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data, -1.5, C=C0)
    assert rel_fro(c3, ref3) <= 1e-12
    assert rel_fro(c1, ref) <= 1e-12


def test_aliased_c_equals_a_times_a():
    rows = np.array([10, 25, 40, 60, 25, 10])
    rng = np.random.default_rng(6)
    mask = rng.random((6, 6)) < 0.5
    np.fill_diagonal(mask, True)
    p = gen.make_problem("alias", 6, rows, rows, rows, mask, mask, b_is_a=True)
    check(p)


def test_empty_products_are_no_ops():
    p = gen.make_problem("none", 0, [3, 4], [5], [2, 2], np.zeros((2, 1), bool), np.zeros((1, 2), bool))
    got, _ = run_gpu(p)
    assert got.size == 0


def test_repeat_launches_bitwise_stable():
    p = gen.random_problem(600, 10, 10, 10, 30, 250, 0.4, 0.4)
    a, plan = run_gpu(p)
    for _ in range(3):
        b, _ = run_gpu(p, plan=plan)
        assert np.array_equal(a, b)


def _sampled_check(p: gen.Problem, nsample: int, seed: int, **kw):
    """Full-size product on the GPU; a random sample of C blocks recomputed by the oracle."""
    _say(f"[fp64 sampled] {p.name} M={p.M} K={p.K} N={p.N}")
    got, plan = run_gpu(p, **kw)
    off = plan.c_offsets()
    present = np.argwhere(off >= 0)
    rng = np.random.default_rng(seed)
    sel = [tuple(int(v) for v in present[q]) for q in rng.choice(len(present), nsample, replace=False)]
    blocks, pres = oracle.bsmm_blocks(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data,
                                      p.b_data, sel)
    num = den = 0.0
    for (i, j), blk, pr in zip(sel, blocks, pres):
        assert pr
        o = int(off[i, j])
        g = got[o:o + blk.size].reshape(blk.shape)
        num += float(np.sum((g - blk) ** 2))
        den += float(np.sum(blk ** 2))
    err = (num / den) ** 0.5
    assert err <= 1e-12, err
    return got


def test_nonuniform_16384_sampled():
    _sampled_check(gen.nonuniform_16384(), nsample=64, seed=1)


def _int_draw(rng, i, j, h, w):
    return rng.integers(-8, 9, (h, w)).astype(np.float64)


@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32, bsm.BF16X3])
def test_block_larger_than_2gib(precision):
    """One B block of 16384 x 17000 FP64 elements (2.2 GB, byte offsets past 2^31) with integer
    values in [-8, 8]: every form reproduces the oracle bit for bit (sums stay below 2^24)."""
    _say(f"[big block] precision={precision}")
    p = gen.make_problem("bigB", 77, [3, 2], [16384], [17000], np.ones((2, 1), bool),
                         np.ones((1, 1), bool), draw=_int_draw)
    got, plan = run_gpu(p, precision=precision)
    plan.verify()
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    assert np.array_equal(got, ref)


def _run_f32_out(p, precision, alpha=1.0, C0=None, **kw):
    plan = bsm.Plan.from_problem(p, precision=precision, out=bsm.OUT_F32, **kw)
    info = plan.info()
    assert info.out == bsm.OUT_F32
    dev = torch.device("cuda:0")
    A = torch.from_numpy(p.a_data).to(dev)
    B = A if p.b_is_a else torch.from_numpy(p.b_data).to(dev)
    C = (torch.full((max(1, info.c_elems),), float("nan"), dtype=torch.float32, device=dev)
         if C0 is None else torch.from_numpy(C0.copy()).to(dev))
    plan.execute(A, B, C, alpha=alpha, accumulate=C0 is not None)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:info.c_elems]


@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32, bsm.BF16X3])
def test_fp32_output(precision):
    """C in FP32: alpha * sum (+ C) is formed in FP64 and rounded once."""
    _say(f"[fp32 out] precision={precision}")
    p = gen.random_problem(1900 + precision, 7, 8, 6, 1, 200, 0.5, 0.5)
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data, -0.75)
    got = _run_f32_out(p, precision, alpha=-0.75)
    assert got.dtype == np.float32 and np.all(np.isfinite(got))
    gate = {bsm.FP64: 1e-12, bsm.FP32: 1e-5, bsm.BF16X3: 1e-6}[precision]
    # the FP32 rounding of C adds at most 2^-24 relative per element
    assert np.all(np.abs(got.astype(np.float64) - ref) <= 2.0 ** -24 * np.abs(ref) + gate * np.abs(ref).max())
    # integers: exact, also with accumulation into an FP32 C and k-windows
    q = gen.integer_problem(1950 + precision, 6, 7, 5, 1, 150, 0.6, 0.6)
    refq = oracle.bsmm(q.rows, q.inner, q.cols, q.a_bits(), q.b_bits(), q.a_data, q.b_data)
    assert np.array_equal(_run_f32_out(q, precision), refq.astype(np.float32))
    C0 = np.random.default_rng(3).integers(-100, 100, refq.size).astype(np.float32)
    want = (2.0 * refq + C0.astype(np.float64)).astype(np.float32)
    assert np.array_equal(_run_f32_out(q, precision, alpha=2.0, C0=C0, k_window=2), want)


def test_execution_counters_catch_a_skipped_task():
    """Every launch counts each task's executions; a task left out by the host-set fault-injection
    flag makes the synchronising checks fail with E_STATE, and the kernel still exits normally."""
    p = gen.random_problem(1990, 6, 6, 6, 16, 200, 0.6, 0.6)
    for use_graph in (0, 1):
        plan = bsm.Plan.from_problem(p, use_graph=use_graph, record_timings=1)
        dev = torch.device("cuda:0")
        A = torch.from_numpy(p.a_data).to(dev)
        B = torch.from_numpy(p.b_data).to(dev)
        C = torch.zeros(plan.info().c_elems, dtype=torch.float64, device=dev)
        for _ in range(3):
            plan.execute(A, B, C)
        plan.verify()
        plan.timings()
        plan.debug_skip_task(2)
        plan.execute(A, B, C)
        with pytest.raises(bsm.BsmError) as ei:
            plan.verify()
        assert ei.value.code == bsm.E_STATE and "task 2" in str(ei.value)
        with pytest.raises(bsm.BsmError) as ei:
            plan.timings()
        assert ei.value.code == bsm.E_STATE
        # a new schedule uploads the tasks again and restarts the counts
        plan.debug_skip_task(-1)
        plan.set_costs(np.ones(plan.info().tasks, np.float32))
        plan.execute(A, B, C)
        plan.verify()
        torch.cuda.synchronize()
        ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
        assert rel_fro(C.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32])
def test_mixed_tile_classes_single_plan(precision):
    """One plan whose size classes use four different tile variants (one launch each): matches
    the oracle, and k-windows give the same bits."""
    p = gen.random_problem(2300 + precision, 9, 9, 9, 8, 200, 0.5, 0.5)
    plan = bsm.Plan.from_problem(p, precision=precision)
    plan.set_tile_classes([4, 3, 2, 1])
    assert plan.info().tile == 0
    got, _ = run_gpu(p, plan=plan)
    plan.verify()
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    assert rel_fro(got, ref) <= (1e-12 if precision == bsm.FP64 else 1e-5)
    win = bsm.Plan.from_problem(p, precision=precision, k_window=2)
    win.set_tile_classes([4, 3, 2, 1])
    got2, _ = run_gpu(p, plan=win)
    win.verify()
    assert np.array_equal(got, got2)


@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32, bsm.BF16X3])
def test_device_built_klists_match_host_lists(precision):
    """k-lists built on the device, batch by batch (also in batches of a few triples), give the
    same bits as the host-built lists, with and without k-windows."""
    _say(f"[device k-lists] precision={precision}")
    p = gen.random_problem(2400 + precision, 9, 12, 8, 4, 180, 0.5, 0.5)
    base, _ = run_gpu(p, precision=precision)
    for dk in (1, 7, 64):
        got, plan = run_gpu(p, precision=precision, device_klists=dk)
        assert plan.info().device_klists == 1
        plan.verify()
        assert np.array_equal(got, base), dk
    got, plan = run_gpu(p, precision=precision, device_klists=7, k_window=3)
    plan.verify()
    assert np.array_equal(got, base)


def test_device_built_klists_decay_cloud_against_oracle():
    """C = A A on a small distance-decay cloud with device-built k-lists and small tiles."""
    p = gen.decay_cloud(seed=5001, npts=300, box=15.0)
    got, plan = run_gpu(p, device_klists=1, tile=4)
    plan.verify()
    ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data)
    assert rel_fro(got, ref) <= 1e-12
    assert np.all(np.abs(got - ref) <= _abs_bound(p) + 1e-300)
