"""Precision forms, k-windows and task timings on the GPU, against the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import bsm, gen
from tests.helpers import rel_fro

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(p, plan=None, alpha=1.0, C0=None, **kw):
    plan = plan or bsm.Plan.from_problem(p, **kw)
    info = plan.info()
    dev = torch.device("cuda:0")
    A = torch.from_numpy(p.a_data).to(dev)
    B = A if p.b_is_a else torch.from_numpy(p.b_data).to(dev)
    C = (torch.full((max(1, info.c_elems),), float("nan"), dtype=torch.float64, device=dev)
         if C0 is None else torch.from_numpy(C0.copy()).to(dev))
    plan.execute(A, B, C, alpha=alpha, accumulate=C0 is not None)
    torch.cuda.synchronize()
    return C.cpu().numpy()[:info.c_elems], plan


def ref(p, alpha=1.0, C0=None):
    return oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data, alpha, C=C0)


@pytest.mark.parametrize("seed", range(3))
def test_fp32_form_error_gate(seed):
    p = gen.random_problem(700 + seed, 8, 9, 7, 1, 200, 0.4, 0.5)
    _say(f"[fp32] {p.name} seed={seed}")
    got, _ = run(p, precision=bsm.FP32)
    err = rel_fro(got, ref(p))
    assert np.all(np.isfinite(got))
    assert err <= 1e-5, err


def test_fp32_form_scaled_blocks():
    """Block values scaled by 10^U(-4,0) as in the precision workload, at a small size."""
    p = gen.nonuniform(4100, 1200, 64, 256, 0.4, draw=gen._scaled_normal(4100), name="prec_small")
    got, _ = run(p, precision=bsm.FP32)
    assert rel_fro(got, ref(p)) <= 1e-5


@pytest.mark.parametrize("tile", range(1, len(bsm.tile_variants()) + 1))
def test_fp32_integer_inputs_bit_exact(tile):
    p = gen.integer_problem(750 + tile, 6, 7, 5, 1, 200, 0.6, 0.6)
    got, _ = run(p, precision=bsm.FP32, tile=tile)
    assert np.array_equal(got, ref(p))


def test_fp32_alpha_accumulate_and_alias():
    p = gen.random_problem(760, 5, 6, 5, 10, 140, 0.6, 0.6)
    C0 = np.random.default_rng(2).standard_normal(ref(p).size)
    got, _ = run(p, precision=bsm.FP32, alpha=-0.5, C0=C0)
    assert rel_fro(got, ref(p, -0.5, C0)) <= 1e-5
    rows = np.array([10, 25, 40, 60, 25])
    mask = np.random.default_rng(3).random((5, 5)) < 0.6
    np.fill_diagonal(mask, True)
    q = gen.make_problem("alias", 9, rows, rows, rows, mask, mask, b_is_a=True)
    got, _ = run(q, precision=bsm.FP32)
    assert rel_fro(got, ref(q)) <= 1e-5


@pytest.mark.parametrize("seed", range(3))
def test_bf16x3_form_error_gate(seed):
    p = gen.random_problem(1700 + seed, 8, 9, 7, 1, 200, 0.4, 0.5)
    _say(f"[bf16x3] {p.name} seed={seed}")
    got, _ = run(p, precision=bsm.BF16X3)
    assert np.all(np.isfinite(got))
    err = rel_fro(got, ref(p))
    assert err <= 1e-6, err


def test_bf16x3_form_scaled_blocks():
    """Block values scaled by 10^U(-4,0) as in the precision workload, at a small size."""
    p = gen.nonuniform(4101, 1500, 64, 256, 0.4, draw=gen._scaled_normal(4101), name="prec_small")
    got, _ = run(p, precision=bsm.BF16X3)
    err = rel_fro(got, ref(p))
    _say(f"[bf16x3] scaled rel err {err:.3e}")
    assert err <= 1e-6, err


def test_bf16x3_ragged_sizes():
    sizes = [1, 3, 15, 16, 17, 31, 33, 63, 64, 65, 127, 129, 255, 256]
    rng = np.random.default_rng(17)
    rows, inner, cols = rng.permutation(sizes), rng.permutation(sizes), rng.permutation(sizes)
    a_mask = rng.random((len(rows), len(inner))) < 0.4
    b_mask = rng.random((len(inner), len(cols))) < 0.4
    p = gen.make_problem("ragged_b3", 17, rows, inner, cols, a_mask, b_mask)
    got, _ = run(p, precision=bsm.BF16X3)
    assert rel_fro(got, ref(p)) <= 1e-6


def test_bf16x3_integer_inputs_bit_exact():
    """Integers in [-8, 8] are exact in bf16 (the second and third slices are 0) and their block
    sums stay below 2^24, so the split form reproduces the FP64 result bit for bit."""
    p = gen.integer_problem(1750, 6, 7, 5, 1, 200, 0.6, 0.6)
    got, _ = run(p, precision=bsm.BF16X3)
    assert np.array_equal(got, ref(p))


def test_bf16x3_alpha_accumulate_and_alias():
    p = gen.random_problem(1760, 5, 6, 5, 10, 140, 0.6, 0.6)
    C0 = np.random.default_rng(2).standard_normal(ref(p).size)
    got, _ = run(p, precision=bsm.BF16X3, alpha=-0.5, C0=C0)
    assert rel_fro(got, ref(p, -0.5, C0)) <= 1e-6
    rows = np.array([10, 25, 40, 60, 25])
    mask = np.random.default_rng(3).random((5, 5)) < 0.6
    np.fill_diagonal(mask, True)
    q = gen.make_problem("alias", 9, rows, rows, rows, mask, mask, b_is_a=True)
    got, _ = run(q, precision=bsm.BF16X3)
    assert rel_fro(got, ref(q)) <= 1e-6


@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32, bsm.BF16X3])
def test_k_window_bitwise_invariant(precision):
    """Issuing the k-iterations I at a time (I = 1, 2, 3, K) gives the same bits."""
    p = gen.random_problem(800 + precision, 7, 9, 6, 8, 150, 0.6, 0.6)
    base, plan = run(p, precision=precision)
    assert plan.info().k_windows == 1
    for I in (1, 2, 3, p.K):
        got, pl = run(p, precision=precision, k_window=I)
        assert pl.info().k_windows == -(-p.K // I)
        assert np.array_equal(got, base), I
    # with accumulation and alpha
    C0 = np.random.default_rng(4).standard_normal(base.size)
    a, _ = run(p, precision=precision, alpha=0.75, C0=C0)
    b, _ = run(p, precision=precision, alpha=0.75, C0=C0, k_window=2)
    assert np.array_equal(a, b)


def test_timings_recorded():
    p = gen.random_problem(900, 6, 6, 6, 16, 200, 0.6, 0.6)
    got, plan = run(p, record_timings=1)
    feats, secs = plan.timings()
    n = plan.info().tasks
    assert feats.shape == (n, 5) and secs.shape == (n,)
    assert np.all(secs > 0) and np.all(secs < 1.0)
    assert np.all(np.isfinite(feats))
    assert rel_fro(got, ref(p)) <= 1e-12
    # the plan without timings refuses
    _, plan2 = run(p)
    with pytest.raises(bsm.BsmError) as ei:
        plan2.timings()
    assert ei.value.code == bsm.E_STATE


@pytest.mark.parametrize("tile", range(1, len(bsm.tile_variants(bsm.BF16X3)) + 1))
def test_bf16x3_every_tile_variant(tile):
    """Every split-bf16 tile variant: integers bit-exact, random values within the gate, also with
    k-windows (resumed partial sums) and ragged sizes."""
    _say(f"[bf16x3 variant] tile={tile}")
    q = gen.integer_problem(1800 + tile, 6, 7, 5, 1, 200, 0.6, 0.6)
    got, plan = run(q, precision=bsm.BF16X3, tile=tile)
    assert plan.info().tile == tile
    assert np.array_equal(got, ref(q))
    p = gen.random_problem(1810 + tile, 8, 9, 7, 1, 260, 0.5, 0.5)
    got, plan = run(p, precision=bsm.BF16X3, tile=tile)
    plan.verify()
    assert rel_fro(got, ref(p)) <= 1e-6
    got2, plan2 = run(p, precision=bsm.BF16X3, tile=tile, k_window=3)
    plan2.verify()
    assert np.array_equal(got, got2)
