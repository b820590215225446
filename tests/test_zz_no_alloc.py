"""The allocation-free entry point (bsm_execute_static) against bsm_execute, through the C ABI:
the same kernels and task order, so C must agree bit for bit; two calls in a row on one stream,
the second on a smaller problem, share the static scratch."""
import sys

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import bsm, gen
from tests.helpers import rel_fro

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _operands(p, info, out_f32, C0=None):
    A = torch.from_numpy(p.a_data).to(DEV)
    B = A if p.b_is_a else torch.from_numpy(p.b_data).to(DEV)
    dt = torch.float32 if out_f32 else torch.float64
    C = (torch.full((max(1, info.c_elems),), float("nan"), dtype=dt, device=DEV) if C0 is None
         else torch.from_numpy(C0.copy()).to(DEV))
    return A, B, C


def _call(fn, plan, A, B, C, alpha, accumulate):
    L = bsm.load()
    st = fn(plan.handle, alpha, A.data_ptr(), B.data_ptr(), C.data_ptr(), int(accumulate),
            torch.cuda.current_stream().cuda_stream)
    assert st == bsm.OK, L.bsm_last_error().decode()


@pytest.mark.parametrize("precision,k_window,out", [
    (bsm.FP64, 0, bsm.OUT_F64), (bsm.FP32, 0, bsm.OUT_F64), (bsm.BF16X3, 0, bsm.OUT_F64),
    (bsm.FP64, 2, bsm.OUT_F64), (bsm.BF16X3, 3, bsm.OUT_F32), (bsm.FP32, 2, bsm.OUT_F32),
])
def test_static_entry_matches_execute(precision, k_window, out):
    print(f"[static] precision={precision} k_window={k_window} out={out}", flush=True)
    L = bsm.load()
    big = gen.random_problem(2100 + precision, 9, 10, 8, 1, 220, 0.5, 0.5)
    small = gen.random_problem(2200 + precision, 3, 4, 3, 1, 60, 0.7, 0.7)
    plans, want, bufs = [], [], []
    for p in (big, small):
        plan = bsm.Plan.from_problem(p, precision=precision, k_window=k_window, out=out)
        info = plan.info()
        C0 = np.random.default_rng(5).standard_normal(info.c_elems).astype(
            np.float32 if out == bsm.OUT_F32 else np.float64)
        A, B, C = _operands(p, info, out == bsm.OUT_F32, C0)
        _call(L.bsm_execute, plan, A, B, C, -0.5, True)
        torch.cuda.synchronize()
        want.append(C.cpu().numpy()[:info.c_elems].copy())
        A2, B2, C2 = _operands(p, info, out == bsm.OUT_F32, C0)
        plans.append(plan)
        bufs.append((A2, B2, C2))
    # two calls in a row on one stream, the second on the smaller problem; no wait in between
    for plan, (A2, B2, C2) in zip(plans, bufs):
        _call(L.bsm_execute_static, plan, A2, B2, C2, -0.5, True)
    torch.cuda.synchronize()
    for plan, (_, _, C2), w, p in zip(plans, bufs, want, (big, small)):
        got = C2.cpu().numpy()[:plan.info().c_elems]
        assert np.array_equal(got, w)
    # and the FP64 result is the oracle's within the FP64 gate
    if precision == bsm.FP64 and out == bsm.OUT_F64:
        p = small
        C0 = np.random.default_rng(5).standard_normal(plans[1].info().c_elems)
        ref = oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data, -0.5, C=C0)
        assert rel_fro(want[1], ref) <= 1e-12


def test_static_entry_aliased_operands_repeated():
    """C = A A through the static entry, called three times on one stream; every result equals
    bsm_execute's."""
    rows = np.array([10, 25, 40, 60, 25])
    mask = np.random.default_rng(8).random((5, 5)) < 0.6
    np.fill_diagonal(mask, True)
    p = gen.make_problem("alias", 8, rows, rows, rows, mask, mask, b_is_a=True)
    L = bsm.load()
    for precision in (bsm.FP64, bsm.FP32, bsm.BF16X3):
        plan = bsm.Plan.from_problem(p, precision=precision)
        info = plan.info()
        A, B, C = _operands(p, info, False)
        _call(L.bsm_execute, plan, A, B, C, 1.0, False)
        torch.cuda.synchronize()
        want = C.cpu().numpy()[:info.c_elems].copy()
        outs = [torch.full_like(C, float("nan")) for _ in range(3)]
        for Cq in outs:
            _call(L.bsm_execute_static, plan, A, B, Cq, 1.0, False)
        torch.cuda.synchronize()
        for Cq in outs:
            assert np.array_equal(Cq.cpu().numpy()[:info.c_elems], want)
