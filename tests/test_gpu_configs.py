"""Parity at full size, in the launch setups the benchmark times, on sampled C blocks the oracle
computes one by one: the 64-product batch (one graph launch, autotuned size classes), the
N=32768 precision workload in all three forms (graph replay), and the 4000-point distance-decay
product (k-lists built on the device, per-class tiles).

Gates: relative Frobenius error over the sampled blocks <= 1e-12 (FP64), 1e-5 (FP32), 1e-6
(split-bf16); the sampled blocks must be present in C and the C-shape must be the boolean product
(checked on the sampled rows)."""
import gc
import sys

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import bsm, gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sampled_err(p, got, off, sel, B_bits=None):
    blocks, pres = oracle.bsmm_blocks(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data,
                                      p.b_data, sel)
    num = den = 0.0
    for (i, j), blk, pr in zip(sel, blocks, pres):
        assert pr and off[i, j] >= 0
        g = got[int(off[i, j]):int(off[i, j]) + blk.size].reshape(blk.shape)
        num += float(np.sum((g - blk) ** 2))
        den += float(np.sum(blk ** 2))
    return (num / den) ** 0.5


def _pick(off, n, seed):
    present = np.argwhere(off >= 0)
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in present[q]) for q in rng.choice(len(present), min(n, len(present)), replace=False)]


def _shape_rows(p, plan, rows):
    """The C-shape on a few block rows equals the boolean product of the shapes."""
    cm = gen.unpack_bits(plan.c_shape(), p.M, p.N)
    for i in rows:
        want = (p.a_mask[i].astype(np.int64) @ p.b_mask.astype(np.int64)) > 0
        assert np.array_equal(cm[i], want)


def test_batch64_sampled():
    probs = gen.batch64()
    _say(f"[batch64] {len(probs)} products")
    plans = [bsm.Plan.from_problem(p) for p in probs]
    batch = bsm.Batch(plans)
    As, Bs, Cs = [], [], []
    for p, pl in zip(probs, plans):
        A = torch.from_numpy(p.a_data).to(DEV)
        As.append(A)
        Bs.append(A if p.b_is_a else torch.from_numpy(p.b_data).to(DEV))
        Cs.append(torch.full((max(1, pl.info().c_elems),), float("nan"), dtype=torch.float64, device=DEV))
    batch.autotune(As, Bs, Cs)
    batch.execute(As, Bs, Cs)
    batch.verify()
    torch.cuda.synchronize()
    worst = 0.0
    for q, (p, pl, C) in enumerate(zip(probs, plans, Cs)):
        off = pl.c_offsets()
        got = C.cpu().numpy()[:pl.info().c_elems]
        assert np.all(np.isfinite(got))
        worst = max(worst, _sampled_err(p, got, off, _pick(off, 3, q)))
    _say(f"[batch64] worst sampled relative error {worst:.3g}")
    assert worst <= 1e-12


@pytest.mark.parametrize("precision,gate", [(bsm.FP64, 1e-12), (bsm.FP32, 1e-5), (bsm.BF16X3, 1e-6)])
def test_precision_32768_sampled(precision, gate):
    p = gen.precision_32768()
    plan = bsm.Plan.from_problem(p, precision=precision, use_graph=1)
    info = plan.info()
    _say(f"[precision_32768] precision={precision} tasks={info.tasks}")
    A = torch.from_numpy(p.a_data).to(DEV)
    B = torch.from_numpy(p.b_data).to(DEV)
    C = torch.full((info.c_elems,), float("nan"), dtype=torch.float64, device=DEV)
    for _ in range(2):  # capture, then a replay
        plan.execute(A, B, C)
    plan.verify()
    torch.cuda.synchronize()
    off = plan.c_offsets()
    got = C.cpu().numpy()
    del A, B, C
    torch.cuda.empty_cache()
    _shape_rows(p, plan, [0, p.M // 2, p.M - 1])
    err = _sampled_err(p, got, off, _pick(off, 16, 100 + precision))
    _say(f"[precision_32768] sampled relative error {err:.3g}")
    assert err <= gate


def test_decay_cloud_4000_sampled():
    """The full 4000-point product (1.04 PFLOP, k-lists built on the device batch by batch), one
    launch per batch as the benchmark runs it."""
    p = gen.decay_cloud()
    plan = bsm.Plan.from_problem(p)
    plan.set_tile_classes([4, 3, 1, 1])
    info = plan.info()
    assert info.device_klists == 1
    _say(f"[decay 4000] C blocks {info.c_blocks}, triples {info.triples}")
    A = torch.from_numpy(p.a_data).to(DEV)
    C = torch.full((info.c_elems,), float("nan"), dtype=torch.float64, device=DEV)
    plan.execute(A, A, C)
    plan.verify()
    torch.cuda.synchronize()
    off = plan.c_offsets()
    sel = _pick(off, 24, 4000)
    got = np.concatenate([C[int(off[i, j]):int(off[i, j]) + int(p.rows[i] * p.cols[j])].cpu().numpy()
                          for i, j in sel])
    del A, C
    gc.collect()
    torch.cuda.empty_cache()
    blocks, pres = oracle.bsmm_blocks(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data,
                                      p.b_data, sel)
    num = den = 0.0
    pos = 0
    for blk, pr in zip(blocks, pres):
        assert pr
        g = got[pos:pos + blk.size].reshape(blk.shape)
        pos += blk.size
        num += float(np.sum((g - blk) ** 2))
        den += float(np.sum(blk ** 2))
    err = (num / den) ** 0.5
    _say(f"[decay 4000] sampled relative error {err:.3g}")
    assert err <= 1e-12
