"""Batches of independent products in one graph-captured launch, graph replay, autotuning and
cost-driven rescheduling, against the oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import bsm, gen
from tests.helpers import rel_fro

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small_batch(seed, count=6):
    out = []
    for b in range(count):
        rng = np.random.default_rng(seed * 100 + b)
        n = int(rng.choice([256, 512, 1024]))
        out.append(gen.nonuniform(seed * 100 + b, n, 16, 192, float(rng.uniform(0.1, 0.9)),
                                  name=f"b{b}_{n}"))
    return out


def ref(p, alpha=1.0, C0=None):
    return oracle.bsmm(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits(), p.a_data, p.b_data, alpha, C=C0)


def operands(probs, plans):
    As = [torch.from_numpy(p.a_data).to(DEV) for p in probs]
    Bs = [a if p.b_is_a else torch.from_numpy(p.b_data).to(DEV) for p, a in zip(probs, As)]
    Cs = [torch.full((max(1, pl.info().c_elems),), float("nan"), dtype=torch.float64, device=DEV)
          for pl in plans]
    return As, Bs, Cs


def host(C, plan):
    return C.cpu().numpy()[:plan.info().c_elems]


@pytest.mark.parametrize("precision,gate", [(bsm.FP64, 1e-12), (bsm.FP32, 1e-5), (bsm.BF16X3, 1e-6)])
def test_batch_matches_oracle_and_single_runs(precision, gate):
    probs = small_batch(3 + precision)
    plans = [bsm.Plan.from_problem(p, precision=precision) for p in probs]
    batch = bsm.Batch(plans)
    As, Bs, Cs = operands(probs, plans)
    alphas = [1.0, -0.5, 2.0, 0.25, 1.0, 3.0]
    _say(f"[batch] precision={precision} tasks={batch.query()[0]}")
    batch.execute(As, Bs, Cs, alphas=alphas)
    torch.cuda.synchronize()
    got = [host(C, pl) for C, pl in zip(Cs, plans)]
    for p, g, al in zip(probs, got, alphas):
        assert rel_fro(g, ref(p, al)) <= gate, p.name
    # each member alone gives the same bits (a task's arithmetic does not depend on the schedule)
    for p, pl, A, B, g, al in zip(probs, plans, As, Bs, got, alphas):
        C1 = torch.full((max(1, pl.info().c_elems),), float("nan"), dtype=torch.float64, device=DEV)
        pl.execute(A, B, C1, alpha=al)
        torch.cuda.synchronize()
        assert np.array_equal(host(C1, pl), g)


def test_batch_graph_replays_with_eager_work_between():
    probs = small_batch(11)
    plans = [bsm.Plan.from_problem(p) for p in probs]
    batch = bsm.Batch(plans)
    As, Bs, Cs = operands(probs, plans)
    batch.execute(As, Bs, Cs)
    torch.cuda.synchronize()
    first = [host(C, pl).copy() for C, pl in zip(Cs, plans)]
    for rep in range(4):
        for C in Cs:
            C.zero_()                      # eager work between replays
        x = torch.randn(1 << 16, device=DEV).sum()
        torch.cuda.synchronize()
        batch.execute(As, Bs, Cs)          # graph replay (same operands)
        torch.cuda.synchronize()
        for C, pl, f in zip(Cs, plans, first):
            assert np.array_equal(host(C, pl), f), rep
        del x
    # accumulate into the previous result: C = AB + C = 2 AB exactly
    batch.execute(As, Bs, Cs, accumulate=True)
    torch.cuda.synchronize()
    for C, pl, f in zip(Cs, plans, first):
        assert np.array_equal(host(C, pl), 2.0 * f)
    # new output buffers force a new capture
    Cs2 = [torch.empty_like(C) for C in Cs]
    batch.execute(As, Bs, Cs2)
    torch.cuda.synchronize()
    for C, pl, f in zip(Cs2, plans, first):
        assert np.array_equal(host(C, pl), f)


def test_single_plan_graph_mode_bitwise_equal():
    p = gen.random_problem(1200, 8, 8, 8, 16, 200, 0.5, 0.5)
    plain = bsm.Plan.from_problem(p)
    graphed = bsm.Plan.from_problem(p, use_graph=1)
    A = torch.from_numpy(p.a_data).to(DEV)
    B = torch.from_numpy(p.b_data).to(DEV)
    C1 = torch.zeros(plain.info().c_elems, dtype=torch.float64, device=DEV)
    C2 = torch.zeros_like(C1)
    plain.execute(A, B, C1)
    for rep in range(3):
        C2.fill_(float("nan"))
        graphed.execute(A, B, C2)
        torch.cuda.synchronize()
        assert np.array_equal(C1.cpu().numpy(), C2.cpu().numpy()), rep


def test_costs_reschedule_without_changing_bits():
    p = gen.random_problem(1300, 9, 9, 9, 16, 220, 0.5, 0.5)
    plan = bsm.Plan.from_problem(p)
    A = torch.from_numpy(p.a_data).to(DEV)
    B = torch.from_numpy(p.b_data).to(DEV)
    C = torch.zeros(plan.info().c_elems, dtype=torch.float64, device=DEV)
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    base = C.cpu().numpy().copy()
    rng = np.random.default_rng(0)
    for _ in range(3):
        plan.set_costs(rng.random(plan.info().tasks).astype(np.float32) * 10)
        C.fill_(float("nan"))
        plan.execute(A, B, C)
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy(), base)


def test_autotune_picks_a_variant_and_stays_correct(tmp_path):
    cache = str(tmp_path / "tune.txt")
    probs = small_batch(21, count=4)
    plans = [bsm.Plan.from_problem(p, tune_cache=cache) for p in probs]
    batch = bsm.Batch(plans)
    As, Bs, Cs = operands(probs, plans)
    v = batch.autotune(As, Bs, Cs)
    assert 0 <= v <= len(bsm.tile_variants())
    assert batch.query()[2] == v
    classes = batch.tile_classes()
    assert all(1 <= c <= len(bsm.tile_variants()) for c in classes)
    _say(f"[autotune] batch class variants {classes}")
    batch.execute(As, Bs, Cs)
    batch.verify()
    for p, C, pl in zip(probs, Cs, plans):
        assert rel_fro(host(C, pl), ref(p)) <= 1e-12
    # the choice was cached: a second tune returns it without timing
    line = (tmp_path / "tune.txt").read_text().strip().splitlines()[-1]
    assert line.endswith(",".join(str(c - 1) for c in classes))
    assert batch.autotune(As, Bs, Cs) == v and batch.tile_classes() == classes
    # single-plan autotune
    p = probs[0]
    plan = bsm.Plan.from_problem(p, tune_cache=cache)
    C = torch.zeros(plan.info().c_elems, dtype=torch.float64, device=DEV)
    w = plan.autotune(As[0], Bs[0], C)
    assert plan.info().tile == w
    plan.execute(As[0], Bs[0], C)
    plan.verify()
    assert rel_fro(C.cpu().numpy(), ref(p)) <= 1e-12


@pytest.mark.parametrize("precision,gate", [(bsm.FP64, 1e-12), (bsm.FP32, 1e-5)])
def test_mixed_variants_in_one_launch(precision, gate):
    """Members cut with different tile variants run in one graph launch (one kernel per variant);
    each product matches the oracle and its own single run bit for bit."""
    probs = small_batch(41 + precision, count=4)
    plans = [bsm.Plan.from_problem(p, precision=precision, tile=1 + q % len(bsm.tile_variants()))
             for q, p in enumerate(probs)]
    batch = bsm.Batch(plans)
    assert batch.query()[2] == 0
    As, Bs, Cs = operands(probs, plans)
    batch.execute(As, Bs, Cs)
    batch.verify()
    for p, pl, A, B, C in zip(probs, plans, As, Bs, Cs):
        g = host(C, pl)
        assert rel_fro(g, ref(p)) <= gate
        C1 = torch.full_like(C, float("nan"))
        pl.execute(A, B, C1)
        torch.cuda.synchronize()
        assert np.array_equal(host(C1, pl), g)


def test_batch_timings():
    probs = small_batch(31, count=3)
    plans = [bsm.Plan.from_problem(p, record_timings=1) for p in probs]
    batch = bsm.Batch(plans)
    As, Bs, Cs = operands(probs, plans)
    batch.execute(As, Bs, Cs)
    f, t = batch.timings()
    assert f.shape == (batch.query()[0], 5)
    assert np.all(t > 0)


def test_fp64_plan_twice_in_a_batch():
    """An FP64 plan may stand for two products of one batch (same structure, different operands)."""
    p = gen.random_problem(1400, 6, 6, 6, 16, 180, 0.5, 0.5)
    q = gen.random_problem(1400, 6, 6, 6, 16, 180, 0.5, 0.5, draw=lambda rng, i, j, h, w: rng.uniform(-2, 2, (h, w)))
    plan = bsm.Plan.from_problem(p)
    batch = bsm.Batch([plan, plan])
    As, Bs, Cs = operands([p, q], [plan, plan])
    batch.execute(As, Bs, Cs, alphas=[1.0, -2.0])
    batch.verify()
    assert rel_fro(host(Cs[0], plan), ref(p)) <= 1e-12
    assert rel_fro(host(Cs[1], plan), ref(q, -2.0)) <= 1e-12
