"""The learned task cost model: GPU forward/backward/Adam against the CPU oracle, training,
persistence, and what the trained model gains over the flop-count model."""
import sys

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import bsm, gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"
F, H = bsm.MLP_IN, bsm.MLP_HIDDEN


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(bsm.mlp_param_count()) * scale).astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def test_forward_matches_oracle():
    p = _params(1)
    X = np.random.default_rng(2).standard_normal((1000, F)).astype(np.float32)
    y = torch.zeros(1000, dtype=torch.float32, device=DEV)
    bsm.mlp_forward(_dev(p), _dev(X), y)
    torch.cuda.synchronize()
    ref = oracle.mlp_forward(F, H, H, p.astype(np.float64), X.astype(np.float64))
    got = y.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 1e-4 * (1 + np.abs(ref)))


@pytest.mark.parametrize("n", [1, 255, 256, 257, 3000])
def test_loss_and_gradient_match_oracle(n):
    p = _params(3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((n, F)).astype(np.float32)
    T = rng.standard_normal(n).astype(np.float32)
    g = torch.zeros(p.size, dtype=torch.float32, device=DEV)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    bsm.mlp_loss_grad(_dev(p), _dev(X), _dev(T), g, loss)
    ref_loss, ref_g = oracle.mlp_loss_grad(F, H, H, p.astype(np.float64), X.astype(np.float64),
                                           T.astype(np.float64))
    got = g.cpu().numpy()
    assert abs(float(loss.item()) - ref_loss) <= 1e-4 * ref_loss
    assert np.linalg.norm(got - ref_g) <= 1e-4 * np.linalg.norm(ref_g)
    assert np.all(np.abs(got - ref_g) <= 1e-4 * (np.abs(ref_g) + np.abs(ref_g).max() * 1e-2))


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(5)
    P = bsm.mlp_param_count()
    p, g = rng.standard_normal(P), rng.standard_normal(P) * 0.1
    m, v = rng.standard_normal(P) * 0.01, np.abs(rng.standard_normal(P)) * 0.01
    dp, dg, dm, dv = _dev(p), _dev(g), _dev(m), _dev(v)
    bsm.adam_step(dp, dg, dm, dv, step=3, lr=1e-2)
    torch.cuda.synchronize()
    pr, mr, vr = p.astype(np.float32).astype(np.float64), m.astype(np.float32).astype(np.float64), v.astype(np.float32).astype(np.float64)
    oracle.adam_step(pr, g.astype(np.float32).astype(np.float64), mr, vr, 3, lr=1e-2)
    assert np.allclose(dp.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)
    assert np.allclose(dm.cpu().numpy(), mr, rtol=1e-5, atol=1e-7)
    assert np.allclose(dv.cpu().numpy(), vr, rtol=1e-5, atol=1e-9)


def _smooth_target(X):
    return (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3 * X[:, 3] + 0.1 * X[:, 4]).astype(np.float32)


def test_training_reduces_loss_is_deterministic_and_persists(tmp_path):
    rng = np.random.default_rng(6)
    X = rng.standard_normal((4000, F)).astype(np.float32) * 2 + 3
    T = _smooth_target(X)
    a = bsm.CostModel(seed=11)
    b = bsm.CostModel(seed=11)
    la = a.train(X, T, epochs=60, batch=512, lr=3e-3)
    lb = b.train(X, T, epochs=60, batch=512, lr=3e-3)
    pa, na = a.params()
    pb, nb = b.params()
    assert np.array_equal(pa, pb) and np.array_equal(na, nb) and la == lb   # deterministic
    assert la < 0.05   # standardised units: the untrained network starts near 1
    pred = a.predict(X)
    assert np.mean((pred - T) ** 2) / np.var(T) < 0.05
    # the prediction is the oracle network on standardised inputs, de-standardised
    Xs = (X - na[:5]) / na[5:10]
    ref = oracle.mlp_forward(F, H, H, pa.astype(np.float64), Xs.astype(np.float64)) * na[11] + na[10]
    assert np.all(np.abs(pred - ref) <= 1e-4 * (1 + np.abs(ref)))
    path = str(tmp_path / "m.bin")
    a.save(path)
    c = bsm.CostModel.load_file(path)
    assert np.array_equal(c.predict(X), pred)
    # training resumes from the saved Adam state exactly as it continues in memory
    a.train(X, T, epochs=5, batch=512, lr=3e-3)
    c.train(X, T, epochs=5, batch=512, lr=3e-3)
    assert np.array_equal(a.params()[0], c.params()[0])


def _harvest(plan, A, B, C, reps=3):
    feats, secs = [], []
    for _ in range(reps):
        plan.execute(A, B, C)
        f, t = plan.timings()
        feats.append(f)
        secs.append(t)
    return np.concatenate(feats), np.concatenate(secs)


def test_learned_model_beats_flop_count_model():
    """Trained on the task timings of one distance-decay workload (blocks of 10..60, where flop
    counts mispredict small tasks), the network predicts the task times of a *different* seeded
    workload better than the flop-count model (log t = log flops + c, c fitted on the training
    workload).  Both task orders are then timed interleaved on the second workload; the makespans
    are reported (the full-size measurement is in the decay-cloud profile) and must give the same
    bits."""
    def harvest(seed, reps):
        p = gen.decay_cloud(seed=seed, npts=600, box=36.0)
        plan = bsm.Plan.from_problem(p, record_timings=1)
        plan.set_tile_classes([4, 3, 1, 1])
        A = torch.from_numpy(p.a_data).to(DEV)
        C = torch.zeros(plan.info().c_elems, dtype=torch.float64, device=DEV)
        plan.execute(A, A, C)  # warm-up
        torch.cuda.synchronize()
        X, T = _harvest(plan, A, A, C, reps=reps)
        return p, A, C, X, np.log(np.maximum(T, 1e-7)).astype(np.float32)
    _, _, _, Xtr, Ttr = harvest(5000, 2)
    p, A, C, Xte, Tte = harvest(5002, 1)
    _say(f"[costmodel] train {Ttr.size} tasks (seed 5000), test {Tte.size} tasks (seed 5002)")
    model = bsm.CostModel(seed=1)
    model.train(Xtr, Ttr, epochs=60, batch=2048, lr=3e-3)
    pred = model.predict(Xte)
    lf_tr = Xtr[:, 0] + Xtr[:, 1] + Xtr[:, 2]
    lf_te = Xte[:, 0] + Xte[:, 1] + Xte[:, 2]
    c = float(np.mean(Ttr - lf_tr))
    err_mlp = float(np.mean(np.abs(pred - Tte)))
    err_flop = float(np.mean(np.abs(lf_te + c - Tte)))
    _say(f"[costmodel] other workload, mean |log error|: MLP {err_mlp:.3f}  flop-count {err_flop:.3f}")
    assert err_mlp < 0.5 * err_flop
    # both orders on the second workload, interleaved
    plan_f = bsm.Plan.from_problem(p)
    plan_f.set_tile_classes([4, 3, 1, 1])
    plan_l = bsm.Plan.from_problem(p)
    plan_l.set_tile_classes([4, 3, 1, 1])
    plan_l.set_costmodel(model)
    times = {"flop": [], "learned": []}
    outs = {}
    for pl in (plan_f, plan_l):
        pl.execute(A, A, C)
    for _ in range(3):
        for name, pl in (("flop", plan_f), ("learned", plan_l)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pl.execute(A, A, C)
            e1.record()
            torch.cuda.synchronize()
            times[name].append(e0.elapsed_time(e1))
            outs[name] = C.cpu().numpy().copy()
    assert np.array_equal(outs["flop"], outs["learned"])
    tf, tl = np.array(times["flop"]), np.array(times["learned"])
    _say(f"[costmodel] makespan flop-count {tf.mean():.2f} +- {tf.std(ddof=1):.2f} ms, "
         f"learned {tl.mean():.2f} +- {tl.std(ddof=1):.2f} ms")


def _wide(seed):
    """Nonuniform blocks of very uneven size (U{4..512}, N=3072, density 0.6): few hundred tasks,
    where the tail of the schedule decides the makespan and flop counts mispredict small tiles."""
    return gen.nonuniform(seed, 3072, 4, 512, 0.6, name=f"wide{seed}")


def test_learned_model_makespan_on_uneven_tasks_is_recorded():
    """Trained on the recorded task times of one seeded workload, the network's costs drive the
    largest-first (LPT) deal of another seed's tasks; the makespans of both cost models are
    recorded with their noise.  Both schedules give the same bits, and the learned one is never
    much slower.  (Measured so far: between 5 % faster and 0.3 % slower depending on the seeds,
    so no gain is asserted.)"""
    ptr = _wide(12100)
    plan = bsm.Plan.from_problem(ptr, record_timings=1)
    A = torch.from_numpy(ptr.a_data).to(DEV)
    B = torch.from_numpy(ptr.b_data).to(DEV)
    C = torch.zeros(plan.info().c_elems, dtype=torch.float64, device=DEV)
    plan.execute(A, B, C)
    torch.cuda.synchronize()
    X, T = _harvest(plan, A, B, C, reps=3)
    model = bsm.CostModel(seed=1)
    model.train(X, np.log(np.maximum(T, 1e-7)).astype(np.float32), epochs=80, batch=1024, lr=3e-3)
    p = _wide(12101)
    A = torch.from_numpy(p.a_data).to(DEV)
    B = torch.from_numpy(p.b_data).to(DEV)
    plan_f = bsm.Plan.from_problem(p, order=bsm.ORDER_LPT, use_graph=1)
    plan_l = bsm.Plan.from_problem(p, order=bsm.ORDER_LPT, use_graph=1)
    plan_l.set_costmodel(model)
    C = torch.zeros(plan_f.info().c_elems, dtype=torch.float64, device=DEV)
    for pl in (plan_f, plan_l, plan_f, plan_l):
        pl.execute(A, B, C)
    torch.cuda.synchronize()
    times = {"flop": [], "learned": []}
    outs = {}
    for _ in range(30):
        for name, pl in (("flop", plan_f), ("learned", plan_l)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pl.execute(A, B, C)
            e1.record()
            torch.cuda.synchronize()
            times[name].append(e0.elapsed_time(e1))
    for name, pl in (("flop", plan_f), ("learned", plan_l)):
        pl.execute(A, B, C)
        torch.cuda.synchronize()
        outs[name] = C.cpu().numpy().copy()
    assert np.array_equal(outs["flop"], outs["learned"])
    tf, tl = np.array(times["flop"]), np.array(times["learned"])
    se = float(np.std(tl - tf, ddof=1) / np.sqrt(tf.size))
    _say(f"[costmodel] uneven tasks ({plan_f.info().tasks}), LPT deal: flop-count costs "
         f"{tf.mean():.4f} ms, learned costs {tl.mean():.4f} ms (difference {tl.mean() - tf.mean():+.4f} "
         f"+- {se:.4f} ms)")
    assert tl.mean() < 1.05 * tf.mean()
