"""The C ABI without a GPU: the library loads and exports every declared function, and the
host-side planning (validation, C-shape, packing, counts) agrees with the oracle."""
import ctypes
import os

import numpy as np
import pytest

import oracle
from paper_1504_05046_amd import bsm, gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_library_exports_every_declared_symbol():
    L = bsm.load()
    names = bsm.declared_symbols()
    assert "bsm_plan_create" in names and "bsm_execute" in names
    for n in names:
        assert hasattr(L, n), n


def _problems():
    yield gen.random_problem(1, 5, 7, 6, 1, 40, 0.4, 0.5)
    yield gen.random_problem(2, 1, 1, 1, 1, 3, 1.0, 1.0)
    yield gen.random_problem(3, 9, 70, 3, 1, 9, 0.05, 0.3)   # inner shape wider than one word
    yield gen.random_problem(4, 66, 3, 130, 1, 5, 0.5, 0.2)
    yield gen.uniform_1024()


@pytest.mark.parametrize("p", list(_problems()), ids=lambda p: p.name)
def test_plan_matches_oracle_shape_and_layout(p):
    plan = bsm.Plan.from_problem(p)
    info = plan.info()
    c_bits = oracle.shape_product(p.M, p.K, p.N, p.a_bits(), p.b_bits())
    assert np.array_equal(plan.c_shape(), c_bits)
    off, total = oracle.block_offsets(p.rows, p.cols, c_bits)
    assert np.array_equal(plan.c_offsets(), off)
    assert info.c_elems == total
    assert info.a_elems == p.a_data.size and info.b_elems == p.b_data.size
    assert info.a_blocks == int(p.a_mask.sum()) and info.b_blocks == int(p.b_mask.sum())
    assert info.c_blocks == int(gen.unpack_bits(c_bits, p.M, p.N).sum())
    assert info.useful_flops == oracle.useful_flops(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits())
    assert info.triples == int((p.a_mask.astype(np.int64) @ p.b_mask.astype(np.int64)).sum())
    assert info.tasks >= info.c_blocks
    plan.close()


def test_tasks_cover_each_c_block_once():
    """Sub-tiles partition every C block: the task count equals the sum over C blocks of the
    number of pieces the cutting rule gives (at most 128 rows/cols, multiples of 16)."""
    p = gen.random_problem(7, 6, 4, 5, 1, 300, 0.6, 0.6)
    info = bsm.Plan.from_problem(p).info()
    c_mask = gen.unpack_bits(oracle.shape_product(p.M, p.K, p.N, p.a_bits(), p.b_bits()), p.M, p.N)
    pieces = lambda m: -(-(-(-m // 16)) // 8)
    want = sum(pieces(int(p.rows[i])) * pieces(int(p.cols[j])) for i, j in zip(*np.nonzero(c_mask)))
    assert info.tasks == want


def test_empty_and_degenerate_plans():
    # no blocks at all
    plan = bsm.Plan([], [], [], [], [])
    i = plan.info()
    assert (i.M, i.K, i.N, i.c_elems, i.tasks) == (0, 0, 0, 0, 0)
    # all-absent shapes: C empty
    p = gen.make_problem("none", 0, [3, 4], [5], [2, 2], np.zeros((2, 1), bool), np.zeros((1, 2), bool))
    i = bsm.Plan.from_problem(p).info()
    assert i.c_blocks == 0 and i.tasks == 0 and i.useful_flops == 0
    # K = 0: nothing to contract, C-shape empty
    p = gen.make_problem("k0", 0, [3], [], [2], np.zeros((1, 0), bool), np.zeros((0, 1), bool))
    assert bsm.Plan.from_problem(p).info().c_blocks == 0


def _expect(code, fn):
    with pytest.raises(bsm.BsmError) as ei:
        fn()
    assert ei.value.code == code
    return str(ei.value)


def test_invalid_inputs_rejected():
    ok_bits = gen.pack_bits(np.ones((1, 1), bool))
    msg = _expect(bsm.E_INVALID, lambda: bsm.Plan([0], [1], [1], ok_bits, ok_bits))
    assert "row_sizes" in msg
    _expect(bsm.E_INVALID, lambda: bsm.Plan([1], [70000], [1], ok_bits, ok_bits))
    _expect(bsm.E_INVALID, lambda: bsm.Plan([1], [1], [-3], ok_bits, ok_bits))
    # stray padding bit in a 1-column shape
    bad = np.array([3], dtype=np.uint64)
    msg = _expect(bsm.E_INVALID, lambda: bsm.Plan([1], [1], [1], bad, ok_bits))
    assert "padding" in msg
    _expect(bsm.E_INVALID, lambda: bsm.Plan([1], [1], [1], ok_bits, bad))
    L = bsm.load()
    h = ctypes.c_void_p()
    rows = np.array([1], np.int64)
    assert L.bsm_plan_create(ctypes.byref(h), 1, None, 1, rows.ctypes.data, 1, rows.ctypes.data,
                             ok_bits.ctypes.data, ok_bits.ctypes.data, None) == bsm.E_INVALID
    assert L.bsm_plan_create(None, 1, rows.ctypes.data, 1, rows.ctypes.data, 1, rows.ctypes.data,
                             ok_bits.ctypes.data, ok_bits.ctypes.data, None) == bsm.E_INVALID
    assert L.bsm_plan_query(None, None) == bsm.E_INVALID
    _expect(bsm.E_INVALID, lambda: bsm.Plan([1], [1], [1], ok_bits, ok_bits, k_window=-1))
    _expect(bsm.E_INVALID, lambda: bsm.Plan([1], [1], [1], ok_bits, ok_bits, precision=7))


def test_block_size_limit_is_exact():
    """Block sizes up to 65535 (16-bit task fields) are accepted on every dimension, 65536 is not."""
    ok_bits = gen.pack_bits(np.ones((1, 1), bool))
    for rows, inner, cols in (([65535], [1], [1]), ([1], [65535], [1]), ([1], [1], [65535])):
        plan = bsm.Plan(rows, inner, cols, ok_bits, ok_bits)
        info = plan.info()
        assert info.c_blocks == 1 and info.useful_flops == 2.0 * 65535
        plan.close()
    for rows, inner, cols in (([65536], [1], [1]), ([1], [65536], [1]), ([1], [1], [65536])):
        msg = _expect(bsm.E_INVALID, lambda: bsm.Plan(rows, inner, cols, ok_bits, ok_bits))
        assert "65535" in msg


def test_execute_argument_errors_need_no_device():
    p = gen.random_problem(8, 2, 2, 2, 2, 4, 1.0, 1.0)
    plan = bsm.Plan.from_problem(p)
    L = bsm.load()
    # null C
    assert L.bsm_execute(plan.handle, 1.0, 16, 4096, None, 0, None) == bsm.E_INVALID
    info = plan.info()
    # C overlapping A
    assert L.bsm_execute(plan.handle, 1.0, 4096, 1 << 30, 4096 + 8, 0, None) == bsm.E_INVALID
    assert L.bsm_execute(plan.handle, 1.0, 4096, 1 << 30, 1 << 40, 3, None) == bsm.E_INVALID
    assert info.c_elems > 0


def test_eq1_matches_golden_table():
    with open(os.path.join(GOLDEN, "eq1_concurrent_iterations.txt")) as f:
        rows = [list(map(int, ln.split())) for ln in f if ln.strip() and not ln.startswith("#")]
    for prow, pcol, K, want in rows:
        assert bsm.concurrent_iterations(prow, pcol, K) == want


def test_tile_variants_listed():
    v = bsm.tile_variants()
    assert len(v) >= 3
    for tm, tn in v:
        assert tm % 16 == 0 and tn % 16 == 0 and 16 <= tm <= 256 and 16 <= tn <= 256
    p = gen.random_problem(9, 3, 3, 3, 1, 300, 1.0, 1.0)
    for t in range(1, len(v) + 1):
        bsm.Plan.from_problem(p, tile=t).close()
    _expect(bsm.E_INVALID, lambda: bsm.Plan.from_problem(p, tile=len(v) + 1))


def test_destroy_null_is_ok():
    assert bsm.load().bsm_plan_destroy(None) == bsm.OK


def test_batch_rules_checked_on_host():
    p = gen.random_problem(40, 3, 3, 3, 1, 50, 0.8, 0.8)
    q = gen.random_problem(41, 4, 2, 3, 1, 50, 0.8, 0.8)
    a = bsm.Plan.from_problem(p)
    b = bsm.Plan.from_problem(q)
    batch = bsm.Batch([a, b])
    tasks, flops, tile = batch.query()
    assert tasks == a.info().tasks + b.info().tasks
    assert flops == a.info().useful_flops + b.info().useful_flops
    assert tile == a.info().tile
    _expect(bsm.E_MISMATCH, lambda: bsm.Batch([a, bsm.Plan.from_problem(q, precision=bsm.FP32)]))
    _expect(bsm.E_MISMATCH, lambda: bsm.Batch([a, bsm.Plan.from_problem(q, k_window=1)]))
    # members may use different tile variants: their tasks run in one launch per variant
    mixed = bsm.Batch([a, bsm.Plan.from_problem(q, tile=3)])
    assert mixed.query()[2] == 0 and mixed.query()[0] == tasks - b.info().tasks + bsm.Plan.from_problem(q, tile=3).info().tasks
    L = bsm.load()
    assert L.bsm_batch_create(None, None, 0) == bsm.E_INVALID


def test_set_costs_validation_and_features():
    p = gen.random_problem(42, 4, 4, 4, 1, 200, 0.7, 0.7)
    plan = bsm.Plan.from_problem(p)
    n = plan.info().tasks
    f = plan.features()
    assert f.shape == (n, 5) and np.all(np.isfinite(f))
    # features: log h, log w in [0, log 128]; density in (0, 1]
    assert np.all(f[:, :2] >= 0) and np.all(f[:, :2] <= np.log(128) + 1e-6)
    assert np.all((f[:, 4] > 0) & (f[:, 4] <= 1))
    _expect(bsm.E_MISMATCH, lambda: plan.set_costs(np.ones(n + 1)))
    bad = np.ones(n)
    bad[0] = np.nan
    _expect(bsm.E_INVALID, lambda: plan.set_costs(bad))
    bad[0] = -1
    _expect(bsm.E_INVALID, lambda: plan.set_costs(bad))
    plan.set_costs(np.arange(n, dtype=np.float32))
    assert plan.info().tasks == n


def test_binding_rejects_short_buffers():
    """The binding checks buffer sizes before a pointer reaches the library (no device needed:
    the check happens before any device call)."""
    torch = pytest.importorskip("torch")
    p = gen.random_problem(43, 3, 3, 3, 4, 40, 1.0, 1.0)
    plan = bsm.Plan.from_problem(p)
    info = plan.info()
    A = torch.zeros(info.a_elems, dtype=torch.float64)
    B = torch.zeros(info.b_elems, dtype=torch.float64)
    with pytest.raises(ValueError, match="C holds"):
        plan.execute(A, B, torch.zeros(info.c_elems - 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="float64"):
        plan.execute(A, B, torch.zeros(info.c_elems, dtype=torch.float32))
    with pytest.raises(ValueError, match="A holds"):
        plan.execute(A[:-1], B, torch.zeros(info.c_elems, dtype=torch.float64))
    with pytest.raises(ValueError, match="device"):
        plan.execute(A, B, torch.zeros(info.c_elems, dtype=torch.float64))


def test_costmodel_host_side():
    m = bsm.CostModel(seed=3)
    p, norm = m.params()
    assert p.size == bsm.mlp_param_count() == 32 * 5 + 32 + 32 * 32 + 32 + 32 + 1
    assert np.all(np.isfinite(p)) and np.all(p[32 * 5:32 * 5 + 32] == 0)        # b1 = 0
    assert np.abs(p[:160]).max() <= np.sqrt(6 / 5) + 1e-6                        # He-uniform
    assert list(norm) == [0] * 5 + [1] * 5 + [0, 1]
    q = bsm.CostModel(seed=3).params()[0]
    assert np.array_equal(p, q)                                                  # seeded
    assert not np.array_equal(p, bsm.CostModel(seed=4).params()[0])
    m.set_params(p * 2, np.array([1, 2, 3, 4, 5, 1, 1, 1, 1, 2, 0.5, 3], np.float32))
    p2, n2 = m.params()
    assert np.array_equal(p2, p * 2) and n2[9] == 2 and n2[11] == 3
    _expect(bsm.E_MISMATCH, lambda: m.set_params(p[:-1]))
    _expect(bsm.E_INVALID, lambda: m.set_params(None, np.array([0] * 5 + [0] + [1] * 4 + [0, 1], np.float32)))


def test_reschedule_does_not_depend_on_the_previous_order():
    """Scheduling deals whole C blocks, in C-block order, to the XCDs: costs that differ reorder
    the tasks, and scheduling again by flop count restores the plan's original order."""
    p = gen.random_problem(11, 6, 6, 6, 16, 200, 0.6, 0.6)
    plan = bsm.Plan.from_problem(p)
    f0 = plan.features().copy()
    rng = np.random.default_rng(0)
    plan.set_costs(rng.uniform(1, 10, len(f0)).astype(np.float32))
    f1 = plan.features().copy()
    assert not np.array_equal(f0, f1)
    # the same multiset of tasks either way
    assert np.array_equal(np.sort(f0.view(np.int32), axis=0), np.sort(f1.view(np.int32), axis=0))
    flops = (2 * np.exp(f1[:, :3].astype(np.float64).sum(1))).astype(np.float32)
    plan.set_costs(flops)
    assert np.array_equal(plan.features(), f0)


def test_options_validated():
    ok_bits = gen.pack_bits(np.ones((1, 1), bool))
    _expect(bsm.E_INVALID, lambda: bsm.Plan([1], [1], [1], ok_bits, ok_bits, out=2))
    _expect(bsm.E_INVALID, lambda: bsm.Plan([1], [1], [1], ok_bits, ok_bits, order=9))
    for order in (bsm.ORDER_DEFAULT, bsm.ORDER_INTERLEAVE, bsm.ORDER_LOCALITY, bsm.ORDER_LPT,
                  bsm.ORDER_PATCH):
        bsm.Plan([1], [1], [1], ok_bits, ok_bits, order=order).close()
    bsm.Plan([1], [1], [1], ok_bits, ok_bits, order=bsm.ORDER_PATCH, patch=(2, 16)).close()
    _expect(bsm.E_INVALID, lambda: bsm.Plan([1], [1], [1], ok_bits, ok_bits, order=bsm.ORDER_PATCH, patch=(-1, 2)))
    plan = bsm.Plan([1], [1], [1], ok_bits, ok_bits, out=bsm.OUT_F32, tune_cache="/tmp/x")
    assert plan.info().out == bsm.OUT_F32
    # the binding wants an FP32 C for such a plan
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError, match="float32"):
        plan.execute(torch.zeros(1, dtype=torch.float64), torch.zeros(1, dtype=torch.float64),
                     torch.zeros(1, dtype=torch.float64))


def test_reduced_precision_plan_only_once_per_batch():
    p = gen.random_problem(44, 3, 3, 3, 1, 50, 0.8, 0.8)
    a = bsm.Plan.from_problem(p)
    bsm.Batch([a, a]).close()                 # FP64: each entry is its own product
    for prec in (bsm.FP32, bsm.BF16X3):
        b = bsm.Plan.from_problem(p, precision=prec)
        msg = _expect(bsm.E_INVALID, lambda: bsm.Batch([b, b]))
        assert "repeats" in msg


def test_debug_skip_task_validated():
    p = gen.random_problem(45, 3, 3, 3, 1, 50, 0.8, 0.8)
    plan = bsm.Plan.from_problem(p)
    n = plan.info().tasks
    plan.debug_skip_task(n - 1)
    plan.debug_skip_task(-1)
    _expect(bsm.E_INVALID, lambda: plan.debug_skip_task(n))
    _expect(bsm.E_INVALID, lambda: plan.debug_skip_task(-2))


def test_static_entry_rejects_plans_beyond_its_scratch():
    """bsm_execute_static refuses, before any device work, a plan whose device buffers exceed its
    64 MiB static scratch (here: FP32 copies of two 4096 x 4096 blocks)."""
    bits = gen.pack_bits(np.ones((1, 1), bool))
    plan = bsm.Plan([4096], [4096], [4096], bits, bits, precision=bsm.FP32)
    L = bsm.load()
    st = L.bsm_execute_static(plan.handle, 1.0, 1 << 32, 1 << 36, 1 << 40, 0, None)
    assert st == bsm.E_NOMEM
    assert "64" in L.bsm_last_error().decode() or "67108864" in L.bsm_last_error().decode()
    assert L.bsm_execute_static(None, 1.0, 0, 0, 0, 0, None) == bsm.E_INVALID


def test_size_classes_and_segments():
    """Tile variants per size class: tasks of a class are cut with its variant; a plan whose
    classes use one variant reports it, and the class table reads back."""
    p = gen.random_problem(46, 6, 5, 6, 8, 200, 0.7, 0.7)
    plan = bsm.Plan.from_problem(p, tile=2)
    assert plan.info().tile == 2 and plan.tile_classes() == [2, 2, 2, 2]
    plan = bsm.Plan.from_problem(p)
    assert plan.tile_classes() == [1, 1, 1, 1]
    plan.set_tile_classes([4, 3, 2, 1])
    assert plan.tile_classes() == [4, 3, 2, 1]
    # sizes 8..200 fall in several classes, so the tasks now mix variants
    assert plan.info().tile == 0
    _expect(bsm.E_INVALID, lambda: plan.set_tile_classes([0, 1, 1, 1]))
    _expect(bsm.E_INVALID, lambda: plan.set_tile_classes([1, 1, 1, 5]))


def test_patch_order_keeps_the_task_set():
    """The patch order deals whole rectangles of C blocks; it reorders tasks, never changes them."""
    p = gen.random_problem(47, 9, 6, 11, 8, 200, 0.6, 0.6)
    base = bsm.Plan.from_problem(p).features()
    pat = bsm.Plan.from_problem(p, order=bsm.ORDER_PATCH, patch=(2, 3)).features()
    assert not np.array_equal(base, pat)
    assert np.array_equal(np.sort(base.view(np.int32), axis=0), np.sort(pat.view(np.int32), axis=0))


@pytest.mark.parametrize("dk", [1, 5, 64])
def test_device_klists_plan_matches_host_lists(dk):
    """Planning with k-lists built on the device keeps the C-shape, layout, counts, useful flops and
    the task set of the host-list plan; only the task order (batches) and the triples' home differ."""
    p = gen.random_problem(48, 7, 9, 8, 4, 150, 0.5, 0.5)
    host = bsm.Plan.from_problem(p)
    dev = bsm.Plan.from_problem(p, device_klists=dk)
    hi, di = host.info(), dev.info()
    assert hi.device_klists == 0 and di.device_klists == 1
    for f in ("c_blocks", "c_elems", "triples", "tasks"):
        assert getattr(hi, f) == getattr(di, f), f
    assert hi.useful_flops == di.useful_flops
    assert np.array_equal(host.c_shape(), dev.c_shape())
    assert np.array_equal(host.c_offsets(), dev.c_offsets())
    fh, fd = host.features(), dev.features()
    assert np.array_equal(np.sort(fh.view(np.int32), axis=0), np.sort(fd.view(np.int32), axis=0))
    _expect(bsm.E_INVALID, lambda: bsm.Plan.from_problem(p, device_klists=-2))


def test_device_klists_limits_on_host():
    p = gen.random_problem(49, 3, 3, 3, 1, 30, 0.8, 0.8)
    dev = bsm.Plan.from_problem(p, device_klists=1)
    _expect(bsm.E_UNSUPPORTED, lambda: bsm.Batch([dev]))
    L = bsm.load()
    assert L.bsm_execute_static(dev.handle, 1.0, 1 << 32, 1 << 36, 1 << 40, 0, None) == bsm.E_UNSUPPORTED


@pytest.mark.parametrize("ta,tb", [(1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("precision", [bsm.FP64, bsm.FP32, bsm.BF16X3])
def test_transposed_operand_plans(precision, ta, tb):
    """With an operand stored transposed the plan reads its shape as stored: C's shape, offsets,
    flop count and triples are those of op(A) op(B) (oracle), and the staged copy of a transposed
    FP64 operand shows in the workspace."""
    p = gen.random_problem(60 + 2 * ta + tb, 5, 7, 4, 1, 90, 0.5, 0.6)
    a_bits = gen.pack_bits(p.a_mask.T) if ta else p.a_bits()
    b_bits = gen.pack_bits(p.b_mask.T) if tb else p.b_bits()
    plan = bsm.Plan(p.rows, p.inner, p.cols, a_bits, b_bits, precision=precision, trans_a=ta,
                    trans_b=tb)
    plain = bsm.Plan.from_problem(p, precision=precision)
    c_bits = oracle.product_shape(p.M, p.K, p.N, a_bits, b_bits, bool(ta), bool(tb))
    assert np.array_equal(plan.c_shape(), c_bits)
    assert np.array_equal(plan.c_offsets(), oracle.block_offsets(p.rows, p.cols, c_bits)[0])
    i, j = plan.info(), plain.info()
    assert (i.a_elems, i.b_elems, i.c_elems, i.triples, i.tasks) == \
        (j.a_elems, j.b_elems, j.c_elems, j.triples, j.tasks)
    assert i.useful_flops == j.useful_flops
    extra = (ta * i.a_elems + tb * i.b_elems) * 8 if precision == bsm.FP64 else 0
    assert i.workspace_bytes >= j.workspace_bytes + extra


def test_transposed_shapes_validated():
    """A transposed operand's bitmap has the stored dimensions: its padding is checked against
    them, the binding checks its length, and trans flags other than 0/1/2 are rejected."""
    M, K, N = 70, 3, 2
    rows, inner, cols = [4] * M, [5] * K, [6] * N
    a_st = gen.pack_bits(np.ones((K, M), bool))      # K x M: 3 rows of 2 words
    b = gen.pack_bits(np.ones((K, N), bool))
    bsm.Plan(rows, inner, cols, a_st, b, trans_a=1).close()
    with pytest.raises(ValueError):                   # M x K layout: 70 rows of 1 word
        bsm.Plan(rows, inner, cols, a_st, b)
    bad = a_st.copy()
    bad[1] |= np.uint64(1) << np.uint64(6)            # column 70 of a 70-column row: padding
    with pytest.raises(bsm.BsmError) as e:
        bsm.Plan(rows, inner, cols, bad, b, trans_a=1)
    assert e.value.code == bsm.E_INVALID
    for flag in ({"trans_a": 3}, {"trans_b": -1}):
        with pytest.raises(bsm.BsmError) as e:
            bsm.Plan(rows, inner, cols, a_st, b, **flag) if "trans_a" in flag else \
                bsm.Plan(rows, inner, cols, gen.pack_bits(np.ones((M, K), bool)), b, **flag)
        assert e.value.code == bsm.E_INVALID


@pytest.mark.parametrize("ops", [(0, 0), (2, 1), (1, 2)])
def test_complex_plans(ops):
    """Complex elements: sizes and offsets count complex elements and follow the oracle's C
    layout; the flop count is the complex product's (8 r s t per triple = the real embedding's)."""
    ta, tb = ops
    p = gen.random_problem(70 + ta + 3 * tb, 5, 6, 4, 1, 90, 0.5, 0.6)
    a_bits = gen.pack_bits(p.a_mask.T) if ta else p.a_bits()
    b_bits = gen.pack_bits(p.b_mask.T) if tb else p.b_bits()
    plan = bsm.Plan(p.rows, p.inner, p.cols, a_bits, b_bits, elem=bsm.COMPLEX, trans_a=ta,
                    trans_b=tb)
    info = plan.info()
    assert info.elem == bsm.COMPLEX
    c_bits = oracle.product_shape(p.M, p.K, p.N, a_bits, b_bits, bool(ta), bool(tb))
    off, total = oracle.block_offsets(p.rows, p.cols, c_bits)
    assert np.array_equal(plan.c_shape(), c_bits)
    assert np.array_equal(plan.c_offsets(), off)
    assert (info.a_elems, info.b_elems, info.c_elems) == (p.a_data.size, p.b_data.size, total)
    real = bsm.Plan.from_problem(p).info()
    assert info.useful_flops == 4 * real.useful_flops
    assert info.triples == real.triples


def test_complex_limits_on_host():
    bits = gen.pack_bits(np.ones((1, 1), bool))
    with pytest.raises(bsm.BsmError) as e:
        bsm.Plan([32768], [4], [4], bits, bits, elem=bsm.COMPLEX)
    assert e.value.code == bsm.E_INVALID
    with pytest.raises(bsm.BsmError) as e:
        bsm.Plan([4], [4], [4], bits, bits, elem=2)
    assert e.value.code == bsm.E_INVALID
    with pytest.raises(bsm.BsmError) as e:
        bsm.Plan([4], [4], [4], bits, bits, elem=bsm.COMPLEX, trans_a=3)
    assert e.value.code == bsm.E_INVALID
    # the adjoint of a real operand is its transpose
    bsm.Plan([4], [4], [4], bits, bits, trans_a=2).close()
    zp = bsm.Plan([4], [4], [4], bits, bits, elem=bsm.COMPLEX)
    with pytest.raises(bsm.BsmError) as e:
        bsm.Batch([zp])
    assert e.value.code == bsm.E_UNSUPPORTED
    L = bsm.load()
    assert L.bsm_execute_static(zp.handle, 1.0, 1 << 32, 1 << 36, 1 << 40, 0, None) == bsm.E_UNSUPPORTED
    assert L.bsm_execute_complex(zp.handle, 1.0, 0.0, (1 << 32) + 8, 1 << 36, 1 << 40, 0, None) == bsm.E_INVALID
    rp = bsm.Plan([4], [4], [4], bits, bits)
    assert L.bsm_execute_complex(rp.handle, 1.0, 0.5, 1 << 32, 1 << 36, 1 << 40, 0, None) == bsm.E_MISMATCH


def test_low_rank_plans_on_host():
    """Block-rank-sparse plans: sizes, C layout (the oracle's), flops of both stages against the
    closed form, the dense-equivalent flops against the oracle's count, and argument errors."""
    p = gen.random_problem(80, 5, 6, 4, 1, 60, 0.7, 0.6)
    rank = lambda i, k, h, d: (i * 3 + k) % 5
    ranks, data = gen.low_rank_operand(p, 81, rank)
    plan = bsm.LowRankPlan(p.rows, p.inner, p.cols, p.a_bits(), ranks, p.b_bits())
    info = plan.info()
    c_bits = oracle.shape_product(p.M, p.K, p.N, p.a_bits(), p.b_bits())
    off, total = oracle.block_offsets(p.rows, p.cols, c_bits)
    assert np.array_equal(plan.c_offsets(), off) and info.c_elems == total
    assert info.a_elems == data.size and info.b_elems == p.b_data.size
    assert info.a_blocks == int(p.a_mask.sum()) and info.factored_blocks == int((ranks > 0).sum())
    assert info.dense_flops == oracle.useful_flops(p.rows, p.inner, p.cols, p.a_bits(), p.b_bits())
    bt = np.array([sum(int(p.cols[j]) for j in range(p.N) if p.b_mask[k, j]) for k in range(p.K)])
    want = 0.0
    for q, (i, k) in enumerate(zip(*np.nonzero(p.a_mask))):
        r, s, rho = int(p.rows[i]), int(p.inner[k]), int(ranks[q])
        want += 2.0 * (r * s if rho == 0 else rho * (r + s)) * bt[k]
    assert info.useful_flops == want
    bad = ranks.copy()
    bad[0] = -2
    with pytest.raises(bsm.BsmError) as e:
        bsm.LowRankPlan(p.rows, p.inner, p.cols, p.a_bits(), bad, p.b_bits())
    assert e.value.code == bsm.E_INVALID
    with pytest.raises(ValueError):
        bsm.LowRankPlan(p.rows, p.inner, p.cols, p.a_bits(), ranks[:-1], p.b_bits())
    with pytest.raises(bsm.BsmError) as e:
        bsm.LowRankPlan(p.rows, p.inner, p.cols, p.a_bits(), ranks, p.b_bits(), elem=bsm.COMPLEX)
    assert e.value.code == bsm.E_UNSUPPORTED
    plan.close()


def test_contraction_plans_on_host():
    """Tensor contraction plans: C's block shape equals the oracle's (boolean contraction of the
    shapes), sizes and flop counts follow, permutation passes only where the mode order needs one,
    and malformed descriptors are rejected."""
    from oracle import contract as tc
    rng = np.random.default_rng(90)
    til = {m: rng.integers(1, 6, int(rng.integers(1, 4))) for m in range(5)}
    cases = [([0, 2], [2, 1], [0, 1], (0, 0, 0)),
             ([0, 3, 2], [2, 1, 3], [1, 0], (0, 1, 1)),
             ([0, 2, 3, 1], [3, 4, 2], [0, 1, 4], (1, 1, 0)),
             ([0, 4], [4, 1, 2, 3], [0, 1, 2, 3], (0, 0, 0))]
    for n, (am, bm, cm, perms) in enumerate(cases):
        pa, da = gen.block_sparse_tensor(91 + n, [til[m] for m in am], 0.6)
        pb, db = gen.block_sparse_tensor(95 + n, [til[m] for m in bm], 0.6)
        plan = bsm.Contraction((am, [til[m] for m in am], gen.tensor_bits(pa)),
                               (bm, [til[m] for m in bm], gen.tensor_bits(pb)), cm)
        info = plan.info()
        shape, data = tc.contract(tc.Tensor(am, [til[m] for m in am], pa, da),
                                  tc.Tensor(bm, [til[m] for m in bm], pb, db), cm)
        assert np.array_equal(plan.c_shape()[:max(1, (shape.size + 63) // 64)], gen.tensor_bits(shape))
        assert (info.a_elems, info.b_elems, info.c_elems) == (da.size, db.size, data.size)
        assert (info.permute_a, info.permute_b, info.permute_c) == perms, (n, info.permute_a, info.permute_b, info.permute_c)
        plan.close()
    bits = gen.tensor_bits(np.ones((2, 2), bool))
    good = ([0, 1], [[2, 3], [4, 5]], bits)
    with pytest.raises(bsm.BsmError) as e:   # contracted tilings differ
        bsm.Contraction(good, ([1, 2], [[4, 6], [1, 1]], bits), [0, 2])
    assert e.value.code == bsm.E_MISMATCH
    with pytest.raises(bsm.BsmError) as e:   # a batch label (in A, B and C)
        bsm.Contraction(good, ([1, 2], [[4, 5], [1, 1]], bits), [0, 1, 2])
    assert e.value.code == bsm.E_UNSUPPORTED
    with pytest.raises(bsm.BsmError) as e:   # a label twice in one operand
        bsm.Contraction(([0, 0], [[2, 3], [2, 3]], bits), ([0, 2], [[2, 3], [1, 1]], bits), [2])
    assert e.value.code == bsm.E_INVALID
    with pytest.raises(bsm.BsmError) as e:   # padding bit
        bsm.Contraction(([0, 1], [[2, 3], [4, 5]], np.array([1 << 5], np.uint64)),
                        ([1, 2], [[4, 5], [1, 1]], bits), [0, 2])
    assert e.value.code == bsm.E_INVALID


def test_k_split_plans_on_host():
    """Reduction variant: every task's k-list cut into pieces (task count grows, C layout and flops
    do not), auto only for products with few tasks, and the combinations it does not support."""
    rng = np.random.default_rng(95)
    rows, inner = np.array([100, 60, 90]), rng.integers(32, 200, 40)
    a_mask = np.ones((3, 40), bool)
    p = gen.make_problem("tall", 95, rows, inner, rows, a_mask, a_mask.T.copy())
    base = bsm.Plan.from_problem(p).info()
    for ks in (2, 5, 16):
        i = bsm.Plan.from_problem(p, k_split=ks).info()
        assert i.k_split == ks and i.tasks == base.tasks * ks
        assert (i.c_elems, i.useful_flops, i.triples) == (base.c_elems, base.useful_flops, base.triples)
        assert i.workspace_bytes > base.workspace_bytes
    auto = bsm.Plan.from_problem(p, k_split=-1).info()
    assert auto.k_split == min(16, -(-2048 // base.tasks)) and base.tasks < 1024
    big = gen.uniform_1024()
    assert bsm.Plan.from_problem(big, k_split=-1).info().k_split == 1 or \
        bsm.Plan.from_problem(big).info().tasks < 1024
    with pytest.raises(bsm.BsmError) as e:
        bsm.Plan.from_problem(p, k_split=4, k_window=3)
    assert e.value.code == bsm.E_UNSUPPORTED
    assert bsm.Plan.from_problem(p, k_split=-1, k_window=3).info().k_split == 1
    with pytest.raises(bsm.BsmError) as e:
        bsm.Plan.from_problem(p, k_split=17)
    assert e.value.code == bsm.E_INVALID
    sp = bsm.Plan.from_problem(p, k_split=3)
    with pytest.raises(bsm.BsmError) as e:
        bsm.Batch([sp])
    assert e.value.code == bsm.E_UNSUPPORTED
    L = bsm.load()
    assert L.bsm_execute_static(sp.handle, 1.0, 1 << 32, 1 << 36, 1 << 40, 0, None) == bsm.E_UNSUPPORTED


def test_add_one_row_blocking():
    """The paper's nonuniform blocking (Sec. 4.1): rows handed out one at a time to uniformly
    chosen blocks.  Sizes sum to N, no block is empty, and for N = 32768 over 128 blocks the sizes
    have the multinomial mean 256 and a spread near sqrt(256 (1 - 1/128))."""
    rng = np.random.default_rng(3)
    sizes = gen.tiling_add_one(32768, 128, rng)
    assert sizes.sum() == 32768 and sizes.size == 128 and sizes.min() >= 1
    assert abs(sizes.mean() - 256) < 1e-9
    assert 12.0 < sizes.std() < 20.0
    few = gen.tiling_add_one(5, 40, np.random.default_rng(4))   # most blocks stay empty: dropped
    assert few.sum() == 5 and few.min() >= 1 and few.size <= 5
