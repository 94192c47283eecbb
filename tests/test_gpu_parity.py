"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Patterns and product lists bit-exact; values within the per-mode relative
Frobenius tolerances of tests/gpu_helpers.py and, block by block, within the
normwise bounds of tests/bounds.py.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_11762_amd import workloads as W
from tests.gpu_helpers import (TOL, TOL_OZAKI_EMULATED, assert_backward, assert_product, check_product,
                               padding_is_zero, pattern_np, units, upload, values_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2011_11762_amd import qbsm
    assert torch.cuda.is_available()
    qbsm.load()
    return qbsm


SMALL = [
    # (m, k, n, bs, p, seed): rectangular, ragged in every dimension
    (300, 260, 200, 64, 0.5, 1),
    (190, 170, 150, 32, 0.5, 2),
    (400, 300, 520, 128, 0.6, 3),
    (1000, 900, 1100, 32, 0.15, 4),   # deeper tree, several units per side
    (64 * 9 + 5, 64 * 7, 64 * 11 + 63, 64, 0.3, 5),
]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-bs{c[3]}")
@pytest.mark.parametrize("mode", ["f64", "f32", "bf16", "bf16x3"])
def test_small_random(q, case, mode):
    m, k, n, bs, p, seed = case
    a, b = W.small_random(m, k, n, bs, p, seed)
    for unit in units(bs, mode):
        C, ref, err, got = check_product(q, a, b, mode, unit)
        assert padding_is_zero(got, ref.brow, ref.bcol, m, n, bs)


def test_config1_full_f64(q):
    c = W.config1()
    for unit in units(32, "f64"):
        C, ref, err, _ = check_product(q, c["A"], c["B"], "f64", unit)
        assert ref.brow.size == 1016 and ref.I.size == 4884


def test_empty_and_degenerate(q):
    bs = 64
    rng = np.random.default_rng(0)
    # A empty
    a = W.random_blocks(200, bs, 0.0, rng, ncols=150)
    b = W.random_blocks(150, bs, 1.0, rng, ncols=100)
    A, B = upload(q, a), upload(q, b)
    C = q.matmul(A, B, "f64")
    assert C.nblk == 0 and C.values().numel() == 0
    # disjoint inner patterns -> no product
    a2 = W.BlockMatrix(128, 128, 64, np.array([0], np.int32), np.array([0], np.int32), rng.uniform(-1, 1, (1, 4096)))
    b2 = W.BlockMatrix(128, 128, 64, np.array([1], np.int32), np.array([1], np.int32), rng.uniform(-1, 1, (1, 4096)))
    C2 = q.matmul(upload(q, a2), upload(q, b2), "f32")
    assert C2.nblk == 0
    # a single block smaller than the leaf (1x1 block grid, ragged)
    for mode in ("f64", "f32", "bf16x3"):
        a3, b3 = W.small_random(37, 50, 21, 64, 1.0, 9)
        check_product(q, a3, b3, mode, 64)
    # depth mismatch: tall-skinny times short-wide
    a4, b4 = W.small_random(64 * 40, 64, 64 * 3, 64, 0.7, 10)
    check_product(q, a4, b4, "f64", 128)


def test_determinism(q):
    a, b = W.small_random(1000, 1000, 1000, 64, 0.3, 11)
    A, B = upload(q, a), upload(q, b)
    for mode in ("f64", "f32", "bf16x3"):
        P = q.Plan(A, B)
        outs = [values_np(P.numeric(mode)) for _ in range(3)]
        assert all(np.array_equal(outs[0], o) for o in outs[1:]), mode


def test_drop_rule_decay(q):
    pts = W.decay_points(2048, 0.1, np.random.default_rng(12))
    a = W.decay_blocks(pts, 64)
    tol = 1e-3  # keeps a visibly sparse pattern at this small size
    assert not np.any(O.borderline(a.vals, 64, tol))
    keep = O.keep_mask(a.vals, 64, tol)
    A = upload(q, a, tol)
    assert A.nblk == int(keep.sum())
    r, c = pattern_np(A)
    oa = O.from_workload(a, tol)
    assert np.array_equal(r, oa.brow) and np.array_equal(c, oa.bcol)
    assert np.array_equal(values_np(A), oa.vals)
    check_product(q, a, a, "f64", 128, drop_tol=tol)


def test_nan_inf_propagate(q):
    a, b = W.small_random(256, 256, 256, 64, 1.0, 13)
    a.vals[5, 17] = np.nan
    a.vals[9, 100] = np.inf
    for mode in ("f64", "f32"):
        A, B = upload(q, a), upload(q, b)
        got = values_np(q.matmul(A, B, mode))
        ref = O.multiply(O.from_workload(a), O.from_workload(b)).vals
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        assert np.array_equal(np.isinf(got), np.isinf(ref))
        fin = np.isfinite(ref)
        assert np.allclose(got[fin], ref[fin], rtol=1e-5 if mode == "f32" else 1e-12, atol=1e-4)
    # NaN norm keeps the block under a drop tolerance
    A = upload(q, a, 1e30)
    assert A.nblk == 2  # only the NaN block and the Inf block survive


def test_error_paths(q):
    lib = q.load()
    a, b = W.small_random(128, 128, 192, 64, 1.0, 14)
    A, B = upload(q, a), upload(q, b)
    with pytest.raises(q.QbsmError) as e:
        q.Plan(B, A)  # 128x192 times 128x128: inner dims differ
    assert e.value.status == 2
    C32 = q.Matrix(128, 128, 32)
    C32.set_blocks(torch.zeros(1, dtype=torch.int32, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda"),
                   torch.zeros(1, 1024, dtype=torch.float64, device="cuda"))
    with pytest.raises(q.QbsmError) as e:
        q.Plan(A, C32)
    assert e.value.status == 2
    M = q.Matrix(128, 128, 64)
    v = torch.zeros(2, 4096, dtype=torch.float64, device="cuda")
    with pytest.raises(q.QbsmError) as e:  # duplicate
        M.set_blocks(torch.tensor([0, 0], dtype=torch.int32, device="cuda"),
                     torch.tensor([1, 1], dtype=torch.int32, device="cuda"), v)
    assert e.value.status == 3
    with pytest.raises(q.QbsmError) as e:  # out of range
        M.set_blocks(torch.tensor([0, 2], dtype=torch.int32, device="cuda"),
                     torch.tensor([1, 0], dtype=torch.int32, device="cuda"), v)
    assert e.value.status == 3
    with pytest.raises(q.QbsmError) as e:  # never given blocks
        q.Plan(M, B)
    assert e.value.status == 7
    # null pointers through the raw ABI
    assert lib.qbsm_matrix_set_blocks(M.handle, 2, None, None, None, 0.0, None, None) == 1
    assert lib.qbsm_multiply_numeric(None, 0, None, None) == 1
    assert lib.qbsm_multiply_numeric(q.Plan(A, B).handle, 9, M.handle, None) == 1
    # output with the wrong shape
    P = q.Plan(A, B)
    with pytest.raises(q.QbsmError) as e:
        P.numeric("f64", q.Matrix(128, 128, 64))
    assert e.value.status == 2
    # the allocator returning NULL -> out of memory, no abort
    fail_alloc = q._ALLOC_FN(lambda n, s, c: None)
    rel = q._RELEASE_FN(lambda p, s, c: None)
    assert lib.qbsm_set_allocator(fail_alloc, rel, None) == 0
    try:
        st = lib.qbsm_multiply_symbolic(A.handle, B.handle, None, None, ctypes.byref(ctypes.c_void_p()), None, None)
        assert st == 4
    finally:
        q._install_torch_allocator()
    # still usable afterwards
    check_product(q, a, b, "f64", 128)


def test_backward_small_vs_oracle(q):
    for (m, k, n, bs, p, seed) in [(300, 260, 200, 64, 0.5, 21), (190, 170, 150, 32, 0.6, 22),
                                    (400, 300, 520, 128, 0.6, 23)]:
        a, b = W.small_random(m, k, n, bs, p, seed)
        oa, ob = O.from_workload(a), O.from_workload(b)
        ref = O.multiply(oa, ob)
        rng = np.random.default_rng(seed)
        dcv = rng.uniform(-1, 1, size=ref.vals.shape)
        W.zero_padding(W.BlockMatrix(m, n, bs, ref.brow, ref.bcol, dcv))
        odc = O.canonical(m, n, bs, ref.brow, ref.bcol, dcv)
        ga, gb = O.backward(oa, ob, odc)
        A, B = upload(q, a), upload(q, b)
        dC = q.Matrix(m, n, bs)
        dC.set_blocks(torch.from_numpy(ref.brow.astype(np.int32)).cuda(),
                      torch.from_numpy(ref.bcol.astype(np.int32)).cuda(), torch.from_numpy(dcv).cuda())
        for mode in ("f64", "f32", "bf16x3"):
            for unit in units(bs, mode):
                dA, dB = q.backward(A, B, dC, mode, unit)
                ra, ca = pattern_np(dA)
                assert np.array_equal(ra, oa.brow) and np.array_equal(ca, oa.bcol)
                rb, cb = pattern_np(dB)
                assert np.array_equal(rb, ob.brow) and np.array_equal(cb, ob.bcol)
                assert_backward(values_np(dA), values_np(dB), oa, ob, odc, ga, gb, mode, f"unit={unit}")


def test_backward_from_forward_plan(q):
    """The backward regrouped from a forward plan: dC on a subset of C's
    blocks (its missing blocks drop their products), every unit side, the
    plan entry point equal bit for bit to the matrix entry point and to
    itself on a repeat; rejected for plans it cannot regroup."""
    for (m, k, n, bs, p, seed) in [(700, 520, 600, 64, 0.5, 24), (450, 390, 330, 32, 0.6, 25),
                                    (640, 600, 700, 128, 0.5, 26)]:
        a, b = W.small_random(m, k, n, bs, p, seed)
        oa, ob = O.from_workload(a), O.from_workload(b)
        ref = O.multiply(oa, ob)
        rng = np.random.default_rng(seed)
        keep = rng.random(ref.brow.size) < 0.7  # dC holds 70% of C's blocks
        dcv = rng.uniform(-1, 1, size=(int(keep.sum()), bs * bs))
        W.zero_padding(W.BlockMatrix(m, n, bs, ref.brow[keep], ref.bcol[keep], dcv))
        odc = O.canonical(m, n, bs, ref.brow[keep], ref.bcol[keep], dcv)
        ga, gb = O.backward(oa, ob, odc)
        A, B = upload(q, a), upload(q, b)
        dC = q.Matrix(m, n, bs)
        dC.set_blocks(torch.from_numpy(ref.brow[keep].astype(np.int32)).cuda(),
                      torch.from_numpy(ref.bcol[keep].astype(np.int32)).cuda(), torch.from_numpy(dcv).cuda())
        for mode in ("f64", "f32"):
            for unit in units(bs, mode):
                P = q.Plan(A, B, unit=unit)
                dA, dB = P.backward(dC, mode)
                assert_backward(values_np(dA), values_np(dB), oa, ob, odc, ga, gb, mode, f"plan unit={unit}")
                dA2, dB2 = q.backward(A, B, dC, mode, unit)
                dA3, _ = P.backward(dC, mode, need_b=False)
                assert np.array_equal(values_np(dA), values_np(dA2)) and np.array_equal(values_np(dB), values_np(dB2))
                assert np.array_equal(values_np(dA), values_np(dA3))
    A, B = upload(q, a), upload(q, b)
    with pytest.raises(q.QbsmError):
        q.Plan(A, B, upper=False, spamm_tol=1e-3).backward(dC, "f64")
    with pytest.raises(q.QbsmError):
        q.Plan(B, A, trans_l=True, trans_r=True).backward(dC, "f64")


def test_masked_plan_products(q):
    a, b = W.small_random(300, 260, 200, 64, 0.5, 31)
    oa, ob = O.from_workload(a), O.from_workload(b)
    ref = O.multiply(oa, ob)
    A, B = upload(q, a), upload(q, b)
    dC = q.Matrix(300, 200, 64)
    dC.set_blocks(torch.from_numpy(ref.brow.astype(np.int32)).cuda(),
                  torch.from_numpy(ref.bcol.astype(np.int32)).cuda(), torch.from_numpy(ref.vals).cuda())
    # dA plan: dC * B^T restricted to A: its products are the forward triples regrouped by (I, K)
    P = q.Plan(dC, B, trans_r=True, mask=A, unit=128)
    I, K, J = (t.cpu().numpy().astype(np.int64) for t in P.products())
    fw = sorted(zip(ref.I.tolist(), ref.K.tolist(), ref.J.tolist()))
    got = sorted(zip(I.tolist(), J.tolist(), K.tolist()))  # (I, Kout=K_A, Jcontr)
    assert got == fw


def test_batched_matches_single_and_graph_replays(q):
    rng = np.random.default_rng(41)
    members = []
    for t, (n, bs) in enumerate([(700, 32), (1000, 64), (513, 64), (900, 32), (1500, 64)]):
        if t % 2 == 0:
            a = W.banded(n, bs, 3, rng, fp32_values=True)
            b = W.banded(n, bs, 3, rng, fp32_values=True)
        else:
            a, b = W.small_random(n, n, n, bs, 0.4, 100 + t, fp32_values=True)
        members.append((a, b))
    As = [(upload(q, a), upload(q, b)) for a, b in members]
    plans = [q.Plan(A, B, unit=128) for A, B in As]
    singles = [values_np(p.numeric("f32")) for p in plans]
    batch = q.Batch(plans, "f32")
    batch.run()
    torch.cuda.synchronize()
    for o, s in zip(batch.outs, singles):
        assert np.array_equal(values_np(o), s)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for rep in range(3):
            # eager work between replays
            junk = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
            for o in batch.outs:
                o.values()
            batch.run_graph()
            stream.synchronize()
            for o, s in zip(batch.outs, singles):
                assert np.array_equal(values_np(o), s), rep
            del junk
    # oracle check of every member
    for (a, b), s in zip(members, singles):
        oa, ob = O.from_workload(a), O.from_workload(b)
        assert_product(s, oa, ob, O.multiply(oa, ob).vals, "f32", what="batch member")


def test_autograd_gradcheck(q):
    a, b = W.small_random(80, 70, 90, 32, 0.6, 51)
    ra, ca = (torch.from_numpy(x.astype(np.int32)).cuda() for x in (a.brow, a.bcol))
    rb, cb = (torch.from_numpy(x.astype(np.int32)).cuda() for x in (b.brow, b.bcol))
    av = torch.from_numpy(a.vals).cuda().requires_grad_(True)
    bv = torch.from_numpy(b.vals).cuda().requires_grad_(True)
    # padding entries are not free parameters of the logical matrix: mask them
    pa = torch.from_numpy((a.vals != 0).astype(np.float64)).cuda()
    pb = torch.from_numpy((b.vals != 0).astype(np.float64)).cuda()

    def f(x, y):
        c, _, _ = q.block_matmul(x * pa, (ra, ca), y * pb, (rb, cb), 80, 70, 90, 32, "f64")
        return c

    assert torch.autograd.gradcheck(f, (av, bv), eps=1e-6, atol=1e-8, rtol=1e-6, fast_mode=True)
    # FP64 oracle gradient of L = sum(C * W)
    c = f(av, bv)
    w = torch.rand_like(c)
    (c * w).sum().backward()
    oa, ob = O.from_workload(a), O.from_workload(b)
    ref = O.multiply(oa, ob)
    odc = O.canonical(80, 90, 32, ref.brow, ref.bcol, w.detach().cpu().numpy())
    ga, gb = O.backward(oa, ob, odc)
    assert O.rel_fro(av.grad.cpu().numpy() * (a.vals != 0), ga * (a.vals != 0)) <= 1e-12
    assert O.rel_fro(bv.grad.cpu().numpy() * (b.vals != 0), gb * (b.vals != 0)) <= 1e-12


def test_autotune_unit(q):
    a, b = W.small_random(2048, 2048, 2048, 64, 0.3, 61)
    A, B = upload(q, a), upload(q, b)
    best, times = q.autotune_unit(A, B, "f32", reps=2)
    assert best in (64, 128, 256) and times[best] > 0
    assert all(times[u] > 0 for u in (64, 128, 256))
    best, times = q.autotune_unit(A, B, "f64", reps=1)
    assert best in (64, 128) and times[256] < 0


def test_batch_autotune(q):
    """The batch tuner times every (unit side, occupancy) that all members
    can run at and returns the fastest; a member with 32-wide leaves rules
    out unit 256, an FP64 batch too; the trial batches leave nothing behind."""
    pairs = []
    for t, (n, bs) in enumerate([(900, 64), (1300, 64), (700, 64)]):
        a, b = W.small_random(n, n, n, bs, 0.4, 400 + t)
        pairs.append((upload(q, a), upload(q, b)))
    r = q.batch_autotune(pairs, "f32", reps=1)
    assert set(r["table"]) == {64, 128, 256}
    assert r["unit"] in r["table"] and r["ms"] == min(min(v.values()) for v in r["table"].values())
    assert all(1 <= o <= 4 and t > 0 for row in r["table"].values() for o, t in row.items())
    # the chosen settings run the batch correctly
    plans = [q.Plan(A, B, unit=r["unit"]) for A, B in pairs]
    singles = [values_np(p.numeric("f32")) for p in plans]
    batch = q.Batch(plans, "f32")
    batch.set_occupancy(r["wg_per_cu"])
    batch.run()
    torch.cuda.synchronize()
    assert all(np.array_equal(values_np(o), s_) for o, s_ in zip(batch.outs, singles))
    a32, b32 = W.small_random(600, 600, 600, 32, 0.4, 410)
    r2 = q.batch_autotune(pairs + [(upload(q, a32), upload(q, b32))], "bf16x3", reps=1)
    assert 256 not in r2["table"] and set(r2["table"]) <= {64, 128}
    r3 = q.batch_autotune(pairs, "f64", reps=1)
    assert 256 not in r3["table"]
    with pytest.raises(q.QbsmError):
        q.batch_autotune(pairs + [(upload(q, a32), upload(q, b32))], "ozaki", reps=1)


UNIT256 = [
    # (m, k, n, bs, p, seed): several 256-wide units per side with ragged
    # edges (a wave's 128 x 128 part partly or wholly outside C), sparse
    # patterns (partial leaf masks inside a wave), 128-wide leaves
    (64 * 9 + 5, 64 * 7 + 33, 64 * 11 + 63, 64, 0.3, 71),
    (1100, 700, 900, 64, 0.08, 72),
    (128 * 5 + 17, 128 * 3, 128 * 4 + 100, 128, 0.5, 73),
    (300, 1500, 200, 64, 1.0, 74),
]


@pytest.mark.parametrize("case", UNIT256, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-bs{c[3]}-p{c[4]}")
@pytest.mark.parametrize("mode", ["f32", "bf16", "bf16x3"])
def test_unit256(q, case, mode):
    m, k, n, bs, p, seed = case
    a, b = W.small_random(m, k, n, bs, p, seed)
    C, ref, err, got = check_product(q, a, b, mode, 256)
    assert padding_is_zero(got, ref.brow, ref.bcol, m, n, bs)


def test_unit256_nonfinite_sparse(q):
    """Unit 256 with Inf/NaN in a sparse pattern: a nil partner of an infinite
    value must contribute nothing (the zero-copy path is not taken)."""
    # whole leaves (no element padding), ragged at the 256-wide units
    a, b = W.small_random(64 * 11, 64 * 9, 64 * 10, 64, 0.35, 77)
    a.vals[3, 100] = np.inf
    a.vals[7, 5] = np.nan
    b.vals[2, 4000] = -np.inf
    ref = O.multiply(O.from_workload(a), O.from_workload(b)).vals
    assert np.isfinite(ref).sum() > 0 and (~np.isfinite(ref)).sum() > 0
    for mode in ("f32", "bf16x3"):
        A, B = upload(q, a), upload(q, b)
        got = values_np(q.matmul(A, B, mode, unit=256))
        if mode == "f32":
            assert np.array_equal(np.isnan(got), np.isnan(ref)), mode
            assert np.array_equal(np.isinf(got), np.isinf(ref)), mode
        else:
            # split products of an infinity may cancel to NaN: non-finite
            # exactly where the FP64 product is
            assert np.array_equal(np.isfinite(got), np.isfinite(ref)), mode
        fin = np.isfinite(ref)
        assert O.rel_fro(got[fin], ref[fin]) <= TOL[mode], mode


def test_unit256_rejects_f64(q):
    a, b = W.small_random(300, 260, 200, 64, 0.5, 75)
    A, B = upload(q, a), upload(q, b)
    P = q.Plan(A, B, unit=256)
    with pytest.raises(q.QbsmError, match="unsupported|FP32"):
        P.numeric("f64")
    assert P.numeric("f32").nblk > 0


def test_unit256_batched(q):
    """Persistent launch at unit 256 over members with 64- and 128-wide leaves."""
    rng = np.random.default_rng(76)
    members = []
    for t, (n, bs) in enumerate([(700, 64), (1000, 128), (513, 64), (1500, 128), (900, 64)]):
        if t % 2 == 0:
            a = W.banded(n, bs, 2, rng, fp32_values=True)
            b = W.banded(n, bs, 2, rng, fp32_values=True)
        else:
            a, b = W.small_random(n, n, n, bs, 0.4, 200 + t, fp32_values=True)
        members.append((a, b))
    As = [(upload(q, a), upload(q, b)) for a, b in members]
    plans = [q.Plan(A, B, unit=256) for A, B in As]
    for mode in ("f32", "bf16x3"):
        singles = [values_np(p.numeric(mode)) for p in plans]
        batch = q.Batch(plans, mode)
        batch.run()
        torch.cuda.synchronize()
        for o, s_ in zip(batch.outs, singles):
            assert np.array_equal(values_np(o), s_)
        for (a, b), s_ in zip(members, singles):
            oa, ob = O.from_workload(a), O.from_workload(b)
            assert_product(s_, oa, ob, O.multiply(oa, ob).vals, mode, what="unit-256 batch member")


@pytest.mark.parametrize("bs", [32, 64, 128])
def test_square_packs_both_roles_at_once(q, bs):
    """A * A through one handle (both operand layouts packed in one pass for
    leaves up to 64) equals A * B with B a second handle of the same values
    (one pack per role), bit for bit, in every mode; the non-finite flags of
    both layouts are set."""
    n = 5 * bs + bs // 2
    a, _ = W.small_random(n, n, n, bs, 0.5, 78)
    A1, A2 = upload(q, a), upload(q, a)
    oa = O.from_workload(a)
    ref = O.multiply(oa, oa)
    for mode in ("f64", "f32", "bf16", "bf16x3"):
        for unit in units(bs, mode):
            same = values_np(q.matmul(A1, A1, mode, unit=unit))
            other = values_np(q.matmul(A1, A2, mode, unit=unit))
            assert np.array_equal(same, other), (mode, unit)
            assert_product(same, oa, oa, ref.vals, mode, what=f"A*A unit={unit}")
    b = W.BlockMatrix(a.nrows, a.ncols, bs, a.brow.copy(), a.bcol.copy(), a.vals.copy())
    b.vals[1, 3] = np.nan
    B1 = upload(q, b)
    got = values_np(q.matmul(B1, B1, "f32", unit=max(units(bs, "f32"))))
    refb = O.multiply(O.from_workload(b), O.from_workload(b)).vals
    assert np.array_equal(np.isnan(got), np.isnan(refb))


def _set_values(A, m):
    """Replaces the content of handle A with the blocks of host matrix m."""
    A.set_blocks(torch.from_numpy(m.brow.astype(np.int32)).cuda(), torch.from_numpy(m.bcol.astype(np.int32)).cuda(),
                 torch.from_numpy(m.vals).cuda(), 0.0)


@pytest.mark.parametrize("bs", [32, 64, 128])
def test_prepack_matches_packing_on_use(q, bs):
    """Packs made ahead on the library's side stream give the same products,
    bit for bit, as packs made on use: one role per operand (A * B), both
    roles of one handle (A * A), every mode and unit.  A prepack made stale by
    new values before use, one followed by the handle's destruction, and one
    consumed by a persistent batch are ordered correctly."""
    n = 5 * bs + bs // 2
    a, b = W.small_random(n, n - bs // 3, n + bs, bs, 0.5, 91)
    sq, _ = W.small_random(n, n, n, bs, 0.5, 92)
    for mode in ("f64", "f32", "bf16", "bf16x3", "ozaki"):
        for unit in units(bs, mode):
            plain = values_np(q.matmul(upload(q, a), upload(q, b), mode, unit=unit))
            A1, B1 = upload(q, a), upload(q, b)
            A1.prepack(mode, 1)
            B1.prepack(mode, 2)
            assert np.array_equal(values_np(q.matmul(A1, B1, mode, unit=unit)), plain), (mode, unit)
            S0, S1 = upload(q, sq), upload(q, sq)
            S1.prepack(mode, 3)
            assert np.array_equal(values_np(q.matmul(S1, S1, mode, unit=unit)),
                                  values_np(q.matmul(S0, S0, mode, unit=unit))), (mode, unit)
    # stale before use: new values replace the prepacked ones
    sq2, _ = W.small_random(n, n, n, bs, 0.5, 93)
    A = upload(q, sq)
    A.prepack("bf16x3", 3)
    _set_values(A, sq2)
    got = values_np(q.matmul(A, A, "bf16x3", unit=units(bs, "bf16x3")[0]))
    o2 = O.from_workload(sq2)
    assert_product(got, o2, o2, O.multiply(o2, o2).vals, "bf16x3", what="stale prepack")
    # destroyed right after the prepack was queued
    D = upload(q, sq)
    D.prepack("f32", 3)
    del D
    torch.cuda.synchronize()
    # a batch over operands packed ahead (FP32 storage keeps the pattern and
    # the plan, makes the packs stale, and packs to the same f32 values)
    A2, B2 = upload(q, a), upload(q, b)
    plan = q.Plan(A2, B2, unit=units(bs, "f32")[0])
    single = values_np(plan.numeric("f32"))
    A2.store_f32()
    B2.store_f32()
    A2.prepack("f32", 1)
    B2.prepack("f32", 2)
    batch = q.Batch([plan], "f32")
    batch.run()
    torch.cuda.synchronize()
    assert np.array_equal(values_np(batch.outs[0]), single)
    with pytest.raises(q.QbsmError):
        A2.prepack("f32", 4)


OZAKI_CASES = [
    (300, 260, 200, 64, 0.5, 81),
    (190, 170, 150, 64, 1.0, 82),
    (2000, 1900, 2100, 64, 0.15, 83),   # deeper tree, many pairs per unit
    (64 * 9 + 5, 64 * 7, 64 * 11 + 63, 64, 0.3, 84),
]


@pytest.mark.parametrize("case", OZAKI_CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-bs{c[3]}")
@pytest.mark.parametrize("unit", [64, 128])
def test_ozaki_against_oracle_split(q, case, unit):
    """Ozaki mode: FP64 result within the stated tolerance of the FP64 oracle
    and within rounding of the oracle's own Ozaki emulation, at unit 64 (one
    leaf per unit) and unit 128 (2 x 2 leaves, nil leaves inside a unit)."""
    m, k, n, bs, p, seed = case
    a, b = W.small_random(m, k, n, bs, p, seed)
    C, ref, err, got = check_product(q, a, b, "ozaki", unit)
    assert C.values().dtype == torch.float64
    oz = O.ozaki_multiply(O.from_workload(a), O.from_workload(b))
    assert O.rel_fro(got, oz.vals) <= TOL_OZAKI_EMULATED
    assert padding_is_zero(got, ref.brow, ref.bcol, m, n, bs)


def test_ozaki_square_pack_pair_matches_single_packs(q):
    """A * A packs both roles of A in one pass (one read per leaf, row and
    column exponents together); a separate copy of A as the right operand
    is packed role by role.  Both give the same digits, so the products are
    bit-identical, also with an infinite entry (its row and column are
    marked in the respective packs) and in FP32 storage."""
    a, _ = W.small_random(900, 900, 900, 64, 0.5, 91)
    a.vals[3, 77] = np.inf
    for f32 in (False, True):
        A, A2 = upload(q, a), upload(q, a)
        if f32:
            A.store_f32()
            A2.store_f32()
        for unit in (64, 128):
            g_pair = values_np(q.Plan(A, A, unit=unit).numeric("ozaki"))
            g_single = values_np(q.Plan(A, A2, unit=unit).numeric("ozaki"))
            assert np.array_equal(np.isfinite(g_pair), np.isfinite(g_single))
            fin = np.isfinite(g_pair)
            assert np.array_equal(g_pair[fin], g_single[fin]), (f32, unit)


def test_ozaki_units_agree(q):
    """Unit 64 and unit 128 add the same leaf products in the same order
    (K ascending, one flush per leaf product), so their results are equal."""
    a, b = W.small_random(900, 1000, 800, 64, 0.4, 90)
    A, B = upload(q, a), upload(q, b)
    g64 = values_np(q.Plan(A, B, unit=64).numeric("ozaki"))
    g128 = values_np(q.Plan(A, B, unit=128).numeric("ozaki"))
    assert np.array_equal(g64, g128)


@pytest.mark.parametrize("decades", [40, 120, 280])
def test_ozaki_wide_dynamic_range(q, decades):
    """Entries spread over 40, 120 and 280 decades (up to about 1e140 and
    down to 1e-140, far outside the FP32 and bfloat16 exponent range; the
    squares that the norms of the checks take stay within FP64): the line
    exponents are applied in FP64, so every block keeps its relative accuracy
    and nothing overflows or underflows that the FP64 product does not."""
    a, b = W.small_random(640, 640, 640, 64, 0.6, 85)
    rng = np.random.default_rng(85)
    # block (I, K) of A scaled by 10^(p_I + q_K), block (K, J) of B by
    # 10^(r_J - q_K): the entries span `decades` decades while every leaf
    # product A_IK B_KJ has the scale 10^(p_I + r_J) of its output block, so
    # no product over- or underflows FP64 (p and r spread over a third of
    # the range, q over the rest)
    nb = 10
    p, r = (rng.uniform(-decades / 6, decades / 6, nb) for _ in range(2))
    qk = rng.uniform(-decades / 3, decades / 3, nb)
    a.vals *= 10.0 ** (p[a.brow] + qk[a.bcol])[:, None]
    b.vals *= 10.0 ** (r[b.bcol] - qk[b.brow])[:, None]
    for unit in (64, 128):
        C, ref, err, got = check_product(q, a, b, "ozaki", unit)
        assert np.all(np.isfinite(ref.vals)) and np.all(np.isfinite(got))
        oz = O.ozaki_multiply(O.from_workload(a), O.from_workload(b))
        assert O.rel_fro(got, oz.vals) <= TOL_OZAKI_EMULATED
        # block by block, relative to each block's own norm
        nrm = np.linalg.norm(ref.vals, axis=1)
        rel = np.linalg.norm(got - ref.vals, axis=1) / np.where(nrm > 0, nrm, 1.0)
        assert np.max(rel) <= 1e-10


def test_ozaki_extreme_values_and_nonfinite(q):
    """Entries near 1e30 and 1e-30 (beyond the bfloat16 and FP32 ranges when
    multiplied), a product that overflows FP64 as in the oracle, and Inf/NaN
    inputs: non-finite exactly where the FP64 product is."""
    a, b = W.small_random(256, 256, 256, 64, 1.0, 88)
    a.vals[:4] *= 1e30
    a.vals[4:8] *= 1e-30
    b.vals[:4] *= 1e30
    b.vals[4:8] *= 1e-30
    C, ref, err, got = check_product(q, a, b, "ozaki", 64)
    assert np.all(np.isfinite(got))
    # an overflowing product: 1e200 * 1e200 is Inf in FP64 too
    a2, b2 = W.small_random(128, 128, 128, 64, 1.0, 89)
    a2.vals[0] *= 1e200
    b2.vals[0] *= 1e200
    r2 = O.multiply(O.from_workload(a2), O.from_workload(b2)).vals
    for unit in (64, 128):
        g2 = values_np(q.matmul(upload(q, a2), upload(q, b2), "ozaki", unit=unit))
        assert np.array_equal(np.isfinite(g2), np.isfinite(r2)) and not np.all(np.isfinite(r2))
        _finite_parts_close(g2, r2)
    # Inf and NaN inputs
    a3, b3 = W.small_random(256, 256, 256, 64, 1.0, 13)
    a3.vals[5, 17] = np.nan
    a3.vals[9, 100] = np.inf
    b3.vals[2, 4000] = -np.inf
    ref3 = O.multiply(O.from_workload(a3), O.from_workload(b3)).vals
    for unit in (64, 128):
        got3 = values_np(q.matmul(upload(q, a3), upload(q, b3), "ozaki", unit=unit))
        assert np.array_equal(np.isfinite(got3), np.isfinite(ref3))
        _finite_parts_close(got3, ref3)


def _finite_parts_close(got, ref, tol=1e-11):
    """Block by block, the finite elements agree within tol relative to the
    norm of the block's finite reference elements (single elements may
    cancel, so they are not compared one by one)."""
    fin = np.isfinite(ref)
    for t in range(ref.shape[0]):
        f = fin[t]
        if not f.any():
            continue
        r, g = ref[t, f], got[t, f]
        s = np.max(np.abs(r))
        if s == 0:
            assert np.all(g == 0)
            continue
        assert np.linalg.norm((g - r) / s) <= tol * np.linalg.norm(r / s), t


def test_ozaki_unit_and_backward(q):
    a, b = W.small_random(320, 256, 288, 64, 0.5, 86)
    A, B = upload(q, a), upload(q, b)
    with pytest.raises(q.QbsmError, match="unit 64 or 128"):
        q.Plan(A, B, unit=256).numeric("ozaki")
    a32, b32 = W.small_random(200, 150, 120, 32, 0.5, 87)
    with pytest.raises(q.QbsmError, match="64 x 64 leaves"):
        q.Plan(upload(q, a32), upload(q, b32), unit=64).numeric("ozaki")
    oa, ob = O.from_workload(a), O.from_workload(b)
    ref = O.multiply(oa, ob)
    rng = np.random.default_rng(86)
    dcv = rng.uniform(-1, 1, size=ref.vals.shape)
    W.zero_padding(W.BlockMatrix(320, 288, 64, ref.brow, ref.bcol, dcv))
    odc = O.canonical(320, 288, 64, ref.brow, ref.bcol, dcv)
    ga, gb = O.backward(oa, ob, odc)
    dC = q.Matrix(320, 288, 64)
    dC.set_blocks(torch.from_numpy(ref.brow.astype(np.int32)).cuda(),
                  torch.from_numpy(ref.bcol.astype(np.int32)).cuda(), torch.from_numpy(dcv).cuda())
    for unit in (64, 128):
        dA, dB = q.backward(A, B, dC, "ozaki", unit)
        assert_backward(values_np(dA), values_np(dB), oa, ob, odc, ga, gb, "ozaki")


def test_ozaki_batched(q):
    rng = np.random.default_rng(87)
    members = [W.small_random(n, n, n, bs, 0.4, 300 + t) for t, (n, bs) in
               enumerate([(700, 64), (1000, 64), (513, 64)])]
    for unit in (64, 128):
        plans = [q.Plan(upload(q, a), upload(q, b), unit=unit) for a, b in members]
        singles = [values_np(p.numeric("ozaki")) for p in plans]
        batch = q.Batch(plans, "ozaki")
        batch.run()
        torch.cuda.synchronize()
        for o, s_, (a, b) in zip(batch.outs, singles, members):
            assert np.array_equal(values_np(o), s_)
            oa, ob = O.from_workload(a), O.from_workload(b)
            assert_product(s_, oa, ob, O.multiply(oa, ob).vals, "ozaki", what=f"ozaki batch member (unit {unit})")
