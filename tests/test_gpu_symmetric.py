"""Symmetric square (only the output blocks with I <= J) on the GPU against the oracle.

Product lists and patterns bit-exact, values within the per-mode tolerances;
the upper blocks of an upper-only plan equal the same blocks of the full
product bit for bit when both run the same kernel configuration.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_11762_amd import workloads as W
from tests.gpu_helpers import assert_values, pattern_np, units, upload, values_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2011_11762_amd import qbsm
    assert torch.cuda.is_available()
    qbsm.load()
    return qbsm


@pytest.mark.parametrize("npoints,bs", [(1500, 32), (3000, 64)])
def test_symmetric_square_decay(q, npoints, bs):
    c = W.config2(npoints=npoints, bs=bs, seed=14)
    a, tol = c["A"], c["drop_tol"]
    oa = O.from_workload(a, tol)
    ref = O.multiply_upper(oa, oa)
    fI, fJ, _, _, _ = O.product_triples(oa, oa)
    fr, fc, _ = O.c_pattern_from_triples(fI, fJ)
    S, npr = (x[fr <= fc] for x in O.block_bound_terms(oa, oa))  # upper blocks of the full product
    A = upload(q, a, tol)
    for mode in ("f64", "f32", "bf16x3", "ozaki"):
        for unit in units(bs, mode):
            P = q.Plan(A, A, unit=unit, upper=True)
            info = P.info()
            assert info["nprod"] == ref.I.size and info["nblk_out"] == ref.brow.size
            assert info["flops"] == O.block_flops(ref.I, ref.J, ref.K, a.nrows, a.ncols, a.ncols, bs)
            gI, gK, gJ = (t.cpu().numpy().astype(np.int64) for t in P.products())
            assert np.array_equal(gI, ref.I) and np.array_equal(gJ, ref.J) and np.array_equal(gK, ref.K)
            C = P.numeric(mode)
            cr, cc = pattern_np(C)
            assert np.array_equal(cr, ref.brow) and np.array_equal(cc, ref.bcol)
            got = values_np(C)
            assert_values(got, ref.vals, S, npr, mode, bs, f"upper unit={unit}")
            # the same blocks of the full product, same configuration: identical
            full = q.Plan(A, A, unit=unit).numeric(mode)
            assert np.array_equal(full.extract(cr, cc).cpu().numpy(), got), (mode, unit)


def test_symmetric_square_rejections(q):
    """A non-square product, or a mask, with the upper-triangle option is an error."""
    a, b = W.small_random(200, 150, 120, 32, 0.5, 15)
    A, B = upload(q, a), upload(q, b)
    with pytest.raises(q.QbsmError):
        q.Plan(A, B, upper=True)  # 200 x 120 output
    S = upload(q, W.small_random(200, 200, 200, 32, 0.5, 17)[0])
    with pytest.raises(q.QbsmError):
        q.Plan(S, S, mask=S, upper=True)


def test_batched_upper_and_spamm_plans(q):
    """Upper-triangle and sparse approximate plans in one persistent launch
    equal their single launches bit for bit."""
    c = W.config2(npoints=2500, bs=64, seed=18)
    a, tol = c["A"], c["drop_tol"]
    A = upload(q, a, tol)
    plans = [q.Plan(A, A, unit=256, upper=True), q.Plan(A, A, unit=256, spamm_tol=1e-6),
             q.Plan(A, A, unit=256), q.Plan(A, A, unit=256, upper=True, spamm_tol=1e-3)]
    for mode in ("f32", "bf16x3"):
        singles = [values_np(p.numeric(mode)) for p in plans]
        batch = q.Batch(plans, mode)
        batch.run()
        torch.cuda.synchronize()
        for o, s_ in zip(batch.outs, singles):
            assert np.array_equal(values_np(o), s_), mode
    # the combined options against the oracle: upper blocks of the approximate product
    oa = O.from_workload(a, tol)
    assert O.spamm_borderline(oa, oa, 1e-3) == 0 and O.spamm_borderline(oa, oa, 1e-6) == 0
    sp = O.multiply_spamm(oa, oa, 1e-3)
    keep = sp.brow <= sp.bcol
    got = values_np(plans[3].numeric("f32"))
    cr, cc = pattern_np(plans[3].numeric("f32"))
    assert np.array_equal(cr, sp.brow[keep]) and np.array_equal(cc, sp.bcol[keep])
    S, npr = (x[keep] for x in O.block_bound_terms(oa, oa, tau=1e-3))
    assert_values(got, sp.vals[keep], S, npr, "f32", 64, "upper spamm")


@pytest.mark.parametrize("bs", [32, 64])
def test_symmetric_rank_k(q, bs):
    """Symmetric rank-k construction (Sec. 2.2): C = A A^T is symmetric for any
    A, and the upper-triangle option with a transposed right operand forms
    exactly its blocks I <= J."""
    a, _ = W.small_random(9 * bs + 5, 6 * bs + 7, 10, bs, 0.4, 60 + bs)  # tall A, m x k
    oa = O.from_workload(a)
    full = O.multiply(oa, oa, trans_b=True)
    keep = full.brow <= full.bcol
    I, J, K, _, _ = O.product_triples(oa, oa, trans_b=True)
    sel = I <= J
    S, npr = (x[keep] for x in O.block_bound_terms(oa, oa, trans_b=True))
    A = upload(q, a)
    for mode in ("f64", "f32", "bf16x3", "ozaki"):
        for unit in units(bs, mode):
            P = q.Plan(A, A, trans_r=True, unit=unit, upper=True)
            gI, gK, gJ = (t.cpu().numpy().astype(np.int64) for t in P.products())
            assert np.array_equal(gI, I[sel]) and np.array_equal(gJ, J[sel]) and np.array_equal(gK, K[sel])
            C = P.numeric(mode)
            cr, cc = pattern_np(C)
            assert np.array_equal(cr, full.brow[keep]) and np.array_equal(cc, full.bcol[keep])
            assert_values(values_np(C), full.vals[keep], S, npr, mode, bs, f"rank-k unit={unit}")


def test_batch_rejects_replaced_operands_and_outputs(q):
    """A batch run after an operand's values were re-stored (new pack
    buffers) or after an output was refilled by another plan is an error
    raised before anything is launched; a fresh batch works."""
    c = W.config2(npoints=1500, bs=64, seed=24)
    A = upload(q, c["A"], c["drop_tol"])
    P = q.Plan(A, A, unit=128)
    batch = q.Batch([P], "f32")
    batch.run()
    torch.cuda.synchronize()
    first = values_np(batch.outs[0])
    A.store_f32()  # same pattern, new value storage: the batch's packs are gone
    with pytest.raises(q.QbsmError):
        batch.run()
    # a multiply packs the re-stored values again, into a buffer of the same
    # size that the pool may place at the old address: still an error (the
    # batch's captured pack kernels would read the freed FP64 values)
    P.numeric("f32")
    torch.cuda.synchronize()
    with pytest.raises(q.QbsmError):
        batch.run()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with pytest.raises(q.QbsmError):
            batch.run_graph()
    stream.synchronize()
    fresh = q.Batch([P], "f32")
    fresh.run()
    torch.cuda.synchronize()
    assert np.array_equal(values_np(fresh.outs[0]), first)  # f32 packs of rounded values are the same
    # an output refilled by a different plan
    P2 = q.Plan(A, A, unit=128)
    P2.numeric("f32", fresh.outs[0])
    with pytest.raises(q.QbsmError):
        fresh.run()
