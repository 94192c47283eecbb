"""GPU parity at the full sizes of the five workloads.

Patterns and product lists are compared bit-exactly wherever the oracle can
enumerate them.  Values are compared on every block against the full FP64
oracle (also for the decay matrix, about 8.5 TFLOP on the host), except for
the batched members and the paper-size random-blocks matrix, whose sampled
output blocks the oracle computes one by one; every compared block is held
to its own normwise bound besides the relative Frobenius norm over all.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_11762_amd import workloads as W
from tests.bounds import assert_blockwise
from tests.gpu_helpers import (TOL, TOL_BF16_ROUNDED, assert_backward, assert_product, assert_sampled, assert_values,
                               pattern_np, rounded, upload, values_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2011_11762_amd import qbsm
    assert torch.cuda.is_available()
    qbsm.load()
    return qbsm


def sampled_values(C, si, sj):
    """GPU values of selected C blocks (zero where a block is not stored)."""
    return C.extract(np.asarray(si), np.asarray(sj)).cpu().numpy()


def test_config2_decay_full(q):
    """16384 points, 64x64 leaves, drop 1e-10: pattern, product list, and the
    whole C in every mode against the full FP64 oracle, globally and block by
    block (block norms span about 15 decades)."""
    c = W.config2()
    a, tol = c["A"], c["drop_tol"]
    assert not np.any(O.borderline(a.vals, 64, tol)), "a block norm lies on the drop threshold"
    oa = O.from_workload(a, tol)
    A = upload(q, a, tol)
    assert A.nblk == oa.nblk
    r, cc = pattern_np(A)
    assert np.array_equal(r, oa.brow) and np.array_equal(cc, oa.bcol)
    P = q.Plan(A, A)
    info = P.info()
    ref = O.multiply(oa, oa)  # the full FP64 product (about 8.5 TFLOP on the host)
    assert info["nprod"] == ref.I.size and info["nblk_out"] == 65536 == ref.brow.size
    assert info["flops"] == O.block_flops(ref.I, ref.J, ref.K, a.nrows, a.ncols, a.ncols, 64)
    gI, gK, gJ = (t.cpu().numpy().astype(np.int64) for t in P.products())
    assert np.array_equal(gI, ref.I) and np.array_equal(gJ, ref.J) and np.array_equal(gK, ref.K)
    del gI, gJ, gK
    S, npr = O.block_bound_terms(oa, oa)
    for mode, unit in (("f64", 128), ("f32", 256), ("bf16x3", 256), ("bf16x3", 128), ("bf16", 256),
                       ("ozaki", 64), ("ozaki", 128)):
        Pm = P if unit == 128 else q.Plan(A, A, unit=unit)
        C = Pm.numeric(mode)
        cr, cc = pattern_np(C)
        assert np.array_equal(cr, ref.brow) and np.array_equal(cc, ref.bcol), (mode, unit)
        got = values_np(C)
        del C
        assert_values(got, ref.vals, S, npr, mode, 64, f"decay unit={unit}")
        del got


def test_config3_random_blocks_full(q):
    """N=65536, 128x128 leaves, p=0.01: BF16 and BF16x3 against the full oracle."""
    c = W.config3()
    a, b = c["A"], c["B"]
    oa, ob = O.from_workload(a), O.from_workload(b)
    ref = O.multiply(oa, ob)
    A, B = upload(q, a), upload(q, b)
    P = q.Plan(A, B)
    gI, gK, gJ = (t.cpu().numpy().astype(np.int64) for t in P.products())
    assert np.array_equal(gI, ref.I) and np.array_equal(gJ, ref.J) and np.array_equal(gK, ref.K)
    for mode in ("bf16", "bf16x3", "f32"):
        C = P.numeric(mode)
        cr, cc = pattern_np(C)
        assert np.array_equal(cr, ref.brow) and np.array_equal(cc, ref.bcol)
        got = values_np(C)
        assert_product(got, oa, ob, ref.vals, mode, what="random blocks")
        if mode == "bf16":
            rr = O.multiply(rounded(oa, O.round_to_bf16), rounded(ob, O.round_to_bf16))
            assert O.rel_fro(got, rr.vals) <= TOL_BF16_ROUNDED


def test_config5_forward_backward_full(q):
    """Banded N=16384, 64x64 leaves, h=6, FP32: forward and masked backward vs the oracle."""
    c = W.config5()
    a, b, dc = c["A"], c["B"], c["dC"]
    oa, ob, odc = O.from_workload(a), O.from_workload(b), O.from_workload(dc)
    ref = O.multiply(oa, ob)
    assert (ref.brow.size, ref.I.size) == (6244, 42354)
    assert np.array_equal(odc.brow, ref.brow) and np.array_equal(odc.bcol, ref.bcol)
    ga, gb = O.backward(oa, ob, odc)
    A, B, dC = upload(q, a), upload(q, b), upload(q, dc)
    for mode in ("f32", "f64", "bf16x3"):
        C = q.matmul(A, B, mode)
        assert_product(values_np(C), oa, ob, ref.vals, mode, what="banded forward")
        dA, dB = q.backward(A, B, dC, mode)
        ra, ca = pattern_np(dA)
        assert np.array_equal(ra, oa.brow) and np.array_equal(ca, oa.bcol)
        assert_backward(values_np(dA), values_np(dB), oa, ob, odc, ga, gb, mode, "banded")
    # adjoint identity on the GPU results: <dA, A> = <dB, B> = <dC, C>
    C = q.matmul(A, B, "f64")
    dA, dB = q.backward(A, B, dC, "f64")
    l0 = float(np.sum(values_np(C) * odc.vals))
    assert abs(float(np.sum(values_np(dA) * oa.vals)) - l0) <= 1e-9 * abs(l0)
    assert abs(float(np.sum(values_np(dB) * ob.vals)) - l0) <= 1e-9 * abs(l0)


def _member_inputs(q, spec):
    """Device handles of one batched member (decay values generated on the GPU)."""
    if spec["kind"] == "banded":
        mem = W.config4_member(spec)
        return upload(q, mem["A"]), upload(q, mem["B"]), mem, None
    rng = np.random.default_rng([4, spec["m"]])
    pts = W.decay_points(spec["n"], 0.1, rng)
    r, c, v = W.decay_blocks_device(pts, spec["bs"])
    A = q.Matrix(spec["n"], spec["n"], spec["bs"])
    A.set_blocks(r, c, v, spec["drop_tol"])
    return A, A, None, (r, c, v)


def test_config4_batched_full(q):
    """256 members (N 1024..16384, leaves 32/64, banded and decay), FP32, one
    persistent launch replayed as a HIP graph; every member checked against
    the oracle on sampled blocks, a subset bit-exact against single launches."""
    specs = W.config4_members()
    plans, handles, samples = [], [], []
    rng = np.random.default_rng(44)
    for spec in specs:
        A, B, mem, dev = _member_inputs(q, spec)
        bs, n = spec["bs"], spec["n"]
        nb = -(-n // bs)
        si, sj = rng.integers(0, nb, 2), rng.integers(0, nb, 2)
        if dev is None:
            oa, ob = O.from_workload(mem["A"]), O.from_workload(mem["B"])
        else:
            # the oracle reads the same FP64 values: the sampled row and column panels
            r, c, v = dev
            sel = torch.isin(r, torch.from_numpy(si.astype(np.int32)).cuda()) | \
                torch.isin(c, torch.from_numpy(sj.astype(np.int32)).cuda())
            oa = O.canonical(n, n, bs, r[sel].cpu().numpy(), c[sel].cpu().numpy(), v[sel].cpu().numpy(),
                             spec["drop_tol"])
            ob = oa
            del dev, r, c, v, sel
        ref = O.multiply_blocks(oa, ob, si, sj)
        samples.append((si, sj, ref, nb) + O.sampled_bound_terms(oa, ob, si, sj))
        if A is B:
            A.store_f32()
        else:
            A.store_f32()
            B.store_f32()
        plans.append(q.Plan(A, B, unit=128))
        handles.append((A, B))
    torch.cuda.empty_cache()
    batch = q.Batch(plans, "f32")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch.run_graph()
        batch.run_graph()
    stream.synchronize()
    # the FP32 tolerance bounds the relative Frobenius error of the result:
    # checked on the union of all sampled blocks; each member's own samples
    # get a looser sanity bound (a single far-field block carries the full
    # long-K FP32 accumulation error relative to its small norm)
    num = den = 0.0
    for k, (C, (si, sj, ref, nb, S, npr)) in enumerate(zip(batch.outs, samples)):
        got = sampled_values(C, si, sj)  # zero where a block has no product
        d2, r2 = float(np.sum((got - ref) ** 2)), float(np.sum(ref ** 2))
        num, den = num + d2, den + r2
        assert_blockwise(got, ref, S, npr, "f32", specs[k]["bs"], f"member {k} {specs[k]}")
    assert (num / den) ** 0.5 <= TOL["f32"], (num / den) ** 0.5
    # bit-exact against single launches for a few members of each kind and leaf size
    for k in (0, 1, 2, 3, 100, 101):
        single = plans[k].numeric("f32")
        assert np.array_equal(values_np(single), values_np(batch.outs[k])), k


@pytest.mark.parametrize("kind", ["banded", "growing", "random"])
def test_paper_workloads_reduced(q, kind):
    """The paper's three sequences (band half-width h plus dense diagonal
    blocks by the doubling rule) at n = 6000, h = 300, 64x64 leaves: product
    list and C pattern bit-exact, FP64 and BF16x3 values against the oracle."""
    from tests.gpu_helpers import check_product, units
    a = W.paper_workload(kind, 6000, 64, 300, seed=31)
    for mode in ("f64", "bf16x3"):
        for unit in units(64, mode):
            check_product(q, a, a, mode, unit)


def test_paper_random_blocks_full(q):
    """Random blocks at the first Table 1 size (n = 1e5: the band plus one
    dense 15716 block at a random diagonal position), 64x64 leaves: product
    count from the block pattern, sampled C blocks in FP64 and BF16x3."""
    a = W.paper_workload("random", 100000)
    assert a.meta["dense_blocks"][0][1] == 15716
    A = upload(q, a)
    P = q.Plan(A, A)
    info = P.info()
    # A * A products: sum over block index K of (blocks in column K) * (blocks in row K)
    ccnt = np.bincount(a.bcol, minlength=a.nbc).astype(np.int64)
    rcnt = np.bincount(a.brow, minlength=a.nbr).astype(np.int64)
    assert info["nprod"] == int((ccnt * rcnt).sum())
    oa = O.from_workload(a)
    rng = np.random.default_rng(41)
    p0, sz = a.meta["dense_blocks"][0]
    lo, hi = p0 // 64, (p0 + sz - 1) // 64
    # samples inside the dense block's square, on the band, and at the band's edge
    si = np.concatenate([rng.integers(lo, hi + 1, 12), rng.integers(0, a.nbr, 12), rng.integers(0, a.nbr - 200, 8)])
    sj = np.concatenate([rng.integers(lo, hi + 1, 12), np.clip(si[12:24] + rng.integers(-90, 91, 12), 0, a.nbc - 1),
                         si[24:] + 94])
    key = np.unique(si * a.nbc + sj)
    si, sj = key // a.nbc, key % a.nbc
    ref = O.multiply_blocks(oa, oa, si, sj)
    assert np.linalg.norm(ref) > 0
    for mode in ("f64", "bf16x3"):
        got = sampled_values(P.numeric(mode), si, sj)
        assert_sampled(got, oa, oa, si, sj, ref, mode, what="paper random blocks")
