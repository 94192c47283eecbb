"""Sparse approximate multiply on the GPU against the oracle's.

The selected leaf products are compared bit-exactly (the inputs are checked
to have no norm product within 1e-9 of the tolerance, where the summation
order of the norms could decide); C's pattern bit-exactly; values within the
per-mode tolerances of the oracle's approximate product, and within the
Frobenius error bound of the exact product.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_11762_amd import workloads as W
from tests.gpu_helpers import TOL, assert_product, assert_sampled, pattern_np, units, upload, values_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2011_11762_amd import qbsm
    assert torch.cuda.is_available()
    qbsm.load()
    return qbsm


def _embed(prod, exact):
    """Values of an approximate product on the exact product's pattern."""
    pos = {(i, j): t for t, (i, j) in enumerate(zip(exact.brow.tolist(), exact.bcol.tolist()))}
    full = np.zeros_like(exact.vals)
    for t, (i, j) in enumerate(zip(prod.brow.tolist(), prod.bcol.tolist())):
        full[pos[(i, j)]] = prod.vals[t]
    return full


@pytest.mark.parametrize("npoints,bs", [(1500, 32), (3000, 64)])
def test_spamm_decay_against_oracle(q, npoints, bs):
    c = W.config2(npoints=npoints, bs=bs, seed=12)
    a, tol = c["A"], c["drop_tol"]
    oa = O.from_workload(a, tol)
    A = upload(q, a, tol)
    exact = O.multiply(oa, oa)
    na = O.block_fnorms(oa.vals, bs)
    _, _, _, ia, ib = O.product_triples(oa, oa)
    prodn = na[ia] * na[ib]
    for tau in (1e-9, 1e-6, 1e-3, 1e-1):
        assert O.spamm_borderline(oa, oa, tau) == 0
        ref = O.multiply_spamm(oa, oa, tau)
        assert 0 < ref.I.size < exact.I.size
        bound = prodn[prodn < tau].sum()
        if tau == 1e-1:  # here leaving a product in would show at every mode's tolerance
            assert O.rel_fro(_embed(ref, exact), exact.vals) > 10 * TOL["bf16x3"]
        for mode in ("f64", "bf16x3", "ozaki"):
            for unit in units(bs, mode):
                P = q.Plan(A, A, unit=unit, spamm_tol=tau)
                info = P.info()
                assert info["nprod"] == ref.I.size, (tau, unit)
                assert info["flops"] == O.block_flops(ref.I, ref.J, ref.K, a.nrows, a.ncols, a.ncols, bs)
                gI, gK, gJ = (t.cpu().numpy().astype(np.int64) for t in P.products())
                assert np.array_equal(gI, ref.I) and np.array_equal(gJ, ref.J) and np.array_equal(gK, ref.K)
                C = P.numeric(mode)
                cr, cc = pattern_np(C)
                assert np.array_equal(cr, ref.brow) and np.array_equal(cc, ref.bcol), (tau, mode, unit)
                got = values_np(C)
                assert_product(got, oa, oa, ref.vals, mode, tau=tau, what=f"spamm tau={tau} unit={unit}")
                if mode == "f64":
                    err = np.linalg.norm(_embed(type(ref)(cr, cc, got, ref.I, ref.J, ref.K, ref.seg), exact)
                                         - exact.vals)
                    assert err <= bound * (1 + 1e-9) + 1e-12 * np.linalg.norm(exact.vals)


def test_spamm_zero_tolerance_and_errors(q):
    """spamm_tol 0 is the regular multiply bit for bit; a negative or
    non-finite tolerance is rejected."""
    c = W.config2(npoints=1200, bs=32, seed=13)
    A = upload(q, c["A"], c["drop_tol"])
    plain = values_np(q.matmul(A, A, "f32", unit=64))
    assert np.array_equal(values_np(q.matmul(A, A, "f32", unit=64, spamm_tol=0.0)), plain)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(q.QbsmError):
            q.Plan(A, A, spamm_tol=bad)


def test_spamm_decay_full_sampled(q):
    """The 16384-point decay matrix with tolerance 1e-8: product count from
    the oracle's selection over all 16 M leaf products, sampled C blocks."""
    c = W.config2()
    a, tol = c["A"], c["drop_tol"]
    oa = O.from_workload(a, tol)
    tau = 1e-8
    _, _, _, ia, ib = O.product_triples(oa, oa)
    keep = O.spamm_keep(oa, oa, ia, ib, tau)
    na = O.block_fnorms(oa.vals, 64)
    assert not np.any(np.abs(na[ia] * na[ib] / tau - 1.0) < 1e-9)
    A = upload(q, a, tol)
    P = q.Plan(A, A, spamm_tol=tau)
    assert P.info()["nprod"] == int(keep.sum())
    del ia, ib, keep
    rng = np.random.default_rng(23)
    si, sj = rng.integers(0, 256, 40), rng.integers(0, 256, 40)
    key = np.unique(si * 256 + sj)
    si, sj = key // 256, key % 256
    ref = O.multiply_blocks(oa, oa, si, sj, tau=tau)
    for mode in ("f64", "bf16x3"):
        got = P.numeric(mode).extract(si, sj).cpu().numpy()
        assert_sampled(got, oa, oa, si, sj, ref, mode, tau=tau, what="spamm decay sampled")
