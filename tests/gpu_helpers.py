"""Shared helpers of the GPU parity tests (device upload, oracle comparison)."""
import numpy as np
import torch

from oracle import oracle as O
from tests.bounds import assert_blockwise

# relative Frobenius tolerances against the FP64 oracle on the original inputs
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2, "bf16x3": 1e-4, "ozaki": 1e-11}
# Ozaki mode against the oracle's own Ozaki splitting and product: the slice
# products are exact on both sides, only the FP64 accumulation order differs
TOL_OZAKI_EMULATED = 1e-13
# BF16: against the FP64 oracle applied to the bf16-rounded inputs (isolates
# the FP32 accumulation)
TOL_BF16_ROUNDED = 1e-5
# work-unit sides valid per leaf size (unit = bs * 2^s, s <= 2); unit 256
# serves the FP32-accumulating modes only
UNITS = {32: (64, 128), 64: (64, 128, 256), 128: (128, 256)}


def units(bs, mode):
    if mode == "ozaki":  # 64-wide integer MFMA: 64 x 64 leaves at unit 64 or 128
        return (64, 128) if bs == 64 else ()
    return tuple(u for u in UNITS[bs] if not (u == 256 and mode == "f64"))


def upload(q, m, drop_tol=0.0):
    return q.from_host(m, drop_tol)


def pattern_np(M):
    r, c = M.pattern()
    return r.cpu().numpy().astype(np.int64), c.cpu().numpy().astype(np.int64)


def values_np(M):
    return M.values().cpu().numpy()


def rounded(om, fn):
    return O.OMatrix(om.nrows, om.ncols, om.bs, om.brow, om.bcol, fn(om.vals))


def check_product(q, a, b, mode, unit, drop_tol=0.0, ref=None, check_products=True):
    """Runs C = A B on the GPU and compares with the oracle; returns (C, ref, err)."""
    A = upload(q, a, drop_tol)
    B = A if b is a else upload(q, b, drop_tol)
    oa = O.from_workload(a, drop_tol)
    ob = oa if b is a else O.from_workload(b, drop_tol)
    if ref is None:
        ref = O.multiply(oa, ob)
    P = q.Plan(A, B, unit=unit)
    info = P.info()
    C = P.numeric(mode)
    torch.cuda.synchronize()
    cr, cc = pattern_np(C)
    assert np.array_equal(cr, ref.brow) and np.array_equal(cc, ref.bcol), "C pattern differs"
    assert info["nblk_out"] == ref.brow.size and info["nprod"] == ref.I.size
    assert info["flops"] == O.block_flops(ref.I, ref.J, ref.K, a.nrows, a.ncols, b.ncols, a.bs)
    if check_products:
        I, K, J = (t.cpu().numpy().astype(np.int64) for t in P.products())
        assert np.array_equal(I, ref.I) and np.array_equal(J, ref.J) and np.array_equal(K, ref.K), \
            "product list differs"
    got = values_np(C)
    err = assert_product(got, oa, ob, ref.vals, mode, what=f"unit={unit}")
    if mode == "bf16":
        rr = O.multiply(rounded(oa, O.round_to_bf16), rounded(ob, O.round_to_bf16))
        e2 = O.rel_fro(got, rr.vals)
        assert e2 <= TOL_BF16_ROUNDED, f"bf16 vs rounded-input oracle {e2:.3e}"
    return C, ref, err, got


def padding_is_zero(vals, brow, bcol, nrows, ncols, bs):
    v = vals.reshape(-1, bs, bs)  # [blk, c, r]
    for t in range(brow.size):
        mr = min(bs, nrows - brow[t] * bs)
        nc = min(bs, ncols - bcol[t] * bs)
        if np.any(v[t, nc:, :] != 0) or np.any(v[t, :, mr:] != 0):
            return False
    return True


def assert_values(got, ref_vals, S, nprod, mode, bs, what=""):
    """Values against the FP64 oracle: the relative Frobenius norm over all
    blocks within TOL[mode], and every block within its own normwise bound
    (tests/bounds.py).  Returns the relative error."""
    err = O.rel_fro(got, ref_vals)
    assert err <= TOL[mode], f"{what} {mode}: rel err {err:.3e} > {TOL[mode]:.1e}"
    assert_blockwise(got, ref_vals, S, nprod, mode, bs, what)
    return err


def assert_product(got, oa, ob, ref_vals, mode, trans_a=False, trans_b=False, tau=0.0, what=""):
    """assert_values for C = op(A) op(B) (sparse approximate when tau > 0),
    with the bound terms taken from the oracle."""
    S, npr = O.block_bound_terms(oa, ob, trans_a, trans_b, tau)
    return assert_values(got, ref_vals, S, npr, mode, oa.bs, what)


def assert_sampled(got, oa, ob, si, sj, ref_vals, mode, tau=0.0, what=""):
    """assert_values on selected C blocks (si[q], sj[q]) of A B."""
    S, npr = O.sampled_bound_terms(oa, ob, si, sj, tau)
    return assert_values(got, ref_vals, S, npr, mode, oa.bs, what)


def _restricted_terms(l, r, trans_l, trans_r, mask):
    """Bound terms of op(L) op(R) on the blocks of `mask` (0 where no product)."""
    I, J, _, _, _ = O.product_triples(l, r, trans_l, trans_r)
    ci, cj, _ = O.c_pattern_from_triples(I, J)
    S, npr = O.block_bound_terms(l, r, trans_l, trans_r)
    nbc = int(max(mask.bcol.max(initial=0), cj.max(initial=0)) + 1)
    pos = {int(k): t for t, k in enumerate((ci * nbc + cj).tolist())}
    Sm, nm = np.zeros(mask.nblk), np.zeros(mask.nblk, dtype=np.int64)
    for q, k in enumerate((mask.brow * nbc + mask.bcol).tolist()):
        t = pos.get(int(k))
        if t is not None:
            Sm[q], nm[q] = S[t], npr[t]
    return Sm, nm


def assert_backward(dA, dB, oa, ob, odc, ga, gb, mode, what=""):
    """Masked adjoints against the oracle: dA = (dC B^T) on A's blocks, dB =
    (A^T dC) on B's blocks, globally and block by block (a mask block with no
    product must be exactly zero)."""
    Sa, na = _restricted_terms(odc, ob, False, True, oa)
    Sb, nb = _restricted_terms(oa, odc, True, False, ob)
    ea = assert_values(dA, ga, Sa, na, mode, oa.bs, what + " dA")
    eb = assert_values(dB, gb, Sb, nb, mode, ob.bs, what + " dB")
    return ea, eb
