"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Every check here is independent of the GPU library: textbook dense GEMM,
brute-force enumeration, algebraic identities, the paper's printed Table 1,
and closed-form counts of the banded workloads.
"""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2011_11762_amd import workloads as W  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def om(m, tol=0.0):
    return O.from_workload(m, tol)


def dense_of(nrows, ncols, bs, brow, bcol, vals):
    nbr, nbc = -(-nrows // bs), -(-ncols // bs)
    out = np.zeros((nbr * bs, nbc * bs))
    for t in range(len(brow)):
        i, j = int(brow[t]), int(bcol[t])
        out[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] = np.asarray(vals[t]).reshape(bs, bs).T
    return out[:nrows, :ncols]


def transpose_matrix(a: O.OMatrix) -> O.OMatrix:
    bs = a.bs
    v = a.vals.reshape(-1, bs, bs).transpose(0, 2, 1).reshape(-1, bs * bs)
    return O.canonical(a.ncols, a.nrows, bs, a.bcol, a.brow, v)


# ---------------------------------------------------------------- dense GEMM
@pytest.mark.parametrize("m,k,n,bs,p,seed", [
    (64, 64, 64, 16, 0.5, 10),
    (100, 70, 90, 16, 0.4, 11),      # ragged in every dimension
    (130, 257, 33, 32, 0.6, 12),     # ragged, rectangular
    (48, 48, 48, 8, 1.0, 13),        # fully dense
    (300, 300, 300, 64, 0.3, 14),
])
def test_dense_gemm(m, k, n, bs, p, seed):
    a, b = W.small_random(m, k, n, bs, p, seed)
    A, B = om(a), om(b)
    C = O.multiply(A, B)
    got = dense_of(m, n, bs, C.brow, C.bcol, C.vals)
    ref = a.to_dense() @ b.to_dense()
    scale = np.abs(a.to_dense()) @ np.abs(b.to_dense())
    assert np.all(np.abs(got - ref) <= 4 * k * 2.0 ** -53 * scale + 1e-300)
    # padding of edge blocks stays zero
    full = np.zeros((C.brow.size, bs, bs))
    full[:] = C.vals.reshape(-1, bs, bs)
    for t in range(C.brow.size):
        mr = min(bs, m - C.brow[t] * bs)
        nc = min(bs, n - C.bcol[t] * bs)
        assert np.all(full[t, nc:, :] == 0) and np.all(full[t, :, mr:] == 0)


def test_all_nil_operands():
    a, b = W.small_random(64, 64, 64, 16, 0.5, 3)
    A, B = om(a), om(b)
    Z = O.canonical(64, 64, 16, [], [], np.zeros((0, 256)))
    for x, y in ((Z, B), (A, Z), (Z, Z)):
        C = O.multiply(x, y)
        assert C.brow.size == 0 and C.vals.shape == (0, 256)


# ------------------------------------------------------- products / pattern
def brute_triples(A, B):
    sa = {(int(i), int(k)) for i, k in zip(A.brow, A.bcol)}
    sb = {(int(k), int(j)) for k, j in zip(B.brow, B.bcol)}
    nbi, nbk, nbj = -(-A.nrows // A.bs), -(-A.ncols // A.bs), -(-B.ncols // B.bs)
    out = []
    for i in range(nbi):
        for j in range(nbj):
            for k in range(nbk):
                if (i, k) in sa and (k, j) in sb:
                    out.append((i, j, k))
    return out


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_products_brute_force(seed):
    a, b = W.small_random(160, 120, 200, 8, 0.2, seed)
    A, B = om(a), om(b)
    I, J, K, ia, ib = O.product_triples(A, B)
    assert list(zip(I.tolist(), J.tolist(), K.tolist())) == brute_triples(A, B)
    # indices point at the right stored blocks
    assert np.array_equal(A.brow[ia], I) and np.array_equal(A.bcol[ia], K)
    assert np.array_equal(B.brow[ib], K) and np.array_equal(B.bcol[ib], J)


def check_pattern(A, B):
    I, J, K, _, _ = O.product_triples(A, B)
    ci, cj, seg = O.c_pattern_from_triples(I, J)
    bi, bj, cnt = O.boolean_pattern_product(A, B)
    assert np.array_equal(ci, bi) and np.array_equal(cj, bj)
    assert np.array_equal(np.diff(seg), cnt)
    return ci.size, I.size


def test_pattern_config1_closed_form():
    c = W.config1()
    A, B = om(c["A"]), om(c["B"])
    assert (A.nblk, B.nblk) == (556, 556)
    nc, npr = check_pattern(A, B)
    assert (nc, npr) == (1016, 4884)


def test_pattern_config5_closed_form():
    c = W.config5()
    A, B = om(c["A"]), om(c["B"])
    assert A.nblk == 3286
    nc, npr = check_pattern(A, B)
    assert (nc, npr) == (6244, 42354)
    dc = om(c["dC"])
    C = O.multiply(A, B)
    assert np.array_equal(dc.brow, C.brow) and np.array_equal(dc.bcol, C.bcol)


def test_pattern_config3():
    c = W.config3()
    A, B = om(c["A"]), om(c["B"])
    nc, npr = check_pattern(A, B)
    assert 2400 < A.nblk < 2850 and 2400 < B.nblk < 2850
    assert npr >= nc > 0


@pytest.mark.slow
def test_pattern_config2_after_drop():
    c = W.config2()
    A = om(c["A"], c["drop_tol"])
    assert not np.any(O.borderline(c["A"].vals, 64, c["drop_tol"]))
    assert 0.97 * 65536 < A.nblk < 0.99 * 65536
    nc, npr = check_pattern(A, A)
    assert nc == 65536


def test_pattern_config4_small_members():
    specs = [s for s in W.config4_members() if s["n"] <= 3000][:4]
    assert specs
    for s in specs:
        mem = W.config4_member(s)
        A, B = om(mem["A"], mem["drop_tol"]), om(mem["B"], mem["drop_tol"])
        check_pattern(A, B)


# --------------------------------------------------------------- identities
def identity_matrix(n, bs):
    nb = -(-n // bs)
    vals = np.zeros((nb, bs * bs))
    for t in range(nb):
        d = min(bs, n - t * bs)
        for e in range(d):
            vals[t, e + e * bs] = 1.0
    return O.canonical(n, n, bs, np.arange(nb), np.arange(nb), vals)


def test_identity_bit_exact():
    a, _ = W.small_random(120, 90, 10, 16, 0.5, 7)
    A = om(a)
    for C in (O.multiply(A, identity_matrix(90, 16)), O.multiply(identity_matrix(120, 16), A)):
        assert np.array_equal(C.brow, A.brow) and np.array_equal(C.bcol, A.bcol)
        assert np.array_equal(C.vals, A.vals)


def test_transpose_bit_exact():
    a, b = W.small_random(100, 140, 75, 16, 0.5, 8)
    A, B = om(a), om(b)
    C = O.multiply(A, B)
    Ct = transpose_matrix(O.canonical(100, 75, 16, C.brow, C.bcol, C.vals))
    D = O.multiply(transpose_matrix(B), transpose_matrix(A))
    assert np.array_equal(D.brow, Ct.brow) and np.array_equal(D.bcol, Ct.bcol)
    assert np.array_equal(D.vals, Ct.vals)
    # the same through the oracle's transposed-operand path
    E = O.multiply(B, A, trans_a=True, trans_b=True)
    assert np.array_equal(E.vals, Ct.vals)


def test_associativity_distributivity():
    rng = np.random.default_rng(9)
    bs = 16
    a = W.random_blocks(96, bs, 0.4, rng, ncols=80)
    b = W.random_blocks(80, bs, 0.4, rng, ncols=112)
    c = W.random_blocks(112, bs, 0.4, rng, ncols=64)
    b2 = W.random_blocks(80, bs, 0.4, rng, ncols=112)
    A, B, Cm, B2 = om(a), om(b), om(c), om(b2)

    def mat(p, nr, nc):
        return O.canonical(nr, nc, bs, p.brow, p.bcol, p.vals)

    AB = mat(O.multiply(A, B), 96, 112)
    BC = mat(O.multiply(B, Cm), 80, 64)
    L, R = O.multiply(AB, Cm), O.multiply(A, BC)
    bi, bj, _ = O.boolean_pattern_product(mat(O.multiply(A, B), 96, 112), Cm)
    assert np.array_equal(L.brow, R.brow) and np.array_equal(L.bcol, R.bcol)
    assert np.array_equal(L.brow, bi) and np.array_equal(L.bcol, bj)
    absd = lambda m: np.abs(m.to_dense()) if hasattr(m, "to_dense") else None  # noqa: E731
    scale = np.abs(a.to_dense()) @ np.abs(b.to_dense()) @ np.abs(c.to_dense())
    gam = 2 * (80 + 112) * 2.0 ** -53
    diff = dense_of(96, 64, bs, L.brow, L.bcol, L.vals) - dense_of(96, 64, bs, R.brow, R.bcol, R.vals)
    assert np.all(np.abs(diff) <= gam * scale)
    # A (B + B2) = A B + A B2 on the union pattern
    dsum = b.to_dense() + b2.to_dense()
    bsum_blocks = np.unique(np.concatenate([B.brow * 1000 + B.bcol, B2.brow * 1000 + B2.bcol]))
    bi_, bj_ = bsum_blocks // 1000, bsum_blocks % 1000
    vals = np.stack([dsum[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs].T.ravel() for i, j in zip(bi_, bj_)])
    S = O.canonical(80, 112, bs, bi_, bj_, vals)
    lhs = O.multiply(A, S)
    lhs_d = dense_of(96, 112, bs, lhs.brow, lhs.bcol, lhs.vals)
    r1, r2 = O.multiply(A, B), O.multiply(A, B2)
    rhs_d = dense_of(96, 112, bs, r1.brow, r1.bcol, r1.vals) + dense_of(96, 112, bs, r2.brow, r2.bcol, r2.vals)
    sc = np.abs(a.to_dense()) @ (np.abs(b.to_dense()) + np.abs(b2.to_dense()))
    assert np.all(np.abs(lhs_d - rhs_d) <= 2 * 80 * 2.0 ** -53 * sc * 2)
    _ = absd


# ----------------------------------------------------------------- flops
def interval_union_len(ivs):
    ivs = sorted(ivs)
    tot, cur_lo, cur_hi = 0, None, None
    for lo, hi in ivs:
        if cur_hi is None or lo > cur_hi + 1:
            if cur_hi is not None:
                tot += cur_hi - cur_lo + 1
            cur_lo, cur_hi = lo, hi
        else:
            cur_hi = max(cur_hi, hi)
    if cur_hi is not None:
        tot += cur_hi - cur_lo + 1
    return tot


def column_counts_banded(n, h, block=0):
    """Nonzeros per column of band(h) plus an optional dense upper-left block,
    from the pattern's definition as a union of row intervals per column."""
    k = np.arange(n, dtype=np.int64)
    band = np.minimum(k + h, n - 1) - np.maximum(k - h, 0) + 1
    if block:
        for kk in range(block):
            band[kk] = interval_union_len([(max(0, kk - h), min(n - 1, kk + h)), (0, block - 1)])
    return band


def test_table1_flops_reproduced():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "table1_tflop.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 7
    for n_s, band_s, blk_s, gb_s in rows:
        n, blk = int(n_s), int(blk_s)
        r = column_counts_banded(n, 3000)
        assert f"{O.element_flops(r, r) / 1e12:.4g}" == band_s
        r2 = column_counts_banded(n, 3000, block=blk)
        assert f"{O.element_flops(r2, r2) / 1e12:.4g}" == gb_s


def test_block_flops_brute_force():
    a, b = W.small_random(70, 45, 52, 16, 0.6, 5)
    A, B = om(a), om(b)
    I, J, K, _, _ = O.product_triples(A, B)
    got = O.block_flops(I, J, K, 70, 45, 52, 16)
    cnt = 0
    for i, j, k in zip(I, J, K):
        for r in range(i * 16, min(70, (i + 1) * 16)):
            for c in range(j * 16, min(52, (j + 1) * 16)):
                cnt += min(45, (k + 1) * 16) - k * 16
    assert got == 2 * cnt
    # fully dense blocks, divisible sizes: block count == element count
    rng = np.random.default_rng(0)
    d = W.random_blocks(64, 16, 1.0, rng)
    D = om(d)
    I, J, K, _, _ = O.product_triples(D, D)
    dense = d.to_dense() != 0
    assert O.block_flops(I, J, K, 64, 64, 64, 16) == O.element_flops(dense.sum(0), dense.sum(1))


# --------------------------------------------------------------- backward
def test_backward_finite_differences_and_adjoint():
    rng = np.random.default_rng(21)
    bs = 8
    a = W.random_blocks(40, bs, 0.5, rng, ncols=48)
    b = W.random_blocks(48, bs, 0.5, rng, ncols=32)
    A, B = om(a), om(b)
    C = O.multiply(A, B)
    dcv = rng.uniform(-1, 1, size=C.vals.shape)
    dC = O.canonical(40, 32, bs, C.brow, C.bcol, dcv)
    dA, dB = O.backward(A, B, dC)

    def loss(Am, Bm):
        P = O.multiply(Am, Bm)
        return float(np.sum(P.vals * dcv))

    for _ in range(12):
        t = int(rng.integers(A.nblk))
        e = int(rng.integers(bs * bs))
        Ap, Am_ = O.OMatrix(**{**A.__dict__, "vals": A.vals.copy()}), O.OMatrix(**{**A.__dict__, "vals": A.vals.copy()})
        Ap.vals[t, e] += 1.0
        Am_.vals[t, e] -= 1.0
        fd = (loss(Ap, B) - loss(Am_, B)) / 2.0
        assert abs(fd - dA[t, e]) <= 1e-12 * (1 + abs(fd))
        t = int(rng.integers(B.nblk))
        Bp, Bm_ = O.OMatrix(**{**B.__dict__, "vals": B.vals.copy()}), O.OMatrix(**{**B.__dict__, "vals": B.vals.copy()})
        Bp.vals[t, e] += 1.0
        Bm_.vals[t, e] -= 1.0
        fd = (loss(A, Bp) - loss(A, Bm_)) / 2.0
        assert abs(fd - dB[t, e]) <= 1e-12 * (1 + abs(fd))
    l0 = float(np.sum(C.vals * dcv))
    assert abs(np.sum(dA * A.vals) - l0) <= 1e-12 * (1 + abs(l0))
    assert abs(np.sum(dB * B.vals) - l0) <= 1e-12 * (1 + abs(l0))
    # against dense autograd-free formulas
    Dd, Bd, Ad = dense_of(40, 32, bs, C.brow, C.bcol, dcv), b.to_dense(), a.to_dense()
    gA, gB = Dd @ Bd.T, Ad.T @ Dd
    got_a = dense_of(40, 48, bs, A.brow, A.bcol, dA)
    got_b = dense_of(48, 32, bs, B.brow, B.bcol, dB)
    ma = dense_of(40, 48, bs, A.brow, A.bcol, np.ones_like(A.vals)) != 0
    mb = dense_of(48, 32, bs, B.brow, B.bcol, np.ones_like(B.vals)) != 0
    assert np.allclose(got_a, np.where(ma, gA, 0), rtol=0, atol=1e-13)
    assert np.allclose(got_b, np.where(mb, gB, 0), rtol=0, atol=1e-13)


# ------------------------------------------------------- norms / drop rule
def test_block_norms_and_drop_rule():
    rng = np.random.default_rng(4)
    v = rng.standard_normal((50, 64))
    n = O.block_fnorms(v, 8)
    ref = np.linalg.norm(v, axis=1)
    assert np.allclose(n, ref, rtol=4e-16 * 64, atol=0)
    blk = np.zeros((4, 4))
    blk[0, 0] = 0.5
    vals = np.stack([blk.ravel(), blk.ravel() * (1 - 2.0 ** -52), np.full(16, np.nan), np.zeros(16)])
    keep = O.keep_mask(vals, 4, 0.5)
    assert keep.tolist() == [True, False, True, False]
    assert O.keep_mask(vals, 4, 0.0).all()


# ------------------------------------------------------ precision roundings
def test_bf16_rounding():
    import torch
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -40, -(1 + 2 ** -8),
                  3.0e38, 3.4e38, 2.0 ** -130, -2.0 ** -133 * 1.5, 0.0, np.inf, -np.inf])
    got = O.round_to_bf16(x)
    exp = [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -1.0, 3.0e38, np.inf, 2.0 ** -130, -2.0 ** -132, 0.0,
           np.inf, -np.inf]
    assert np.allclose(got[[0, 1, 2, 3, 4, 7, 8, 9]], np.array(exp)[[0, 1, 2, 3, 4, 7, 8, 9]], rtol=0, atol=0)
    assert abs(got[5] - 3.0e38) / 3.0e38 < 2 ** -8 and np.isinf(got[6]) and np.isinf(got[10])
    assert np.isnan(O.round_to_bf16(np.array([np.nan]))[0])
    # values exactly representable in binary32: torch's binary32 -> bfloat16 RNE
    rng = np.random.default_rng(0)
    f = (rng.standard_normal(100000) * np.exp(rng.uniform(-30, 30, 100000))).astype(np.float32)
    ref = torch.from_numpy(f).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.round_to_bf16(f.astype(np.float64)), ref)
    # split: hi + lo carries ~16 bits
    xd = rng.uniform(-1, 1, 100000)
    hi, lo = O.split_bf16(xd)
    assert np.array_equal(O.round_to_bf16(hi), hi) and np.array_equal(O.round_to_bf16(lo), lo)
    assert np.all(np.abs(xd - hi - lo) <= 2.0 ** -16 * np.abs(xd) + 1e-300)
    # non-finite hi part: zero residual (Inf stays Inf in hi*lo + lo*hi + hi*hi)
    hi, lo = O.split_bf16(np.array([np.inf, -np.inf, np.nan, 1e39, -4e38, 3.0e38]))
    assert np.isposinf(hi[0]) and np.isneginf(hi[1]) and np.isnan(hi[2])
    assert np.isposinf(hi[3]) and np.isneginf(hi[4]) and np.isfinite(hi[5])
    assert np.array_equal(lo[:5], np.zeros(5)) and np.isfinite(lo[5])


def test_canonical_rejects_bad_input():
    v = np.zeros((2, 4))
    with pytest.raises(ValueError):
        O.canonical(4, 4, 2, [0, 0], [1, 1], v)
    with pytest.raises(ValueError):
        O.canonical(4, 4, 2, [0, 2], [0, 0], v)


def test_multiply_blocks_matches_full():
    a, b = W.small_random(200, 160, 180, 16, 0.3, 17)
    A, B = om(a), om(b)
    C = O.multiply(A, B)
    pick = np.arange(0, C.brow.size, 3)
    got = O.multiply_blocks(A, B, C.brow[pick], C.bcol[pick])
    assert np.array_equal(got, C.vals[pick])


def _balanced_digits(m_int: int, n: int, bits: int):
    """Digits d_1 .. d_n (highest first) of the integer m_int in balanced base
    2^bits, each in [-2^(bits-1), 2^(bits-1)), by plain integer arithmetic;
    None if n digits do not reach m_int."""
    half, base = 1 << (bits - 1), 1 << bits
    out = []
    for _ in range(n):
        d = (m_int + half) % base - half
        out.append(d)
        m_int = (m_int - d) // base
    return None if m_int else out[::-1]


def test_ozaki_split_exact_slices_and_reconstruction():
    """Slices are 8-bit integers (balanced digits in [-128, 127]) on the
    grid 2^(e + 1 - 8 t) of the line's exponent, they are the balanced base-256
    digits of the element truncated to 47 bits below the line exponent (checked
    against Python integer arithmetic element by element), and a line whose
    maximum lies within 0.4 % below a power of two takes the next exponent."""
    rng = np.random.default_rng(5)
    bs = 16
    vals = rng.standard_normal((7, bs * bs)) * np.exp(rng.uniform(-20, 20, (7, 1)))
    vals[2, :] = 0.0                        # an all-zero block
    vals[3, 5] = 2.0 ** 10                  # an exact power of two as a line maximum
    vals[4, 0:bs] *= -1.0
    vals[5, 3] = (2.0 ** 47 - 5) * 2.0 ** -40          # just below 2^7: its line is raised
    vals[6, 7 * bs + 2] = -(2.0 ** 47 - 5) * 2.0 ** -60
    assert O.OZ_SLICES * O.OZ_BITS == 48 and O.OZ_MANT == 47 and O.OZ_MAXM == 127 * (2 ** 48 - 1) // 255
    for line in ("row", "col"):
        sl = O.ozaki_split(vals, bs, line)
        assert sl.shape == (O.OZ_SLICES, 7, bs * bs)
        v = vals.reshape(-1, bs, bs)
        m = np.abs(v).max(axis=1 if line == "row" else 2, keepdims=True)
        _, e0 = np.frexp(m)
        e = O.ozaki_exponent(m)
        assert np.all((e == e0) | (e == e0 + 1))
        raised = e != e0
        assert np.all(m[raised] >= 0.996 * np.ldexp(1.0, e0[raised])) and raised.any()
        e = np.broadcast_to(e, v.shape).reshape(-1, bs * bs)
        q = np.stack([np.ldexp(sl[t - 1], -(e + 1 - O.OZ_BITS * t)) for t in range(1, O.OZ_SLICES + 1)])
        assert np.array_equal(q, np.rint(q)) and q.min() >= -128 and q.max() <= 127
        # element by element against integer arithmetic
        for blk, idx in [(0, 0), (0, 17), (1, 100), (3, 5), (4, 3), (5, 3), (6, 7 * bs + 2), (6, 200)]:
            x = vals[blk, idx]
            mint = int(np.sign(x)) * int(np.floor(np.ldexp(abs(x), O.OZ_MANT - int(e[blk, idx]))))
            want = _balanced_digits(mint, O.OZ_SLICES, O.OZ_BITS)
            assert want is not None and [int(d) for d in q[:, blk, idx]] == want
        rec = sl.sum(axis=0)
        err = np.abs(vals - rec)
        assert np.all(err < np.ldexp(1.0, e - O.OZ_MANT))
        assert np.all(np.abs(rec) <= np.abs(vals))           # truncation toward zero
        assert np.all(sl[:, 2] == 0)
    # values with at most 46 bits below the line exponent split exactly
    ints = rng.integers(-(2 ** 46), 2 ** 46, (3, bs * bs)).astype(np.float64)
    ints[:, 0] = 2.0 ** 46 - 1                                # line maxima just below 2^46
    x = np.ldexp(ints, -30)
    for line in ("row", "col"):
        assert np.array_equal(O.ozaki_split(x, bs, line).sum(axis=0), x)


def test_ozaki_split_nonfinite_and_sign():
    bs = 4
    v = np.zeros((1, 16))
    v[0, :] = np.arange(1, 17, dtype=np.float64)
    v[0, 5] = np.inf
    v[0, 6] = -3.5
    sl = O.ozaki_split(v, bs, "col")
    assert np.isposinf(sl[0, 0, 5]) and np.all(sl[1:, 0, 5] == 0)
    assert sl.sum(axis=0)[0, 6] == -3.5                       # finite neighbours exact
    assert np.all(np.isfinite(np.delete(sl.sum(axis=0)[0], 5)))


def test_ozaki_multiply_against_fp64():
    """Slice products are exact, so inputs on the grid 2^(e - 22) of their
    line exponents (their expansions end at the third digit, and every pair of
    the first three slices is kept) give the FP64 product up to the FP64
    accumulation; general inputs differ from it by the 47-bit truncation and
    the dropped pairs only."""
    a, b = W.small_random(150, 130, 170, 32, 0.6, 7)
    oa, ob = O.from_workload(a), O.from_workload(b)
    ref = O.multiply(oa, ob)
    oz = O.ozaki_multiply(oa, ob)
    assert np.array_equal(oz.brow, ref.brow) and np.array_equal(oz.bcol, ref.bcol)
    assert O.rel_fro(oz.vals, ref.vals) < 1e-13

    def on_grid(m, line):
        v = m.vals.reshape(-1, m.bs, m.bs)
        mx = np.abs(v).max(axis=1 if line == "row" else 2, keepdims=True)
        _, e0 = np.frexp(mx)
        g = np.ldexp(np.rint(np.ldexp(v, 22 - e0)), e0 - 22)
        return O.OMatrix(m.nrows, m.ncols, m.bs, m.brow, m.bcol, g.reshape(m.vals.shape))

    ag, bg = on_grid(oa, "row"), on_grid(ob, "col")
    for sl in (O.ozaki_split(ag.vals, ag.bs, "row"), O.ozaki_split(bg.vals, bg.bs, "col")):
        assert not np.any(sl[3:])                            # three digits carry them
    rg, zg = O.multiply(ag, bg), O.ozaki_multiply(ag, bg)
    scale = np.abs(rg.vals).max()
    assert np.max(np.abs(zg.vals - rg.vals)) <= 64 * 2.0 ** -52 * scale
    # a dropped term is visible: with 2 slices of 8 bits the error is ~2^-15
    r2 = O.ozaki_multiply(oa, ob, slices=2)
    assert 1e-7 < O.rel_fro(r2.vals, ref.vals) < 1e-3


# ---------------------------------------------------------------- sparse approximate multiply
def _decay_like(n, bs, seed):
    """Small matrix with entries decaying away from the diagonal (block norms spread over decades)."""
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    dense = rng.uniform(-1, 1, (n, n)) * np.exp(-0.35 * np.abs(i - j))
    nb = -(-n // bs)
    blocks, br, bc = [], [], []
    for I in range(nb):
        for J in range(nb):
            blk = np.zeros((bs, bs))
            sub = dense[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
            blk[:sub.shape[0], :sub.shape[1]] = sub
            br.append(I)
            bc.append(J)
            blocks.append(blk.T.ravel())  # column-major
    return O.canonical(n, n, bs, np.array(br), np.array(bc), np.array(blocks))


def test_spamm_zero_tolerance_is_the_multiply():
    a = _decay_like(150, 16, 1)
    b = _decay_like(150, 16, 2)
    s, r = O.multiply_spamm(a, b, 0.0), O.multiply(a, b)
    assert np.array_equal(s.brow, r.brow) and np.array_equal(s.bcol, r.bcol)
    assert np.array_equal(s.vals, r.vals) and np.array_equal(s.K, r.K)


def test_spamm_brute_force():
    """Against explicit loops over (I, K, J) with norms summed element by element."""
    bs, n = 8, 45
    a, b = _decay_like(n, bs, 3), _decay_like(n, bs, 4)
    tau = 0.05
    nb = -(-n // bs)

    def blk(m, I, J):
        for t in range(m.nblk):
            if m.brow[t] == I and m.bcol[t] == J:
                return m.vals[t].reshape(bs, bs).T
        return None

    want = {}
    kept = []
    for I in range(nb):
        for J in range(nb):
            acc, any_ = np.zeros((bs, bs)), False
            for K in range(nb):
                x, y = blk(a, I, K), blk(b, K, J)
                if x is None or y is None:
                    continue
                nx = sum(float(v) * float(v) for v in x.ravel()) ** 0.5
                ny = sum(float(v) * float(v) for v in y.ravel()) ** 0.5
                if nx * ny < tau:
                    continue
                kept.append((I, J, K))
                acc += x @ y
                any_ = True
            if any_:
                want[(I, J)] = acc
    got = O.multiply_spamm(a, b, tau)
    assert O.spamm_borderline(a, b, tau) == 0
    assert list(zip(got.I.tolist(), got.J.tolist(), got.K.tolist())) == kept
    assert list(zip(got.brow.tolist(), got.bcol.tolist())) == sorted(want)
    for t, key in enumerate(zip(got.brow.tolist(), got.bcol.tolist())):
        np.testing.assert_allclose(got.vals[t].reshape(bs, bs).T, want[key], rtol=0, atol=1e-13)
    assert 0 < len(kept) < O.product_triples(a, b)[0].size  # the test really skips products


def test_spamm_error_bound_and_monotone():
    """||C_spamm - C||_F <= sum over skipped products of ||A_IK|| ||B_KJ|| (sub-
    multiplicativity of the Frobenius norm); a larger tolerance keeps a subset."""
    a, b = _decay_like(256, 16, 5), _decay_like(256, 16, 6)
    exact = O.multiply(a, b)
    na, nb = O.block_fnorms(a.vals, 16), O.block_fnorms(b.vals, 16)
    _, _, _, ia, ib = O.product_triples(a, b)
    prev = None
    for tau in (1e-8, 1e-5, 1e-3, 1e-1):
        s = O.multiply_spamm(a, b, tau)
        # embed the approximate result in the exact pattern
        pos = {(i, j): t for t, (i, j) in enumerate(zip(exact.brow.tolist(), exact.bcol.tolist()))}
        full = np.zeros_like(exact.vals)
        for t, (i, j) in enumerate(zip(s.brow.tolist(), s.bcol.tolist())):
            full[pos[(i, j)]] = s.vals[t]
        err = np.linalg.norm(full - exact.vals)
        skipped = na[ia] * nb[ib]
        bound = skipped[skipped < tau].sum()
        assert err <= bound * (1 + 1e-12) + 1e-300
        triples = set(zip(s.I.tolist(), s.J.tolist(), s.K.tolist()))
        if prev is not None:
            assert triples <= prev
        prev = triples


def _decay_rect(m, n, bs, rate, seed, shift=0):
    """Rectangular block matrix whose entries decay away from the line i = j + shift."""
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    dense = rng.uniform(-1, 1, (m, n)) * np.exp(-rate * np.abs(i - j - shift))
    nbr, nbc = -(-m // bs), -(-n // bs)
    br, bc, blocks = [], [], []
    for I in range(nbr):
        for J in range(nbc):
            blk = np.zeros((bs, bs))
            sub = dense[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
            blk[:sub.shape[0], :sub.shape[1]] = sub
            br.append(I)
            bc.append(J)
            blocks.append(blk.T.ravel())
    return O.canonical(m, n, bs, np.array(br), np.array(bc), np.array(blocks))


def test_sampled_spamm_blocks_match_the_approximate_product():
    """multiply_blocks with tau > 0 (the sampled path of the sparse
    approximate multiply) gives exactly the blocks of multiply_spamm, and its
    bound terms those of block_bound_terms.  A and B differ in shape, decay
    rate and offset, so a norm taken from the wrong operand or index changes
    the kept set."""
    bs = 16
    a = _decay_rect(200, 120, bs, 0.30, 21, shift=40)
    b = _decay_rect(120, 168, bs, 0.08, 22, shift=-25)
    tau = 0.5
    full = O.multiply_spamm(a, b, tau)
    exact = O.multiply(a, b)
    assert 0 < full.I.size < exact.I.size  # the test really leaves products out
    nbr, nbc = -(-200 // bs), -(-168 // bs)
    si, sj = np.meshgrid(np.arange(nbr), np.arange(nbc), indexing="ij")
    si, sj = si.ravel(), sj.ravel()
    got = O.multiply_blocks(a, b, si, sj, tau)
    pos = {(i, j): t for t, (i, j) in enumerate(zip(full.brow.tolist(), full.bcol.tolist()))}
    for q, (i, j) in enumerate(zip(si.tolist(), sj.tolist())):
        t = pos.get((i, j))
        if t is None:
            assert not np.any(got[q])
        else:
            assert np.array_equal(got[q], full.vals[t]), (i, j)
    # selected blocks whose products are all left out exist and come back zero
    assert any((i, j) not in pos for i, j in zip(exact.brow.tolist(), exact.bcol.tolist()))
    S, npr = O.block_bound_terms(a, b, tau=tau)
    sS, snpr = O.sampled_bound_terms(a, b, si, sj, tau)
    for q, (i, j) in enumerate(zip(si.tolist(), sj.tolist())):
        t = pos.get((i, j))
        assert (snpr[q], sS[q]) == ((npr[t], S[t]) if t is not None else (0, 0.0))


def test_block_bound_terms_brute_force():
    """S_IJ and the product count per C block against explicit loops with
    norms summed element by element, also for transposed operands."""
    bs = 8
    a = _decay_rect(40, 56, bs, 0.2, 23)
    b = _decay_rect(40, 33, bs, 0.1, 24, shift=5)
    S, npr = O.block_bound_terms(a, b, trans_a=True)
    c = O.multiply(a, b, trans_a=True)

    def nrm(m, t):
        return sum(float(v) * float(v) for v in m.vals[t]) ** 0.5

    ia = {(int(i), int(j)): t for t, (i, j) in enumerate(zip(a.brow, a.bcol))}
    ib = {(int(i), int(j)): t for t, (i, j) in enumerate(zip(b.brow, b.bcol))}
    want = {}
    for (k, i), ta in ia.items():          # op(A) = A^T: block (i, k) of op(A) is A's (k, i)
        for (k2, j), tb in ib.items():
            if k2 == k:
                s0, n0 = want.get((i, j), (0.0, 0))
                want[(i, j)] = (s0 + nrm(a, ta) * nrm(b, tb), n0 + 1)
    assert sorted(want) == list(zip(c.brow.tolist(), c.bcol.tolist()))
    for t, key in enumerate(zip(c.brow.tolist(), c.bcol.tolist())):
        assert npr[t] == want[key][1]
        assert abs(S[t] - want[key][0]) <= 1e-13 * want[key][0]
    # the scale bounds the block itself
    assert np.all(np.linalg.norm(c.vals, axis=1) <= S * (1 + 1e-13))


def _emulate(mode, a, b):
    """Plain numpy emulation of a precision mode, block by block (each leaf
    product one float32 GEMM, summed over K in float32; the Ozaki mode is the
    oracle's own splitting), in C's canonical order."""
    from tests.bounds import SAFETY  # noqa: F401  (same module as the GPU checks)
    bs = a.bs
    if mode == "ozaki":
        return O.ozaki_multiply(a, b).vals
    I, J, K, ia, ib = O.product_triples(a, b)
    _, _, seg = O.c_pattern_from_triples(I, J)

    def mats(vals, fn):
        return np.ascontiguousarray(fn(vals).reshape(-1, bs, bs).transpose(0, 2, 1))

    out = np.zeros((seg.size - 1, bs * bs))
    if mode == "f64":
        A, B = mats(a.vals, lambda x: x), mats(b.vals, lambda x: x)
        for q in range(seg.size - 1):  # K descending: another order than the oracle's
            acc = np.zeros((bs, bs))
            for t in range(seg[q + 1] - 1, seg[q] - 1, -1):
                acc = acc + A[ia[t]] @ B[ib[t]]
            out[q] = acc.T.ravel()
        return out
    if mode == "bf16x3":
        ah, al = (mats(x, lambda v: v).astype(np.float32) for x in O.split_bf16(a.vals))
        bh, bl = (mats(x, lambda v: v).astype(np.float32) for x in O.split_bf16(b.vals))
        for q in range(seg.size - 1):
            acc = np.zeros((bs, bs), np.float32)
            for t in range(seg[q], seg[q + 1]):
                x, y = ia[t], ib[t]
                acc = acc + ah[x] @ bl[y]
                acc = acc + al[x] @ bh[y]
                acc = acc + ah[x] @ bh[y]
            out[q] = acc.astype(np.float64).T.ravel()
        return out
    rnd = O.round_to_f32 if mode == "f32" else O.round_to_bf16
    A = mats(a.vals, rnd).astype(np.float32)
    B = mats(b.vals, rnd).astype(np.float32)
    for q in range(seg.size - 1):
        acc = np.zeros((bs, bs), np.float32)
        for t in range(seg[q], seg[q + 1]):
            acc = acc + A[ia[t]] @ B[ib[t]]
        out[q] = acc.astype(np.float64).T.ravel()
    return out


@pytest.mark.parametrize("mode", ["f64", "f32", "bf16", "bf16x3", "ozaki"])
def test_blockwise_bound_holds_and_catches_mistakes(mode):
    """The per-block bound of every mode holds for a plain emulation of that
    mode's arithmetic on block norms spread over many decades, and it catches
    a zeroed block and a dropped leaf product that a relative Frobenius norm
    over the whole C lets through."""
    from tests.bounds import rel_bound, violations
    bs = 16
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2, "bf16x3": 1e-4, "ozaki": 1e-11}[mode]
    for case, (a, b) in enumerate(((_decay_rect(192, 160, bs, 0.25, 25), _decay_rect(160, 176, bs, 0.2, 26, shift=8)),
                                   W_small_pair(bs))):
        ref = O.multiply(a, b)
        S, npr = O.block_bound_terms(a, b)
        got = _emulate(mode, a, b)
        bad, err, lim = violations(got, ref.vals, S, npr, mode, bs)
        assert bad.size == 0, (mode, bad[:5], err[bad[:5]], lim[bad[:5]])
        # planted mistake 1: the block with the smallest norm relative to the total comes back zero
        nrm = np.linalg.norm(ref.vals, axis=1)
        k = int(np.argmin(np.where(nrm > 0, nrm, np.inf)))
        wrong = got.copy()
        wrong[k] = 0.0
        assert k in violations(wrong, ref.vals, S, npr, mode, bs)[0]
        if case == 0:  # decaying blocks: the mistake passes the global check at the mode's tolerance
            assert O.rel_fro(wrong, ref.vals) <= tol
        # planted mistake 2: one block misses its largest leaf product
        I, J, K, ia, ib = O.product_triples(a, b)
        _, _, seg = O.c_pattern_from_triples(I, J)
        na, nb = O.block_fnorms(a.vals, bs), O.block_fnorms(b.vals, bs)
        q = int(np.argmax(npr))
        ts = np.arange(seg[q], seg[q + 1])
        t = ts[np.argmax(na[ia[ts]] * nb[ib[ts]])]
        lo = O.OMatrix(a.nrows, a.ncols, bs, a.brow[[ia[t]]], a.bcol[[ia[t]]], a.vals[[ia[t]]])
        hi = O.OMatrix(b.nrows, b.ncols, bs, b.brow[[ib[t]]], b.bcol[[ib[t]]], b.vals[[ib[t]]])
        term = O.multiply(lo, hi).vals[0]
        wrong = got.copy()
        wrong[q] -= term
        if np.linalg.norm(term) > 4 * rel_bound(mode, npr[q], bs) * S[q]:
            assert q in violations(wrong, ref.vals, S, npr, mode, bs)[0]


def W_small_pair(bs):
    a, b = W.small_random(150, 130, 120, bs, 0.4, 27)
    return O.from_workload(a), O.from_workload(b)


# ---------------------------------------------------------------- symmetric square
def _symmetric(n, bs, p, seed):
    """Block-sparse symmetric matrix (pattern and values mirrored)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, (n, n))
    nb = -(-n // bs)
    keep = rng.random((nb, nb)) < p
    keep = keep | keep.T
    mask = np.kron(keep, np.ones((bs, bs), dtype=bool))[:n, :n]
    dense = np.where(mask, x, 0.0)
    dense = np.triu(dense) + np.triu(dense, 1).T
    br, bc = np.nonzero(keep)
    blocks = []
    for I, J in zip(br, bc):
        blk = np.zeros((bs, bs))
        sub = dense[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs]
        blk[:sub.shape[0], :sub.shape[1]] = sub
        blocks.append(blk.T.ravel())
    return O.canonical(n, n, bs, br, bc, np.array(blocks)), dense


def test_symmetric_square_reconstructs_the_product():
    """For a symmetric A, the upper blocks with the mirror of the strictly
    upper ones give the regular product, block for block (the product of a
    symmetric matrix with itself is symmetric)."""
    a, _ = _symmetric(300, 16, 0.3, 7)
    up, full = O.multiply_upper(a, a), O.multiply(a, a)
    assert np.all(up.brow <= up.bcol) and np.all(up.I <= up.J)
    got = {}
    for t, (i, j) in enumerate(zip(up.brow.tolist(), up.bcol.tolist())):
        got[(i, j)] = up.vals[t].reshape(16, 16).T
        if i < j:
            got[(j, i)] = got[(i, j)].T
    assert sorted(got) == list(zip(full.brow.tolist(), full.bcol.tolist()))
    for t, (i, j) in enumerate(zip(full.brow.tolist(), full.bcol.tolist())):
        np.testing.assert_allclose(got[(i, j)], full.vals[t].reshape(16, 16).T, rtol=0, atol=1e-12)


def test_symmetric_square_against_dense():
    a, dense = _symmetric(70, 8, 0.4, 8)
    up = O.multiply_upper(a, a)
    c = dense @ dense
    for t, (i, j) in enumerate(zip(up.brow.tolist(), up.bcol.tolist())):
        want = np.zeros((8, 8))
        sub = c[i * 8:(i + 1) * 8, j * 8:(j + 1) * 8]
        want[:sub.shape[0], :sub.shape[1]] = sub
        np.testing.assert_allclose(up.vals[t].reshape(8, 8).T, want, rtol=0, atol=1e-12)
    # every upper block of the boolean pattern product is present
    bi, bj, _ = O.boolean_pattern_product(a, a)
    sel = bi <= bj
    assert np.array_equal(up.brow, bi[sel]) and np.array_equal(up.bcol, bj[sel])


# ---------------------------------------------------------------- elements and truncation
def test_elements_round_trip_dense():
    rng = np.random.default_rng(9)
    n, m, bs = 70, 53, 16
    dense = np.zeros((n, m))
    pos = rng.choice(n * m, 400, replace=False)
    r, c = pos // m, pos % m
    v = rng.uniform(-1, 1, 400)
    dense[r, c] = v
    a = O.from_elements(n, m, bs, r, c, v)
    full = np.zeros((-(-n // bs) * bs, -(-m // bs) * bs))
    for t in range(a.nblk):
        full[a.brow[t] * bs:(a.brow[t] + 1) * bs, a.bcol[t] * bs:(a.bcol[t] + 1) * bs] = a.vals[t].reshape(bs, bs).T
    assert np.array_equal(full[:n, :m], dense) and not np.any(full[n:, :]) and not np.any(full[:, m:])
    held = sorted(set(zip((r // bs).tolist(), (c // bs).tolist())))
    assert list(zip(a.brow.tolist(), a.bcol.tolist())) == held
    qr, qc = rng.integers(0, n, 300), rng.integers(0, m, 300)
    assert np.array_equal(O.get_elements(a, qr, qc), dense[qr, qc])
    with pytest.raises(ValueError):
        O.from_elements(n, m, bs, np.append(r, r[0]), np.append(c, c[0]), np.append(v, 1.0))
    with pytest.raises(ValueError):
        O.from_elements(n, m, bs, np.array([n]), np.array([0]), np.array([1.0]))


def test_truncation_error_control():
    """The removed part is within eps in the Frobenius norm, removing one more
    leaf (the next smallest) would exceed it, and the kept leaves are the
    largest ones (brute force over the sorted norms)."""
    rng = np.random.default_rng(10)
    a = O.from_workload(W.random_blocks(300, 16, 0.5, rng))
    a.vals *= np.exp(rng.uniform(-12, 0, a.nblk))[:, None]  # norms over many decades
    norms = np.array([np.sqrt(np.sum(v * v)) for v in a.vals])
    for eps in (1e-9, 1e-5, 1e-3, 0.1):
        t = O.truncate_error_control(a, eps)
        kept = set(zip(t.brow.tolist(), t.bcol.tolist()))
        dropped = [i for i in range(a.nblk) if (a.brow[i], a.bcol[i]) not in kept]
        err = np.sqrt(sum(norms[i] ** 2 for i in dropped))
        assert err <= eps
        rest = sorted(norms[i] for i in range(a.nblk) if (a.brow[i], a.bcol[i]) in kept)
        if rest:
            assert np.sqrt(err ** 2 + rest[0] ** 2) > eps
            assert max((norms[i] for i in dropped), default=0.0) <= rest[0]
    assert O.truncate_error_control(a, 0.0).nblk == a.nblk


def test_truncation_keeps_infinite_norms():
    """A leaf with an infinite element has an infinite norm, which no eps
    bounds: it stays even where eps^2 overflows, while the finite small
    leaves still go.  Leaves whose squared norms overflow are kept too (the
    removed part must be shown to be within eps)."""
    rng = np.random.default_rng(11)
    a = O.from_workload(W.random_blocks(96, 16, 0.6, rng))
    a.vals[3, 5] = np.inf
    a.vals[7] *= 1e170                       # squared norm overflows
    for eps in (1e-3, 1e200, np.finfo(np.float64).max):
        with np.errstate(over="ignore"):
            t = O.truncate_error_control(a, eps)
        kept = set(zip(t.brow.tolist(), t.bcol.tolist()))
        assert (a.brow[3], a.bcol[3]) in kept and (a.brow[7], a.bcol[7]) in kept
        dropped = [i for i in range(a.nblk) if (a.brow[i], a.bcol[i]) not in kept]
        err = np.sqrt(sum(float(np.sum(a.vals[i] ** 2)) for i in dropped))
        assert err <= eps
        if eps >= 1e200:                     # every finite, non-overflowing leaf goes
            assert t.nblk == 2


# ---------------------------------------------------------------- addition
def test_addition_against_dense():
    rng = np.random.default_rng(12)
    a = W.random_blocks(150, 16, 0.3, rng, ncols=130)
    b = W.random_blocks(150, 16, 0.3, rng, ncols=130)
    A, B = om(a), om(b)
    c = O.add(0.5, A, -2.0, B)
    dense = 0.5 * a.to_dense() - 2.0 * b.to_dense()
    got = W.BlockMatrix(150, 130, 16, c.brow.astype(np.int32), c.bcol.astype(np.int32), c.vals).to_dense()
    assert np.array_equal(got, dense)
    pat = set(zip(A.brow.tolist(), A.bcol.tolist())) | set(zip(B.brow.tolist(), B.bcol.tolist()))
    assert list(zip(c.brow.tolist(), c.bcol.tolist())) == sorted(pat)
    # the multiply distributes over the sum: (A + B) X = A X + B X within rounding
    X = om(W.random_blocks(130, 16, 0.4, rng, ncols=90))
    left = O.multiply(O.add(1.0, A, 1.0, B), X)
    ax, bx = O.multiply(A, X), O.multiply(B, X)
    right = O.add(1.0, O.OMatrix(150, 90, 16, ax.brow, ax.bcol, ax.vals), 1.0,
                  O.OMatrix(150, 90, 16, bx.brow, bx.bcol, bx.vals))
    assert np.array_equal(left.brow, right.brow) and np.array_equal(left.bcol, right.bcol)
    assert O.rel_fro(left.vals, right.vals) < 1e-14


def test_add_identity_against_dense():
    rng = np.random.default_rng(13)
    a = W.random_blocks(100, 16, 0.2, rng, ncols=90)
    A = om(a)
    c = O.add_identity(A, 3.5)
    dense = a.to_dense()[:100, :90].copy()
    dense[np.arange(90), np.arange(90)] += 3.5
    got = W.BlockMatrix(100, 90, 16, c.brow.astype(np.int32), c.bcol.astype(np.int32), c.vals).to_dense()
    assert np.array_equal(got[:100, :90], dense) and not np.any(got[100:, :]) and not np.any(got[:, 90:])


def _brute_pairs(a, b, i, j, tau):
    """Every stored pair (A_iK, B_Kj), K ascending, enumerated over all pairs
    of stored blocks; for tau > 0 only pairs whose norm product (each norm a
    plain sum of squares) is not below tau."""
    na = np.sqrt(np.einsum("ij,ij->i", a.vals, a.vals))
    nb = np.sqrt(np.einsum("ij,ij->i", b.vals, b.vals))
    out = []
    for l in range(a.brow.size):
        if a.brow[l] != i:
            continue
        for r in range(b.brow.size):
            if b.bcol[r] == j and b.brow[r] == a.bcol[l] and not (tau > 0 and na[l] * nb[r] < tau):
                out.append((int(a.bcol[l]), l, r))
    return [(l, r) for _, l, r in sorted(out)]


@pytest.mark.parametrize("case", ["sparse-exact", "decay-approx"])
def test_sampled_products_brute_force(case):
    """sampled_products (the product lists behind multiply_blocks) lists, for
    every selected C block, exactly the pairs of stored blocks with a shared
    contraction index, K ascending, and for tau > 0 only those whose norm
    product is not below tau (Sec. 2.2 regular multiply; Sec. 1 and 2.2
    sparse approximate multiply): brute-force enumeration over all pairs of
    stored blocks of two different, ragged operands, on every (I, J) of the
    grid, empty blocks included."""
    bs = 16
    if case == "sparse-exact":
        wa, wb = W.small_random(150, 120, 170, bs, 0.3, 31)
        a, b, tau = om(wa), om(wb), 0.0
    else:
        a = _decay_rect(200, 120, bs, 0.30, 21, shift=40)
        b = _decay_rect(120, 168, bs, 0.08, 22, shift=-25)
        tau = 0.5
        # no norm product sits so close to tau that the summation order of a
        # norm could decide it
        na = np.sqrt(np.einsum("ij,ij->i", a.vals, a.vals))
        nb = np.sqrt(np.einsum("ij,ij->i", b.vals, b.vals))
        assert np.min(np.abs(np.outer(na, nb) / tau - 1.0)) > 1e-9
    nbr, nbc = -(-a.nrows // bs), -(-b.ncols // bs)
    si, sj = (g.ravel() for g in np.meshgrid(np.arange(nbr), np.arange(nbc), indexing="ij"))
    seg, lidx, ridx = O.sampled_products(a, b, si, sj, tau)
    assert seg.size == si.size + 1
    kept = dropped = 0
    empty = 0
    for q, (i, j) in enumerate(zip(si.tolist(), sj.tolist())):
        got = list(zip(np.asarray(lidx[seg[q]:seg[q + 1]]).tolist(), np.asarray(ridx[seg[q]:seg[q + 1]]).tolist()))
        exp = _brute_pairs(a, b, i, j, tau)
        assert got == exp, (i, j)
        kept += len(exp)
        empty += not exp
        if tau > 0:
            dropped += len(_brute_pairs(a, b, i, j, 0.0)) - len(exp)
    assert kept > 0 and empty > 0
    if tau > 0:
        assert dropped > 0


def test_truncate_borderline_closed_form():
    """truncate_borderline counts the partial sums of the ascending squared
    leaf norms that lie within rel of eps^2 (where the truncation's cut could
    depend on summation order).  Blocks with one entry each, 1, -1 and 2:
    squared norms 1, 1, 4, partial sums 1, 2, 6 exactly."""
    bs = 4
    vals = np.zeros((3, bs * bs))
    vals[0, 0], vals[1, 5], vals[2, 10] = 1.0, -1.0, 2.0
    a = O.canonical(12, 4, bs, [0, 1, 2], [0, 0, 0], vals)
    assert O.truncate_borderline(a, np.sqrt(2.0)) == 1
    assert O.truncate_borderline(a, np.sqrt(6.0)) == 1
    assert O.truncate_borderline(a, 1.0) == 1
    assert O.truncate_borderline(a, 2.0) == 0
    assert O.truncate_borderline(a, np.sqrt(3.0)) == 0
    assert O.truncate_borderline(a, 0.0) == 0
    assert O.truncate_borderline(O.canonical(12, 4, bs, [], [], np.zeros((0, bs * bs))), 1.0) == 0
