"""CPU oracle for the block-sparse quadtree multiply -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this module.  The GPU library never uses it,
and the two share no code.

The oracle computes the plain definitions that the paper's recursive
sparse-quadtree algorithms reach (no quadtree here):

* Sparse quadtree semantics (paper Sec. 2 and Sec. 2.1): a matrix is zero, a
  leaf, or four quadrants; a nil chunk is a zero submatrix and a task with a
  nil input yields nil.  At leaf-block granularity the product pattern is
  therefore the boolean product of the block patterns,
  ``P_C = {(I,J) : exists K, (I,K) in P_A and (K,J) in P_B}``, and
  ``C_IJ = sum_K A_IK B_KJ`` over exactly those K.
* Truncation (paper Sec. 2.2, block-level variant): a block is dropped iff its
  FP64 Frobenius norm is strictly below the tolerance (NaN norms are kept).
* Matrix-matrix multiplication (paper Sec. 2.2): regular multiply; its masked
  adjoints dA = (dC B^T) restricted to P_A and dB = (A^T dC) restricted to P_B;
  the sparse approximate multiply (Sec. 1 and 2.2) as the regular multiply
  over the leaf products whose norm product is not below a tolerance.
* Flop counts: element level ``2 * sum_k r(k) c(k)`` (the convention that
  reproduces the paper's Table 1) and block level ``2 * sum m_I k_K n_J`` over
  the nonzero leaf products with logical (unpadded) sizes.

Readings of points the paper leaves open are listed with each function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qbsm_oracle.c")
_LIB = os.path.join(_HERE, "_qbsm_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-std=c99", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, p = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.oracle_block_fnorm.argtypes = [i64, i32, p, p]
        lib.oracle_block_fnorm.restype = None
        lib.oracle_segmented_products.argtypes = [i32, i64, p, p, p, p, p,
                                                  ctypes.c_int, ctypes.c_int, p]
        lib.oracle_segmented_products.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> int:
    """OpenMP threads of the C part for the calls that follow; returns the
    previous count (used to time the oracle on all threads and on one)."""
    return int(_load().oracle_set_threads(int(n)))


# --------------------------------------------------------------------------
# Block norms and truncation
# --------------------------------------------------------------------------

def block_fnorms(vals: np.ndarray, bs: int) -> np.ndarray:
    """FP64 Frobenius norm of each block (column-major summation order)."""
    vals = np.ascontiguousarray(vals, dtype=np.float64).reshape(-1, bs * bs)
    out = np.empty(vals.shape[0], dtype=np.float64)
    if vals.shape[0]:
        _load().oracle_block_fnorm(vals.shape[0], bs, _ptr(vals), _ptr(out))
    return out


def keep_mask(vals: np.ndarray, bs: int, tol: float) -> np.ndarray:
    """Blocks kept by truncation: not (norm < tol).  Equality and NaN keep.

    Reading: the paper names truncation with error control (Sec. 2.2) without
    a formula; the block-level rule here drops iff ||X||_F < tol in FP64.
    """
    if tol <= 0.0:
        return np.ones(vals.shape[0], dtype=bool)
    return ~(block_fnorms(vals, bs) < tol)


def borderline(vals: np.ndarray, bs: int, tol: float, rel: float = 1e-9) -> np.ndarray:
    """Blocks whose squared norm lies within ``rel`` of tol^2 (order-sensitive)."""
    if tol <= 0.0:
        return np.zeros(vals.shape[0], dtype=bool)
    n = block_fnorms(vals, bs)
    return np.abs(n * n / (tol * tol) - 1.0) < rel


@dataclass
class OMatrix:
    """Oracle-side block matrix: canonical row-major pattern + FP64 blocks."""

    nrows: int
    ncols: int
    bs: int
    brow: np.ndarray  # int64
    bcol: np.ndarray  # int64
    vals: np.ndarray  # float64 [nblk, bs*bs], column-major blocks

    @property
    def nblk(self):
        return int(self.brow.shape[0])


def canonical(nrows, ncols, bs, brow, bcol, vals, drop_tol=0.0) -> OMatrix:
    """Sort blocks row-major, apply truncation, reject duplicates / out-of-range."""
    brow = np.asarray(brow, dtype=np.int64)
    bcol = np.asarray(bcol, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64).reshape(-1, bs * bs)
    nbr, nbc = -(-nrows // bs), -(-ncols // bs)
    if brow.size and (brow.min() < 0 or bcol.min() < 0 or brow.max() >= nbr or bcol.max() >= nbc):
        raise ValueError("block index out of range")
    order = np.lexsort((bcol, brow))
    brow, bcol, vals = brow[order], bcol[order], vals[order]
    if brow.size > 1 and np.any((np.diff(brow) == 0) & (np.diff(bcol) == 0)):
        raise ValueError("duplicate block")
    keep = keep_mask(vals, bs, drop_tol)
    return OMatrix(nrows, ncols, bs, brow[keep], bcol[keep], np.ascontiguousarray(vals[keep]))


def from_elements(nrows, ncols, bs, row, col, val) -> OMatrix:
    """Assignment from vectors of row indices, column indices and values
    (Sec. 2.2): the leaves are the blocks holding at least one given element;
    every other element of a leaf is zero.  Reading: the paper does not say
    what a repeated (row, col) means; it is rejected (as a repeated block is).
    """
    row = np.asarray(row, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    if row.size and (row.min() < 0 or col.min() < 0 or row.max() >= nrows or col.max() >= ncols):
        raise ValueError("element index out of range")
    key = row * ncols + col
    if np.unique(key).size != key.size:
        raise ValueError("repeated element")
    nbc = -(-ncols // bs)
    bkey = (row // bs) * nbc + col // bs
    ub, inv = np.unique(bkey, return_inverse=True)
    vals = np.zeros((ub.size, bs * bs))
    vals[inv, (row % bs) + (col % bs) * bs] = val
    return OMatrix(nrows, ncols, bs, ub // nbc, ub % nbc, vals)


def get_elements(a: OMatrix, row, col) -> np.ndarray:
    """Extraction of the elements given by row and column index vectors
    (Sec. 2.2); zero where no leaf is stored."""
    row = np.asarray(row, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    bs = a.bs
    nbc = -(-a.ncols // bs)
    pos = {int(k): t for t, k in enumerate((a.brow * nbc + a.bcol).tolist())}
    out = np.zeros(row.size)
    for q, (r, c) in enumerate(zip(row.tolist(), col.tolist())):
        t = pos.get((r // bs) * nbc + c // bs)
        if t is not None:
            out[q] = a.vals[t, (r % bs) + (c % bs) * bs]
    return out


def truncate_error_control(a: OMatrix, eps: float) -> OMatrix:
    """Truncation with error control (Sec. 2.2), at leaf-block granularity:
    with the leaves ordered by FP64 Frobenius norm ascending (ties by storage
    position), the longest leading run whose squared norms sum to at most
    eps^2 is removed, so the removed part has Frobenius norm <= eps.  Leaves
    with a NaN norm stay, and so does every leaf from the first one at which
    the running sum of squared norms stops being finite (an infinite norm is
    never within eps; a sum that overflows only makes the cut conservative).
    Reading: the paper names truncation with several variants of error
    control without formulas; this is the Frobenius-norm variant.
    """
    if a.nblk == 0:
        return a
    n = block_fnorms(a.vals, a.bs)
    sq = n * n
    order = np.lexsort((np.arange(a.nblk), sq))  # NaN last
    csum = np.cumsum(sq[order])
    k = int(np.count_nonzero((csum <= eps * eps) & np.isfinite(csum)))
    keep = np.ones(a.nblk, dtype=bool)
    keep[order[:k]] = False
    return OMatrix(a.nrows, a.ncols, a.bs, a.brow[keep], a.bcol[keep], np.ascontiguousarray(a.vals[keep]))


def truncate_borderline(a: OMatrix, eps: float, rel: float = 1e-9) -> int:
    """Partial sums of the squared norms within ``rel`` of eps^2 (their
    comparison depends on the summation order)."""
    if a.nblk == 0:
        return 0
    n = block_fnorms(a.vals, a.bs)
    sq = np.sort(n * n)
    csum = np.cumsum(sq)
    return int(np.count_nonzero(np.abs(csum / (eps * eps) - 1.0) < rel)) if eps > 0 else 0


def add(alpha: float, a: OMatrix, beta: float, b: OMatrix) -> OMatrix:
    """Matrix addition (Sec. 2.2): alpha A + beta B on the union of the two
    leaf patterns, each block alpha*A_IJ + beta*B_IJ in FP64 (a missing block
    is zero).  Reading: the paper lists regular addition without a rule for
    the pattern; every leaf of either operand is kept, none is dropped."""
    if (a.nrows, a.ncols, a.bs) != (b.nrows, b.ncols, b.bs):
        raise ValueError("shapes differ")
    nbc = -(-a.ncols // a.bs)
    ka, kb = a.brow * nbc + a.bcol, b.brow * nbc + b.bcol
    keys = np.union1d(ka, kb)
    vals = np.zeros((keys.size, a.bs * a.bs))
    ia, ib = np.searchsorted(keys, ka), np.searchsorted(keys, kb)
    vals[ia] += alpha * a.vals
    vals[ib] += beta * b.vals
    return OMatrix(a.nrows, a.ncols, a.bs, keys // nbc, keys % nbc, vals)


def add_identity(a: OMatrix, sigma: float) -> OMatrix:
    """A + sigma I (Sec. 2.2, addition of a scaled identity): sigma is added to
    the diagonal elements (r, r), r < min(nrows, ncols); diagonal leaves that
    are not stored are created."""
    bs = a.bs
    nd = min(a.nrows, a.ncols)
    nb = -(-nd // bs)
    diag = np.zeros((nb, bs * bs))
    for t in range(nb):
        for r in range(bs):
            if t * bs + r < nd:
                diag[t, r + r * bs] = sigma
    d = OMatrix(a.nrows, a.ncols, bs, np.arange(nb, dtype=np.int64), np.arange(nb, dtype=np.int64), diag)
    return add(1.0, a, 1.0, d)


def from_workload(m, drop_tol=0.0) -> OMatrix:
    return canonical(m.nrows, m.ncols, m.bs, m.brow, m.bcol, m.vals, drop_tol)


# --------------------------------------------------------------------------
# Symbolic part: product triples and the C pattern
# --------------------------------------------------------------------------

def _row_index(brow: np.ndarray, nrows_blk: int) -> np.ndarray:
    """Row pointer of a row-major sorted pattern."""
    return np.searchsorted(brow, np.arange(nrows_blk + 1), side="left")


def product_triples(a: OMatrix, b: OMatrix, trans_a=False, trans_b=False):
    """All nonzero leaf products of op(A) op(B), canonical (I, J, K) order.

    Returns (I, J, K, ia, ib): ``ia``/``ib`` index the stored blocks of A/B.
    Plain definition: for every stored block (I,K) of op(A) and every stored
    block (K,J) of op(B), the triple (I,K,J) is a product.
    """
    # logical coordinates of op(X)
    ai, ak = (a.bcol, a.brow) if trans_a else (a.brow, a.bcol)
    bk, bj = (b.bcol, b.brow) if trans_b else (b.brow, b.bcol)
    # index B's blocks by their K (block row of op(B))
    order_b = np.lexsort((bj, bk))
    bk_s, bj_s = bk[order_b], bj[order_b]
    nk = int(max(ak.max(initial=-1), bk.max(initial=-1)) + 1)
    ptr = np.searchsorted(bk_s, np.arange(nk + 1), side="left")
    cnt = (ptr[ak + 1] - ptr[ak]) if ak.size else np.zeros(0, dtype=np.int64)
    total = int(cnt.sum())
    ia = np.repeat(np.arange(a.nblk, dtype=np.int64), cnt)
    start = np.repeat(ptr[ak] if ak.size else np.zeros(0, np.int64), cnt)
    off = np.arange(total, dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    ib = order_b[start + off]
    I, K, J = ai[ia], ak[ia], bj[ib]
    o = np.lexsort((K, J, I))
    return I[o], J[o], K[o], ia[o], ib[o]


def c_pattern_from_triples(I, J):
    """Unique (I, J) of the triples in row-major order, with segment offsets."""
    if I.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(1, np.int64)
    new = np.ones(I.size, dtype=bool)
    new[1:] = (I[1:] != I[:-1]) | (J[1:] != J[:-1])
    starts = np.nonzero(new)[0]
    seg = np.append(starts, I.size).astype(np.int64)
    return I[starts], J[starts], seg


def boolean_pattern_product(a: OMatrix, b: OMatrix):
    """C pattern as the boolean matrix product of the block masks (pin)."""
    nbi, nbk = -(-a.nrows // a.bs), -(-a.ncols // a.bs)
    nbj = -(-b.ncols // b.bs)
    ma = np.zeros((nbi, nbk), dtype=np.int64)
    mb = np.zeros((nbk, nbj), dtype=np.int64)
    ma[a.brow, a.bcol] = 1
    mb[b.brow, b.bcol] = 1
    prod = ma @ mb
    ii, jj = np.nonzero(prod)
    return ii.astype(np.int64), jj.astype(np.int64), prod[ii, jj]


# --------------------------------------------------------------------------
# Numeric part
# --------------------------------------------------------------------------

@dataclass
class OProduct:
    brow: np.ndarray
    bcol: np.ndarray
    vals: np.ndarray
    I: np.ndarray
    J: np.ndarray
    K: np.ndarray
    seg: np.ndarray


def _segmented(bs, seg, lidx, ridx, L, R, transL, transR):
    nout = seg.size - 1
    out = np.empty((nout, bs * bs), dtype=np.float64)
    if nout:
        seg = np.ascontiguousarray(seg, dtype=np.int64)
        lidx = np.ascontiguousarray(lidx, dtype=np.int64)
        ridx = np.ascontiguousarray(ridx, dtype=np.int64)
        L = np.ascontiguousarray(L, dtype=np.float64)
        R = np.ascontiguousarray(R, dtype=np.float64)
        _load().oracle_segmented_products(bs, nout, _ptr(seg), _ptr(lidx), _ptr(ridx),
                                          _ptr(L), _ptr(R), int(transL), int(transR), _ptr(out))
    return out


def multiply(a: OMatrix, b: OMatrix, trans_a=False, trans_b=False) -> OProduct:
    """C = op(A) op(B): structural pattern (no numerical dropping) + FP64 values.

    Readings: C keeps every structurally nonzero block even when its value is
    numerically zero (truncation is a separate operation, paper Sec. 2.2);
    each C block sums its leaf products with K ascending.
    """
    if a.bs != b.bs:
        raise ValueError("leaf sizes differ")
    I, J, K, ia, ib = product_triples(a, b, trans_a, trans_b)
    ci, cj, seg = c_pattern_from_triples(I, J)
    vals = _segmented(a.bs, seg, ia, ib, a.vals, b.vals, trans_a, trans_b)
    return OProduct(ci, cj, vals, I, J, K, seg)


def spamm_keep(a: OMatrix, b: OMatrix, ia: np.ndarray, ib: np.ndarray, tau: float) -> np.ndarray:
    """Leaf products kept by the sparse approximate multiply: not
    (||A_IK||_F * ||B_KJ||_F < tau), both norms and their product in FP64.

    Reading: the paper lists sparse approximate multiplication for matrices
    with decay among the library's multiply task types (Sec. 1 and 2.2)
    without a formula; the rule here is the norm-product test at leaf-block
    granularity, with the same strict comparison as truncation.
    """
    if tau <= 0.0:
        return np.ones(ia.shape[0], dtype=bool)
    return _spamm_test(block_fnorms(a.vals, a.bs), block_fnorms(b.vals, b.bs), ia, ib, tau)


def _spamm_test(na: np.ndarray, nb: np.ndarray, ia: np.ndarray, ib: np.ndarray, tau: float) -> np.ndarray:
    """The norm-product test itself: product (ia, ib) is kept unless
    na[ia] * nb[ib] < tau (FP64, strict)."""
    return ~(na[ia] * nb[ib] < tau)


def multiply_spamm(a: OMatrix, b: OMatrix, tau: float) -> OProduct:
    """Sparse approximate C = A B: the regular multiply over the kept leaf
    products only; C holds the blocks with at least one kept product.
    tau <= 0 is the regular multiply."""
    if a.bs != b.bs:
        raise ValueError("leaf sizes differ")
    I, J, K, ia, ib = product_triples(a, b)
    keep = spamm_keep(a, b, ia, ib, tau)
    I, J, K, ia, ib = I[keep], J[keep], K[keep], ia[keep], ib[keep]
    ci, cj, seg = c_pattern_from_triples(I, J)
    vals = _segmented(a.bs, seg, ia, ib, a.vals, b.vals, False, False)
    return OProduct(ci, cj, vals, I, J, K, seg)


def multiply_upper(a: OMatrix, b: OMatrix) -> OProduct:
    """The blocks I <= J of C = A B with their leaf products.

    Reading: the paper lists symmetric multiplication and the symmetric
    matrix square among the multiply task types (Sec. 2.2) without a storage
    convention; for a symmetric A the square A A is symmetric, and here its
    representation is the upper triangle of the regular product at block
    granularity (diagonal blocks whole).
    """
    if a.bs != b.bs:
        raise ValueError("leaf sizes differ")
    I, J, K, ia, ib = product_triples(a, b)
    keep = I <= J
    I, J, K, ia, ib = I[keep], J[keep], K[keep], ia[keep], ib[keep]
    ci, cj, seg = c_pattern_from_triples(I, J)
    vals = _segmented(a.bs, seg, ia, ib, a.vals, b.vals, False, False)
    return OProduct(ci, cj, vals, I, J, K, seg)


def spamm_borderline(a: OMatrix, b: OMatrix, tau: float, rel: float = 1e-9) -> int:
    """Number of leaf products whose norm product lies within ``rel`` of tau
    (their selection depends on the summation order of the norms)."""
    if tau <= 0.0:
        return 0
    _, _, _, ia, ib = product_triples(a, b)
    na, nb = block_fnorms(a.vals, a.bs), block_fnorms(b.vals, b.bs)
    return int(np.count_nonzero(np.abs(na[ia] * nb[ib] / tau - 1.0) < rel))


def sampled_products(a: OMatrix, b: OMatrix, sample_i, sample_j, tau: float = 0.0):
    """The leaf products of selected C blocks (I, J) = (sample_i[q], sample_j[q]).

    Returns (seg, lidx, ridx): the products of selected block q are the
    stored-block pairs (lidx[t], ridx[t]) for t in [seg[q], seg[q+1]), with
    the contraction index K ascending -- the same products, in the same
    order, that ``multiply`` (tau = 0) or ``multiply_spamm`` (tau > 0) uses
    for that block.  A selected block with no product has an empty range.
    """
    sample_i = np.asarray(sample_i, dtype=np.int64)
    sample_j = np.asarray(sample_j, dtype=np.int64)
    bs = a.bs
    if tau > 0.0:
        na, nb = block_fnorms(a.vals, bs), block_fnorms(b.vals, bs)
    segs = [0]
    lid, rid = [], []
    a_rowptr = _row_index(a.brow, -(-a.nrows // bs))
    bt_order = np.lexsort((b.brow, b.bcol))  # B sorted by column, then row
    b_col = b.bcol[bt_order]
    b_colptr = np.searchsorted(b_col, np.arange(-(-b.ncols // bs) + 1), side="left")
    for i, j in zip(sample_i.tolist(), sample_j.tolist()):
        ra = np.arange(a_rowptr[i], a_rowptr[i + 1])
        cb = bt_order[b_colptr[j]:b_colptr[j + 1]]
        common, xa, xb = np.intersect1d(a.bcol[ra], b.brow[cb], assume_unique=True, return_indices=True)
        la, lb = ra[xa], cb[xb]
        if tau > 0.0:
            kept = _spamm_test(na, nb, la, lb, tau)
            la, lb = la[kept], lb[kept]
        lid.append(la)
        rid.append(lb)
        segs.append(segs[-1] + la.size)
    seg = np.asarray(segs, dtype=np.int64)
    lidx = np.concatenate(lid) if lid else np.zeros(0, np.int64)
    ridx = np.concatenate(rid) if rid else np.zeros(0, np.int64)
    return seg, lidx, ridx


def multiply_blocks(a: OMatrix, b: OMatrix, sample_i, sample_j, tau: float = 0.0) -> np.ndarray:
    """Values of selected C blocks only (for sampling very large products).

    A selected (I, J) with no product gets a zero block.  tau > 0 applies the
    sparse approximate multiply's selection (the norm-product test of
    ``spamm_keep``).
    """
    seg, lidx, ridx = sampled_products(a, b, sample_i, sample_j, tau)
    return _segmented(a.bs, seg, lidx, ridx, a.vals, b.vals, False, False)


def _norm_product_sums(na, nb, seg, lidx, ridx):
    """Per segment: (sum of na[l] * nb[r] over its products, product count)."""
    terms = na[lidx] * nb[ridx]
    out = np.zeros(seg.size - 1)
    nz = np.nonzero(np.diff(seg))[0]  # reduceat needs non-empty segments
    if nz.size:
        out[nz] = np.add.reduceat(terms, seg[nz])
    return out, np.diff(seg).astype(np.int64)


def block_bound_terms(a: OMatrix, b: OMatrix, trans_a=False, trans_b=False, tau: float = 0.0):
    """For every block of C = op(A) op(B) (canonical order of ``multiply``,
    or of ``multiply_spamm`` when tau > 0): S_IJ = sum over its leaf products
    of ||op(A)_IK||_F ||op(B)_KJ||_F, and the number of those products.

    S_IJ bounds the block: ||C_IJ||_F <= S_IJ, and ||(|A| |B|)_IJ||_F <= S_IJ
    (triangle inequality and submultiplicativity of the Frobenius norm), which
    is the scale of every rounding-error bound of the block.
    """
    I, J, K, ia, ib = product_triples(a, b, trans_a, trans_b)
    if tau > 0.0:
        keep = spamm_keep(a, b, ia, ib, tau)
        I, J, ia, ib = I[keep], J[keep], ia[keep], ib[keep]
    _, _, seg = c_pattern_from_triples(I, J)
    return _norm_product_sums(block_fnorms(a.vals, a.bs), block_fnorms(b.vals, b.bs), seg, ia, ib)


def sampled_bound_terms(a: OMatrix, b: OMatrix, sample_i, sample_j, tau: float = 0.0):
    """``block_bound_terms`` of selected C blocks (zero and 0 where a block has
    no product)."""
    seg, lidx, ridx = sampled_products(a, b, sample_i, sample_j, tau)
    return _norm_product_sums(block_fnorms(a.vals, a.bs), block_fnorms(b.vals, b.bs), seg, lidx, ridx)


def _restrict(prod: OProduct, mask: OMatrix) -> np.ndarray:
    """Values of ``prod`` on the blocks of ``mask`` (zero where no product)."""
    bs = mask.bs
    out = np.zeros((mask.nblk, bs * bs), dtype=np.float64)
    if prod.brow.size == 0 or mask.nblk == 0:
        return out
    nbc = int(max(mask.bcol.max(), prod.bcol.max()) + 1)
    key_p = prod.brow * nbc + prod.bcol
    key_m = mask.brow * nbc + mask.bcol
    pos = np.searchsorted(key_p, key_m)
    pos = np.minimum(pos, key_p.size - 1)
    hit = key_p[pos] == key_m
    out[hit] = prod.vals[pos[hit]]
    return out


def backward(a: OMatrix, b: OMatrix, dc: OMatrix):
    """Masked adjoints of C = A B.

    dA = (dC B^T) restricted to A's pattern; dB = (A^T dC) restricted to B's
    pattern.  Each block sums over the free index ascending (J for dA, I for
    dB).  Blocks of the mask with no contributing product are zero.
    """
    pa = multiply(dc, b, trans_a=False, trans_b=True)   # (I,K) = sum_J dC_IJ B_KJ^T
    pb = multiply(a, dc, trans_a=True, trans_b=False)   # (K,J) = sum_I A_IK^T dC_IJ
    return _restrict(pa, a), _restrict(pb, b)


# --------------------------------------------------------------------------
# Flop counts
# --------------------------------------------------------------------------

def element_flops(col_counts_a: np.ndarray, row_counts_b: np.ndarray) -> int:
    """2 * sum_k r(k) c(k): r(k) nonzeros in column k of A, c(k) in row k of B.

    This is the element-level count of scalar multiply-adds (two flops each)
    that the paper's Table 1 reports for A*A.
    """
    r = np.asarray(col_counts_a, dtype=np.int64)
    c = np.asarray(row_counts_b, dtype=np.int64)
    return int(2 * np.sum(r * c, dtype=np.int64))


def block_flops(I, J, K, m_rows: int, k_dim: int, n_cols: int, bs: int) -> int:
    """2 * sum over leaf products of m_I * k_K * n_J with logical sizes."""
    def ext(idx, n):
        idx = np.asarray(idx, dtype=np.int64)
        return np.minimum(bs, n - idx * bs)
    return int(2 * np.sum(ext(I, m_rows) * ext(K, k_dim) * ext(J, n_cols), dtype=np.int64))


# --------------------------------------------------------------------------
# Precision-mode input roundings (used to isolate accumulation error)
# --------------------------------------------------------------------------

def round_to_f32(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even to binary32 (returned as float64)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even of an FP64 value straight to bfloat16 (no double rounding).

    bfloat16: 8 significant bits, the binary32 exponent range (normal
    exponents -126..127, subnormal quantum 2^-133), overflow to infinity.
    """
    x = np.asarray(x, dtype=np.float64)
    out = np.array(x, copy=True)
    fin = np.isfinite(x)
    ax = np.abs(x)
    normal = fin & (ax >= 2.0 ** -126)
    m, e = np.frexp(x[normal])               # x = m * 2^e, 0.5 <= |m| < 1
    out[normal] = np.ldexp(np.rint(m * 256.0) / 256.0, e)   # 8 significant bits
    sub = fin & ~normal
    out[sub] = np.rint(x[sub] * 2.0 ** 133) * 2.0 ** -133
    big = np.isfinite(out) & (np.abs(out) >= 2.0 ** 128)
    out[big] = np.sign(out[big]) * np.inf
    return out


def split_bf16(x: np.ndarray):
    """hi = bf16(x), lo = bf16(x - hi) with x - hi formed in FP64 (exact).

    Where hi is not finite (x is Inf or NaN, or overflows bfloat16) the
    residual is undefined and lo is taken as zero, so that hi + lo keeps the
    infinity (a NaN stays NaN through hi).
    """
    x = np.asarray(x, dtype=np.float64)
    hi = round_to_bf16(x)
    fin = np.isfinite(hi)
    lo = np.zeros_like(x)
    lo[fin] = round_to_bf16(x[fin] - hi[fin])
    return hi, lo


# Ozaki splitting (Ozaki, Ogita, Oishi and Rump, "Error-free transformations
# of matrix multiplication by using fast routines of matrix multiplication
# and its applications", Numer. Algorithms 59, 2012): an addition to the
# paper's FP64-only leaves.  Reading taken here: one exponent per leaf row of
# the left operand and per leaf column of the right operand; each element is
# truncated to an integer M of OZ_MANT bits on the line's grid and M is
# written in OZ_SLICES balanced base-2^OZ_BITS digits (every digit in
# [-128, 127], an 8-bit integer); the slice pairs with t + u <= OZ_SLICES + 1
# are kept.
OZ_SLICES, OZ_BITS, OZ_MANT = 6, 8, 47
# the largest M whose balanced digits all fit in [-128, 127]: 127 (2^48 - 1) / 255
OZ_MAXM = 127 * ((1 << (OZ_SLICES * OZ_BITS)) - 1) // ((1 << OZ_BITS) - 1)


def ozaki_exponent(m: np.ndarray) -> np.ndarray:
    """Line exponents for line maxima m (finite, >= 0): the e of m = f 2^e,
    0.5 <= f < 1 (0 for m = 0), raised by one where floor(m 2^(OZ_MANT - e))
    would exceed OZ_MAXM (m within 0.4 % below 2^e), so that every element of
    the line has a digit expansion."""
    _, e = np.frexp(m)
    mmax = np.floor(np.ldexp(m, OZ_MANT - e))
    return np.where(mmax > OZ_MAXM, e + 1, e)


def ozaki_split(vals: np.ndarray, bs: int, line: str, slices: int = OZ_SLICES) -> np.ndarray:
    """Exponent-aligned slices of leaf blocks: returns [slices, nblk, bs*bs].

    line = "row" (left operand: one exponent per leaf row) or "col" (right
    operand: one per leaf column).  With e the line's exponent
    (ozaki_exponent of its largest finite magnitude), every finite element x
    becomes M = sign(x) floor(|x| 2^(OZ_MANT - e)), |M| <= OZ_MAXM, written
    from the lowest digit up as M = sum_t d_t 2^(OZ_BITS (OZ_SLICES - t)) with
    d_t = ((M + 128) mod 256) - 128; slice t (t = 1 .. slices, the highest
    digits) is d_t 2^(e + 1 - OZ_BITS t).  An Inf or NaN element is its own
    first slice (the rest zero).
    """
    v = np.asarray(vals, dtype=np.float64).reshape(-1, bs, bs)   # [block, column, row]
    fin = np.isfinite(v)
    a = np.where(fin, np.abs(v), 0.0)
    m = a.max(axis=1, keepdims=True) if line == "row" else a.max(axis=2, keepdims=True)
    e = ozaki_exponent(m)
    big = np.sign(v) * np.floor(np.ldexp(a, OZ_MANT - e))   # exact integers, |M| < 2^47
    half = 2.0 ** (OZ_BITS - 1)
    digits = np.zeros((OZ_SLICES,) + v.shape)
    for t in range(OZ_SLICES, 0, -1):
        d = np.mod(big + half, 2.0 ** OZ_BITS) - half
        digits[t - 1] = d
        big = (big - d) / 2.0 ** OZ_BITS
    assert not np.any(big[fin]), "balanced digits do not cover an element"
    out = np.zeros((slices,) + v.shape)
    for t in range(1, slices + 1):
        out[t - 1] = np.where(fin, np.ldexp(digits[t - 1], e + 1 - OZ_BITS * t), 0.0)
    out[0] = np.where(fin, out[0], v)
    return out.reshape(slices, -1, bs * bs)


def ozaki_multiply(a: OMatrix, b: OMatrix, slices: int = OZ_SLICES) -> OProduct:
    """C = sum over t + u <= slices + 1 of A_t B_u (the first `slices`
    slices of each operand), every slice product in FP64 through the plain
    multiply (the slice products are exact; only their accumulation rounds)."""
    sa = ozaki_split(a.vals, a.bs, "row", slices)
    sb = ozaki_split(b.vals, b.bs, "col", slices)
    total = None
    for t in range(1, slices + 1):
        for u in range(1, slices + 2 - t):
            at = OMatrix(a.nrows, a.ncols, a.bs, a.brow, a.bcol, np.ascontiguousarray(sa[t - 1]))
            bu = OMatrix(b.nrows, b.ncols, b.bs, b.brow, b.bcol, np.ascontiguousarray(sb[u - 1]))
            p = multiply(at, bu)
            if total is None:
                total = p
            else:
                total.vals = total.vals + p.vals
    return total


def rel_fro(x: np.ndarray, ref: np.ndarray) -> float:
    """Relative Frobenius error ||x - ref|| / ||ref||."""
    num = np.linalg.norm((np.asarray(x) - np.asarray(ref)).ravel())
    den = np.linalg.norm(np.asarray(ref).ravel())
    return float(num / den) if den > 0 else float(num)
