"""Element-level assignment / extraction and error-controlled truncation on
the GPU against the oracle: patterns bit-exact, values exact (they are
copies), truncation's kept set bit-exact away from ties with eps."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_11762_amd import workloads as W
from tests.gpu_helpers import assert_product, pattern_np, upload, values_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2011_11762_amd import qbsm
    assert torch.cuda.is_available()
    qbsm.load()
    return qbsm


def _elements(n, m, count, seed):
    rng = np.random.default_rng(seed)
    pos = rng.choice(n * m, count, replace=False)
    return pos // m, pos % m, rng.uniform(-1, 1, count)


@pytest.mark.parametrize("n,m,bs", [(300, 250, 32), (1000, 700, 64), (513, 513, 128)])
def test_set_and_get_elements(q, n, m, bs):
    r, c, v = _elements(n, m, 5000, 40 + bs)
    ref = O.from_elements(n, m, bs, r, c, v)
    A = q.Matrix(n, m, bs)
    nb = A.set_elements(torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda(), torch.from_numpy(v).cuda())
    assert nb == ref.nblk
    pr, pc = pattern_np(A)
    assert np.array_equal(pr, ref.brow) and np.array_equal(pc, ref.bcol)
    assert np.array_equal(values_np(A), ref.vals)
    rng = np.random.default_rng(7)
    qr = np.concatenate([r[:500], rng.integers(0, n, 500)])
    qc = np.concatenate([c[:500], rng.integers(0, m, 500)])
    assert np.array_equal(A.get_elements(qr, qc).cpu().numpy(), O.get_elements(ref, qr, qc))
    # the element-built matrix multiplies like any other
    b = W.random_blocks(m, bs, 0.4, np.random.default_rng(8), ncols=300)
    B = upload(q, b)
    got = values_np(q.matmul(A, B, "f64"))
    ob = O.from_workload(b)
    assert_product(got, ref, ob, O.multiply(ref, ob).vals, "f64", what="element-built operand")


def test_element_errors(q):
    n, bs = 200, 32
    A = q.Matrix(n, n, bs)
    r, c, v = _elements(n, n, 100, 3)
    T = lambda x, dt=torch.int64: torch.as_tensor(x, dtype=dt).cuda()
    with pytest.raises(q.QbsmError):  # repeated (row, col)
        A.set_elements(T(np.append(r, r[5])), T(np.append(c, c[5])), T(np.append(v, 2.0), torch.float64))
    with pytest.raises(q.QbsmError):  # outside the matrix
        A.set_elements(T([n]), T([0]), T([1.0], torch.float64))
    A.set_elements(T(r), T(c), T(v, torch.float64))
    with pytest.raises(q.QbsmError):
        A.get_elements([0, n], [0, 0])
    assert A.get_elements([int(r[0])], [int(c[0])]).item() == v[0]


@pytest.mark.parametrize("store_f32", [False, True])
def test_truncate_error_control(q, store_f32):
    rng = np.random.default_rng(11)
    a = W.random_blocks(900, 32, 0.4, rng)
    a.vals *= np.exp(rng.uniform(-14, 0, a.nblk))[:, None]
    a.vals[3] = 0.0                  # an identically zero leaf
    a.vals[7, 5] = np.nan            # a NaN leaf stays
    oa = O.from_workload(a)
    if store_f32:
        oa = O.OMatrix(oa.nrows, oa.ncols, oa.bs, oa.brow, oa.bcol, O.round_to_f32(oa.vals))
    for eps in (0.0, 1e-9, 1e-6, 1e-3, 1e-1):
        assert O.truncate_borderline(oa, eps) == 0
        ref = O.truncate_error_control(oa, eps)
        A = upload(q, a)
        if store_f32:
            A.store_f32()
        assert A.truncate(eps) == ref.nblk
        pr, pc = pattern_np(A)
        assert np.array_equal(pr, ref.brow) and np.array_equal(pc, ref.bcol), eps
        got = values_np(A)
        assert np.array_equal(np.isnan(got), np.isnan(ref.vals))
        assert np.array_equal(np.nan_to_num(got), np.nan_to_num(ref.vals))
    with pytest.raises(q.QbsmError):
        A.truncate(-1.0)


def test_truncate_keeps_infinite_norms(q):
    """A leaf with an infinite norm stays for every eps, also where eps^2
    overflows; so does a leaf whose squared norm overflows."""
    rng = np.random.default_rng(12)
    a = W.random_blocks(600, 32, 0.4, rng)
    a.vals[4, 9] = np.inf
    a.vals[8] *= 1e170
    oa = O.from_workload(a)
    with np.errstate(over="ignore"):
        for eps in (1e-3, 1e200, np.finfo(np.float64).max):
            ref = O.truncate_error_control(oa, eps)
            A = upload(q, a)
            assert A.truncate(eps) == ref.nblk
            pr, pc = pattern_np(A)
            assert np.array_equal(pr, ref.brow) and np.array_equal(pc, ref.bcol), eps
            assert np.array_equal(values_np(A), ref.vals)
    assert ref.nblk == 2


def test_truncate_product(q):
    """Truncation of a multiply's FP32 result, then a second multiply with it."""
    c = W.config2(npoints=2000, bs=32, seed=19)
    a, tol = c["A"], c["drop_tol"]
    A = upload(q, a, tol)
    C = q.matmul(A, A, "f32")
    oc = O.OMatrix(C.nrows, C.ncols, 32, *pattern_np(C), values_np(C))
    eps = 1e-4 * np.linalg.norm(oc.vals)
    assert O.truncate_borderline(oc, eps) == 0
    ref = O.truncate_error_control(oc, eps)
    assert C.truncate(eps) == ref.nblk < oc.nblk
    pr, pc = pattern_np(C)
    assert np.array_equal(pr, ref.brow) and np.array_equal(pc, ref.bcol)
    assert np.array_equal(values_np(C), ref.vals)
    got = values_np(q.matmul(C, A, "f64"))
    oa2 = O.from_workload(a, tol)
    assert_product(got, ref, oa2, O.multiply(ref, oa2).vals, "f64", what="truncated operand")


def test_empty_and_degenerate_new_operations(q):
    """Zero elements, truncation of an empty matrix, empty queries, packing an
    empty matrix ahead, and a tolerance that leaves out every product."""
    bs = 32
    E = q.Matrix(100, 90, bs)
    T = lambda x, dt=torch.int64: torch.as_tensor(x, dtype=dt).cuda()
    assert E.set_elements(T([]), T([]), T([], torch.float64)) == 0
    assert E.nblk == 0 and E.truncate(1.0) == 0
    assert E.get_elements([], []).numel() == 0
    E.prepack("bf16x3", 3)
    b = W.random_blocks(90, bs, 0.5, np.random.default_rng(3), ncols=70)
    B = upload(q, b)
    C = q.matmul(E, B, "f32")
    assert C.nblk == 0
    # one element: one leaf; squares and products of it
    one = q.Matrix(40, 40, bs)
    assert one.set_elements(T([33]), T([5]), T([2.0], torch.float64)) == 1
    assert one.get_elements([33, 0], [5, 0]).cpu().numpy().tolist() == [2.0, 0.0]
    sq = q.matmul(one, one, "f64")   # (33,5) * (33,5): no product (5 != 33 // 32 block)
    assert sq.nblk == (1 if 33 // bs == 5 // bs else 0)
    # every product left out: empty output, zero units
    c = W.config2(npoints=1200, bs=32, seed=21)
    A = upload(q, c["A"], c["drop_tol"])
    P = q.Plan(A, A, spamm_tol=1e30)
    assert P.info()["nprod"] == 0 and P.info()["nblk_out"] == 0
    assert P.numeric("bf16x3").nblk == 0
    # the upper triangle of a single-leaf product is that leaf
    s1 = W.small_random(30, 30, 30, bs, 1.0, 22)[0]
    S1 = upload(q, s1)
    U1 = q.Plan(S1, S1, upper=True).numeric("f64")
    full = q.matmul(S1, S1, "f64")
    assert np.array_equal(values_np(U1), values_np(full))


@pytest.mark.parametrize("bs", [32, 64])
def test_matrix_addition(q, bs):
    """alpha A + beta B and A + sigma I against the oracle, bit for bit (each
    element is two rounded products and one rounded sum on both sides);
    FP32-stored operands; the sum then feeds a multiply."""
    rng = np.random.default_rng(30 + bs)
    n, m = 9 * bs + 3, 7 * bs + 11
    a = W.random_blocks(n, bs, 0.3, rng, ncols=m)
    b = W.random_blocks(n, bs, 0.3, rng, ncols=m)
    oa, ob = O.from_workload(a), O.from_workload(b)
    A, B = upload(q, a), upload(q, b)
    C = q.add(0.75, A, -1.5, B)
    ref = O.add(0.75, oa, -1.5, ob)
    cr, cc = pattern_np(C)
    assert np.array_equal(cr, ref.brow) and np.array_equal(cc, ref.bcol)
    assert np.array_equal(values_np(C), ref.vals)
    # FP32 storage of one operand: its values widened exactly
    B.store_f32()
    ob32 = O.OMatrix(ob.nrows, ob.ncols, bs, ob.brow, ob.bcol, O.round_to_f32(ob.vals))
    assert np.array_equal(values_np(q.add(2.0, A, 1.0, B)), O.add(2.0, oa, 1.0, ob32).vals)
    # scaled identity, in place, creating missing diagonal leaves
    S = upload(q, a)
    S.add_identity(-3.25)
    refi = O.add_identity(oa, -3.25)
    sr, sc = pattern_np(S)
    assert np.array_equal(sr, refi.brow) and np.array_equal(sc, refi.bcol)
    assert np.array_equal(values_np(S), refi.vals)
    # (A + B) X through the multiply
    x = W.random_blocks(m, bs, 0.4, rng, ncols=5 * bs)
    got = values_np(q.matmul(q.add(1.0, A, 1.0, upload(q, b)), upload(q, x), "f64"))
    osum, ox = O.add(1.0, oa, 1.0, ob), O.from_workload(x)
    assert_product(got, osum, ox, O.multiply(osum, ox).vals, "f64", what="sum operand")
    with pytest.raises(q.QbsmError):
        q.add(1.0, A, 1.0, upload(q, W.random_blocks(n, bs, 0.3, rng, ncols=m + bs)))
