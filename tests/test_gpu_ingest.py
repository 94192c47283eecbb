"""Construction from leaf blocks (set_blocks) on both of its device paths:
one workgroup for small inputs (at most 16384 blocks on a block grid of side
at most 512), the multi-launch path otherwise.  Each is checked against the
stored pattern and values worked out on the host (kept blocks in row-major
order, padding beyond the logical size zero), with and without a drop
tolerance, and on its error cases (repeated and out-of-range coordinates
leave the matrix as it was)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2011_11762_amd import qbsm
    assert torch.cuda.is_available()
    qbsm.load()
    return qbsm


def _blocks(nbr, nbc, nblk, bs, seed):
    """nblk distinct random block coordinates in shuffled order, values with
    block norms spread over several decades (so that a drop tolerance keeps
    some and drops others)."""
    rng = np.random.default_rng(seed)
    cells = rng.choice(nbr * nbc, size=nblk, replace=False)
    brow, bcol = (cells // nbc).astype(np.int32), (cells % nbc).astype(np.int32)
    scale = 10.0 ** rng.uniform(-6, 0, size=(nblk, 1))
    vals = rng.standard_normal((nblk, bs * bs)) * scale
    return brow, bcol, vals


def _expected(nrows, ncols, bs, brow, bcol, vals, tol):
    """Kept blocks in row-major block order, padding zeroed; a block is kept
    unless the FP64 Frobenius norm of its logical part is below tol."""
    v = vals.reshape(-1, bs, bs).copy()  # [blk, col, row] (column-major blocks)
    for t in range(v.shape[0]):
        mr = min(bs, nrows - int(brow[t]) * bs)
        nc = min(bs, ncols - int(bcol[t]) * bs)
        v[t, nc:, :] = 0.0
        v[t, :, mr:] = 0.0
    norms = np.sqrt((v.reshape(v.shape[0], -1) ** 2).sum(axis=1))
    keep = ~(norms < tol) if tol > 0 else np.ones(v.shape[0], dtype=bool)
    order = np.lexsort((bcol[keep], brow[keep]))
    return brow[keep][order], bcol[keep][order], v.reshape(v.shape[0], -1)[keep][order]


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# (nrows, ncols, bs, nblk, seed): which path the shape selects
CASES = [
    (100 * 32 - 5, 90 * 32 - 17, 32, 3000, 1),       # one workgroup, ragged edges
    (512 * 32, 512 * 32, 32, 16384, 2),              # one workgroup at both limits
    (200 * 32 - 3, 200 * 32, 32, 20000, 3),          # more blocks than one workgroup takes
    (600 * 32 - 9, 700 * 32 - 1, 32, 700, 4),        # grid side above 512
    (40 * 64, 30 * 64 + 7, 64, 1, 5),                # a single block
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}-bs{c[2]}-n{c[3]}")
@pytest.mark.parametrize("tol", [0.0, 1e-3])
def test_set_blocks_against_host(q, case, tol):
    nrows, ncols, bs, nblk, seed = case
    nbr, nbc = -(-nrows // bs), -(-ncols // bs)
    brow, bcol, vals = _blocks(nbr, nbc, nblk, bs, seed)
    er, ec, ev = _expected(nrows, ncols, bs, brow, bcol, vals, tol)
    M = q.Matrix(nrows, ncols, bs)
    nk = M.set_blocks(_dev(brow), _dev(bcol), _dev(vals), tol)
    torch.cuda.synchronize()
    assert nk == er.size == M.nblk
    r, c = M.pattern()
    assert np.array_equal(r.cpu().numpy(), er) and np.array_equal(c.cpu().numpy(), ec)
    assert np.array_equal(M.values().cpu().numpy(), ev)  # a copy: bit for bit
    # the stored matrix multiplies like its host copy (the walk reads the keys)
    if nbr == nbc and nrows == ncols:
        P = q.Plan(M, M)
        assert P.info()["nblk_out"] > 0


@pytest.mark.parametrize("grid", [(64, 64, 32), (600, 600, 32)], ids=["one-workgroup", "multi-launch"])
def test_set_blocks_empty_and_errors(q, grid):
    nbr, nbc, bs = grid
    M = q.Matrix(nbr * bs, nbc * bs, bs)
    e32 = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert M.set_blocks(e32, e32, torch.zeros(0, bs * bs, dtype=torch.float64, device="cuda")) == 0
    assert M.nblk == 0
    brow, bcol, vals = _blocks(nbr, nbc, 50, bs, 9)
    assert M.set_blocks(_dev(brow), _dev(bcol), _dev(vals)) == 50
    before = M.values().cpu().numpy()
    bad = [
        (np.r_[brow, brow[7]], np.r_[bcol, bcol[7]]),     # repeated coordinate
        (np.r_[brow, nbr], np.r_[bcol, 0]),               # row past the grid
        (np.r_[brow, 0], np.r_[bcol, -1]),                # negative column
    ]
    for br, bc in bad:
        v = np.vstack([vals, vals[:1]])
        for tol in (0.0, 1e-3):
            with pytest.raises(q.QbsmError) as e:
                M.set_blocks(_dev(br.astype(np.int32)), _dev(bc.astype(np.int32)), _dev(v), tol)
            assert e.value.status == 3
            assert M.nblk == 50
            assert np.array_equal(M.values().cpu().numpy(), before)


def test_set_blocks_many_with_repeat(q):
    """A repeated coordinate among more blocks than one workgroup takes."""
    nbr = nbc = 200
    bs = 32
    brow, bcol, vals = _blocks(nbr, nbc, 20000, bs, 11)
    brow[19999], bcol[19999] = brow[3], bcol[3]
    M = q.Matrix(nbr * bs, nbc * bs, bs)
    with pytest.raises(q.QbsmError) as e:
        M.set_blocks(_dev(brow), _dev(bcol), _dev(vals))
    assert e.value.status == 3


@pytest.mark.parametrize("nblk", [6, 20000], ids=["one-workgroup-tree", "multi-launch-tree"])
def test_depth16_grid_against_oracle(q, nblk):
    """A block grid of side 65536 (quadtree depth 16, the largest): the root
    level's keys shift by all 32 bits of a key.  Blocks include the grid's
    corners; the product's pattern and values against the oracle."""
    from oracle import oracle as O

    bs, side = 32, 65536
    n = side * bs
    rng = np.random.default_rng(17)
    if nblk == 6:
        ar = np.array([0, 0, side - 1, 40000, side - 1, 123], dtype=np.int32)
        ac = np.array([0, side - 1, side - 1, 123, 0, 40000], dtype=np.int32)
    else:
        cells = rng.choice(side * side, size=nblk, replace=False)
        ar, ac = (cells // side).astype(np.int32), (cells % side).astype(np.int32)
    # B's rows are A's columns (so every A block meets B blocks), columns random
    br = np.concatenate([ac, rng.integers(0, side, size=nblk // 2).astype(np.int32)])
    bc = np.concatenate([ar[::-1], rng.integers(0, side, size=nblk // 2).astype(np.int32)])
    keyb = np.unique(br.astype(np.int64) * side + bc, return_index=True)[1]
    br, bc = br[keyb], bc[keyb]
    av = rng.uniform(-1, 1, size=(ar.size, bs * bs))
    bv = rng.uniform(-1, 1, size=(br.size, bs * bs))
    A, B = q.Matrix(n, n, bs), q.Matrix(n, n, bs)
    assert A.set_blocks(_dev(ar), _dev(ac), _dev(av)) == ar.size
    assert B.set_blocks(_dev(br), _dev(bc), _dev(bv)) == br.size
    oa = O.canonical(n, n, bs, ar, ac, av, 0.0)
    ob = O.canonical(n, n, bs, br, bc, bv, 0.0)
    ref = O.multiply(oa, ob)
    P = q.Plan(A, B)
    assert P.info()["nprod"] == ref.I.size
    C = P.numeric("f64")
    torch.cuda.synchronize()
    r, c = C.pattern()
    assert np.array_equal(r.cpu().numpy(), ref.brow) and np.array_equal(c.cpu().numpy(), ref.bcol)
    got = C.values().cpu().numpy()
    err = np.linalg.norm(got - ref.vals) / max(np.linalg.norm(ref.vals), 1e-300)
    assert err < 1e-12
