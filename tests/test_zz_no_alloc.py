"""The allocation-free numeric entry point against the regular one.

qbsm_multiply_numeric_noalloc packs the operands into the library's static
scratch array and writes the result to a caller-owned array; it runs the same
kernels as qbsm_multiply_numeric, so its blocks must equal that entry point's
bit for bit.  Two calls in a row, the second on a smaller input (the scratch
keeps the first call's contents), per mode; a masked plan; the size limit.
"""
import numpy as np
import pytest
import torch

from paper_2011_11762_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    from paper_2011_11762_amd import qbsm
    assert torch.cuda.is_available()
    qbsm.load()
    return qbsm


def morton(i, j):
    """Interleaved bits of (I, J), I's bit above J's."""
    i = np.asarray(i, dtype=np.uint64)
    j = np.asarray(j, dtype=np.uint64)
    k = np.zeros(i.shape, dtype=np.uint64)
    for b in range(16):
        k |= ((i >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
        k |= ((j >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
    return k


def regular_in_storage_order(C):
    """Values of a result matrix, FP64, in ascending Morton order of its blocks."""
    r, c = (t.cpu().numpy() for t in C.pattern())
    order = np.argsort(morton(r, c), kind="stable")
    return C.values().cpu().numpy()[order]


def run_noalloc(q, P, mode, nblk, bs):
    dt = torch.float64 if mode in ("f64", "ozaki") else torch.float32
    out = torch.full((nblk, bs * bs), float("nan"), dtype=dt, device="cuda")
    P.numeric_noalloc(mode, out)
    torch.cuda.synchronize()
    return out.to(torch.float64).cpu().numpy()


CASES = [("f64", 128), ("f32", 256), ("bf16", 128), ("bf16x3", 256), ("bf16x3", 64), ("ozaki", 64)]


@pytest.mark.parametrize("mode,unit", CASES)
def test_noalloc_matches_regular_twice(q, mode, unit):
    bs = 64
    # first call on the larger input, second on a smaller one
    for (m, k, n, dens, seed) in ((900, 700, 800, 0.5, 11), (300, 260, 200, 0.6, 12)):
        a, b = W.small_random(m, k, n, bs, dens, seed)
        A, B = q.from_host(a), q.from_host(b)
        P = q.Plan(A, B, unit=unit)
        nout = P.info()["nblk_out"]
        ref = regular_in_storage_order(P.numeric(mode))
        got = run_noalloc(q, P, mode, nout, bs)
        assert got.shape == ref.shape
        assert np.array_equal(got, ref), (mode, unit, m, k, n, "differs from the regular numeric phase")


def test_noalloc_square_and_masked(q):
    bs = 32
    a, _ = W.small_random(500, 500, 500, bs, 0.4, 21)
    A = q.from_host(a)
    # A * A: one matrix in both roles (two packs in the scratch)
    P = q.Plan(A, A, unit=64)
    ref = regular_in_storage_order(P.numeric("f64"))
    assert np.array_equal(run_noalloc(q, P, "f64", P.info()["nblk_out"], bs), ref)
    # A^T * A: the same matrix in the same role on both sides (one pack)
    P2 = q.Plan(A, A, trans_l=True, unit=64)
    ref2 = regular_in_storage_order(P2.numeric("f32"))
    assert np.array_equal(run_noalloc(q, P2, "f32", P2.info()["nblk_out"], bs), ref2)
    # a masked plan: the mask's blocks without products are written as zero
    m, _ = W.small_random(500, 500, 500, bs, 0.3, 22)
    M = q.from_host(m)
    P3 = q.Plan(A, A, mask=M, unit=64)
    ref3 = regular_in_storage_order(P3.numeric("f64"))
    assert np.array_equal(run_noalloc(q, P3, "f64", P3.info()["nblk_out"], bs), ref3)


def test_noalloc_rejects_packs_beyond_the_scratch(q):
    c = W.config5()  # banded N = 16384, 64x64 leaves: 2 x 3286 FP64 leaves = 215 MB of packs
    A, B = q.from_host(c["A"]), q.from_host(c["B"])
    P = q.Plan(A, B)
    out = torch.zeros((P.info()["nblk_out"], 64 * 64), dtype=torch.float64, device="cuda")
    with pytest.raises(q.QbsmError) as e:
        P.numeric_noalloc("f64", out)
    assert e.value.status == 6 and "scratch" in str(e.value)
    assert bool(torch.all(out == 0))  # nothing was launched
    # the same plan in BF16 (2 bytes per element) fits: 27 MB
    ref = regular_in_storage_order(P.numeric("bf16"))
    out32 = torch.empty((P.info()["nblk_out"], 64 * 64), dtype=torch.float32, device="cuda")
    P.numeric_noalloc("bf16", out32)
    torch.cuda.synchronize()
    assert np.array_equal(out32.to(torch.float64).cpu().numpy(), ref)
