"""The streamed numeric schedule (resident workgroups that each run every
G-th unit, the next unit's metadata and first copies issued before this
unit's output is stored) against one workgroup per unit and the oracle.

Both schedules run the same steps of every unit in the same order, so their
outputs are compared bit for bit; the streamed one is also checked against
the FP64 oracle where the oracle finishes in seconds.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2011_11762_amd import workloads as W
from tests.gpu_helpers import assert_product, assert_sampled, pattern_np, upload, values_np

pytestmark = pytest.mark.gpu

MODES = ["f64", "f32", "bf16", "bf16x3"]


@pytest.fixture(scope="module")
def q():
    from paper_2011_11762_amd import qbsm
    assert torch.cuda.is_available()
    qbsm.load()
    return qbsm


def _both(q, A, B, mode, unit, **kw):
    """Values of op(A) op(B) under schedule 1 (one workgroup per unit) and 2 (streamed)."""
    out = []
    for sched in (1, 2):
        P = q.Plan(A, B, unit=unit, schedule=sched, **kw)
        C = P.numeric(mode)
        torch.cuda.synchronize()
        out.append((pattern_np(C), values_np(C), P.info()))
    (p1, v1, i1), (p2, v2, i2) = out
    assert np.array_equal(p1[0], p2[0]) and np.array_equal(p1[1], p2[1])
    assert i1 == i2
    return v1, v2, i1


def _bitwise(v1, v2, what):
    assert v1.dtype == v2.dtype and v1.shape == v2.shape, what
    same = (v1 == v2) | (np.isnan(v1) & np.isnan(v2))
    assert same.all(), f"{what}: {int((~same).sum())} values differ"


# (n, bs, p, seed): random-block matrices with about one leaf product per C
# block; the larger ones have more units than the resident workgroups of the
# streamed grid (2 per CU), so every workgroup runs many units, with a ragged
# last round
SPARSE = [
    (128 * 40 + 17, 128, 0.05, 1),    # fewer units than workgroups
    (128 * 256, 128, 0.01, 2),        # about 1700 units
    (64 * 300 + 5, 64, 0.012, 3),     # unit 64 and 128, ragged edge
    (32 * 600, 32, 0.006, 4),
]


@pytest.mark.parametrize("case", SPARSE, ids=lambda c: f"n{c[0]}-bs{c[1]}-p{c[2]}")
@pytest.mark.parametrize("mode", MODES)
def test_stream_sparse_against_oracle(q, case, mode):
    n, bs, p, seed = case
    rng = np.random.default_rng(seed)
    a = W.random_blocks(n, bs, p, rng)
    b = W.random_blocks(n, bs, p, rng)
    oa, ob = O.from_workload(a), O.from_workload(b)
    ref = O.multiply(oa, ob)
    A, B = upload(q, a), upload(q, b)
    for unit in (u for u in (64, 128) if u >= bs):
        v1, v2, info = _both(q, A, B, mode, unit)
        assert info["nprod"] == ref.I.size and info["nblk_out"] == ref.brow.size
        _bitwise(v1, v2, f"{mode} unit {unit}")
        assert_product(v2, oa, ob, ref.vals, mode, what=f"streamed unit={unit}")


@pytest.mark.parametrize("mode", MODES)
def test_stream_long_units(q, mode):
    """Units with more pairs than one LDS batch of metadata holds (213 pairs
    at unit 64 with 32-wide leaves), more units than resident workgroups: the
    streamed loop runs a unit's later batches before it begins the next
    unit."""
    a, b = W.small_random(32 * 48 + 7, 32 * 480, 32 * 48, 32, 0.97, 21)
    A, B = upload(q, a), upload(q, b)
    v1, v2, info = _both(q, A, B, mode, 64)
    assert info["npairs"] > 213 * info["nunits"] // 2
    _bitwise(v1, v2, mode)
    # a sample of C blocks against the oracle (the whole product has about a
    # million leaf products)
    oa, ob = O.from_workload(a), O.from_workload(b)
    C = q.Plan(A, B, unit=64, schedule=2).numeric(mode)
    cr, cc = pattern_np(C)
    pick = np.sort(np.random.default_rng(5).choice(cr.size, size=8, replace=False))
    si, sj = cr[pick], cc[pick]
    got = C.extract(si, sj).cpu().numpy()
    assert_sampled(got, oa, ob, si, sj, O.multiply_blocks(oa, ob, si, sj), mode, what="long units")


def test_stream_banded_f32_and_masks(q):
    """Banded FP32 inputs (a few pairs per unit, the shape of the masked
    backward's plans): forward, a masked plan and a sparse approximate plan
    agree bit for bit between the schedules."""
    rng = np.random.default_rng(7)
    a = W.banded(64 * 96 + 3, 64, 2, rng, fp32_values=True)
    b = W.banded(64 * 96 + 3, 64, 2, rng, fp32_values=True)
    A, B = upload(q, a), upload(q, b)
    for mode in MODES:
        for unit in (64, 128):
            v1, v2, _ = _both(q, A, B, mode, unit)
            _bitwise(v1, v2, f"{mode} unit {unit}")
    # masked: A^T * B restricted to B's pattern
    v1, v2, _ = _both(q, A, B, "f32", 128, trans_l=True, mask=B)
    _bitwise(v1, v2, "masked")
    norms = O.block_fnorms(O.from_workload(a).vals, 64)
    tau = float(np.median(norms)) ** 2
    v1, v2, info = _both(q, A, B, "bf16x3", 64, spamm_tol=tau)
    assert info["nprod"] > 0
    _bitwise(v1, v2, "spamm")
    # the masked adjoints from a forward plan take its schedule
    dC = q.Plan(A, B, unit=128).numeric("f64")
    grads = []
    for sched in (1, 2):
        dA, dB = q.Plan(A, B, unit=128, schedule=sched).backward(dC, "f32")
        grads.append((values_np(dA), values_np(dB)))
    _bitwise(grads[0][0], grads[1][0], "dA")
    _bitwise(grads[0][1], grads[1][1], "dB")


def test_stream_nonfinite(q):
    """Inf and NaN travel the same way under both schedules."""
    rng = np.random.default_rng(9)
    a = W.random_blocks(128 * 60, 128, 0.04, rng)
    b = W.random_blocks(128 * 60, 128, 0.04, rng)
    a.vals[1, 7] = np.inf
    a.vals[4, 300] = np.nan
    b.vals[2, 9] = -np.inf
    A, B = upload(q, a), upload(q, b)
    for mode in ("f64", "f32", "bf16x3"):
        v1, v2, _ = _both(q, A, B, mode, 128)
        _bitwise(v1, v2, mode)
        assert (~np.isfinite(v2)).any()


def test_schedule_option_checked(q):
    a, b = W.small_random(300, 260, 200, 64, 0.5, 11)
    A, B = upload(q, a), upload(q, b)
    for bad in (-1, 3):
        with pytest.raises(q.QbsmError, match="schedule"):
            q.Plan(A, B, schedule=bad)
    # streamed where not available (unit 256; the Ozaki mode) runs one
    # workgroup per unit
    ref = values_np(q.Plan(A, B, unit=256, schedule=1).numeric("f32"))
    _bitwise(values_np(q.Plan(A, B, unit=256, schedule=2).numeric("f32")), ref, "unit 256")
    ref = values_np(q.Plan(A, B, unit=64, schedule=1).numeric("ozaki"))
    _bitwise(values_np(q.Plan(A, B, unit=64, schedule=2).numeric("ozaki")), ref, "ozaki")


def _from_mask(mask, bs, rng):
    """Block matrix (U[-1,1] values) with the leaves of a boolean mask."""
    ii, jj = np.nonzero(mask)
    n = mask.shape[0] * bs
    return W.BlockMatrix(n, n, bs, ii.astype(np.int32), jj.astype(np.int32),
                         rng.uniform(-1.0, 1.0, size=(ii.size, bs * bs)), {"kind": "test"})


@pytest.mark.parametrize("mode", ["bf16", "bf16x3", "f64"])
def test_single_stage_schedule(q, mode):
    """The automatic schedule's single-stage kernel (BF16 modes at unit 128,
    about one unit-level pair per unit) against the double-buffered kernel,
    bit for bit, and against the oracle.  One unit holds 50 pairs, more than
    one metadata batch (28 pairs of 2 x 2 leaves), among about 5500 units of
    about one pair each."""
    bs, nb = 64, 400
    rng = np.random.default_rng(31)
    ma = np.zeros((nb, nb), dtype=bool)
    mb = np.zeros((nb, nb), dtype=bool)
    ma[0, :100] = True      # C block (0, 0): 100 leaf products over K < 100
    mb[:100, 0] = True
    ma[2:, 200:] = rng.random((nb - 2, nb - 200)) < 0.01
    mb[200:, 2:] = rng.random((nb - 200, nb - 2)) < 0.01
    a, b = _from_mask(ma, bs, rng), _from_mask(mb, bs, rng)
    oa, ob = O.from_workload(a), O.from_workload(b)
    ref = O.multiply(oa, ob)
    A, B = upload(q, a), upload(q, b)
    vals = {}
    for sched in (0, 1):
        P = q.Plan(A, B, unit=128, schedule=sched)
        info = P.info()
        C = P.numeric(mode)
        torch.cuda.synchronize()
        cr, cc = pattern_np(C)
        assert np.array_equal(cr, ref.brow) and np.array_equal(cc, ref.bcol)
        vals[sched] = values_np(C)
    # the automatic schedule's condition for the single-stage kernel holds
    assert 4 * info["npairs"] <= 5 * info["nunits"] and info["nunits"] > 1000
    _bitwise(vals[0], vals[1], mode)
    assert_product(vals[0], oa, ob, ref.vals, mode, what="single-stage")


@pytest.mark.parametrize("case", [(300, 260, 200, 64, 0.5, 1), (400, 300, 520, 128, 0.6, 3),
                                  (64 * 9 + 5, 64 * 7, 64 * 11 + 63, 64, 0.3, 5)],
                         ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-bs{c[3]}")
def test_single_stage_f64_dense(q, case):
    """FP64 at unit 128 takes the single-stage kernel under the automatic
    schedule on every plan: against the double-buffered kernel (bit for bit)
    and the oracle, on ragged rectangular products with several pairs per
    unit."""
    m, k, n, bs, p, seed = case
    a, b = W.small_random(m, k, n, bs, p, seed)
    oa, ob = O.from_workload(a), O.from_workload(b)
    ref = O.multiply(oa, ob)
    A, B = upload(q, a), upload(q, b)
    vals = {}
    for sched in (0, 1):
        C = q.Plan(A, B, unit=128, schedule=sched).numeric("f64")
        torch.cuda.synchronize()
        vals[sched] = values_np(C)
    _bitwise(vals[0], vals[1], "f64")
    assert_product(vals[0], oa, ob, ref.vals, "f64", what="single-stage f64")
