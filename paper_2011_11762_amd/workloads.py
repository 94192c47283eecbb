"""Seeded synthetic inputs with the shapes of the paper's block-sparse workloads.

This module only draws inputs.  It holds none of the multiply's arithmetic
(no norms, no dropping, no products): both the GPU path and the CPU oracle
receive the same FP64 arrays produced here.

Conventions shared by every generator
-------------------------------------
* A block-sparse matrix is a set of dense ``bs x bs`` leaf blocks at block
  coordinates ``(I, J)``; blocks not listed are identically zero (the nil
  child of the sparse quadtree, paper Sec. 2 and 2.1).
* Leaf blocks use the column-wise element layout of the paper's basic dense
  leaf type (Sec. 2.1): element ``(r, c)`` of a block sits at flat index
  ``r + c * bs``.
* Blocks are listed in canonical row-major block order ``(I, J)``.
* When the logical size is not a multiple of ``bs`` the last block row /
  column is zero-padded inside the block (the paper's N = 1e5 with 2048
  leaves is such a ragged case, Sec. 3).
* Random draws use ``numpy.random.default_rng(seed)`` (PCG64).  For one
  matrix the pattern is drawn first, then the values of the stored blocks in
  canonical order, each block as ``bs*bs`` numbers filling the block
  column-major.  When a workload has two random operands, A is drawn
  completely before B from the same stream.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "BlockMatrix",
    "banded",
    "random_blocks",
    "decay_points",
    "decay_blocks",
    "config1",
    "config2",
    "config3",
    "config4_members",
    "config4_member",
    "config5",
    "small_random",
    "zero_padding",
    "decay_blocks_device",
    "PAPER_TABLE1",
    "paper_block_size",
    "paper_workload",
    "paper_dense_blocks",
    "paper_element_flops",
]


@dataclass
class BlockMatrix:
    """Host-side block-sparse matrix in the library's exchange format."""

    nrows: int
    ncols: int
    bs: int
    brow: np.ndarray  # int32 [nblk], canonical row-major order
    bcol: np.ndarray  # int32 [nblk]
    vals: np.ndarray  # float64 [nblk, bs*bs], column-major inside a block
    meta: dict = field(default_factory=dict)

    @property
    def nblk(self) -> int:
        return int(self.brow.shape[0])

    @property
    def nbr(self) -> int:
        return -(-self.nrows // self.bs)

    @property
    def nbc(self) -> int:
        return -(-self.ncols // self.bs)

    def to_dense(self) -> np.ndarray:
        """Assemble the logical dense matrix (small sizes only)."""
        bs = self.bs
        out = np.zeros((self.nbr * bs, self.nbc * bs), dtype=np.float64)
        for t in range(self.nblk):
            i, j = int(self.brow[t]), int(self.bcol[t])
            out[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs] = self.vals[t].reshape(bs, bs).T
        return out[: self.nrows, : self.ncols]


def _pad_mask(n_logical: int, bs: int, b: int) -> int:
    """Number of valid rows (or columns) in block row/column ``b``."""
    return max(0, min(bs, n_logical - b * bs))


def zero_padding(m: BlockMatrix) -> None:
    """Zero the elements of edge blocks that lie beyond the logical size."""
    bs = m.bs
    if m.nrows % bs == 0 and m.ncols % bs == 0:
        return
    v = m.vals.reshape(-1, bs, bs)  # [blk, c, r]
    for t in range(m.nblk):
        mr = _pad_mask(m.nrows, bs, int(m.brow[t]))
        nc = _pad_mask(m.ncols, bs, int(m.bcol[t]))
        if mr < bs:
            v[t, :, mr:] = 0.0
        if nc < bs:
            v[t, nc:, :] = 0.0


def _fill_uniform(rng, nblk: int, bs: int, fp32_values: bool) -> np.ndarray:
    vals = rng.uniform(-1.0, 1.0, size=(nblk, bs * bs))
    if fp32_values:
        vals = vals.astype(np.float32).astype(np.float64)
    return vals


def _from_mask(mask: np.ndarray):
    ii, jj = np.nonzero(mask)  # row-major order
    return ii.astype(np.int32), jj.astype(np.int32)


def banded(n: int, bs: int, h: int, rng, ncols: int | None = None,
           fp32_values: bool = False) -> BlockMatrix:
    """Block-banded pattern |I - J| <= h with U[-1, 1] entries."""
    ncols = n if ncols is None else ncols
    nbr, nbc = -(-n // bs), -(-ncols // bs)
    ii, jj = np.meshgrid(np.arange(nbr), np.arange(nbc), indexing="ij")
    mask = np.abs(ii - jj) <= h
    brow, bcol = _from_mask(mask)
    m = BlockMatrix(n, ncols, bs, brow, bcol,
                    _fill_uniform(rng, brow.shape[0], bs, fp32_values),
                    {"kind": "banded", "h": h})
    zero_padding(m)
    return m


def random_blocks(n: int, bs: int, p: float, rng, ncols: int | None = None,
                  fp32_values: bool = False) -> BlockMatrix:
    """Each block present independently with probability ``p``."""
    ncols = n if ncols is None else ncols
    nbr, nbc = -(-n // bs), -(-ncols // bs)
    mask = rng.random((nbr, nbc)) < p
    brow, bcol = _from_mask(mask)
    m = BlockMatrix(n, ncols, bs, brow, bcol,
                    _fill_uniform(rng, brow.shape[0], bs, fp32_values),
                    {"kind": "random", "p": p})
    zero_padding(m)
    return m


def decay_points(npoints: int, density: float, rng) -> np.ndarray:
    """Points uniform in a cube of the given density, sorted along a Morton curve.

    Each coordinate is quantised to 21 bits over [0, side); the three codes
    are bit-interleaved with x in the highest position of each triple; ties
    keep the original draw order (stable sort).
    """
    side = (npoints / density) ** (1.0 / 3.0)
    pts = rng.uniform(0.0, side, size=(npoints, 3))
    q = np.clip(np.floor(pts / side * (1 << 21)), 0, (1 << 21) - 1).astype(np.uint64)
    code = np.zeros(npoints, dtype=np.uint64)
    for b in range(21):
        for axis, shift in ((0, 2), (1, 1), (2, 0)):
            bit = (q[:, axis] >> np.uint64(b)) & np.uint64(1)
            code |= bit << np.uint64(3 * b + shift)
    order = np.argsort(code, kind="stable")
    return pts[order]


def decay_blocks(points: np.ndarray, bs: int, alpha: float = 0.5) -> BlockMatrix:
    """All blocks of the matrix exp(-alpha * |p_i - p_j|) (Euclidean, no images).

    Every block of the block grid is returned; dropping small blocks is the
    multiply's job, not the generator's.
    """
    n = points.shape[0]
    nb = -(-n // bs)
    brow, bcol = _from_mask(np.ones((nb, nb), dtype=bool))
    vals = np.zeros((nb * nb, bs * bs), dtype=np.float64)
    v = vals.reshape(nb, nb, bs, bs)  # [I, J, c, r]
    for bi in range(nb):
        r0, r1 = bi * bs, min(n, (bi + 1) * bs)
        diff = points[r0:r1, None, :] - points[None, :, :]
        dist = np.sqrt(np.sum(diff * diff, axis=2))
        rowblk = np.exp(-alpha * dist)  # [r, col]
        full = np.zeros((bs, nb * bs), dtype=np.float64)
        full[: r1 - r0, :n] = rowblk
        # [r, J, c] -> [J, c, r]
        v[bi] = full.reshape(bs, nb, bs).transpose(1, 2, 0)
    return BlockMatrix(n, n, bs, brow, bcol, vals, {"kind": "decay", "alpha": alpha})


def decay_blocks_device(points: np.ndarray, bs: int, alpha: float = 0.5, device="cuda"):
    """Same blocks as :func:`decay_blocks`, generated with torch on a device.

    Returns (brow, bcol, vals) as int32 / int32 / float64 device tensors in
    canonical order.  Elementwise FP64 arithmetic on the device may differ
    from numpy's ``exp`` in the last bit, so consumers that compare against
    a reference must read the values back from these tensors.
    """
    import torch

    n = points.shape[0]
    nb = -(-n // bs)
    p = torch.from_numpy(np.ascontiguousarray(points)).to(device=device, dtype=torch.float64)
    vals = torch.zeros((nb, nb, bs, bs), dtype=torch.float64, device=device)  # [I, J, c, r]
    for bi in range(nb):
        r0, r1 = bi * bs, min(n, (bi + 1) * bs)
        diff = p[r0:r1, None, :] - p[None, :, :]
        rowblk = torch.exp(-alpha * torch.sqrt((diff * diff).sum(dim=2)))  # [r, col]
        full = torch.zeros((bs, nb * bs), dtype=torch.float64, device=device)
        full[: r1 - r0, :n] = rowblk
        vals[bi] = full.reshape(bs, nb, bs).permute(1, 2, 0)
    ii, jj = torch.meshgrid(torch.arange(nb, device=device), torch.arange(nb, device=device), indexing="ij")
    return (ii.reshape(-1).to(torch.int32).contiguous(), jj.reshape(-1).to(torch.int32).contiguous(),
            vals.reshape(nb * nb, bs * bs))


# --------------------------------------------------------------------------
# The five workloads (sizes and seeds fixed; see the module docstring)
# --------------------------------------------------------------------------

def config1():
    """N=2048, 32x32 leaves, block-banded half-bandwidth 4, FP64, seed 1."""
    rng = np.random.default_rng(1)
    a = banded(2048, 32, 4, rng)
    b = banded(2048, 32, 4, rng)
    return {"name": "banded-n2048-bs32-h4", "A": a, "B": b, "drop_tol": 0.0}


def config2(npoints: int = 16384, bs: int = 64, seed: int = 2):
    """3-D exponential decay, 16384 points at density 0.1 per cubic Angstrom,
    64x64 leaves, drop tolerance 1e-10; A and B are the same matrix."""
    rng = np.random.default_rng(seed)
    pts = decay_points(npoints, 0.1, rng)
    a = decay_blocks(pts, bs)
    return {"name": f"decay3d-n{npoints}-bs{bs}", "A": a, "B": a, "drop_tol": 1e-10,
            "points": pts}


def config3(n: int = 65536, bs: int = 128, p: float = 0.01, seed: int = 3):
    """N=65536, 128x128 leaves, each block present with probability 0.01."""
    rng = np.random.default_rng(seed)
    a = random_blocks(n, bs, p, rng)
    b = random_blocks(n, bs, p, rng)
    return {"name": f"randblk-n{n}-bs{bs}-p{p}", "A": a, "B": b, "drop_tol": 0.0}


def config4_members(nmembers: int = 256, seed: int = 4):
    """Parameters of the batched workload's members (cheap; no values).

    Member m: N ~ U_int[1024, 16384], leaf size 32 or 64 with probability 1/2;
    even m banded with half-bandwidth U_int[2, 8]; odd m 3-D decay as in
    config 2 at the same density (drop tolerance 1e-10).
    """
    rng = np.random.default_rng(seed)
    out = []
    for m in range(nmembers):
        n = int(rng.integers(1024, 16384, endpoint=True))
        bs = int(rng.choice([32, 64]))
        if m % 2 == 0:
            h = int(rng.integers(2, 8, endpoint=True))
            out.append({"m": m, "n": n, "bs": bs, "kind": "banded", "h": h, "drop_tol": 0.0})
        else:
            out.append({"m": m, "n": n, "bs": bs, "kind": "decay", "drop_tol": 1e-10})
    return out


def config4_member(spec: dict, seed: int = 4):
    """Values of one batched member, drawn from its own stream (seed, m)."""
    rng = np.random.default_rng([seed, spec["m"]])
    if spec["kind"] == "banded":
        a = banded(spec["n"], spec["bs"], spec["h"], rng, fp32_values=True)
        b = banded(spec["n"], spec["bs"], spec["h"], rng, fp32_values=True)
        return {"A": a, "B": b, "drop_tol": 0.0}
    pts = decay_points(spec["n"], 0.1, rng)
    a = decay_blocks(pts, spec["bs"])
    return {"A": a, "B": a, "drop_tol": spec["drop_tol"], "points": pts}


def config5(n: int = 16384, bs: int = 64, h: int = 6, seed: int = 5):
    """Forward + masked backward: banded h=6, FP32 entries, dC on C's pattern."""
    rng = np.random.default_rng(seed)
    a = banded(n, bs, h, rng, fp32_values=True)
    b = banded(n, bs, h, rng, fp32_values=True)
    dc = banded(n, bs, 2 * h, rng, fp32_values=True)
    return {"name": f"banded-n{n}-bs{bs}-h{h}-bwd", "A": a, "B": b, "dC": dc, "drop_tol": 0.0}


def small_random(m: int, k: int, n: int, bs: int, p: float, seed: int,
                 fp32_values: bool = False):
    """Small rectangular pair with random block patterns (tests)."""
    rng = np.random.default_rng(seed)
    a = random_blocks(m, bs, p, rng, ncols=k, fp32_values=fp32_values)
    b = random_blocks(k, bs, p, rng, ncols=n, fp32_values=fp32_values)
    return a, b


# ---------------------------------------------------------------------------
# The paper's weak-scaling workloads (Sec. 3, Table 1): element-level band of
# half-width 3000 (bandwidth 2*3000 + 1), optionally with dense square blocks
# on the diagonal, stored as block-sparse matrices of 64 x 64 leaves.

# Table 1: n -> (growing-block size, random-blocks size, number of random blocks)
PAPER_TABLE1 = {
    100000: (15716, 15716, 1),
    200000: (19652, 15705, 2),
    400000: (24621, 15700, 4),
    800000: (30899, 15697, 8),
    1600000: (38825, 15696, 16),
    3200000: (48828, 15695, 32),
    6400000: (61446, 15695, 64),
}
PAPER_HALF_BAND = 3000


def _column_counts(n: int, h: int, blocks) -> np.ndarray:
    """Nonzeros per column of band(h) united with dense diagonal blocks
    [p, p + s) (symmetric pattern: also the nonzeros per row)."""
    k = np.arange(n, dtype=np.int64)
    lo, hi = np.maximum(k - h, 0), np.minimum(k + h, n - 1)
    c = hi - lo + 1
    for p, sz in blocks:
        l1, h1 = lo[p:p + sz], hi[p:p + sz]
        ov = np.maximum(0, np.minimum(h1, p + sz - 1) - np.maximum(l1, p) + 1)
        c[p:p + sz] = (h1 - l1 + 1) + sz - ov
    return c


def _mults(c: np.ndarray) -> int:
    # scalar multiplications of A * A for a symmetric pattern: sum_k c_k^2
    return int((c.astype(np.int64) ** 2).sum())


def paper_block_size(n: int, h: int = PAPER_HALF_BAND) -> int:
    """Side of the upper-left dense block that doubles the multiplications of
    A * A against the band alone (the growing-block rule, nearest size)."""
    target = 2 * _mults(_column_counts(n, h, []))
    lo, hi = 1, n
    while lo < hi:
        mid = (lo + hi) // 2
        if _mults(_column_counts(n, h, [(0, mid)])) >= target:
            hi = mid
        else:
            lo = mid + 1
    cands = [sz for sz in (lo - 1, lo) if sz >= 1]
    return min(cands, key=lambda sz: abs(_mults(_column_counts(n, h, [(0, sz)])) - target))


def paper_dense_blocks(kind: str, n: int, h: int, rng) -> list:
    """Dense diagonal blocks [(start, size)] of one paper workload; draws the
    random positions from ``rng`` (the first draws of the workload)."""
    if kind == "banded":
        return []
    if kind not in ("growing", "random"):
        raise ValueError(f"unknown paper workload {kind!r}")
    if n in PAPER_TABLE1 and h == PAPER_HALF_BAND:
        sg, sr, k = PAPER_TABLE1[n]
    else:
        sg = paper_block_size(n, h)
        sr, k = sg, 1
    if kind == "growing":
        return [(0, sg)]
    assert k * sr <= n, "dense blocks do not fit"
    x = np.sort(rng.integers(0, n - k * sr + 1, size=k))
    return [(int(x[i]) + i * sr, sr) for i in range(k)]


def paper_element_flops(kind: str, n: int = 100000, h: int = PAPER_HALF_BAND, seed: int = 11) -> int:
    """Element-level flops (two per scalar multiply-add) of A * A for the
    workload ``paper_workload(kind, n, h=h, seed=seed)``; Table 1's count."""
    return 2 * _mults(_column_counts(n, h, paper_dense_blocks(kind, n, h, np.random.default_rng(seed))))


def paper_workload(kind: str, n: int = 100000, bs: int = 64, h: int = PAPER_HALF_BAND, seed: int = 11,
                   chunk: int = 4096) -> BlockMatrix:
    """One matrix of the paper's Banded / Growing block / Random blocks sequences.

    ``kind``: "banded", "growing" (one dense block at the upper-left corner) or
    "random" (equally sized dense blocks at random non-overlapping diagonal
    positions).  Block sizes and counts are Table 1's where ``n`` is printed
    there, else the growing-block doubling rule with one block.  Entries of the
    element structure are U[-1, 1] (the paper does not give values); every
    other element, and the padding past ``n``, is zero.  The block pattern is
    exactly the set of leaves that hold structure elements.  Draw order: the
    random block positions, then the values of the stored blocks (canonical
    order, each block column-major).
    """
    rng = np.random.default_rng(seed)
    dense = paper_dense_blocks(kind, n, h, rng)
    nb = -(-n // bs)
    # candidate leaves: the block band plus the blocks covering each dense block
    hb = (h + bs - 1) // bs
    cand = set()
    ii = np.arange(nb)
    for d in range(-hb, hb + 1):
        jj = ii + d
        ok = (jj >= 0) & (jj < nb)
        cand.update(zip(ii[ok].tolist(), jj[ok].tolist()))
    for p, sz in dense:
        r = range(p // bs, (p + sz - 1) // bs + 1)
        cand.update((a, b) for a in r for b in r)
    key = np.array(sorted(cand), dtype=np.int64).reshape(-1, 2)
    a_in = np.arange(bs * bs) % bs  # row inside the leaf
    b_in = np.arange(bs * bs) // bs  # column inside the leaf

    def masks(t0, t1):
        R = (key[t0:t1, 0:1] * bs).astype(np.int32) + a_in[None, :].astype(np.int32)
        C = (key[t0:t1, 1:2] * bs).astype(np.int32) + b_in[None, :].astype(np.int32)
        m = np.abs(R - C) <= h
        for p, sz in dense:
            m |= (R >= p) & (R < p + sz) & (C >= p) & (C < p + sz)
        m &= (R < n) & (C < n)
        return m

    keep = np.zeros(key.shape[0], dtype=bool)
    for t0 in range(0, key.shape[0], chunk):
        keep[t0:t0 + chunk] = masks(t0, t0 + chunk).any(axis=1)
    key = key[keep]
    vals = rng.uniform(-1.0, 1.0, size=(key.shape[0], bs * bs))
    for t0 in range(0, key.shape[0], chunk):
        vals[t0:t0 + chunk] *= masks(t0, t0 + chunk)
    return BlockMatrix(n, n, bs, key[:, 0].astype(np.int32), key[:, 1].astype(np.int32), vals,
                       {"kind": f"paper-{kind}", "h": h, "dense_blocks": dense,
                        "element_flops": 2 * _mults(_column_counts(n, h, dense))})
