"""Per-block error bounds of the precision modes (test infrastructure).

Every block C_IJ = sum_K A_IK B_KJ of a GPU result is compared with the FP64
oracle's block through a normwise bound

    ||C_IJ - ref_IJ||_F <= c * r_mode(n) * S_IJ,   S_IJ = sum_K ||A_IK||_F ||B_KJ||_F,

where n = (leaf products of the block) * bs is the length of the inner
products that form each element, and c = 2 is a safety factor that also
covers the oracle's own FP64 rounding.  S_IJ is the Frobenius norm scale of
|A||B| restricted to the block (triangle inequality and submultiplicativity),
so a zero or wrong block fails the check whatever the norms of the other
blocks are, which a single relative Frobenius norm over the whole C cannot
guarantee when block norms span many decades.

r_mode(n) is the worst-case relative bound of the mode's arithmetic with unit
roundoffs u64 = 2^-53 and u32 = 2^-24 (gamma_n ~ n u for sums in any order,
products exact or rounded once):

* F64:    n u64 (FP64 products and sums).
* F32:    (n + 3) u32: inputs rounded to binary32 (2 u32 per product), FP32
          sums (n u32), the FP32 result rounded once more (u32).
* BF16:   n u32 + 2 * 2^-8 + 2^-16 + u32: inputs rounded to bfloat16
          (8 significant bits, 2^-8 each), exact products, FP32 sums.
* BF16X3: 3 n u32 + 4 * 2^-16 + u32: a = hi + lo + d with |d| <= 2^-16 |a|;
          the three kept terms hi hi + hi lo + lo hi miss lo lo and the d
          terms (below 3.1 * 2^-16 |a||b|), and 3 n products are summed in FP32.
* OZAKI:  n u64 + (29 bs + 4) 2^-48: an element a of a line with maximum m
          gets the line exponent e with 2^e < 2.01 m (the frexp exponent, or
          one more for a maximum within 0.4 % below a power of two); a is cut
          to M = floor(|a| 2^(47-e)) on the grid 2^(e-47), a = sum of six
          slices + d with |d| < 2^(e-47) < 4.02 2^-48 m, slice t a balanced
          digit of at most 128 on the grid 2^(e+1-8t); the kept pairs
          t + u <= 7 are summed exactly in integers, the dropped pairs
          (t + u = 8..12, 15 of them) add below 128^2 2^(e+f+2)
          (5 2^-64 + 4 2^-72 + ...) <= 20.3 2^-48 m m' per element product,
          the truncations 8.04 2^-48 m m'; over bs terms and with
          m <= ||A_IK row||, m' <= ||B_KJ column|| this is below
          29 bs 2^-48 ||A_IK||_F ||B_KJ||_F per leaf product, plus a few FP64
          roundings of the per-leaf conversion (the 4) and the FP64
          accumulation.
"""
from __future__ import annotations

import numpy as np

SAFETY = 2.0
U64, U32 = 2.0 ** -53, 2.0 ** -24


def rel_bound(mode: str, nprod, bs: int):
    """r_mode(n) of the module docstring for blocks with ``nprod`` leaf products."""
    n = np.asarray(nprod, dtype=np.float64) * bs
    if mode == "f64":
        return n * U64
    if mode == "f32":
        return (n + 3) * U32
    if mode == "bf16":
        return n * U32 + 2 * 2.0 ** -8 + 2.0 ** -16 + U32
    if mode == "bf16x3":
        return 3 * n * U32 + 4 * 2.0 ** -16 + U32
    if mode == "ozaki":
        return n * U64 + (29 * bs + 4) * 2.0 ** -48
    raise ValueError(mode)


def block_errors(got, ref, bs):
    """||got_IJ - ref_IJ||_F per block (rows of [nblk, bs*bs] arrays), in chunks."""
    got = np.asarray(got).reshape(-1, bs * bs)
    ref = np.asarray(ref).reshape(-1, bs * bs)
    out = np.empty(got.shape[0])
    step = 4096
    for s in range(0, got.shape[0], step):
        out[s:s + step] = np.linalg.norm(got[s:s + step] - ref[s:s + step], axis=1)
    return out


def violations(got, ref, S, nprod, mode, bs):
    """Indices of the blocks whose error exceeds SAFETY * r_mode(n) * S_IJ
    (a block without products, S_IJ = 0, must match exactly).  Blocks whose
    reference is not finite are left to the non-finite checks."""
    err = block_errors(got, ref, bs)
    S = np.asarray(S, dtype=np.float64)
    lim = SAFETY * rel_bound(mode, nprod, bs) * S
    r = np.asarray(ref).reshape(-1, bs * bs)
    fin = np.all(np.isfinite(r), axis=1)
    bad = fin & ~(err <= lim)
    # blocks without products: exactly equal (a norm could underflow to zero)
    z = np.nonzero(S == 0)[0]
    if z.size:
        g = np.asarray(got).reshape(-1, bs * bs)
        bad[z] |= np.any(g[z] != r[z], axis=1)
    return np.nonzero(bad)[0], err, lim


def assert_blockwise(got, ref, S, nprod, mode, bs, what=""):
    bad, err, lim = violations(got, ref, S, nprod, mode, bs)
    if bad.size:
        k = bad[np.argmax(err[bad] / np.maximum(lim[bad], 1e-300))]
        raise AssertionError(
            f"{what} {mode}: {bad.size} of {err.size} blocks exceed the per-block bound; worst block {k}: "
            f"error {err[k]:.3e} > bound {lim[k]:.3e} (S = {float(np.asarray(S)[k]):.3e}, "
            f"{int(np.asarray(nprod)[k])} products)")
