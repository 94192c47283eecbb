"""Benchmark: block-sparse C = A A on the 3-D exponential-decay workload.

Workload: 16384 points uniform in a cube at 0.1 points per cubic Angstrom,
Morton-ordered, A_ij = exp(-0.5 |p_i - p_j|), 64 x 64 leaves, blocks with
Frobenius norm < 1e-10 dropped (about 98% of the 256 x 256 blocks stay), A
and B the same matrix.

One step = the whole device path from FP64 leaf blocks already resident in
HBM: construction (block norms + drop, Morton ranking, quadtree), symbolic
phase (quadtree walk, work list, C pattern) and numeric phase (operand
packing + the leaf-product kernel).  The packing is queued right after the
construction on the library's side stream, so it runs while the host works
through the symbolic phase.  ``value`` is the chosen precision
mode's effective GFLOP/s = block-level flops of the nonzero leaf products
(2 m k n each) / step time; the plain FP64 GPU path is reported beside it,
with each mode's relative Frobenius error on a sampled set of C blocks
against the FP64 CPU oracle (the cpu_baseline leg).

Usage: python bench.py [--steps K] [--warmup W] [--mode bf16x3] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective GFLOP/s on nonzero leaf products, plain FP64 vs chosen form at stated error"
# dense MFMA peaks of the instruction type each mode runs (TFLOP/s; int8 in TOP/s)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0, "ozaki": 5000.0}
MFMA_TERMS = {"f64": 1, "f32": 1, "bf16": 1, "bf16x3": 3, "ozaki": 21}
DTYPE = {"f64": "f64", "f32": "f32", "bf16": "bf16", "bf16x3": "bf16", "ozaki": "i8"}
# bytes per element of the packed operands and of the result, per mode (the
# Ozaki packs: seven 1-byte digits plus a 4-byte exponent per 64-element line)
OPERAND_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "bf16x3": 4, "ozaki": 6 + 4 / 64}
RESULT_BYTES = {"f64": 8, "f32": 4, "bf16": 4, "bf16x3": 4, "ozaki": 8}
KERNEL_SOURCES = ("numeric.hip", "numeric_oz.hip", "common.h", "device_math.h")
# HBM bytes of one numeric-kernel launch on the default workload, per
# "mode@unit", from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE in KiB
# per dispatch), scaled by what the same counters read for a 1 GiB
# device-to-device copy in the same runs (FETCH_SIZE x2.0, WRITE_SIZE x1.0);
# at unit 256 the two kernels of one launch (branch-free and tile-skipping
# paths) are summed.
# They describe only the kernel sources with this digest; for any other
# source, mode, unit or workload the traffic is reported as null.
TRAFFIC = {
    "sources_sha256_16": "fef3b78a2915da3e",
    "npoints": 16384,
    "bytes": {
        "bf16x3@128": 121468077205,
        "bf16x3@256": 49774483538,
        "bf16x3@64": 327485731776,
        "f32@128": 203662038683,
        "f32@256": 67679619840,
        "f32@64": 338423548032,
        "f64@128": 430586429760,
        "f64@64": 710156404224,
        "ozaki@128": 117787017198,
        "ozaki@64": 555307313621,
    },
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="bf16x3", choices=["f64", "f32", "bf16", "bf16x3", "ozaki"])
    ap.add_argument("--unit", type=int, default=0,
                    help="work-unit side; 0 = chosen per mode by the library's autotuner before timing")
    ap.add_argument("--npoints", type=int, default=16384)
    ap.add_argument("--workload", default="decay", choices=["decay", "banded", "growing", "random", "batched", "backward", "sparse"],
                    help="decay: the 3-D decay matrix (headline); banded/growing/random: the paper's "
                         "weak-scaling sequences (Sec. 3, Table 1) at size --n; batched: 256 FP32 "
                         "multiplies of uneven sizes in one persistent launch replayed as a HIP graph; "
                         "backward: forward and masked backward on banded N 16384 with FP32 entries; "
                         "sparse: random 128x128 blocks at density 0.01, N 65536 (bound by HBM)")
    ap.add_argument("--n", type=int, default=100000, help="matrix size of the paper's sequences")
    ap.add_argument("--sym-square", action="store_true",
                    help="also time the symmetric square (upper-triangle blocks only) of the chosen mode")
    ap.add_argument("--spamm-tol", type=float, default=0.0,
                    help="also time the sparse approximate multiply of the chosen mode with this tolerance "
                         "(reported beside the headline, which is always the full multiply)")
    ap.add_argument("--modes", default="f64,f32,ozaki", help="reference modes timed beside the chosen one")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (no error statement)")
    ap.add_argument("--no-legs", action="store_true",
                    help="decay workload only: leave out the compact legs of the other workloads (N 2048 "
                         "banded FP64, random blocks, batched, forward + backward)")
    ap.add_argument("--leg-steps", type=int, default=3,
                    help="timed steps of the batched leg (the millisecond-scale legs time 20 times as many)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be >= 1 and --warmup >= 0")
    return args


def kernel_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2011_11762_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(mode, unit, npoints, workload="decay"):
    t = TRAFFIC
    if workload != "decay" or (t["sources_sha256_16"], t["npoints"]) != (kernel_digest(), npoints):
        return None
    return t["bytes"].get(f"{mode}@{unit}")


def cpu_baseline_leg(wl, tol, bs, seconds):
    """Times the FP64 oracle on a bounded random sample of C blocks.

    Returns the baseline record and the oracle's values of the sampled
    blocks (the reference for the error statement of every mode).
    """
    from oracle import oracle as O

    oa = O.from_workload(wl["A"], tol)
    nb = -(-wl["A"].nrows // bs)
    rng = np.random.default_rng(99)
    rowsets, colsets = {}, {}

    def common(i, j):
        # products of C block (i, j): common K of row i of A and column j of A
        if i not in rowsets:
            rowsets[i] = set(oa.bcol[oa.brow == i].tolist())
        if j not in colsets:
            colsets[j] = set(oa.brow[oa.bcol == j].tolist())
        return len(rowsets[i] & colsets[j])

    def draw(count):
        # C blocks that have at least one product, uniformly among those
        si, sj = [], []
        for _ in range(200):
            ci, cj = rng.integers(0, nb, 4 * count), rng.integers(0, nb, 4 * count)
            for i, j in zip(ci.tolist(), cj.tolist()):
                if common(i, j):
                    si.append(i)
                    sj.append(j)
            if len(si) >= count:
                break
        key = np.unique(np.asarray(si[:count], dtype=np.int64) * nb + np.asarray(sj[:count], dtype=np.int64))
        return key // nb, key % nb

    # calibration on a few blocks, then a sample sized to the time budget
    cal_i, cal_j = draw(16)
    t0 = time.perf_counter()
    O.multiply_blocks(oa, oa, cal_i, cal_j)
    dt = max(time.perf_counter() - t0, 1e-3)
    nsample = int(min(nb * nb, max(64, 16 * seconds / dt)))
    si, sj = draw(nsample)
    ncommon = sum(common(i, j) for i, j in zip(si.tolist(), sj.tolist()))
    flops = 2.0 * bs ** 3 * ncommon
    t0 = time.perf_counter()
    ref = O.multiply_blocks(oa, oa, si, sj)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rec = {"value": round(flops / el / 1e9, 3), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"{si.size} random C blocks of the workload ({ncommon} leaf products, "
                     f"{flops / 1e9:.1f} GFLOP) in {el:.1f} s, FP64 oracle, OpenMP over C blocks"}
    return rec, (si, sj, ref)


# --------------------------------------------------------------------------
# Compact legs for the other workloads, added to the default run's JSON line.
# Each leg times one pass of its hot path, reports the dominant kernel's
# roofline (HIP events around every launch of it during the timed steps) and
# times the FP64 oracle on the same inputs on the host (all threads and one
# thread where the oracle finishes in seconds).

def _oracle_timed(fn, flops, sample, one_thread=True):
    """Runs fn (an oracle computation) on all threads, then on one; returns
    the cpu_baseline record and fn's result."""
    from oracle import oracle as O

    nthr = O.set_threads(0)  # query (n < 1 leaves the count as it is)
    t0 = time.perf_counter()
    res = fn()
    el = time.perf_counter() - t0
    rec = {"value": round(flops / el / 1e9, 3), "unit": "GFLOP/s", "cores": nthr, "kind": "oracle",
           "sample": f"{sample}; {flops / 1e9:.2f} GFLOP in {el:.2f} s on {nthr} threads"}
    if one_thread:
        O.set_threads(1)
        t0 = time.perf_counter()
        fn()
        el1 = time.perf_counter() - t0
        O.set_threads(nthr)
        rec["value_1_thread"] = round(flops / el1 / 1e9, 3)
        rec["seconds_1_thread"] = round(el1, 3)
    return rec, res


def _timed_steps(torch, qbsm, fn, steps, warmup):
    """Average wall time of fn over `steps` calls (after `warmup`), and the
    average numeric-kernel launch time recorded meanwhile."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    qbsm.profile_reset()
    qbsm.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    qbsm.profile_enable(False)
    n, tot = qbsm.profile_read(qbsm.PROF_NUMERIC)
    qbsm.profile_reset()
    return ms, tot / max(n, 1), n


def _upload_raw(torch, m):
    return (torch.from_numpy(m.brow.astype(np.int32)).cuda(), torch.from_numpy(m.bcol.astype(np.int32)).cuda(),
            torch.from_numpy(m.vals).cuda())


def _mfma_roofline(mode, flops, kern_ms, kernel):
    ach = MFMA_TERMS[mode] * flops / (kern_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_TFLOPS[mode],
            "unit": "TOP/s" if mode == "ozaki" else "TFLOP/s", "frac": round(ach / PEAK_TFLOPS[mode], 4),
            "traffic": None, "kernel": kernel}


def leg_config1(torch, qbsm, W, steps, warmup):
    """Banded N 2048, 32x32 leaves, half-bandwidth 4, FP64: one whole pass
    (set_blocks of A and B, symbolic, numeric with packing; the unit side from
    the library's autotuner); a latency-bound workload."""
    from oracle import oracle as O

    c = W.config1()
    a, b = c["A"], c["B"]
    ra, rb = _upload_raw(torch, a), _upload_raw(torch, b)
    A, B = qbsm.Matrix(a.nrows, a.ncols, a.bs), qbsm.Matrix(b.nrows, b.ncols, b.bs)
    C = qbsm.Matrix(a.nrows, b.ncols, a.bs)
    st = {}
    A.set_blocks(*ra)
    B.set_blocks(*rb)
    unit, tune = qbsm.autotune_unit(A, B, "f64", reps=3)

    def step():
        A.set_blocks(*ra)
        B.set_blocks(*rb)
        # (no packing ahead on the side stream: at this size its events cost
        # more than the overlap gains)
        st["P"] = qbsm.Plan(A, B, unit=unit)
        st["P"].numeric("f64", C)

    ms, kern, _ = _timed_steps(torch, qbsm, step, steps, warmup)
    info = st["P"].info()
    oa, ob = O.from_workload(a), O.from_workload(b)
    cpu, ref = _oracle_timed(lambda: O.multiply(oa, ob), info["flops"], "the whole product, FP64 oracle")
    err = O.rel_fro(C.values().cpu().numpy(), ref.vals)
    return {"workload": f"{c['name']} ({info['nblk_out']} C blocks, {info['nprod']} leaf products)",
            "mode": "f64", "unit": info["unit"], "ms_per_step": round(ms, 4), "kernel_ms": round(kern, 4),
            "value": round(info["flops"] / (ms * 1e-3) / 1e9, 3), "unit_value": "GFLOP/s",
            "autotune_ms": {str(k): round(v, 4) for k, v in tune.items() if v > 0},
            "step": "set_blocks(A, B) + symbolic + numeric", "rel_err_vs_fp64_oracle": float(f"{err:.3e}"),
            "roofline": _mfma_roofline("f64", info["flops"], kern, "numeric leaf-product kernel (f64): "
                                       "latency-bound at this size"),
            "cpu_baseline": cpu}


def leg_config3(torch, qbsm, W, steps, warmup, modes=("bf16x3", "bf16")):
    """Random 128x128 blocks at density 0.01, N 65536: BF16 and BF16X3 (the
    last mode listed is the leg's chosen one); bound by HBM."""
    from oracle import oracle as O

    c = W.config3()
    a, b = c["A"], c["B"]
    bs = a.bs
    ra, rb = _upload_raw(torch, a), _upload_raw(torch, b)
    A, B = qbsm.Matrix(a.nrows, a.ncols, bs), qbsm.Matrix(b.nrows, b.ncols, bs)
    C = qbsm.Matrix(a.nrows, b.ncols, bs)
    A.set_blocks(*ra)
    B.set_blocks(*rb)
    res, st = {}, {}
    for mode in modes:
        unit = qbsm.autotune_unit(A, B, mode, reps=2)[0]

        def step():
            A.set_blocks(*ra)
            B.set_blocks(*rb)
            A.prepack(mode, 1)
            B.prepack(mode, 2)
            st["P"] = qbsm.Plan(A, B, unit=unit)
            st["P"].numeric(mode, C)

        ms, kern, _ = _timed_steps(torch, qbsm, step, steps, warmup)

        def multiply():
            st["P"] = qbsm.Plan(A, B, unit=unit)
            st["P"].numeric(mode, C)

        # symbolic + numeric with the operands stored and packed (the HBM-bound multiply alone)
        mms, _, _ = _timed_steps(torch, qbsm, multiply, max(steps, 10), warmup)
        info = st["P"].info()
        alg = (A.nblk + B.nblk) * bs * bs * OPERAND_BYTES[mode] + info["nblk_out"] * bs * bs * RESULT_BYTES[mode]
        res[mode] = {"ms_per_step": round(ms, 4), "symbolic_numeric_ms": round(mms, 4), "kernel_ms": round(kern, 4),
                     "unit": unit,
                     "value": round(info["flops"] / (ms * 1e-3) / 1e9, 3), "algorithmic_bytes": int(alg),
                     "kernel_gbps": round(alg / (kern * 1e-3) / 1e9, 1), "_vals": C.values().cpu().numpy()}
    oa, ob = O.from_workload(a), O.from_workload(b)
    cpu, ref = _oracle_timed(lambda: O.multiply(oa, ob), info["flops"], "the whole product, FP64 oracle")
    for mode in modes:
        res[mode]["rel_err_vs_fp64_oracle"] = float(f"{O.rel_fro(res[mode].pop('_vals'), ref.vals):.3e}")
    ch = res[modes[-1]]
    return {"workload": f"{c['name']} ({A.nblk} + {B.nblk} blocks, {info['nblk_out']} C blocks, "
                        f"{info['nprod']} leaf products)",
            "mode": modes[-1], "modes": res, "ms_per_step": ch["ms_per_step"], "value": ch["value"],
            "symbolic_numeric_ms": ch["symbolic_numeric_ms"],
            "unit_value": "GFLOP/s", "step": "set_blocks(A, B) + packing + symbolic + numeric "
                                             "(symbolic_numeric_ms: the multiply with A and B stored and packed)",
            "roofline": {"bound": "hbm", "achieved": ch["kernel_gbps"], "peak": 8000.0, "unit": "GB/s",
                         "frac": round(ch["kernel_gbps"] / 8000.0, 4), "traffic": None,
                         "algorithmic_bytes": ch["algorithmic_bytes"],
                         "kernel": f"numeric leaf-product kernel, mode {modes[-1]}, unit {ch['unit']}"},
            "cpu_baseline": cpu}


def leg_config5(torch, qbsm, W, steps, warmup, mode="f32"):
    """Banded N 16384, 64x64 leaves, h 6, FP32 entries: forward C = A B and
    the masked backward (dA on A's pattern, dB on B's) from stored operands,
    as a training step runs them: the forward's plan (symbolic phase) is kept
    and the backward regroups its product list (no second walk)."""
    from oracle import oracle as O

    c = W.config5()
    A, B, dC = qbsm.from_host(c["A"]), qbsm.from_host(c["B"]), qbsm.from_host(c["dC"])
    st = {}

    def fwd():
        st["P"] = qbsm.Plan(A, B)
        st["C"] = st["P"].numeric(mode)

    def bwd():
        st["g"] = st["P"].backward(dC, mode)

    info = qbsm.Plan(A, B).info()
    fms, fkern, _ = _timed_steps(torch, qbsm, fwd, steps, warmup)
    bms, bkern, nb = _timed_steps(torch, qbsm, bwd, steps, warmup)
    fl_f, fl_b = info["flops"], 2 * info["flops"]
    oa, ob, odc = O.from_workload(c["A"]), O.from_workload(c["B"]), O.from_workload(c["dC"])

    def oracle_pass():
        return O.multiply(oa, ob), O.backward(oa, ob, odc)

    cpu, (ref, (ga, gb)) = _oracle_timed(oracle_pass, fl_f + fl_b, "forward + masked backward, FP64 oracle")
    dA, dB = st["g"]
    err = {"forward": float(f"{O.rel_fro(st['C'].values().cpu().numpy(), ref.vals):.3e}"),
           "dA": float(f"{O.rel_fro(dA.values().cpu().numpy(), ga):.3e}"),
           "dB": float(f"{O.rel_fro(dB.values().cpu().numpy(), gb):.3e}")}
    ms = fms + bms
    return {"workload": f"{c['name']} ({info['nprod']} leaf products; each reused for dA and for dB)",
            "mode": mode, "ms_per_step": round(ms, 4), "forward_ms": round(fms, 4), "backward_ms": round(bms, 4),
            "value": round((fl_f + fl_b) / (ms * 1e-3) / 1e9, 3), "unit_value": "GFLOP/s",
            "backward_gflops": round(fl_b / (bms * 1e-3) / 1e9, 3),
            "step": "forward (symbolic + numeric) + backward (dA and dB), operands stored",
            "rel_err_vs_fp64_oracle": err,
            "roofline": _mfma_roofline(mode, fl_b / 2, bkern, f"numeric leaf-product kernel of the backward "
                                       f"({mode}; one of its two launches)"),
            "cpu_baseline": cpu}


def batched_member_builder(torch, qbsm, W, spec):
    """Callable leaf size -> the member's (A, B) handles, stored in FP32.
    Banded members are defined at their own leaf size (their half-bandwidth
    counts blocks); decay members are given by their points, so any leaf
    size stores the same matrix (before the block drop)."""

    def build(bs):
        if spec["kind"] == "banded":
            assert bs == spec["bs"], "a banded member keeps its leaf size"
            mem = W.config4_member(spec)
            A, B = qbsm.from_host(mem["A"]), qbsm.from_host(mem["B"])
            A.store_f32()
            B.store_f32()
            return A, B
        # decay values generated on the device (FP64), then stored in FP32
        pts = W.decay_points(spec["n"], 0.1, np.random.default_rng([4, spec["m"]]))
        r, c, v = W.decay_blocks_device(pts, bs)
        A = qbsm.Matrix(spec["n"], spec["n"], bs)
        A.set_blocks(r, c, v, spec["drop_tol"])
        del r, c, v
        A.store_f32()
        return A, A

    return build


def build_batched(torch, qbsm, W, unit=128, leaf="given"):
    """The batched workload: 256 multiplies of uneven sizes (N 1024..16384,
    leaves 32 or 64, banded members with independent A and B, decay members
    squared), stored in FP32, with one plan per member at `unit`; decay
    members stored at `leaf` (32 or 64) unless it is "given"."""
    specs = W.config4_members()
    plans, handles = [], []
    for spec in specs:
        bs = spec["bs"] if (leaf == "given" or spec["kind"] == "banded") else int(leaf)
        A, B = batched_member_builder(torch, qbsm, W, spec)(bs)
        plans.append(qbsm.Plan(A, B, unit=unit))
        handles.append((A, B))
    torch.cuda.empty_cache()
    return specs, plans, handles


def tuned_batch_settings(torch, qbsm, W, log=None):
    """The autotuner's (leaf option, unit, occupancy) for the batched
    workload, from the cache when the batch's key is there.  The key needs the
    plan infos of the batch as given; returns them with the built batch so
    that a "given" choice reuses it."""
    from paper_2011_11762_amd import autotune

    specs, plans, handles = build_batched(torch, qbsm, W, 128, "given")
    infos = [p.info() for p in plans]
    members = [{"bs": s["bs"], "flexible": s["kind"] == "decay", "build": batched_member_builder(torch, qbsm, W, s)}
               for s in specs]
    t0 = time.perf_counter()
    choice, key, cached = autotune.tune_batch(qbsm, "f32", members, infos=infos, log=log)
    return choice, key, cached, time.perf_counter() - t0, (specs, plans, handles)


def leg_config4(torch, qbsm, W, steps, warmup, unit=0, oracle_members=(0, 2, 4, 6, 1, 3)):
    """The batched form: one persistent launch over all 256 members' work
    units, captured once as a HIP graph and replayed; a step is one replay
    (operand re-packing + the persistent kernel).  unit 0: the unit side,
    the occupancy and the decay members' leaf size come from the autotuner
    (its cache, or a tuning run on a sample of the members).  The oracle
    checks and is timed on a bounded sample: whole banded members and sampled
    output blocks of decay members (their FP32-stored values read back)."""
    from oracle import oracle as O

    t_gen = time.perf_counter()
    tuning = None
    if unit:
        specs, plans, handles = build_batched(torch, qbsm, W, unit)
        occ = 0
    else:
        log = lambda msg: print(f"[bench] {msg}", file=sys.stderr, flush=True)  # noqa: E731
        choice, key, cached, tune_s, built = tuned_batch_settings(torch, qbsm, W, log=log)
        unit, occ = choice["unit"], choice["wg_per_cu"]
        tuning = {"key": key, "cached": cached, "tuning_s": round(tune_s, 2), "leaf": choice["leaf"],
                  "unit": unit, "wg_per_cu": occ, "sample_ms": choice.get("ms"), "sample": choice.get("sample")}
        log(f"batched settings ({'cached' if cached else 'tuned'}): leaf {choice['leaf']}, unit {unit}, "
            f"{occ} WG/CU")
        if choice["leaf"] == "given" and unit == 128:
            specs, plans, handles = built
        else:
            del built
            torch.cuda.empty_cache()
            specs, plans, handles = build_batched(torch, qbsm, W, unit, choice["leaf"])
    infos = [p.info() for p in plans]
    flops = sum(i["flops"] for i in infos)
    batch = qbsm.Batch(plans, "f32")
    if occ:
        batch.set_occupancy(occ)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t_gen
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ms, _, _ = _timed_steps(torch, qbsm, batch.run_graph, steps, max(warmup, 1))
        # GPU time of one replay (the graph holds the packing and the
        # persistent kernel; the library's own kernel events are not captured)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            batch.run_graph()
        e1.record(stream)
        e1.synchronize()
        kern = e0.elapsed_time(e1) / steps
    # oracle sample
    refs, gots, oflops, nblocks = [], [], 0, 0
    work = []
    for m in oracle_members:
        A, B = handles[m]
        oa = O.canonical(A.nrows, A.ncols, A.bs, *[t.cpu().numpy() for t in A.pattern()], A.values().cpu().numpy())
        ob = oa if B is A else O.canonical(B.nrows, B.ncols, B.bs, *[t.cpu().numpy() for t in B.pattern()],
                                          B.values().cpu().numpy())
        out = batch.outs[m]
        cr, cc = (t.cpu().numpy() for t in out.pattern())
        if specs[m]["kind"] == "banded":
            work.append((oa, ob, None, None, out.values().cpu().numpy()))
            oflops += infos[m]["flops"]
            nblocks += cr.size
        else:
            rng = np.random.default_rng(40 + m)
            pick = np.sort(rng.choice(cr.size, size=min(48, cr.size), replace=False))
            si, sj = cr[pick].astype(np.int64), cc[pick].astype(np.int64)
            work.append((oa, ob, si, sj, out.extract(si, sj).cpu().numpy()))
            I, J, K, _, _ = O.product_triples(oa, ob)
            sel = np.isin(I * (1 << 20) + J, si * (1 << 20) + sj)
            oflops += O.block_flops(I[sel], J[sel], K[sel], oa.nrows, oa.ncols, ob.ncols, oa.bs)
            nblocks += si.size

    def oracle_pass():
        return [O.multiply(oa, ob).vals if si is None else O.multiply_blocks(oa, ob, si, sj)
                for oa, ob, si, sj, _ in work]

    cpu, err = None, None
    if work:
        cpu, outs = _oracle_timed(oracle_pass, oflops, f"members {list(oracle_members)}: whole banded members "
                                  f"and 48 sampled C blocks of each decay member ({nblocks} C blocks)",
                                  one_thread=False)
        num = sum(float(np.sum((w[4] - r) ** 2)) for w, r in zip(work, outs))
        den = sum(float(np.sum(r ** 2)) for r in outs)
        err = float(f"{(num / den) ** 0.5:.3e}")
    tflops = flops / (ms * 1e-3) / 1e12
    return {"workload": f"batched-{len(plans)}-members-n1024..16384-bs32/64-banded+decay "
                        f"({sum(i['nblk_out'] for i in infos)} C blocks, {sum(i['nprod'] for i in infos)} "
                        "leaf products)",
            "mode": "f32", "unit": unit, "ms_per_step": round(ms, 4), "kernel_ms": round(kern, 4),
            "value": round(tflops * 1e3, 3), "unit_value": "GFLOP/s", "flops_per_step": flops,
            "build_s": round(build_s, 2), "autotune": tuning,
            "step": "one HIP-graph replay: operand re-packing + one persistent MFMA kernel over every member",
            "rel_err_vs_fp64_oracle": err,
            "roofline": _mfma_roofline("f32", flops, kern, f"one graph replay: packing + persistent numeric kernel "
                                       f"(f32, unit {unit}), HIP events on the replay stream"),
            "cpu_baseline": cpu}


def batched_main(args, torch, qbsm, W):
    """The batched form as its own JSON line (see leg_config4)."""
    leg = leg_config4(torch, qbsm, W, args.steps, args.warmup, unit=args.unit,
                      oracle_members=() if args.no_cpu else (0, 2, 4, 6, 1, 3))
    print(f"[bench] batched f32: {leg['ms_per_step']:.3f} ms/step, {leg['value']} GFLOP/s", file=sys.stderr,
          flush=True)
    out = {
        "metric": METRIC,
        "value": leg["value"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": leg["workload"], "mode": "f32", "unit": leg["unit"],
                   "flops_per_step": leg["flops_per_step"], "step": leg["step"], "autotune": leg["autotune"]},
        "roofline": leg["roofline"],
        "cpu_baseline": leg["cpu_baseline"] if not args.no_cpu else None,
        "rel_err_vs_fp64_oracle": leg["rel_err_vs_fp64_oracle"] if not args.no_cpu else None,
    }
    print(json.dumps(out), flush=True)


def backward_main(args, torch, qbsm, W):
    """Forward C = A*B and the masked backward (dA on A's pattern, dB on B's)
    on the banded workload with FP32 entries (N 16384, 64x64 leaves, block
    half-bandwidth 6, dC on C's pattern).  A step is one backward from the
    forward's plan: the forward product list regrouped by A node and by B
    node (no symbolic walk) and both numeric phases, with the inputs in HBM;
    the forward (symbolic + numeric) is timed beside it, and so is the
    stand-alone backward call that first builds the forward plan.  The
    backward reuses every forward leaf product once for dA and once for dB."""
    c = W.config5()
    A, B, dC = qbsm.from_host(c["A"]), qbsm.from_host(c["B"]), qbsm.from_host(c["dC"])
    info = qbsm.Plan(A, B).info()
    fwd_flops, bwd_flops = info["flops"], 2 * info["flops"]

    def timed(fn):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps * 1e3

    modes = [m for m in args.modes.split(",") if m and m != args.mode] + [args.mode]
    results = {}
    st = {}
    for mode in modes:
        def forward():
            st["P"] = qbsm.Plan(A, B)
            st["C"] = st["P"].numeric(mode)

        fwd = timed(forward)
        bwd = timed(lambda: st["P"].backward(dC, mode))
        alone = timed(lambda: qbsm.backward(A, B, dC, mode))
        results[mode] = {"forward_ms": round(fwd, 4), "forward_gflops": round(fwd_flops / (fwd * 1e-3) / 1e9, 2),
                         "backward_ms": round(bwd, 4), "backward_gflops": round(bwd_flops / (bwd * 1e-3) / 1e9, 2),
                         "backward_standalone_ms": round(alone, 4)}
        print(f"[bench] {mode}: forward {fwd:.3f} ms, backward from the forward plan {bwd:.3f} ms "
              f"({results[mode]['backward_gflops']} GFLOP/s), stand-alone backward {alone:.3f} ms",
              file=sys.stderr, flush=True)
    ch = results[args.mode]
    achieved = MFMA_TERMS[args.mode] * bwd_flops / (ch["backward_ms"] * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        oa, ob, odc = O.from_workload(c["A"]), O.from_workload(c["B"]), O.from_workload(c["dC"])
        cpu, _ = _oracle_timed(lambda: O.backward(oa, ob, odc), bwd_flops,
                               "the whole masked backward (dA and dB), FP64 oracle")
    out = {
        "metric": METRIC,
        "value": ch["backward_gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": ch["backward_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.mode],
        "data": "synthetic",
        "config": {
            "workload": f"banded-n16384-bs64-h6-fp32-entries masked backward ({info['nprod']} forward leaf "
                        f"products, each used for dA and for dB)",
            "mode": args.mode,
            "flops_per_step": bwd_flops,
            "step": "one backward from the forward's plan: product list regrouped for dA and dB + both "
                    "numeric phases",
        },
        "roofline": {
            "bound": "mfma",
            "achieved": round(achieved, 2),
            "peak": PEAK_TFLOPS[args.mode],
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_TFLOPS[args.mode], 4),
            "traffic": None,
            "kernel": "whole backward (regrouping included): a small, launch-bound workload",
        },
        "modes": results,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def sparse_main(args, torch, qbsm, W):
    """C = A*B for independent random-block matrices (N 65536, 128x128 leaves,
    each block present with probability 0.01): almost every C block has one
    leaf product, so the numeric kernel is bound by HBM (C written once, the
    operands read once).  A step is the symbolic and numeric phases with the
    operands stored and packed; the roofline is over HBM bytes."""
    c = W.config3()
    A, B = qbsm.from_host(c["A"]), qbsm.from_host(c["B"])
    bs = c["A"].bs
    C = qbsm.Matrix(A.nrows, B.ncols, bs)
    # (the Ozaki mode's int8 MFMA needs 64-wide leaves: not timed on these 128-wide ones)
    modes = [m for m in args.modes.split(",") if m and m != args.mode and not (m == "ozaki" and bs != 64)]
    modes.append(args.mode)
    results, info = {}, None
    for mode in modes:
        unit = args.unit or qbsm.autotune_unit(A, B, mode, reps=2)[0]
        for _ in range(max(args.warmup, 1)):
            qbsm.Plan(A, B, unit=unit).numeric(mode, C)
        torch.cuda.synchronize()
        qbsm.profile_reset()
        qbsm.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            P = qbsm.Plan(A, B, unit=unit)
            P.numeric(mode, C)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        qbsm.profile_enable(False)
        n, tot = qbsm.profile_read(qbsm.PROF_NUMERIC)
        qbsm.profile_reset()
        kern = tot / max(n, 1)
        info = P.info()
        alg = (A.nblk + B.nblk) * bs * bs * OPERAND_BYTES[mode] + info["nblk_out"] * bs * bs * RESULT_BYTES[mode]
        results[mode] = {"ms_per_step": round(ms, 4), "kernel_ms": round(kern, 4), "unit": unit,
                         "effective_gflops": round(info["flops"] / (ms * 1e-3) / 1e9, 2),
                         "algorithmic_bytes": alg, "kernel_gbps": round(alg / (kern * 1e-3) / 1e9, 1)}
        print(f"[bench] {mode}: {ms:.3f} ms/step, kernel {kern:.3f} ms, {results[mode]['kernel_gbps']} GB/s "
              f"(unit {unit})", file=sys.stderr, flush=True)
    ch = results[args.mode]
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        oa, ob = O.from_workload(c["A"]), O.from_workload(c["B"])
        cpu, _ = _oracle_timed(lambda: O.multiply(oa, ob), info["flops"], "the whole product, FP64 oracle")
    out = {
        "metric": METRIC,
        "value": ch["effective_gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": ch["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.mode],
        "data": "synthetic",
        "config": {
            "workload": f"random-blocks-n65536-bs128-p0.01 ({A.nblk} + {B.nblk} blocks, {info['nblk_out']} C "
                        f"blocks, {info['nprod']} leaf products)",
            "mode": args.mode,
            "unit": ch["unit"],
            "flops_per_step": info["flops"],
            "step": "symbolic (quadtree walk, work list) + numeric (MFMA kernel), operands stored and packed",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": ch["kernel_gbps"],
            "peak": 8000.0,
            "unit": "GB/s",
            "frac": round(ch["kernel_gbps"] / 8000.0, 4),
            "traffic": None,
            "algorithmic_bytes": ch["algorithmic_bytes"],
            "kernel": f"numeric leaf-product kernel, mode {args.mode}, unit {ch['unit']}",
        },
        "modes": results,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not built "
                                   "(the library has no cross-GPU path)", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2011_11762_amd import qbsm
    from paper_2011_11762_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    qbsm.load()
    if args.workload == "batched":
        batched_main(args, torch, qbsm, W)
        return
    if args.workload == "backward":
        backward_main(args, torch, qbsm, W)
        return
    if args.workload == "sparse":
        sparse_main(args, torch, qbsm, W)
        return
    bs = 64
    t_gen = time.perf_counter()
    if args.workload == "decay":
        tol = 1e-10
        wl = W.config2(npoints=args.npoints, bs=bs)
    else:
        tol = 0.0
        wl = {"A": W.paper_workload(args.workload, args.n, bs)}
    a = wl["A"]
    brow = torch.from_numpy(a.brow.astype(np.int32)).cuda()
    bcol = torch.from_numpy(a.bcol.astype(np.int32)).cuda()
    vals = torch.from_numpy(a.vals).cuda()
    torch.cuda.synchronize()
    print(f"[bench] workload generated and resident in HBM in {time.perf_counter() - t_gen:.1f} s",
          file=sys.stderr, flush=True)

    # device-to-device copy bandwidth (read + write bytes / time) for scale;
    # left out of counter runs, whose only large copy is the calibration copy
    copy_gbps = None
    if not args.calibrate_copy:
        src = torch.empty(1 << 31, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t_copy = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        copy_gbps = round(2 * (1 << 31) * 5 / (time.perf_counter() - t_copy) / 1e9, 1)
        del src, dst
        torch.cuda.empty_cache()

    if args.calibrate_copy:
        src = torch.empty(args.calibrate_copy << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    A = qbsm.Matrix(a.nrows, a.ncols, bs)
    C = qbsm.Matrix(a.nrows, a.ncols, bs)
    state = {}

    units, tuning = {}, {}

    def step(mode, spamm=0.0, upper=False):
        A.set_blocks(brow, bcol, vals, tol)
        A.prepack(mode, 3)  # operand packing overlaps the symbolic phase (side stream)
        P = qbsm.Plan(A, A, unit=units[mode] if spamm <= 0 else spamm_unit[mode], spamm_tol=spamm, upper=upper)
        P.numeric(mode, C)
        state["plan"] = P

    def time_mode(mode, steps, warmup, profile, spamm=0.0, upper=False):
        for _ in range(warmup):
            step(mode, spamm, upper)
        torch.cuda.synchronize()
        if profile:
            qbsm.profile_reset()
            qbsm.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step(mode, spamm, upper)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kern = None
        if profile:
            qbsm.profile_enable(False)
            n, tot = qbsm.profile_read(qbsm.PROF_NUMERIC)
            kern = tot / max(n, 1)
            qbsm.profile_reset()
        info = state["plan"].info()
        # numeric phase alone on the last plan (operands already packed)
        P = state["plan"]
        P.numeric(mode, C)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            P.numeric(mode, C)
        torch.cuda.synchronize()
        num_ms = (time.perf_counter() - t1) / steps * 1e3
        # spread of single steps (each bracketed by a synchronisation), after the timed run
        single = []
        for _ in range(steps):
            t2 = time.perf_counter()
            step(mode, spamm, upper)
            torch.cuda.synchronize()
            single.append((time.perf_counter() - t2) * 1e3)
        state["spread"] = {"median": round(float(np.median(single)), 4), "min": round(min(single), 4),
                           "max": round(max(single), 4)}
        return el / steps * 1e3, kern, num_ms, info

    modes = [m for m in args.modes.split(",") if m and m != args.mode] + [args.mode]
    A.set_blocks(brow, bcol, vals, tol)
    for mode in modes:
        if args.unit:
            units[mode] = args.unit
        else:
            best, times = qbsm.autotune_unit(A, A, mode, reps=2)
            units[mode] = best
            tuning[mode] = {str(u): round(t, 3) for u, t in times.items() if t > 0}
            print(f"[bench] {mode}: unit {best} (autotune ms per numeric phase: {tuning[mode]})",
                  file=sys.stderr, flush=True)
    results = {}
    for mode in modes:
        ms, kern, num_ms, info = time_mode(mode, args.steps, args.warmup, profile=True)
        flops = info["flops"]
        results[mode] = {
            "ms_per_step": round(ms, 4),
            "effective_gflops": round(flops / (ms * 1e-3) / 1e9, 2),
            "numeric_ms": round(num_ms, 4),
            "numeric_gflops": round(flops / (num_ms * 1e-3) / 1e9, 2),
            "kernel_ms": round(kern, 4),
            "kernel_mfma_tflops": round(MFMA_TERMS[mode] * flops / (kern * 1e-3) / 1e12, 2),
            "unit": units[mode],
            "single_step_ms": state["spread"],
        }
        if mode in tuning:
            results[mode]["autotune_ms"] = tuning[mode]
        print(f"[bench] {mode}: {ms:.3f} ms/step, {results[mode]['effective_gflops']} GFLOP/s "
              f"(kernel {kern:.3f} ms)", file=sys.stderr, flush=True)
        results[mode]["_vals"] = None
    info = state["plan"].info()
    spamm = None
    spamm_unit = {}
    if args.spamm_tol > 0:
        # the unit side for the approximate multiply: numeric phase timed per candidate
        A.set_blocks(brow, bcol, vals, tol)
        cand = {}
        for u in (64, 128, 256):
            if u % bs or u // bs > 4 or (u == 256 and args.mode == "f64") or (args.mode == "ozaki" and u == 256):
                continue
            P = qbsm.Plan(A, A, unit=u, spamm_tol=args.spamm_tol)
            P.numeric(args.mode, C)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                P.numeric(args.mode, C)
            torch.cuda.synchronize()
            cand[u] = (time.perf_counter() - t0) / 2 * 1e3
            del P
        spamm_unit[args.mode] = min(cand, key=cand.get)
        ms, kern, num_ms, sinfo = time_mode(args.mode, args.steps, args.warmup, profile=True, spamm=args.spamm_tol)
        spamm = {"tol": args.spamm_tol, "mode": args.mode, "ms_per_step": round(ms, 4),
                 "kernel_ms": round(kern, 4), "nprod_kept": sinfo["nprod"], "nprod_full": info["nprod"],
                 "flops_kept": sinfo["flops"], "kept_gflops": round(sinfo["flops"] / (ms * 1e-3) / 1e9, 2),
                 "speedup_vs_full": round(results[args.mode]["ms_per_step"] / ms, 3),
                 "unit": spamm_unit[args.mode], "unit_ms": {str(u): round(t, 3) for u, t in cand.items()}}
        print(f"[bench] spamm tol {args.spamm_tol:g} ({args.mode}): {ms:.3f} ms/step, "
              f"{sinfo['nprod']}/{info['nprod']} products kept", file=sys.stderr, flush=True)

    sym = None
    if args.sym_square:
        ms, kern, num_ms, yinfo = time_mode(args.mode, args.steps, args.warmup, profile=True, upper=True)
        sym = {"mode": args.mode, "ms_per_step": round(ms, 4), "kernel_ms": round(kern, 4),
               "nblk_out": yinfo["nblk_out"], "nprod": yinfo["nprod"], "flops": yinfo["flops"],
               "gflops": round(yinfo["flops"] / (ms * 1e-3) / 1e9, 2),
               "speedup_vs_full": round(results[args.mode]["ms_per_step"] / ms, 3)}
        print(f"[bench] symmetric square ({args.mode}): {ms:.3f} ms/step, {yinfo['nprod']} products",
              file=sys.stderr, flush=True)

    # CPU oracle leg: baseline timing + reference values of sampled C blocks
    cpu = None
    if not args.no_cpu:
        cpu, (si, sj, ref) = cpu_baseline_leg(wl, tol, bs, args.cpu_seconds)
        for mode in modes:
            step(mode)
            got = C.extract(si, sj).cpu().numpy()
            err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            results[mode]["rel_err_vs_fp64_oracle"] = float(f"{err:.3e}")
        if spamm is not None:
            step(args.mode, args.spamm_tol)
            got = C.extract(si, sj).cpu().numpy()
            spamm["rel_err_vs_exact_fp64_oracle"] = float(f"{np.linalg.norm(got - ref) / np.linalg.norm(ref):.3e}")
        print(f"[bench] cpu oracle: {cpu['value']} GFLOP/s on {cpu['cores']} threads", file=sys.stderr,
              flush=True)
    for mode in modes:
        results[mode].pop("_vals", None)

    ch = results[args.mode]
    f64 = results.get("f64")
    peak = PEAK_TFLOPS[args.mode]
    achieved = ch["kernel_mfma_tflops"]
    bs2 = bs * bs
    # algorithmic bytes of one launch: both packed operands read once, C written once
    alg_bytes = (2 * A.nblk * bs2 * OPERAND_BYTES[args.mode]
                 + info["nblk_out"] * bs2 * RESULT_BYTES[args.mode])
    out = {
        "metric": METRIC,
        "value": ch["effective_gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ch["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.mode],
        "data": "synthetic",
        "config": {
            "workload": (f"decay3d-n{args.npoints}-bs{bs}-tol1e-10" if args.workload == "decay" else
                         f"paper-{args.workload}-n{args.n}-h3000-bs{bs}")
                        + f" (C = A*A, {info['nblk_out']} C blocks, {info['nprod']} leaf products)",
            "mode": args.mode,
            "unit": info["unit"],
            "flops_per_step": info["flops"],
            "step": "set_blocks(norms+drop, Morton rank) + operand packing (side stream, overlapping the "
                    "symbolic phase) + symbolic (quadtree, walk, work list) + numeric (MFMA kernel)",
        },
        "roofline": {
            "bound": "mfma",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(args.mode, info["unit"], args.npoints, args.workload),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes": alg_bytes,
            "kernel": f"numeric leaf-product kernel, mode {args.mode}, unit {info['unit']} "
                      f"({MFMA_TERMS[args.mode]} MFMA term(s) per leaf product)",
        },
        "modes": results,
        "vs_f64_gpu": round(ch["effective_gflops"] / f64["effective_gflops"], 3) if f64 else None,
        "cpu_baseline": cpu,
        "copy_gbps": copy_gbps,
        "spamm": spamm,
        "symmetric_square": sym,
    }
    if args.workload != "decay":
        # the paper's own count (Table 1): element-level multiply-adds of the structure
        ef = a.meta["element_flops"]
        out["config"]["element_flops_table1"] = ef
        out["element_gflops"] = round(ef / (ch["ms_per_step"] * 1e-3) / 1e9, 2)
    if args.workload == "decay" and not args.no_legs:
        # the other workloads, each with its own roofline and oracle timing
        del A, C, state, brow, bcol, vals
        torch.cuda.empty_cache()
        legs = {}
        ls, lw = max(args.leg_steps, 1), 1
        # the millisecond-scale legs time 20 times as many steps (a few tens of
        # ms each), after a few warmup steps
        ms_s, ms_w = 20 * ls, 5
        for name, fn in (("banded-n2048-f64", lambda: leg_config1(torch, qbsm, W, ms_s, ms_w)),
                         ("random-blocks-n65536", lambda: leg_config3(torch, qbsm, W, ms_s, ms_w)),
                         ("forward-backward-n16384-f32", lambda: leg_config5(torch, qbsm, W, ms_s, ms_w)),
                         ("batched-256-f32", lambda: leg_config4(torch, qbsm, W, ls, lw))):
            t_leg = time.perf_counter()
            legs[name] = fn()
            torch.cuda.empty_cache()
            print(f"[bench] leg {name}: {legs[name]['ms_per_step']} ms/step, {legs[name]['value']} GFLOP/s, "
                  f"roofline {legs[name]['roofline']['frac']} ({time.perf_counter() - t_leg:.1f} s)",
                  file=sys.stderr, flush=True)
        out["configs"] = legs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
