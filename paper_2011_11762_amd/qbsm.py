"""Thin Python binding of libqbsm (the C ABI in ``include/qbsm.h``).

Argument marshalling only: every step of the multiply runs in the library's
HIP kernels.  PyTorch provides device memory (the library allocates through
torch's caching allocator once :func:`load` has installed the hooks) and
streams (every call uses ``torch.cuda.current_stream()``).

The library must have been built (``python -m paper_2011_11762_amd.build``);
importing works without it, but every call raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqbsm.so")

F64, F32, BF16, BF16X3, OZAKI_I8 = 0, 1, 2, 3, 4
MODES = {"f64": F64, "f32": F32, "bf16": BF16, "bf16x3": BF16X3, "ozaki": OZAKI_I8}
MODE_NAMES = {v: k for k, v in MODES.items()}

STATUS = {0: "ok", 1: "invalid argument", 2: "shape mismatch", 3: "invalid block pattern",
          4: "out of device memory", 5: "HIP runtime error", 6: "unsupported", 7: "invalid state"}


class QbsmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class BatchTuning(ctypes.Structure):
    _fields_ = [("unit", c_int32), ("wg_per_cu", c_int32), ("ms", c_double), ("times_ms", (c_double * 4) * 3)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("unit", c_int32), ("upper", c_int32), ("spamm_tol", c_double), ("schedule", c_int32),
                ("reserved", c_int32 * 3)]


_ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p, c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)

_lib = None
_hooks = None

_SIGS = {
    "qbsm_set_allocator": [_ALLOC_FN, _RELEASE_FN, c_void_p],
    "qbsm_status_string": [c_int32],
    "qbsm_last_error": [],
    "qbsm_version": [],
    "qbsm_matrix_create": [c_int64, c_int64, c_int32, POINTER(c_void_p)],
    "qbsm_matrix_destroy": [c_void_p],
    "qbsm_matrix_set_blocks": [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                               POINTER(c_int64)],
    "qbsm_matrix_store_f32": [c_void_p, c_void_p],
    "qbsm_matrix_prepack": [c_void_p, c_int32, c_int32, c_void_p],
    "qbsm_matrix_set_elements": [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_int64)],
    "qbsm_matrix_get_elements": [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p],
    "qbsm_matrix_truncate": [c_void_p, c_double, c_void_p, POINTER(c_int64)],
    "qbsm_matrix_add": [c_double, c_void_p, c_double, c_void_p, c_void_p, c_void_p],
    "qbsm_matrix_add_identity": [c_void_p, c_double, c_void_p],
    "qbsm_matrix_info": [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32), POINTER(c_int64)],
    "qbsm_matrix_get_pattern": [c_void_p, c_void_p, c_void_p, c_void_p],
    "qbsm_matrix_get_values": [c_void_p, c_void_p, c_void_p],
    "qbsm_matrix_extract_blocks": [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p],
    "qbsm_multiply_symbolic": [c_void_p, c_void_p, POINTER(PlanOpts), c_void_p, POINTER(c_void_p),
                               POINTER(c_int64), POINTER(c_int64)],
    "qbsm_multiply_symbolic_ex": [c_void_p, c_int32, c_void_p, c_int32, c_void_p, POINTER(PlanOpts), c_void_p,
                                  POINTER(c_void_p), POINTER(c_int64), POINTER(c_int64)],
    "qbsm_plan_info": [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int64), POINTER(c_int32),
                       POINTER(c_int64), POINTER(c_int64)],
    "qbsm_plan_get_products": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
    "qbsm_plan_destroy": [c_void_p],
    "qbsm_multiply_numeric": [c_void_p, c_int32, c_void_p, c_void_p],
    "qbsm_multiply_numeric_noalloc": [c_void_p, c_int32, c_void_p, c_void_p],
    "qbsm_multiply_backward": [c_void_p, c_void_p, c_void_p, c_int32, POINTER(PlanOpts), c_void_p, c_void_p,
                               c_void_p],
    "qbsm_multiply_backward_plan": [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p],
    "qbsm_batch_create": [c_int32, POINTER(c_void_p), c_int32, POINTER(c_void_p), c_void_p, POINTER(c_void_p)],
    "qbsm_batch_run": [c_void_p, c_void_p],
    "qbsm_batch_run_graph": [c_void_p, c_void_p],
    "qbsm_batch_set_occupancy": [c_void_p, c_int32],
    "qbsm_batch_destroy": [c_void_p],
    "qbsm_autotune_unit": [c_void_p, c_void_p, c_int32, c_int32, c_void_p, POINTER(c_int32), POINTER(c_double)],
    "qbsm_batch_autotune": [c_int32, POINTER(c_void_p), POINTER(c_void_p), c_int32, c_int32, c_void_p,
                            POINTER(BatchTuning)],
    "qbsm_profile_enable": [c_int32],
    "qbsm_profile_reset": [],
    "qbsm_profile_read": [c_int32, POINTER(c_int64), POINTER(c_double)],
}

ABI_SYMBOLS = tuple(_SIGS)


def load(install_torch_allocator: bool = True):
    """Loads libqbsm.so (raises if it has not been built)."""
    global _lib, _hooks
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2011_11762_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_char_p if name in ("qbsm_status_string", "qbsm_last_error") else c_int32
    _lib = lib
    if install_torch_allocator and torch.cuda.is_available():
        _install_torch_allocator()
    return lib


def _install_torch_allocator():
    global _hooks

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                      int(stream or 0))
        except Exception:  # out of memory -> NULL, the library reports it
            return None

    def _release(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    _hooks = (_ALLOC_FN(_alloc), _RELEASE_FN(_release))
    _check(_lib.qbsm_set_allocator(_hooks[0], _hooks[1], None))


def _check(st: int):
    if st != 0:
        msg = _lib.qbsm_last_error()
        raise QbsmError(st, msg.decode() if msg else "")


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return c_void_p(t.data_ptr() if t is not None and t.numel() else None)


def mode_id(mode) -> int:
    return MODES[mode] if isinstance(mode, str) else int(mode)


# --------------------------------------------------------------------------
class Matrix:
    """A block-sparse matrix handle (device-resident sparse quadtree)."""

    def __init__(self, nrows: int, ncols: int, bs: int):
        load()
        h = c_void_p()
        _check(_lib.qbsm_matrix_create(int(nrows), int(ncols), int(bs), ctypes.byref(h)))
        self._h = h
        self.nrows, self.ncols, self.bs = int(nrows), int(ncols), int(bs)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.qbsm_matrix_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def set_blocks(self, brow: torch.Tensor, bcol: torch.Tensor, vals: torch.Tensor,
                   drop_tol: float = 0.0) -> int:
        """brow/bcol: int32 cuda [n]; vals: float64 cuda [n, bs*bs] column-major blocks."""
        n = int(brow.numel())
        assert brow.dtype == torch.int32 and bcol.dtype == torch.int32 and vals.dtype == torch.float64
        assert brow.is_contiguous() and bcol.is_contiguous() and vals.is_contiguous()
        assert vals.numel() == n * self.bs * self.bs
        kept = c_int64()
        _check(_lib.qbsm_matrix_set_blocks(self._h, n, _ptr(brow), _ptr(bcol), _ptr(vals),
                                           float(drop_tol), _stream(), ctypes.byref(kept)))
        return kept.value

    def store_f32(self):
        """Round stored values to binary32 and drop the FP64 copy (halves memory)."""
        _check(_lib.qbsm_matrix_store_f32(self._h, _stream()))

    def set_elements(self, row: torch.Tensor, col: torch.Tensor, val: torch.Tensor) -> int:
        """row/col: int64 cuda [n]; val: float64 cuda [n].  Returns the number of leaves."""
        assert row.dtype == torch.int64 and col.dtype == torch.int64 and val.dtype == torch.float64
        row, col, val = row.contiguous(), col.contiguous(), val.contiguous()
        nb = c_int64()
        _check(_lib.qbsm_matrix_set_elements(self._h, int(row.numel()), _ptr(row), _ptr(col), _ptr(val),
                                             _stream(), ctypes.byref(nb)))
        return nb.value

    def get_elements(self, row, col) -> torch.Tensor:
        """FP64 values at (row[q], col[q]) (zero where no leaf is stored)."""
        row = torch.as_tensor(row, dtype=torch.int64).cuda().contiguous()
        col = torch.as_tensor(col, dtype=torch.int64).cuda().contiguous()
        out = torch.empty(row.numel(), dtype=torch.float64, device="cuda")
        _check(_lib.qbsm_matrix_get_elements(self._h, int(row.numel()), _ptr(row), _ptr(col), _ptr(out),
                                             _stream()))
        return out

    def truncate(self, eps: float) -> int:
        """Removes the smallest leaves while their Frobenius norm stays <= eps; returns leaves kept."""
        k = c_int64()
        _check(_lib.qbsm_matrix_truncate(self._h, float(eps), _stream(), ctypes.byref(k)))
        return k.value

    def add_identity(self, sigma: float):
        """In place: self += sigma * I."""
        _check(_lib.qbsm_matrix_add_identity(self._h, float(sigma), _stream()))

    def prepack(self, mode="bf16x3", roles: int = 3):
        """Pack the values for `mode` ahead of use on the library's side stream.

        roles: 1 = as a left operand, 2 = as a right operand, 3 = both.  The
        packing overlaps the symbolic phase that follows; later uses wait for it.
        """
        _check(_lib.qbsm_matrix_prepack(self._h, mode_id(mode), int(roles), _stream()))

    @property
    def nblk(self) -> int:
        n = c_int64()
        _check(_lib.qbsm_matrix_info(self._h, None, None, None, ctypes.byref(n)))
        return n.value

    def pattern(self):
        n = self.nblk
        brow = torch.empty(n, dtype=torch.int32, device="cuda")
        bcol = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(_lib.qbsm_matrix_get_pattern(self._h, _ptr(brow), _ptr(bcol), _stream()))
        return brow, bcol

    def values(self) -> torch.Tensor:
        n = self.nblk
        out = torch.empty((n, self.bs * self.bs), dtype=torch.float64, device="cuda")
        _check(_lib.qbsm_matrix_get_values(self._h, _ptr(out), _stream()))
        return out


    def extract(self, brow, bcol) -> torch.Tensor:
        """FP64 values of blocks (brow[q], bcol[q]) (zero blocks where not stored)."""
        brow = torch.as_tensor(brow, dtype=torch.int32).cuda().contiguous()
        bcol = torch.as_tensor(bcol, dtype=torch.int32).cuda().contiguous()
        out = torch.empty((brow.numel(), self.bs * self.bs), dtype=torch.float64, device="cuda")
        _check(_lib.qbsm_matrix_extract_blocks(self._h, brow.numel(), _ptr(brow), _ptr(bcol), _ptr(out),
                                               _stream()))
        return out


class Plan:
    """Symbolic phase result (work list + output pattern) of op(L) op(R) [masked]."""

    def __init__(self, L: Matrix, R: Matrix, trans_l=False, trans_r=False, mask: Matrix | None = None,
                 unit: int = 0, spamm_tol: float = 0.0, upper: bool = False, schedule: int = 0):
        """spamm_tol > 0: sparse approximate multiply (leaf products with
        ||L_leaf|| * ||R_leaf|| < spamm_tol are left out).  upper: only the
        output blocks with I <= J (symmetric square of a symmetric matrix).
        schedule: numeric-phase schedule, 0 automatic, 1 one workgroup per
        unit, 2 streamed (same results)."""
        load()
        h = c_void_p()
        nout, nprod = c_int64(), c_int64()
        opts = PlanOpts(unit=int(unit), spamm_tol=float(spamm_tol), upper=int(bool(upper)),
                        schedule=int(schedule))
        _check(_lib.qbsm_multiply_symbolic_ex(L.handle, int(trans_l), R.handle, int(trans_r),
                                              mask.handle if mask is not None else None, ctypes.byref(opts),
                                              _stream(), ctypes.byref(h), ctypes.byref(nout),
                                              ctypes.byref(nprod)))
        self._h = h
        self._keep = (L, R, mask)  # the plan refers to these handles
        self.nrows = L.ncols if trans_l else L.nrows
        self.ncols = R.nrows if trans_r else R.ncols
        self.bs = L.bs

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.qbsm_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        v = [c_int64(), c_int64(), c_int64(), c_int32(), c_int64(), c_int64()]
        _check(_lib.qbsm_plan_info(self._h, *[ctypes.byref(x) for x in v]))
        keys = ("nblk_out", "nprod", "flops", "unit", "nunits", "npairs")
        return {k: x.value for k, x in zip(keys, v)}

    def products(self):
        n = self.info()["nprod"]
        I, K, J = (torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(3))
        _check(_lib.qbsm_plan_get_products(self._h, _ptr(I), _ptr(K), _ptr(J), _stream()))
        return I, K, J

    def numeric(self, mode, out: Matrix | None = None) -> Matrix:
        if out is None:
            out = Matrix(self.nrows, self.ncols, self.bs)
        _check(_lib.qbsm_multiply_numeric(self._h, mode_id(mode), out.handle, _stream()))
        return out


    def backward(self, dC: Matrix, mode="f64", need_a=True, need_b=True):
        """dA = (dC R^T) on L's pattern, dB = (L^T dC) on R's pattern from this
        (forward) plan's product list: no symbolic walk."""
        L, R, _ = self._keep
        dA = Matrix(L.nrows, L.ncols, L.bs) if need_a else None
        dB = Matrix(R.nrows, R.ncols, R.bs) if need_b else None
        _check(_lib.qbsm_multiply_backward_plan(self._h, dC.handle, mode_id(mode),
                                                dA.handle if dA is not None else None,
                                                dB.handle if dB is not None else None, _stream()))
        return dA, dB

    def numeric_noalloc(self, mode, out: torch.Tensor) -> torch.Tensor:
        """Numeric phase into a caller-owned tensor (float64 for f64/ozaki,
        float32 otherwise; [nblk_out, bs*bs], blocks in ascending Morton order
        of (I, J)); the library allocates nothing."""
        assert out.is_cuda and out.is_contiguous()
        _check(_lib.qbsm_multiply_numeric_noalloc(self._h, mode_id(mode), _ptr(out), _stream()))
        return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def add(alpha: float, A: Matrix, beta: float, B: Matrix) -> Matrix:
    """alpha A + beta B on the union of the leaf patterns (FP64)."""
    C = Matrix(A.nrows, A.ncols, A.bs)
    _check(_lib.qbsm_matrix_add(float(alpha), A.handle, float(beta), B.handle, C.handle, _stream()))
    return C


def matmul(A: Matrix, B: Matrix, mode="f64", unit: int = 0, spamm_tol: float = 0.0) -> Matrix:
    """C = A B (symbolic + numeric); spamm_tol > 0 for the sparse approximate multiply."""
    return Plan(A, B, unit=unit, spamm_tol=spamm_tol).numeric(mode)


def backward(A: Matrix, B: Matrix, dC: Matrix, mode="f64", unit: int = 0, need_a=True, need_b=True):
    """dA = (dC B^T) on A's pattern, dB = (A^T dC) on B's pattern."""
    dA = Matrix(A.nrows, A.ncols, A.bs) if need_a else None
    dB = Matrix(B.nrows, B.ncols, B.bs) if need_b else None
    opts = PlanOpts(unit=int(unit))
    _check(_lib.qbsm_multiply_backward(A.handle, B.handle, dC.handle, mode_id(mode), ctypes.byref(opts),
                                       dA.handle if dA is not None else None,
                                       dB.handle if dB is not None else None, _stream()))
    return dA, dB


class Batch:
    """Batched numeric phase: one persistent launch (optionally a replayed HIP graph)."""

    def __init__(self, plans, mode, outs=None):
        load()
        self.plans = list(plans)
        self.outs = outs if outs is not None else [Matrix(p.nrows, p.ncols, p.bs) for p in self.plans]
        n = len(self.plans)
        ph = (c_void_p * n)(*[p.handle.value for p in self.plans])
        oh = (c_void_p * n)(*[o.handle.value for o in self.outs])
        h = c_void_p()
        _check(_lib.qbsm_batch_create(n, ph, mode_id(mode), oh, _stream(), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.qbsm_batch_destroy(h)
            self._h = None

    def run(self):
        _check(_lib.qbsm_batch_run(self._h, _stream()))

    def run_graph(self):
        _check(_lib.qbsm_batch_run_graph(self._h, _stream()))

    def set_occupancy(self, wg_per_cu: int):
        _check(_lib.qbsm_batch_set_occupancy(self._h, int(wg_per_cu)))


def autotune_unit(A: Matrix, B: Matrix, mode, reps: int = 3):
    best = c_int32()
    times = (c_double * 3)()
    _check(_lib.qbsm_autotune_unit(A.handle, B.handle, mode_id(mode), int(reps), _stream(),
                                   ctypes.byref(best), times))
    return best.value, {64: times[0], 128: times[1], 256: times[2]}


def batch_autotune(pairs, mode, reps: int = 1) -> dict:
    """Times every valid (unit side, persistent occupancy) for a batch over
    the (A, B) pairs; returns the fastest and the table {unit: {occ: ms}}."""
    n = len(pairs)
    lh = (c_void_p * n)(*[a.handle.value for a, _ in pairs])
    rh = (c_void_p * n)(*[b.handle.value for _, b in pairs])
    res = BatchTuning()
    _check(_lib.qbsm_batch_autotune(n, lh, rh, mode_id(mode), int(reps), _stream(), ctypes.byref(res)))
    table = {u: {o + 1: res.times_ms[i][o] for o in range(4) if res.times_ms[i][o] >= 0}
             for i, u in enumerate((64, 128, 256))}
    return {"unit": res.unit, "wg_per_cu": res.wg_per_cu, "ms": res.ms,
            "table": {u: t for u, t in table.items() if t}}


PROF_NUMERIC, PROF_PACK = 0, 1


def profile_enable(on: bool = True):
    load()
    _check(_lib.qbsm_profile_enable(1 if on else 0))


def profile_reset():
    _check(_lib.qbsm_profile_reset())


def profile_read(kernel_class: int = PROF_NUMERIC):
    """(launches, total_ms) of the recorded launches of a kernel class."""
    n, t = c_int64(), c_double()
    _check(_lib.qbsm_profile_read(int(kernel_class), ctypes.byref(n), ctypes.byref(t)))
    return n.value, t.value


# --------------------------------------------------------------------------
# Convenience: host BlockMatrix (paper_2011_11762_amd.workloads) -> device handle
def from_host(m, drop_tol: float = 0.0) -> Matrix:
    h = Matrix(m.nrows, m.ncols, m.bs)
    brow = torch.from_numpy(m.brow.astype("int32")).cuda()
    bcol = torch.from_numpy(m.bcol.astype("int32")).cuda()
    vals = torch.from_numpy(m.vals).cuda()
    h.set_blocks(brow, bcol, vals, drop_tol)
    return h


# --------------------------------------------------------------------------
# Autograd: gradients with respect to the block values
class _MatmulFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a_vals, b_vals, a_pat, b_pat, shapes, mode, unit):
        (m, k, n, bs) = shapes
        A = Matrix(m, k, bs)
        B = Matrix(k, n, bs)
        A.set_blocks(a_pat[0], a_pat[1], a_vals.detach().contiguous())
        B.set_blocks(b_pat[0], b_pat[1], b_vals.detach().contiguous())
        P = Plan(A, B, unit=unit)
        C = P.numeric(mode)
        cr, cc = C.pattern()
        ctx.save_for_backward(cr, cc)
        ctx.handles = (A, B, P)
        ctx.meta = (m, n, bs, mode, unit)
        ctx.mark_non_differentiable(cr, cc)
        return C.values(), cr, cc

    @staticmethod
    def backward(ctx, g_vals, _g1, _g2):
        cr, cc = ctx.saved_tensors
        A, B, P = ctx.handles
        m, n, bs, mode, unit = ctx.meta
        dC = Matrix(m, n, bs)
        dC.set_blocks(cr, cc, g_vals.contiguous().to(torch.float64))
        dA, dB = P.backward(dC, mode, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        ga = dA.values() if dA is not None else None
        gb = dB.values() if dB is not None else None
        return ga, gb, None, None, None, None, None


def block_matmul(a_vals, a_pat, b_vals, b_pat, m, k, n, bs, mode="f64", unit=0):
    """Differentiable C = A B on block values.

    a_pat / b_pat are (brow, bcol) int32 cuda tensors in canonical row-major
    order (the order the library reports patterns in), so that gradients
    line up with the value rows.  Returns (c_vals, c_brow, c_bcol).
    """
    for r, c in (a_pat, b_pat):
        key = r.to(torch.int64) * (max(k, n) // bs + 2) + c.to(torch.int64)
        if key.numel() > 1 and not bool((key[1:] > key[:-1]).all()):
            raise ValueError("block patterns must be in canonical row-major order")
    return _MatmulFn.apply(a_vals, b_vals, a_pat, b_pat, (m, k, n, bs), mode_id(mode), int(unit))
