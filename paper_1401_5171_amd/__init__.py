"""Oblique QR factorisation Z = QR, Q^T A Q = I, on one MI355X.

A thin ctypes binding over liboqr.so (C ABI in include/oqr.h).  Every step of
every algorithm runs in the library's HIP kernels; this module only marshals
arguments: it checks shapes, allocates outputs and the workspace with torch on
the current device and stream, and raises OQRError on a non-zero status or
device `info`.  There is no CPU fallback: importing works without a GPU, but
every call needs the built library and a HIP device.

Matrices are column-major: an (m, n) tensor with stride (1, ld), ld >= m, as
produced by `colmajor(x)`.  The dense operator A is an (m, m) contiguous
float64 tensor holding a symmetric matrix (its row- and column-major readings
coincide).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboqr.so")

OQR_OK, OQR_E_ARG, OQR_E_NOT_SPD, OQR_E_HIP, OQR_E_WORKSPACE, OQR_E_UNSUPPORTED, OQR_E_SCRATCH = range(7)
OQR_F64, OQR_F32 = 0, 1
OQR_BATCH_BAD_ITEM = -1          # info of a batch item outside the entry point's limits
OQR_OP_DENSE, OQR_OP_STENCIL7, OQR_OP_TRIDIAG = 0, 1, 2
PREC = {"fp64": 0, "fp32": 1, "bf16x2": 2, "bf16x3": 3}
GS = {"cgs": 0, "mgs_row": 1, "mgs_col": 2, "cgs2": 3}
ALG = {"cholqr": 0, "cholqr2": 1, "chol_a": 2, "eig_a": 3, "gs": 4, "pre_cholqr": 5}
MAX_N = 256

EXPORTS = (
    "oqr_default_opts", "oqr_workspace_bytes", "oqr_cholqr", "oqr_cholqr2", "oqr_pre_cholqr", "oqr_chol_a", "oqr_eig_a",
    "oqr_gs", "oqr_check", "oqr_batched_workspace_bytes", "oqr_cholqr2_batched", "oqr_batched_default_tuning",
    "oqr_status_string", "oqr_version", "oqr_trace_start", "oqr_trace_stop", "oqr_gls", "oqr_gls_workspace_bytes",
    "oqr_cholqr2_noalloc", "oqr_noalloc_scratch_bytes",
)


class OQRError(RuntimeError):
    def __init__(self, msg, status=None, info=None):
        super().__init__(msg)
        self.status = status
        self.info = info


class _Op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("a", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("center", ctypes.c_double), ("off", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("pass1", ctypes.c_int32), ("pass2", ctypes.c_int32), ("shift_c", ctypes.c_double),
                ("max_retries", ctypes.c_int32), ("gs_variant", ctypes.c_int32)]


BATCH_MBUCKETS, BATCH_NCLASSES, BATCH_SHAPES = 6, 4, 4
BATCH_SHAPE_NAMES = ("128x32", "64x32", "128x16", "64x16")       # rows per row block x K step
TUNING_PATH = os.path.join(_HERE, "batch_tuning.json")


class BatchTuning(ctypes.Structure):
    _fields_ = [("wg_per_cu", ctypes.c_int32), ("sort", ctypes.c_int32),
                ("shape", (ctypes.c_uint8 * BATCH_NCLASSES) * BATCH_MBUCKETS),
                ("split_m", ctypes.c_int32), ("parts", ctypes.c_int32)]

    def to_dict(self):
        return {"wg_per_cu": int(self.wg_per_cu), "sort": int(self.sort),
                "shape": [[int(self.shape[b][c]) for c in range(BATCH_NCLASSES)] for b in range(BATCH_MBUCKETS)],
                "split_m": int(self.split_m), "parts": int(self.parts)}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        t.wg_per_cu, t.sort = int(d["wg_per_cu"]), int(d["sort"])
        for b in range(BATCH_MBUCKETS):
            for c in range(BATCH_NCLASSES):
                t.shape[b][c] = int(d["shape"][b][c])
        t.split_m, t.parts = int(d.get("split_m", 0)), int(d.get("parts", 1))
        return t


def batch_m_bucket(m: int) -> int:
    """m bucket of the batched tuning table: m < 512, < 1024, < 2048, < 4096, < 8192, >= 8192."""
    b, lim = 0, 512
    while b < BATCH_MBUCKETS - 1 and m >= lim:
        b, lim = b + 1, lim * 2
    return b


def batch_n_class(n: int) -> int:
    """n class of the batched tuning table: n <= 8, <= 16, <= 32, <= 64."""
    return 0 if n <= 8 else 1 if n <= 16 else 2 if n <= 32 else 3


def default_batch_tuning() -> "BatchTuning":
    t = BatchTuning()
    lib().oqr_batched_default_tuning(ctypes.byref(t))
    return t


def stored_batch_tuning(dtype: str) -> Optional["BatchTuning"]:
    """The tuning table checked in beside the library for storage `dtype` ("f64" or "f32"), or None."""
    import json
    if not os.path.exists(TUNING_PATH):
        return None
    with open(TUNING_PATH) as f:
        d = json.load(f)
    return BatchTuning.from_dict(d[dtype]) if dtype in d else None


class BatchItem(ctypes.Structure):
    _fields_ = [("a", ctypes.c_void_p), ("z", ctypes.c_void_p), ("q", ctypes.c_void_p), ("r", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("ldz", ctypes.c_int64), ("ldq", ctypes.c_int64), ("ldr", ctypes.c_int64),
                ("m", ctypes.c_int32), ("n", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded liboqr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OQRError(f"{LIB_PATH} is missing: build it with `python -m paper_1401_5171_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        sig = [ctypes.POINTER(_Op), vp, i64, i64, i64, vp, i64, vp, i64, ctypes.POINTER(_Opts), vp, sz, vp, vp]
        for name in ("oqr_cholqr", "oqr_cholqr2", "oqr_pre_cholqr", "oqr_chol_a", "oqr_eig_a", "oqr_gs"):
            f = getattr(L, name)
            f.argtypes = sig
            f.restype = ctypes.c_int
        L.oqr_cholqr2_noalloc.argtypes = sig[:10] + [vp, vp]
        L.oqr_cholqr2_noalloc.restype = ctypes.c_int
        L.oqr_noalloc_scratch_bytes.restype = sz
        L.oqr_workspace_bytes.argtypes = [i32, ctypes.POINTER(_Op), i64, i64, ctypes.POINTER(_Opts)]
        L.oqr_workspace_bytes.restype = sz
        L.oqr_gls.argtypes = [ctypes.POINTER(_Op), vp, i64, vp, i64, i64, i64, vp, i64, i64, vp, i64, vp, sz, vp]
        L.oqr_gls.restype = ctypes.c_int
        L.oqr_gls_workspace_bytes.argtypes = [ctypes.POINTER(_Op), i64, i64, i64]
        L.oqr_gls_workspace_bytes.restype = sz
        L.oqr_check.argtypes = [ctypes.POINTER(_Op), vp, i64, i64, i64, vp, i64, vp, i64, vp, sz, vp, vp]
        L.oqr_check.restype = ctypes.c_int
        L.oqr_batched_workspace_bytes.argtypes = [i64, i32, i32, i32]
        L.oqr_batched_workspace_bytes.restype = sz
        L.oqr_cholqr2_batched.argtypes = [i64, vp, i32, i32, i32, ctypes.POINTER(_Opts), ctypes.POINTER(BatchTuning),
                                          vp, sz, vp, vp]
        L.oqr_cholqr2_batched.restype = ctypes.c_int
        L.oqr_batched_default_tuning.argtypes = [ctypes.POINTER(BatchTuning)]
        L.oqr_status_string.argtypes = [ctypes.c_int]
        L.oqr_status_string.restype = ctypes.c_char_p
        L.oqr_default_opts.argtypes = [ctypes.POINTER(_Opts)]
        L.oqr_version.restype = ctypes.c_int
        L.oqr_trace_start.argtypes = [ctypes.c_char_p]
        L.oqr_trace_start.restype = ctypes.c_int
        L.oqr_trace_stop.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
        L.oqr_trace_stop.restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().oqr_status_string(int(code)).decode()


def _raise(code, what):
    if code != OQR_OK:
        raise OQRError(f"{what}: {status_string(code)}", status=code)


@dataclasses.dataclass(frozen=True)
class Stencil7:
    """Matrix-free 7-point operator (A z)_p = center z_p + off * sum of in-grid face neighbours,
    p = x + nx (y + ny z)."""

    nx: int
    ny: int
    nz: int
    center: float
    off: float

    @property
    def m(self):
        return self.nx * self.ny * self.nz


class Tridiag:
    """Symmetric tridiagonal operator: A(i, i) = diag[i], A(i, i+1) = A(i+1, i) = sub[i].  The two
    arrays (numpy or torch) are copied into one device buffer [diag, sub] (the layout of the C ABI)."""

    def __init__(self, diag, sub, device=None):
        torch = _torch()
        d = torch.as_tensor(diag, dtype=torch.float64)
        e = torch.as_tensor(sub, dtype=torch.float64)
        if d.dim() != 1 or e.dim() != 1 or e.numel() != max(d.numel() - 1, 0) or d.numel() < 1:
            raise ValueError("need diag (m,) and sub (m - 1,)")
        dev = device or (d.device if d.is_cuda else torch.device("cuda", torch.cuda.current_device()))
        self.buf = torch.cat([d.to(dev), e.to(dev)]).contiguous()
        self.m = int(d.numel())
        self.device = self.buf.device


def _torch():
    import torch
    return torch


def colmajor(x):
    """Column-major view (stride (1, m)) of a 2D tensor, copying only if needed."""
    if x.dim() != 2:
        raise ValueError("expected a 2D tensor")
    if (x.stride(0) == 1 or x.shape[0] <= 1) and (x.shape[1] <= 1 or x.stride(1) >= max(1, x.shape[0])):
        return x
    return x.t().contiguous().t()


def _ld(x):
    """Leading dimension of a column-major tensor (size-1 dimensions carry arbitrary strides)."""
    if x.shape[1] <= 1:
        return max(1, x.shape[0])
    return max(1, x.stride(1))


def make_op(A) -> Tuple[_Op, int]:
    """oqr_op for a dense symmetric float64 tensor or a Stencil7; returns (op, m)."""
    op = _Op()
    if isinstance(A, Tridiag):
        op.kind, op.dtype = OQR_OP_TRIDIAG, OQR_F64
        op.a, op.lda = A.buf.data_ptr(), A.m
        return op, A.m
    if isinstance(A, Stencil7) or hasattr(A, "nx"):
        op.kind, op.dtype = OQR_OP_STENCIL7, OQR_F64
        op.nx, op.ny, op.nz = int(A.nx), int(A.ny), int(A.nz)
        op.center, op.off = float(A.center), float(A.off)
        return op, op.nx * op.ny * op.nz
    torch = _torch()
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    if A.dtype != torch.float64 or not A.is_cuda:
        raise ValueError("A must be a float64 CUDA tensor")
    m = A.shape[0]
    # symmetric: rows of a row-major view are columns; either unit stride gives a column-major lda
    if A.stride(1) == 1 and A.stride(0) >= m:
        lda = A.stride(0)
    elif A.stride(0) == 1 and A.stride(1) >= m:
        lda = A.stride(1)
    elif m <= 1:
        lda = 1
    else:
        raise ValueError("A must have one unit stride and a leading dimension >= m")
    op.kind, op.dtype = OQR_OP_DENSE, OQR_F64
    op.a, op.lda = A.data_ptr(), lda
    return op, m


def make_opts(pass1="fp64", pass2="fp64", shift_c=1.0, max_retries=3, gs_variant="cgs") -> _Opts:
    o = _Opts()
    o.pass1, o.pass2 = PREC[pass1], PREC[pass2]
    o.shift_c, o.max_retries = float(shift_c), int(max_retries)
    o.gs_variant = GS[gs_variant]
    return o


class Plan:
    """Pre-allocated call of one algorithm on a fixed operator and shape (no allocation per run)."""

    def __init__(self, alg: str, A, n: int, **opts):
        torch = _torch()
        self.alg = alg
        self.A = A                      # keep the operand alive
        self.op, self.m = make_op(A)
        self.n = int(n)
        self.opts = make_opts(**opts)
        self.device = A.device if hasattr(A, "device") else torch.device("cuda", torch.cuda.current_device())
        L = lib()
        nbytes = L.oqr_workspace_bytes(ALG[alg], ctypes.byref(self.op), self.m, self.n, ctypes.byref(self.opts))
        if nbytes == 0 and self.n > 0:
            raise OQRError(f"workspace query failed for {alg} (m={self.m}, n={self.n})")
        self.ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        self.info = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.fn = getattr(L, "oqr_" + alg)

    def run(self, Z, Q, R, stream=None):
        """Enqueue the factorisation of column-major Z into Q (may be Z) and R; returns nothing."""
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        rc = self.fn(ctypes.byref(self.op), Z.data_ptr(), _ld(Z), self.m, self.n, Q.data_ptr(), _ld(Q),
                     R.data_ptr(), _ld(R), ctypes.byref(self.opts), self.ws.data_ptr(), self.ws.numel(),
                     self.info.data_ptr(), s)
        _raise(rc, "oqr_" + self.alg)

    def capture(self, Z, Q, R):
        """Capture one call on these tensors into a HIP graph (a torch.cuda.CUDAGraph) and return it:
        `graph.replay()` re-runs the factorisation of whatever Z then holds into the same Q, R and
        `info`, as one graph launch instead of one launch per kernel.  The call is made once eagerly on
        the capture stream first, so that the library's one-time device queries run outside the
        capture.  The library issues no memset or allocation, so every replay repeats the eager
        result bit for bit."""
        torch = _torch()
        s = torch.cuda.Stream(self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.run(Z, Q, R)
        torch.cuda.current_stream(self.device).wait_stream(s)
        torch.cuda.synchronize(self.device)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.run(Z, Q, R)
        return g

    def __call__(self, Z, check_info=True):
        torch = _torch()
        Z = colmajor(Z)
        if Z.dtype != torch.float64 or not Z.is_cuda:
            raise ValueError("Z must be a float64 CUDA tensor")
        if Z.shape != (self.m, self.n):
            raise ValueError(f"Z must be {self.m} x {self.n}")
        Q = torch.empty(self.n, self.m, dtype=torch.float64, device=Z.device).t()
        R = torch.empty(self.n, self.n, dtype=torch.float64, device=Z.device).t()
        self.run(Z, Q, R)
        info = int(self.info.item()) if check_info else None
        if check_info and info != 0:
            raise OQRError(f"oqr_{self.alg}: numerical failure, info = {info}", info=info)
        return Q, R


class KernelTimer:
    """Context manager: summed HIP-event time of every launch of one library kernel."""

    def __init__(self, kernel: str):
        self.kernel = kernel
        self.total_ms = 0.0
        self.count = 0

    def __enter__(self):
        _raise(lib().oqr_trace_start(self.kernel.encode()), "oqr_trace_start")
        return self

    def __exit__(self, *exc):
        t = ctypes.c_double()
        c = ctypes.c_int32()
        rc = lib().oqr_trace_stop(ctypes.byref(t), ctypes.byref(c))
        if exc[0] is None:
            _raise(rc, "oqr_trace_stop")
        self.total_ms, self.count = t.value, c.value
        return False

    @property
    def avg_ms(self):
        return self.total_ms / self.count if self.count else float("nan")


class BatchPlan:
    """Batched CholQR2-A (one persistent launch) over dense instances A_i (m_i x m_i, symmetric,
    contiguous) and Z_i (m_i x n_i, column-major), storage float64 or float32, n_i <= 64.

    Outputs Q_i (column-major, same dtype) and R_i (n_i x n_i) are allocated here; `run()` enqueues
    the launch on the current stream and allocates nothing, so it can be captured in a graph.
    `tuning`: a BatchTuning (tile shape per (m bucket, n class), workgroups per compute unit, order);
    None takes the table checked in beside the library for this storage type, else the built-in one."""

    def __init__(self, As, Zs, tuning: Optional[BatchTuning] = None, shift_c: float = 1.0, max_retries: int = 3,
                 q_in_place=False):
        torch = _torch()
        if len(As) != len(Zs) or not As:
            raise ValueError("need as many A_i as Z_i, at least one")
        dt = As[0].dtype
        if dt not in (torch.float64, torch.float32):
            raise ValueError("batch storage must be float64 or float32")
        self.dtype = OQR_F64 if dt == torch.float64 else OQR_F32
        self.device = As[0].device
        self.As, self.Zs = list(As), [colmajor(z) for z in Zs]
        items = (BatchItem * len(As))()
        self.Qs, self.Rs = [], []
        max_m = max_n = 1
        for k, (a, z) in enumerate(zip(self.As, self.Zs)):
            m, n = z.shape
            if a.shape != (m, m) or a.dtype != dt or z.dtype != dt or not a.is_contiguous():
                raise ValueError(f"instance {k}: shapes or dtypes do not match")
            q = z if q_in_place else torch.empty(n, m, dtype=dt, device=self.device).t()
            r = torch.empty(n, n, dtype=dt, device=self.device).t()
            self.Qs.append(q)
            self.Rs.append(r)
            it = items[k]
            it.a, it.z, it.q, it.r = a.data_ptr(), z.data_ptr(), q.data_ptr(), r.data_ptr()
            it.lda, it.ldz, it.ldq, it.ldr = m, _ld(z), _ld(q), _ld(r)
            it.m, it.n = m, n
            max_m, max_n = max(max_m, m), max(max_n, n)
        self._items_host = items
        raw = bytes(items)
        self.items = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)
        self.batch, self.max_m, self.max_n = len(As), max_m, max_n
        if tuning is None:
            tuning = stored_batch_tuning("f64" if self.dtype == OQR_F64 else "f32") or default_batch_tuning()
        self.tuning = tuning
        self.opts = make_opts(shift_c=shift_c, max_retries=max_retries)
        L = lib()
        nbytes = L.oqr_batched_workspace_bytes(self.batch, max_m, max_n, self.dtype)
        self.ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        self.info = torch.zeros(self.batch, dtype=torch.int32, device=self.device)

    def _launch(self, items, count, info, tuning, stream=None):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        rc = lib().oqr_cholqr2_batched(count, items.data_ptr(), self.dtype, self.max_m, self.max_n,
                                       ctypes.byref(self.opts), ctypes.byref(tuning), self.ws.data_ptr(),
                                       self.ws.numel(), info.data_ptr(), s)
        _raise(rc, "oqr_cholqr2_batched")

    def run(self, stream=None, tuning: Optional[BatchTuning] = None):
        self._launch(self.items, self.batch, self.info, tuning or self.tuning, stream)

    def _time(self, items, count, info, tuning, reps):
        torch = _torch()
        self._launch(items, count, info, tuning)
        torch.cuda.synchronize()
        with KernelTimer("batch") as kt:
            for _ in range(reps):
                self._launch(items, count, info, tuning)
            torch.cuda.synchronize()
        return kt.avg_ms

    def autotune(self, reps: int = 3) -> dict:
        """Choose the tuning on this batch: for every (m bucket, n class) that holds instances, launch
        those instances alone with each tile shape (`reps` timed launches each, HIP events around the
        batched launch) and keep the fastest shape; then time the whole batch with 1, 2 and 3 workgroups
        per compute unit (largest instances first), then with the largest instances split over several
        workgroups (SPLIT_CANDIDATES: m threshold x parts, or none), keeping the fastest each time.  Inputs are read only; outputs
        are overwritten.  Sets and returns `self.tuning` with the timings in a dict."""
        torch = _torch()
        classes = {}
        for k in range(self.batch):
            it = self._items_host[k]
            classes.setdefault((batch_m_bucket(it.m), batch_n_class(it.n)), []).append(k)
        tu = BatchTuning.from_dict(self.tuning.to_dict())
        report = {"classes": {}, "wg_per_cu": {}}
        for (b, c), idx in sorted(classes.items()):
            sub = (BatchItem * len(idx))(*[self._items_host[k] for k in idx])
            sub_items = torch.frombuffer(bytearray(bytes(sub)), dtype=torch.uint8).to(self.device)
            sub_info = torch.zeros(len(idx), dtype=torch.int32, device=self.device)
            times = {}
            for shp in range(BATCH_SHAPES):
                trial = BatchTuning.from_dict(tu.to_dict())
                trial.shape[b][c] = shp
                times[shp] = self._time(sub_items, len(idx), sub_info, trial, reps)
            best = min(times, key=times.get)
            tu.shape[b][c] = best
            report["classes"][f"m{b}_n{c}"] = {"count": len(idx), "ms": {BATCH_SHAPE_NAMES[k]: round(v, 4)
                                                                      for k, v in times.items()},
                                               "shape": BATCH_SHAPE_NAMES[best]}
        for wg in (1, 2, 3):
            trial = BatchTuning.from_dict(tu.to_dict())
            trial.wg_per_cu, trial.sort = wg, 1
            report["wg_per_cu"][wg] = round(self._time(self.items, self.batch, self.info, trial, reps), 4)
        tu.wg_per_cu, tu.sort = min(report["wg_per_cu"], key=report["wg_per_cu"].get), 1
        # cooperative instances: the largest ones (m >= split_m) split over `parts` workgroups per pass
        report["split"] = {}
        for split_m, parts in self.SPLIT_CANDIDATES:
            if split_m > self.max_m:
                continue
            trial = BatchTuning.from_dict(tu.to_dict())
            trial.split_m, trial.parts = split_m, parts
            report["split"][f"{split_m}x{parts}"] = round(self._time(self.items, self.batch, self.info, trial, reps), 4)
        best = min(report["split"], key=report["split"].get)
        tu.split_m, tu.parts = (int(v) for v in best.split("x"))
        self.tuning = tu
        report["tuning"] = tu.to_dict()
        return report

    SPLIT_CANDIDATES = ((0, 1), (3584, 4), (3584, 8), (3072, 4), (3072, 8), (2048, 4), (2048, 8))


def save_batch_tuning(tuning: BatchTuning, dtype: str, path: str = TUNING_PATH) -> None:
    """Store `tuning` for storage `dtype` ("f64" or "f32") in the JSON table at `path` (merged)."""
    import json
    d = {}
    if os.path.exists(path):
        with open(path) as f:
            d = json.load(f)
    d[dtype] = tuning.to_dict()
    with open(path, "w") as f:
        json.dump(d, f, indent=1)
        f.write("\n")


def _run(alg, A, Z, **opts):
    Z = colmajor(Z)
    return Plan(alg, A, Z.shape[1], **opts)(Z)


def cholqr(A, Z, prec="fp64", shift_c=1.0, max_retries=3):
    """CHOLQR-A (Algorithm 1): returns (Q, R)."""
    return _run("cholqr", A, Z, pass1=prec, shift_c=shift_c, max_retries=max_retries)


def cholqr2(A, Z, pass1="fp64", pass2="fp64", shift_c=1.0, max_retries=3):
    """CholQR2-A (CHOLQR-A twice, R = R2 R1): returns (Q, R)."""
    return _run("cholqr2", A, Z, pass1=pass1, pass2=pass2, shift_c=shift_c, max_retries=max_retries)


def noalloc_scratch_bytes() -> int:
    """Size of the library's fixed scratch used by cholqr2_noalloc (per device)."""
    return int(lib().oqr_noalloc_scratch_bytes())


def cholqr2_noalloc_into(A, Z, Q, R, info, pass1="fp64", pass2="fp64", shift_c=1.0, max_retries=3, stream=None):
    """oqr_cholqr2_noalloc on caller-owned column-major Z, Q (may be Z), R and a 1-element int32
    `info`: enqueues CholQR2-A on the library's own scratch and allocates nothing (graph-capturable
    after a first call on the device).  Raises OQRError on a host status; `info` is left on the device."""
    torch = _torch()
    op, m = make_op(A)
    n = Z.shape[1]
    if Z.shape[0] != m or Q.shape != (m, n) or R.shape != (n, n):
        raise ValueError("shapes of A, Z, Q and R do not match")
    opts = make_opts(pass1=pass1, pass2=pass2, shift_c=shift_c, max_retries=max_retries)
    s = stream if stream is not None else torch.cuda.current_stream(Z.device).cuda_stream
    rc = lib().oqr_cholqr2_noalloc(ctypes.byref(op), Z.data_ptr(), _ld(Z), m, n, Q.data_ptr(), _ld(Q), R.data_ptr(),
                                   _ld(R), ctypes.byref(opts), info.data_ptr(), s)
    _raise(rc, "oqr_cholqr2_noalloc")


def cholqr2_noalloc(A, Z, pass1="fp64", pass2="fp64", shift_c=1.0, max_retries=3):
    """CholQR2-A through the allocation-free entry point (outputs allocated here): returns (Q, R)."""
    torch = _torch()
    Z = colmajor(Z)
    m, n = Z.shape
    Q = torch.empty(n, m, dtype=torch.float64, device=Z.device).t()
    R = torch.empty(n, n, dtype=torch.float64, device=Z.device).t()
    info = torch.zeros(1, dtype=torch.int32, device=Z.device)
    cholqr2_noalloc_into(A, Z, Q, R, info, pass1, pass2, shift_c, max_retries)
    k = int(info.item())
    if k != 0:
        raise OQRError(f"oqr_cholqr2_noalloc: numerical failure, info = {k}", info=k)
    return Q, R


def pre_cholqr(A, Z, prec="fp64", shift_c=1.0, max_retries=3):
    """PRE-CHOLQR-A (Algorithm 2): Householder QR Z = Y U, CHOLQR-A on Y, R = S U; returns (Q, R)."""
    return _run("pre_cholqr", A, Z, pass1=prec, shift_c=shift_c, max_retries=max_retries)


def chol_a(A, Z):
    """CHOL-EQR (Algorithm 3): returns (Q, R)."""
    return _run("chol_a", A, Z)


def eig_a(A, Z):
    """EQR-SYEV (Algorithm 4): returns (Q, R)."""
    return _run("eig_a", A, Z)


def gs(A, Z, variant="cgs"):
    """Gram-Schmidt in the A inner product (cgs, mgs_row, mgs_col, cgs2): returns (Q, R)."""
    return _run("gs", A, Z, gs_variant=variant)


def gls(A, Q, R, B):
    """Generalised least squares (Section 1): X = R^{-1} Q^T A B minimises ||Z x - b||_A for every
    column b of B, given the oblique QR (Q, R) of Z.  B may be a vector.  Returns X (n, k) or (n,)."""
    torch = _torch()
    op, m = make_op(A)
    Q, R = colmajor(Q), colmajor(R)
    vec = B.dim() == 1
    Bm = colmajor(B[:, None] if vec else B)
    n, k = Q.shape[1], Bm.shape[1]
    if Q.shape[0] != m or R.shape != (n, n) or Bm.shape[0] != m:
        raise ValueError("shapes of A, Q, R and B do not match")
    X = torch.empty(k, n, dtype=torch.float64, device=Q.device).t()
    L = lib()
    nbytes = L.oqr_gls_workspace_bytes(ctypes.byref(op), m, n, k)
    if nbytes == 0:
        raise OQRError("gls workspace query failed")
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=Q.device)
    s = torch.cuda.current_stream(Q.device).cuda_stream
    rc = L.oqr_gls(ctypes.byref(op), Q.data_ptr(), _ld(Q), R.data_ptr(), _ld(R), m, n, Bm.data_ptr(), _ld(Bm), k,
                   X.data_ptr(), _ld(X), ws.data_ptr(), ws.numel(), s)
    _raise(rc, "oqr_gls")
    return X[:, 0] if vec else X


def check(A, Z, Q, R):
    """Device report: (||I - Q^T A Q||_F, ||Z - QR||_F / ||Z||_F)."""
    torch = _torch()
    op, m = make_op(A)
    Z, Q, R = colmajor(Z), colmajor(Q), colmajor(R)
    n = Z.shape[1]
    L = lib()
    # workspace: W (m x n) + Gram partials + G + per-block partial sums; generous upper bound
    nbytes = L.oqr_workspace_bytes(ALG["cholqr"], ctypes.byref(op), m, n, None) + 4 * m * 8 + (1 << 20)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=Z.device)
    out = torch.zeros(2, dtype=torch.float64, device=Z.device)
    s = torch.cuda.current_stream(Z.device).cuda_stream
    rc = L.oqr_check(ctypes.byref(op), Z.data_ptr(), _ld(Z), m, n, Q.data_ptr(), _ld(Q), R.data_ptr(), _ld(R),
                     ws.data_ptr(), ws.numel(), out.data_ptr(), s)
    _raise(rc, "oqr_check")
    o = out.cpu()
    return float(o[0]), float(o[1])
