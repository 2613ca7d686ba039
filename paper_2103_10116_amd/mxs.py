"""ctypes binding of libmxs (include/mxs.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python and
torch arguments to the C ABI, raises MxsError on a non-OK status, and hands
torch's current HIP stream to the library.  Importing it loads
``libmxs.so`` from this package directory and fails loudly if it has not
been built (``python -c "import __graft_entry__ as g; g.build()"``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmxs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(paper_2103_10116_amd/build.py or __graft_entry__.build())")
# torch first: its HIP runtime is then already in the process when libmxs is
# loaded, so both bind to the same runtime and share devices and streams
# (loading libmxs first brings in a second runtime, on which context
# creation fails).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

OK, INVALID_ARG, INVALID_MATRIX, UNSUPPORTED, OOM, HIP = 0, 1, 2, 3, 4, 5
NOT_CONVERGED, BREAKDOWN, NONFINITE, BUDGET, PENDING = 6, 7, 8, 9, 10

CSR, COO, ELL, HYB = 0, 1, 2, 3
F64, F32, F16_ROWSCALED, C128, C64 = 0, 1, 2, 3, 4
FORMATS = {"csr": CSR, "coo": COO, "ell": ELL, "hyb": HYB}
DTYPES = {"f64": F64, "f32": F32, "f16": F16_ROWSCALED, "c128": C128, "c64": C64}
CG, BICGSTAB, GMRES, CGS, PIPECG = 0, 1, 2, 3, 4
SOLVERS = {"cg": CG, "bicgstab": BICGSTAB, "gmres": GMRES, "cgs": CGS, "pipecg": PIPECG}
HOST_PTRS, DEVICE_PTRS, SORT_AND_SUM = 0, 1, 2
IR_LAST_STEP, IR_CARRY_DIRECTION = 1, 2

(ARR_ROWPTR, ARR_COL, ARR_VAL, ARR_ROW, ARR_ELL_COL, ARR_ELL_VAL,
 ARR_COO_ROW, ARR_COO_COL, ARR_COO_VAL, ARR_SCALE) = range(10)


class Allocator(C.Structure):
    _fields_ = [("alloc", C.c_void_p), ("free", C.c_void_p), ("user", C.c_void_p)]


class ConvertOpts(C.Structure):
    _fields_ = [("ell_width", C.c_int64), ("max_ell_bytes", C.c_int64),
                ("block_nnz", C.c_int32), ("csr_kernel", C.c_int32),
                ("lanes_per_row", C.c_int32), ("rows_per_group", C.c_int32),
                ("waves_per_group", C.c_int32), ("coo_kernel", C.c_int32),
                ("col_panels", C.c_int32)]


CSR_AUTO, CSR_STREAM, CSR_VECTOR, CSR_ROWS_LDS, CSR_PRODUCTS = 0, 1, 2, 3, 4
CSR_KERNELS = {"auto": CSR_AUTO, "stream": CSR_STREAM, "vector": CSR_VECTOR,
               "rows_lds": CSR_ROWS_LDS, "products": CSR_PRODUCTS, "merge": 5}
CSR_MERGE = 5
COO_AUTO, COO_LDS, COO_RUNS = 0, 1, 2
COO_KERNELS = {"auto": COO_AUTO, "lds": COO_LDS, "runs": COO_RUNS}


class MatrixDesc(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("nnz", C.c_int64),
                ("format", C.c_int32), ("dtype", C.c_int32), ("ell_width", C.c_int64),
                ("ell_stride", C.c_int64), ("coo_nnz", C.c_int64), ("blocks", C.c_int64),
                ("bytes", C.c_int64), ("block_nnz", C.c_int32),
                ("lanes_per_row", C.c_int32), ("rows_per_group", C.c_int32),
                ("waves_per_group", C.c_int32), ("csr_kernel", C.c_int32),
                ("coo_kernel", C.c_int32), ("col_panels", C.c_int32)]


class Stop(C.Structure):
    _fields_ = [("max_iters", C.c_int64), ("rel_tol", C.c_double), ("abs_tol", C.c_double),
                ("baseline", C.c_int32), ("check_every", C.c_int32),
                ("max_replacements", C.c_int32)]


class PageRankInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("delta", C.c_double), ("status", C.c_int32)]


class SolverOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("reserved", C.c_int32), ("precond", C.c_void_p)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("relres_recurrence", C.c_double),
                ("relres_true", C.c_double), ("replacements", C.c_int64),
                ("restarts", C.c_int64), ("status", C.c_int32)]


# the same record as a numpy dtype (for arrays of results)
_SOLVE_INFO_DTYPE = np.dtype({"names": [f for f, _ in SolveInfo._fields_],
                              "formats": [np.dtype(t) for _, t in SolveInfo._fields_],
                              "offsets": [getattr(SolveInfo, f).offset
                                          for f, _ in SolveInfo._fields_],
                              "itemsize": C.sizeof(SolveInfo)})


class IRInfo(C.Structure):
    _fields_ = [("outer_iters", C.c_int64), ("inner_iters_total", C.c_int64),
                ("relres_true", C.c_double), ("status", C.c_int32)]


class BwResult(C.Structure):
    _fields_ = [("read_gbs", C.c_double), ("copy_gbs", C.c_double),
                ("triad_gbs", C.c_double), ("best_gbs", C.c_double)]


class BatchOpts(C.Structure):
    _fields_ = [("budget_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("iters_per_step", C.c_int32), ("nclasses", C.c_int32),
                ("class_max_n", C.c_int32 * 8), ("class_block", C.c_int32 * 8),
                ("class_slots", C.c_int32 * 8), ("staging_bytes", C.c_size_t)]


class BatchStats(C.Structure):
    _fields_ = [("active", C.c_int32), ("pending", C.c_int32), ("slots", C.c_int32),
                ("reserved", C.c_int32), ("completed", C.c_int64),
                ("arena_used", C.c_int64), ("arena_size", C.c_int64)]


_P = C.c_void_p
_S = C.c_int32
_I64 = C.c_int64
_SIGS = {
    "mxs_ctx_create": (_S, [C.c_int, _P, C.POINTER(Allocator), C.POINTER(_P)]),
    "mxs_ctx_destroy": (_S, [_P]),
    "mxs_ctx_set_stream": (_S, [_P, _P]),
    "mxs_ctx_synchronize": (_S, [_P]),
    "mxs_matrix_create_csr": (_S, [_P, _I64, _I64, _I64, _P, _P, _P, C.c_int, C.POINTER(_P)]),
    "mxs_matrix_convert": (_S, [_P, _P, C.c_int, C.c_int, C.POINTER(ConvertOpts), C.POINTER(_P)]),
    "mxs_matrix_info": (_S, [_P, C.POINTER(MatrixDesc)]),
    "mxs_matrix_export": (_S, [_P, _P, C.c_int, _P, C.c_size_t]),
    "mxs_matrix_destroy": (_S, [_P]),
    "mxs_matrix_create_csr_complex": (_S, [_P, _I64, _I64, _I64, _P, _P, _P, C.c_int,
                                           C.POINTER(_P)]),
    "mxs_spmv": (_S, [_P, _P, _P, _P, _P, _P]),
    "mxs_spmv_noalloc": (_S, [_P, _P, _P, _P, _P, _P]),
    "mxs_solve": (_S, [_P, C.c_int, _P, _P, _P, C.POINTER(Stop), C.POINTER(SolverOpts),
                       C.POINTER(SolveInfo)]),
    "mxs_solve_ir": (_S, [_P, _P, _P, _P, _P, C.POINTER(Stop), C.c_double, _I64, _S, _P,
                          C.POINTER(IRInfo)]),
    "mxs_graph_create": (_S, [_P, _I64, _I64, _P, _P, _S, C.POINTER(_P)]),
    "mxs_graph_destroy": (_S, [_P]),
    "mxs_graph_transition": (_P, [_P]),
    "mxs_pagerank": (_S, [_P, _P, _P, C.c_double, C.c_double, _I64, _P,
                          C.POINTER(PageRankInfo)]),
    "mxs_precond_create": (_S, [_P, _P, _S, _S, C.POINTER(_P)]),
    "mxs_precond_destroy": (_S, [_P]),
    "mxs_precond_export": (_S, [_P, _P, _P, C.c_size_t]),
    "mxs_batch_create": (_S, [_P, C.POINTER(BatchOpts), C.POINTER(_P)]),
    "mxs_batch_destroy": (_S, [_P]),
    "mxs_batch_submit": (_S, [_P, _I64, _I64, _P, _P, _P, _P, C.c_double, _I64,
                              C.POINTER(C.c_uint64)]),
    "mxs_batch_submit_many": (_S, [_P, _I64, _P, _P, _P]),
    "mxs_batch_step": (_S, [_P, C.POINTER(BatchStats)]),
    "mxs_batch_step_launch": (_S, [_P]),
    "mxs_batch_step_finish": (_S, [_P, C.POINTER(BatchStats)]),
    "mxs_batch_poll": (_S, [_P, C.c_uint64, _P, C.POINTER(SolveInfo)]),
    "mxs_batch_poll_many": (_S, [_P, _I64, _P, _P, _P, _P, _P]),
    "mxs_batch_completed": (_S, [_P, C.POINTER(C.c_uint64), _I64, C.POINTER(_I64)]),
    "mxs_batch_config": (_S, [_P, _S, C.POINTER(_S), C.POINTER(_S), C.POINTER(_S),
                              C.POINTER(_S), C.POINTER(_S)]),
    "mxs_hbm_probe": (_S, [_P, C.c_size_t, C.c_int, C.POINTER(BwResult)]),
    "mxs_gather_probe": (_S, [_P, C.c_int64, C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    "mxs_flush_cache": (_S, [_P, C.c_size_t]),
    "mxs_status_string": (C.c_char_p, [_S]),
    "mxs_last_error": (C.c_char_p, [_P]),
    "mxs_version": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    """Names of the C functions this binding declares (all must resolve)."""
    return list(_SIGS)


class MxsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{_lib.mxs_status_string(status).decode()}: {message}")
        self.status = status


def _check(status, ctx=None):
    if status != OK:
        msg = _lib.mxs_last_error(ctx.handle if ctx is not None else None)
        raise MxsError(status, msg.decode() if msg else "")


def version() -> str:
    return _lib.mxs_version().decode()


def status_string(s: int) -> str:
    return _lib.mxs_status_string(s).decode()


# ---------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class TorchAllocator:
    """Device memory for a context from torch's caching allocator: each block
    is a uint8 tensor kept alive until the library frees it.  `offset` shifts
    every pointer by that many bytes (a way to hand out misaligned blocks)."""

    def __init__(self, device: int = 0, offset: int = 0):
        self.device, self.offset = device, int(offset)
        self.live = {}
        self.calls = 0
        self._alloc = _ALLOC_FN(self._on_alloc)
        self._free = _FREE_FN(self._on_free)
        self.struct = Allocator(C.cast(self._alloc, C.c_void_p), C.cast(self._free, C.c_void_p),
                                None)

    def _on_alloc(self, nbytes, stream, user):
        import torch
        try:
            t = torch.empty(int(nbytes) + self.offset, dtype=torch.uint8,
                            device=f"cuda:{self.device}")
        except RuntimeError:
            return None
        p = t.data_ptr() + self.offset
        self.live[p] = t
        self.calls += 1
        return p

    def _on_free(self, ptr, stream, user):
        self.live.pop(ptr, None)


class Context:
    """A libmxs context bound to torch's current HIP stream on `device`;
    device memory from hipMalloc, or from `allocator` (a TorchAllocator)."""

    def __init__(self, device: int = 0, stream=None, allocator=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libmxs needs a ROCm GPU; torch.cuda is not available")
        self.device = device
        torch.cuda.set_device(device)
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        self.allocator = allocator
        h = C.c_void_p()
        a = C.byref(allocator.struct) if allocator is not None else None
        _check(_lib.mxs_ctx_create(device, C.c_void_p(s.cuda_stream), a, C.byref(h)))
        self.handle = h

    def synchronize(self):
        _check(_lib.mxs_ctx_synchronize(self.handle), self)

    def close(self):
        if getattr(self, "handle", None):
            _lib.mxs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---------------------------------------------------------------------------
# matrices
# ---------------------------------------------------------------------------
_VDT = {F64: np.float64, F32: np.float32, F16_ROWSCALED: np.uint16, C128: np.complex128,
        C64: np.complex64}


class Matrix:
    def __init__(self, ctx: Context, handle, owner=None):
        """owner: the object that owns `handle` (then close() leaves it be)."""
        self.ctx = ctx
        self.handle = handle
        self._owner = owner
        d = MatrixDesc()
        _check(_lib.mxs_matrix_info(handle, C.byref(d)), ctx)
        self.desc = d

    @classmethod
    def from_csr(cls, ctx: Context, n, ncols, rowptr, col, val,
                 sort_and_sum=False) -> "Matrix":
        """mxs_matrix_create_csr from host numpy arrays or device torch tensors
        (sort_and_sum: MXS_SORT_AND_SUM, unordered and repeated columns allowed)."""
        import torch
        if isinstance(rowptr, torch.Tensor):
            flags = DEVICE_PTRS
            for t, dt in ((rowptr, torch.int32), (col, torch.int32), (val, torch.float64)):
                if t.dtype != dt or not t.is_contiguous() or t.device.type != "cuda":
                    raise TypeError("device CSR arrays must be contiguous int32/int32/float64 on the GPU")
            ptrs = [C.c_void_p(t.data_ptr()) for t in (rowptr, col, val)]
            keep = None
            nnz = int(col.numel())
        else:
            flags = HOST_PTRS
            keep = [np.ascontiguousarray(rowptr, np.int32), np.ascontiguousarray(col, np.int32),
                    np.ascontiguousarray(val, np.float64)]
            ptrs = [a.ctypes.data_as(C.c_void_p) for a in keep]
            nnz = len(keep[1])
        if sort_and_sum:
            flags |= SORT_AND_SUM
        h = C.c_void_p()
        _check(_lib.mxs_matrix_create_csr(ctx.handle, int(n), int(ncols), nnz, *ptrs, flags,
                                          C.byref(h)), ctx)
        return cls(ctx, h)

    @classmethod
    def from_host(cls, ctx: Context, A) -> "Matrix":
        """From any object with n, ncols, rowptr, col, val (numpy)."""
        return cls.from_csr(ctx, A.n, A.ncols, A.rowptr, A.col, A.val)

    @classmethod
    def from_host_complex(cls, ctx: Context, n, ncols, rowptr, col, val,
                          sort_and_sum=False) -> "Matrix":
        """mxs_matrix_create_csr_complex from host numpy arrays (val complex)."""
        rp = np.ascontiguousarray(rowptr, np.int32)
        ci = np.ascontiguousarray(col, np.int32)
        v = np.ascontiguousarray(np.asarray(val, np.complex128))
        h = C.c_void_p()
        _check(_lib.mxs_matrix_create_csr_complex(ctx.handle, int(n), int(ncols), len(ci),
                                                  rp.ctypes.data_as(_P), ci.ctypes.data_as(_P),
                                                  v.ctypes.data_as(_P),
                                                  HOST_PTRS | (SORT_AND_SUM if sort_and_sum else 0),
                                                  C.byref(h)),
               ctx)
        return cls(ctx, h)

    def convert(self, fmt="csr", dtype="f64", ell_width=0, max_ell_bytes=0,
                block_nnz=0, csr_kernel="auto", lanes_per_row=0,
                rows_per_group=0, waves_per_group=0, coo_kernel="auto",
                col_panels=0) -> "Matrix":
        o = ConvertOpts(int(ell_width), int(max_ell_bytes), int(block_nnz),
                        CSR_KERNELS.get(csr_kernel, csr_kernel), int(lanes_per_row),
                        int(rows_per_group), int(waves_per_group),
                        COO_KERNELS.get(coo_kernel, coo_kernel), int(col_panels))
        h = C.c_void_p()
        _check(_lib.mxs_matrix_convert(self.ctx.handle, self.handle, FORMATS.get(fmt, fmt),
                                       DTYPES.get(dtype, dtype), C.byref(o), C.byref(h)),
               self.ctx)
        return Matrix(self.ctx, h)

    @property
    def n(self):
        return self.desc.nrows

    @property
    def dtype(self):
        return self.desc.dtype

    def info(self) -> dict:
        d = self.desc
        return {f: getattr(d, f) for f, _ in MatrixDesc._fields_}

    def export(self, which: int) -> np.ndarray:
        d = self.desc
        vdt = _VDT[d.dtype]
        sizes = {
            ARR_ROWPTR: (d.nrows + 1, np.int32), ARR_COL: (d.nnz, np.int32),
            ARR_VAL: (d.nnz, vdt), ARR_ROW: (d.nnz, np.int32),
            ARR_ELL_COL: (d.ell_width * d.ell_stride, np.int32),
            ARR_ELL_VAL: (d.ell_width * d.ell_stride, vdt),
            ARR_COO_ROW: (d.coo_nnz, np.int32), ARR_COO_COL: (d.coo_nnz, np.int32),
            ARR_COO_VAL: (d.coo_nnz, vdt), ARR_SCALE: (d.nrows, np.float32),
        }
        count, dt = sizes[which]
        out = np.empty(int(count), dt)
        _check(_lib.mxs_matrix_export(self.ctx.handle, self.handle, which,
                                      out.ctypes.data_as(C.c_void_p), out.nbytes), self.ctx)
        return out

    def close(self):
        if getattr(self, "handle", None):
            if getattr(self, "_owner", None) is None:
                _lib.mxs_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """mxs_graph_create: a directed graph by in-links (row j lists the
    sources of the edges into j) with its transition matrix on the GPU."""

    def __init__(self, ctx: Context, G):
        rp = np.ascontiguousarray(G.rowptr, np.int32)
        ci = np.ascontiguousarray(G.col, np.int32)
        h = C.c_void_p()
        _check(_lib.mxs_graph_create(ctx.handle, int(G.n), len(ci), rp.ctypes.data_as(_P),
                                     ci.ctypes.data_as(_P), HOST_PTRS, C.byref(h)), ctx)
        self.ctx = ctx
        self.handle = h
        self.n = int(G.n)

    def transition(self) -> "Matrix":
        """T (owned by the graph): convert it to run PageRank in another format."""
        return Matrix(self.ctx, _lib.mxs_graph_transition(self.handle), owner=self)

    def close(self):
        if getattr(self, "handle", None):
            _lib.mxs_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class PageRankResult:
    status: int
    iters: int
    delta: float


def pagerank(ctx: Context, G: Graph, x, damping=0.85, tol=1e-10, max_iters=0, op=None,
             raise_on_error=True) -> PageRankResult:
    """mxs_pagerank into the FP64 device vector x (n entries)."""
    import torch
    info = PageRankInfo()
    s = _lib.mxs_pagerank(ctx.handle, G.handle, op.handle if op is not None else None,
                          float(damping), float(tol), int(max_iters), _vec(x, G.n, torch.float64),
                          C.byref(info))
    if raise_on_error and s != OK:
        _check(s, ctx)
    return PageRankResult(s, info.iters, info.delta)


PRECOND_JACOBI, PRECOND_BLOCK_JACOBI = 1, 2
PRECONDS = {"jacobi": PRECOND_JACOBI, "block_jacobi": PRECOND_BLOCK_JACOBI}


class Precond:
    """mxs_precond_create: Jacobi or block-Jacobi preconditioner of an F64
    CSR matrix (device-resident, FP64 and FP32 copies)."""

    def __init__(self, ctx: Context, A: "Matrix", kind="jacobi", block_size=1):
        h = C.c_void_p()
        _check(_lib.mxs_precond_create(ctx.handle, A.handle, PRECONDS.get(kind, kind),
                                       int(block_size), C.byref(h)), ctx)
        self.ctx = ctx
        self.handle = h
        self.kind = PRECONDS.get(kind, kind)
        self.n = A.n
        self.bs = int(block_size) if self.kind == PRECOND_BLOCK_JACOBI else 1

    def export(self) -> np.ndarray:
        cnt = self.n if self.kind == PRECOND_JACOBI else -(-self.n // self.bs) * self.bs ** 2
        out = np.empty(cnt, np.float64)
        _check(_lib.mxs_precond_export(self.ctx.handle, self.handle,
                                       out.ctypes.data_as(C.c_void_p), out.nbytes), self.ctx)
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib.mxs_precond_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# operations
# ---------------------------------------------------------------------------
def _vec(t, n, want):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("vectors must be torch tensors on the GPU")
    if t.dtype != want or not t.is_contiguous() or t.numel() != n:
        raise TypeError(f"expected a contiguous {want} vector of {n} entries, "
                        f"got {t.dtype} {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _compute_dtype(A: Matrix):
    import torch
    return {F64: torch.float64, C128: torch.complex128,
            C64: torch.complex64}.get(A.dtype, torch.float32)


def spmv(ctx: Context, A: Matrix, x, y, alpha=1.0, beta=0.0, noalloc=False):
    """mxs_spmv: y = alpha*A*x + beta*y (asynchronous on the ctx stream);
    noalloc=True calls mxs_spmv_noalloc (scratch from the library's fixed
    per-GPU array, no allocation)."""
    if A.dtype in (C128, C64):
        ct = C.c_double if A.dtype == C128 else C.c_float
        a = (ct * 2)(complex(alpha).real, complex(alpha).imag)
        b = (ct * 2)(complex(beta).real, complex(beta).imag)
    else:
        ct = C.c_double if A.dtype == F64 else C.c_float
        a, b = ct(alpha), ct(beta)
    dt = _compute_dtype(A)
    fn = _lib.mxs_spmv_noalloc if noalloc else _lib.mxs_spmv
    _check(fn(ctx.handle, C.byref(a), A.handle, _vec(x, A.desc.ncols, dt),
              C.byref(b), _vec(y, A.n, dt)), ctx)


@dataclass
class Result:
    status: int
    iters: int
    relres_recurrence: float
    relres_true: float
    replacements: int = 0
    restarts: int = 0


def solve(ctx: Context, kind, A: Matrix, b, x, tol=1e-10, max_iters=0, abs_tol=0.0,
          baseline=0, check_every=0, max_replacements=-1, restart=30, raise_on_error=True,
          precond: Precond | None = None):
    """mxs_solve: A x = b with x holding x0 on entry (FP64 device vectors);
    `precond` makes CG the preconditioned CG."""
    import torch
    st = Stop(int(max_iters), float(tol), float(abs_tol), int(baseline), int(check_every),
              int(max_replacements))
    opts = SolverOpts(int(restart), 0, precond.handle if precond is not None else None)
    info = SolveInfo()
    s = _lib.mxs_solve(ctx.handle, SOLVERS.get(kind, kind), A.handle,
                       _vec(b, A.n, torch.float64), _vec(x, A.n, torch.float64), C.byref(st),
                       C.byref(opts), C.byref(info))
    if raise_on_error and s not in (OK,):
        _check(s, ctx)
    return Result(s, info.iters, info.relres_recurrence, info.relres_true, info.replacements,
                  info.restarts)


@dataclass
class IRResult:
    status: int
    outer_iters: int
    inner_iters_total: int
    relres_true: float


def solve_ir(ctx: Context, A64: Matrix, Alow: Matrix, b, x, tol=1e-10, outer_max=50,
             inner_tol=1e-4, inner_max=20000, last_step_variant=False, check_every=0,
             raise_on_error=True, precond: Precond | None = None, carry_direction=False):
    """mxs_solve_ir: FP64 refinement around an FP32 CG on the low-precision
    copy (preconditioned with the FP32 copy of `precond` when given);
    `carry_direction` keeps the inner CG's direction across refinement steps
    (MXS_IR_CARRY_DIRECTION)."""
    flags = (IR_LAST_STEP if last_step_variant else 0) | \
        (IR_CARRY_DIRECTION if carry_direction else 0)
    import torch
    st = Stop(int(outer_max), float(tol), 0.0, 0, int(check_every), -1)
    info = IRInfo()
    s = _lib.mxs_solve_ir(ctx.handle, A64.handle, Alow.handle, _vec(b, A64.n, torch.float64),
                          _vec(x, A64.n, torch.float64), C.byref(st), float(inner_tol),
                          int(inner_max), flags,
                          precond.handle if precond is not None else None, C.byref(info))
    if raise_on_error and s != OK:
        _check(s, ctx)
    return IRResult(s, info.outer_iters, info.inner_iters_total, info.relres_true)


def hbm_probe(ctx: Context, nbytes=1 << 30, reps=5) -> dict:
    r = BwResult()
    _check(_lib.mxs_hbm_probe(ctx.handle, int(nbytes), int(reps), C.byref(r)), ctx)
    return {"read_gbs": r.read_gbs, "copy_gbs": r.copy_gbs, "triad_gbs": r.triad_gbs,
            "best_gbs": r.best_gbs}


def _as(a, dt):
    """a itself when it is already a C-contiguous array of dtype dt."""
    if type(a) is np.ndarray and a.dtype == dt and a.flags.c_contiguous:
        return a
    return np.ascontiguousarray(a, dt)


def gather_probe(ctx: Context, nx: int, count: int, value_bytes=8, reps=5) -> float:
    """Random gathers per second from an x of nx values (see mxs_gather_probe)."""
    r = C.c_double(0.0)
    _check(_lib.mxs_gather_probe(ctx.handle, int(nx), int(count), int(value_bytes), int(reps),
                                 C.byref(r)), ctx)
    return r.value


def flush_cache(ctx: Context, nbytes=1 << 30):
    _check(_lib.mxs_flush_cache(ctx.handle, int(nbytes)), ctx)


# ---------------------------------------------------------------------------
# batched CG engine
# ---------------------------------------------------------------------------
class Batch:
    """mxs_batch_*: continuous batching of independent SPD solves.

    classes: None for the library defaults, or a list of
    (max_n, threads_per_system, slots) tuples (slots 0 = even share)."""

    def __init__(self, ctx: Context, budget_bytes=2 << 30, max_slots=512,
                 iters_per_step=16, classes=None, staging_bytes=0):
        o = BatchOpts()
        o.budget_bytes = int(budget_bytes)
        o.staging_bytes = int(staging_bytes)
        o.max_slots = int(max_slots)
        o.iters_per_step = int(iters_per_step)
        if classes:
            o.nclasses = len(classes)
            for i, (mn, blk, sl) in enumerate(classes):
                o.class_max_n[i] = int(mn)
                o.class_block[i] = int(blk)
                o.class_slots[i] = int(sl)
        h = C.c_void_p()
        _check(_lib.mxs_batch_create(ctx.handle, C.byref(o), C.byref(h)), ctx)
        self.ctx = ctx
        self.handle = h
        self._buf = (C.c_uint64 * 4096)()

    def submit(self, A, b, tol=1e-10, max_iters=0) -> int:
        rp = np.ascontiguousarray(A.rowptr, np.int32)
        ci = np.ascontiguousarray(A.col, np.int32)
        v = np.ascontiguousarray(A.val, np.float64)
        bb = np.ascontiguousarray(b, np.float64)
        t = C.c_uint64()
        _check(_lib.mxs_batch_submit(self.handle, int(A.n), len(ci), rp.ctypes.data_as(_P),
                                     ci.ctypes.data_as(_P), v.ctypes.data_as(_P),
                                     bb.ctypes.data_as(_P), float(tol), int(max_iters),
                                     C.byref(t)), self.ctx)
        return t.value

    # mxs_batch_request, field for field
    _REQ = np.dtype([("n", "<i8"), ("nnz", "<i8"), ("rowptr", "<u8"), ("col", "<u8"),
                     ("val", "<u8"), ("b", "<u8"), ("rel_tol", "<f8"), ("max_iters", "<i8"),
                     ("mode", "<i4"), ("reserved", "<i4"), ("inner_rel_tol", "<f8")])
    MODES = {"f64": 0, "ir32": 1}

    def submit_many(self, systems, tol=1e-10, max_iters=0, mode="f64", inner_tol=0.0):
        """Queues [(A, b), ...] in one call (validated and packed on host
        threads).  mode "f64" (CG in FP64) or "ir32" (FP32-storage CG inside
        FP64 iterative refinement, inner tolerance inner_tol, 0 = 1e-4).
        Returns (tickets, statuses) as numpy arrays; ticket 0 marks a
        rejected request, whose status says why."""
        md = self.MODES.get(mode, mode)
        k = len(systems)
        req = np.zeros(k, self._REQ)
        keep = []
        ns = np.empty(k, np.int64)
        nnzs = np.empty(k, np.int64)
        ptrs = np.empty((4, k), np.uint64)
        for i, (A, b) in enumerate(systems):
            arrs = (_as(A.rowptr, np.int32), _as(A.col, np.int32), _as(A.val, np.float64),
                    _as(b, np.float64))
            keep.append(arrs)
            ns[i] = A.n
            nnzs[i] = arrs[1].size
            for q in range(4):
                ptrs[q, i] = arrs[q].__array_interface__["data"][0]
        req["n"] = ns
        req["nnz"] = nnzs
        for q, f in enumerate(("rowptr", "col", "val", "b")):
            req[f] = ptrs[q]
        req["rel_tol"] = tol
        req["max_iters"] = max_iters
        req["mode"] = md
        req["inner_rel_tol"] = inner_tol
        tickets = np.zeros(k, np.uint64)
        statuses = np.zeros(k, np.int32)
        _check(_lib.mxs_batch_submit_many(self.handle, k, req.ctypes.data, tickets.ctypes.data,
                                          statuses.ctypes.data), self.ctx)
        del keep
        return tickets, statuses

    def step(self) -> dict:
        s = BatchStats()
        _check(_lib.mxs_batch_step(self.handle, C.byref(s)), self.ctx)
        return {f: getattr(s, f) for f, _ in BatchStats._fields_}

    def step_launch(self):
        """First half of step(): admit and launch without waiting."""
        _check(_lib.mxs_batch_step_launch(self.handle), self.ctx)

    def step_finish(self) -> dict:
        """Second half of step(): wait, retire, report."""
        s = BatchStats()
        _check(_lib.mxs_batch_step_finish(self.handle, C.byref(s)), self.ctx)
        return {f: getattr(s, f) for f, _ in BatchStats._fields_}

    def completed(self) -> list:
        out = []
        while True:
            cnt = C.c_int64()
            _check(_lib.mxs_batch_completed(self.handle, self._buf, len(self._buf),
                                            C.byref(cnt)), self.ctx)
            out.extend(self._buf[i] for i in range(cnt.value))
            if cnt.value < len(self._buf):
                return out

    def poll(self, ticket: int, n: int):
        """(status, x or None, Result); status PENDING while running."""
        x = np.empty(int(n), np.float64)
        info = SolveInfo()
        s = _lib.mxs_batch_poll(self.handle, int(ticket), x.ctypes.data_as(_P), C.byref(info))
        if s == PENDING:
            return s, None, None
        if s == INVALID_ARG:
            _check(s, self.ctx)
        return s, x, Result(s, info.iters, info.relres_recurrence, info.relres_true,
                            info.replacements, info.restarts)

    def poll_many(self, tickets, ns):
        """mxs_batch_poll_many: (statuses, x, off, info) for the tickets, with
        ns their system sizes.  Request i's x is x[off[i]:off[i] + ns[i]] (one
        shared buffer); info is a structured array of SolveInfo records
        (fields iters, relres_recurrence, relres_true, replacements,
        restarts, status).  A pending request keeps status PENDING and its
        slice of x is left unwritten."""
        t = np.ascontiguousarray(np.asarray(tickets, dtype=np.uint64))
        ns = np.asarray(ns, dtype=np.int64)
        k = int(t.size)
        off = np.zeros(k, np.int64)
        if k > 1:
            np.cumsum(ns[:-1], out=off[1:])
        x = np.empty(int(ns.sum()), np.float64)
        info = np.zeros(k, _SOLVE_INFO_DTYPE)
        sts = np.zeros(k, np.int32)
        _check(_lib.mxs_batch_poll_many(self.handle, k, t.ctypes.data, x.ctypes.data,
                                        off.ctypes.data, info.ctypes.data, sts.ctypes.data),
               self.ctx)
        if (sts == INVALID_ARG).any():
            _check(INVALID_ARG, self.ctx)
        return sts, x, off, info

    def config(self, cls: int) -> dict:
        vals = [C.c_int32() for _ in range(5)]
        _check(_lib.mxs_batch_config(self.handle, int(cls), *[C.byref(v) for v in vals]),
               self.ctx)
        return dict(zip(("max_n", "block", "rows_per_thread", "slots", "uses_lds"),
                        (v.value for v in vals)))

    def close(self):
        if getattr(self, "handle", None):
            _lib.mxs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
