"""CPU oracle for the SpMV + Krylov hot path (TEST INFRASTRUCTURE ONLY).

This package wraps ``oracle.c``, a plain single-threaded FP64 C implementation
of the operations the GPU library computes: CSR/COO/ELL/hybrid storage and
conversions, the sparse matrix-vector product, CG, pipelined CG, BiCGSTAB,
CGS, GMRES(m),
Jacobi and block-Jacobi preconditioned CG, PageRank by power iteration,
mixed-precision iterative refinement and a dense LU solver.  Each C function
cites the passage of the paper (or the textbook the paper refers to) that it
writes out.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library neither links nor calls
it, and the two share no code: the only thing both sides consume is the
seeded input generators in ``paper_2103_10116_amd.inputs``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source built with OpenMP: the host baseline's all-core timing only
# (parity always uses the single-thread build)
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

OK, INVALID_ARG, INVALID_MATRIX, UNSUPPORTED = 0, 1, 2, 3
NOT_CONVERGED, BREAKDOWN, NONFINITE = 6, 7, 8


def _compile(out: str, openmp: bool) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
         *(["-fopenmp"] if openmp else []),
         "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
         _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, no FP contraction, no fast-math),
    and liboracle_omp.so, the same source with OpenMP (timing only)."""
    for out, omp in ((_LIB, False), (_LIB_OMP, True)):
        if force or not os.path.exists(out):
            _compile(out, omp)
    return _LIB


_lib = None
_libs = {}
_threads = 1


def _load(path, openmp):
    if path not in _libs:
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            _compile(path, openmp)
        L = C.CDLL(path)
        _declare(L)
        _libs[path] = L
    return _libs[path]


def use_threads(n: int) -> int:
    """n == 1: the single-thread parity build (the default); n > 1: the
    OpenMP build of the same source on n threads, for host-baseline timing
    (its inner products are summed in another order).  Returns the previous
    setting."""
    global _lib, _threads
    prev = _threads
    _threads = max(1, int(n))
    if _threads == 1:
        _lib = _load(_LIB, False)
    else:
        _lib = _load(_LIB_OMP, True)
        C.CDLL("libgomp.so.1").omp_set_num_threads(_threads)
    return prev


def lib():
    global _lib
    if _lib is None:
        _lib = _load(_LIB, False)
    return _lib


class Stop(C.Structure):
    _fields_ = [("max_iters", C.c_int64), ("rel_tol", C.c_double),
                ("abs_tol", C.c_double), ("baseline", C.c_int32),
                ("max_replacements", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("relres_recurrence", C.c_double),
                ("relres_true", C.c_double), ("replacements", C.c_int64),
                ("restarts", C.c_int64)]


class IRInfo(C.Structure):
    _fields_ = [("outer_iters", C.c_int64), ("inner_iters_total", C.c_int64),
                ("relres_true", C.c_double)]


_P = C.c_void_p
_I64 = C.c_int64
_D = C.c_double


def _declare(L):
    sig = {
        "orc_csr_validate": (C.c_int, [_I64, _I64, _I64, _P, _P]),
        "orc_csr_sort_and_sum": (C.c_int, [_I64, _I64, _I64, _P, _P, _P, C.c_int, _P, _P, _P,
                                           C.POINTER(_I64)]),
        "orc_csr_to_coo": (None, [_I64, _P, _P]),
        "orc_coo_to_csr": (None, [_I64, _I64, _P, _P]),
        "orc_ell_width": (_I64, [_I64, _P]),
        "orc_ell_stride": (_I64, [_I64]),
        "orc_csr_to_ell": (None, [_I64, _P, _P, _P, _I64, _I64, _P, _P]),
        "orc_hyb_width": (_I64, [_I64, _P, C.c_int]),
        "orc_csr_to_hyb": (_I64, [_I64, _P, _P, _P, _I64, _I64, _P, _P, _P, _P, _P]),
        "orc_cast_f32": (C.c_int, [_I64, _P, _P]),
        "orc_f64_to_f16": (C.c_uint16, [_D]),
        "orc_f16_to_f64": (_D, [C.c_uint16]),
        "orc_rowscale_f16": (C.c_int, [_I64, _P, _P, _P, _P]),
        "orc_spmv_csr": (None, [_I64, _P, _P, _P, _P, _D, _D, _P, C.c_int]),
        "orc_spmv_coo": (None, [_I64, _I64, _P, _P, _P, _P, _D, _D, _P]),
        "orc_spmv_ell": (None, [_I64, _I64, _I64, _P, _P, _P, _D, _D, _P]),
        "orc_spmv_hyb": (None, [_I64, _I64, _I64, _P, _P, _I64, _P, _P, _P, _P, _D, _D, _P]),
        "orc_spmv_csr_f16": (None, [_I64, _P, _P, _P, _P, _P, _D, _D, _P]),
        "orc_absrow": (None, [_I64, _P, _P, _P, _P, _P]),
        "orc_spmv_csr_z": (None, [_I64, _P, _P, _P, _P, _P, _P, _P]),
        "orc_absrow_z": (None, [_I64, _P, _P, _P, _P, _P]),
        "orc_dense_matvec": (None, [_I64, _I64, _P, _P, _P]),
        "orc_dense_lu_solve": (C.c_int, [_I64, _P, _P, _P]),
        "orc_cg": (C.c_int, [_I64, _P, _P, _P, _P, _P, C.POINTER(Stop), C.POINTER(Info), _P, _I64]),
        "orc_bicgstab": (C.c_int, [_I64, _P, _P, _P, _P, _P, C.POINTER(Stop), C.POINTER(Info)]),
        "orc_cgs": (C.c_int, [_I64, _P, _P, _P, _P, _P, C.POINTER(Stop), C.POINTER(Info)]),
        "orc_pipecg": (C.c_int, [_I64, _P, _P, _P, _P, _P, C.POINTER(Stop), C.POINTER(Info)]),
        "orc_pagerank": (C.c_int, [_I64, _P, _P, _D, _D, _I64, _P, C.POINTER(_I64), C.POINTER(_D)]),
        "orc_gmres": (C.c_int, [_I64, _P, _P, _P, _P, _P, _I64, C.POINTER(Stop), C.POINTER(Info), _P, _I64]),
        "orc_ir": (C.c_int, [_I64, _P, _P, _P, C.c_int, _P, _P, _P, _P, _P, _D, _I64, _D, _I64, C.c_int, C.POINTER(IRInfo)]),
        "orc_ir_pc": (C.c_int, [_I64, _P, _P, _P, C.c_int, _P, _P, _P, _P, _P, _D, _I64, _D, _I64, C.c_int, C.c_int, _I64, _P, C.POINTER(IRInfo)]),
        "orc_jacobi": (C.c_int, [_I64, _P, _P, _P, _P]),
        "orc_block_jacobi": (C.c_int, [_I64, _P, _P, _P, _I64, _P]),
        "orc_prec_apply": (None, [_I64, C.c_int, _I64, _P, _P, _P]),
        "orc_pcg": (C.c_int, [_I64, _P, _P, _P, C.c_int, _I64, _P, _P, _P, C.POINTER(Stop), C.POINTER(Info)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


# ---------------------------------------------------------------------------
# array helpers
# ---------------------------------------------------------------------------
def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _csr(A):
    rp = _c(A.rowptr, np.int32)
    ci = _c(A.col, np.int32)
    v = _c(A.val, np.float64)
    return int(A.n), rp, ci, v


# ---------------------------------------------------------------------------
# ingest and conversions
# ---------------------------------------------------------------------------
def validate(n, ncols, rowptr, col) -> int:
    rp = _c(rowptr, np.int32)
    ci = _c(col, np.int32)
    return lib().orc_csr_validate(n, ncols, int(rp[-1]) if len(rp) else 0, _p(rp), _p(ci))


def csr_sort_and_sum(n, ncols, rowptr, col, val):
    """(status, CSRMatrix-like tuple (rowptr, col, val)) of the row-grouped
    list with each row ordered by column and repeated columns summed in input
    order; val may be real (float64) or complex (complex128)."""
    rp = _c(rowptr, np.int32)
    ci = _c(col, np.int32)
    cplx = np.iscomplexobj(val)
    v = _c(np.asarray(val, np.complex128).view(np.float64) if cplx else val, np.float64)
    nnz = int(rp[n]) if len(rp) > n else 0
    vpe = 2 if cplx else 1
    orp = np.zeros(n + 1, np.int32)
    oc = np.zeros(max(nnz, 1), np.int32)
    ov = np.zeros(max(nnz, 1) * vpe, np.float64)
    nout = _I64(0)
    st = lib().orc_csr_sort_and_sum(n, ncols, len(ci), _p(rp), _p(ci), _p(v), vpe, _p(orp),
                                    _p(oc), _p(ov), C.byref(nout))
    if st != OK:
        return st, None
    k = nout.value
    ov = ov[:k * vpe]
    return st, (orp, oc[:k].copy(), (ov.view(np.complex128) if cplx else ov).copy())


def csr_to_coo(n, rowptr):
    rp = _c(rowptr, np.int32)
    row = np.empty(int(rp[n]), np.int32)
    lib().orc_csr_to_coo(n, _p(rp), _p(row))
    return row


def coo_to_csr(n, row):
    r = _c(row, np.int32)
    rp = np.empty(n + 1, np.int32)
    lib().orc_coo_to_csr(n, len(r), _p(r), _p(rp))
    return rp


@dataclass
class ELL:
    n: int
    K: int
    stride: int
    col: np.ndarray
    val: np.ndarray


@dataclass
class HYB:
    n: int
    K: int
    stride: int
    ecol: np.ndarray
    eval: np.ndarray
    crow: np.ndarray
    ccol: np.ndarray
    cval: np.ndarray


def csr_to_ell(A, K=None) -> ELL:
    n, rp, ci, v = _csr(A)
    L = lib()
    if K is None:
        K = L.orc_ell_width(n, _p(rp))
    stride = L.orc_ell_stride(n)
    ecol = np.empty(K * stride, np.int32)
    ev = np.empty(K * stride, np.float64)
    L.orc_csr_to_ell(n, _p(rp), _p(ci), _p(v), K, stride, _p(ecol), _p(ev))
    return ELL(n, K, stride, ecol, ev)


def hyb_width(n, rowptr, value_bytes) -> int:
    rp = _c(rowptr, np.int32)
    return lib().orc_hyb_width(n, _p(rp), value_bytes)


def csr_to_hyb(A, value_bytes=8, K=None) -> HYB:
    n, rp, ci, v = _csr(A)
    L = lib()
    if K is None:
        K = L.orc_hyb_width(n, _p(rp), value_bytes)
    stride = L.orc_ell_stride(n)
    lens = np.diff(rp.astype(np.int64))
    cn = int(np.maximum(lens - K, 0).sum())
    ecol = np.empty(K * stride, np.int32)
    ev = np.empty(K * stride, np.float64)
    crow = np.empty(cn, np.int32)
    ccol = np.empty(cn, np.int32)
    cval = np.empty(cn, np.float64)
    got = L.orc_csr_to_hyb(n, _p(rp), _p(ci), _p(v), K, stride, _p(ecol), _p(ev),
                           _p(crow), _p(ccol), _p(cval))
    assert got == cn
    return HYB(n, K, stride, ecol, ev, crow, ccol, cval)


def cast_f32(val):
    v = _c(val, np.float64)
    out = np.empty(len(v), np.float32)
    st = lib().orc_cast_f32(len(v), _p(v), _p(out))
    return st, out


def f64_to_f16_bits(vals):
    L = lib()
    return np.array([L.orc_f64_to_f16(float(v)) for v in np.ravel(vals)], np.uint16)


def f16_bits_to_f64(bits):
    L = lib()
    return np.array([L.orc_f16_to_f64(int(b)) for b in np.ravel(bits)], np.float64)


def rowscale_f16(A):
    n, rp, ci, v = _csr(A)
    h = np.empty(len(v), np.uint16)
    s = np.empty(n, np.float32)
    st = lib().orc_rowscale_f16(n, _p(rp), _p(v), _p(h), _p(s))
    return st, h, s


# ---------------------------------------------------------------------------
# SpMV
# ---------------------------------------------------------------------------
def _y(n, y, beta):
    if y is None:
        out = np.zeros(n, np.float64)
    else:
        out = np.array(y, dtype=np.float64, copy=True)
    return out


def spmv_csr(A, x, alpha=1.0, beta=0.0, y=None, mode="accurate"):
    n, rp, ci, v = _csr(A)
    xx = _c(x, np.float64)
    out = _y(n, y, beta)
    lib().orc_spmv_csr(n, _p(rp), _p(ci), _p(v), _p(xx), alpha, beta, _p(out),
                       0 if mode == "accurate" else 1)
    return out



def spmv_csr_z(n, rowptr, col, val, x, alpha=1.0, beta=0.0, y=None):
    """Complex CSR product; val, x, y complex128 numpy arrays."""
    rp = _c(rowptr, np.int32)
    ci = _c(col, np.int32)
    v = _c(np.asarray(val, np.complex128).view(np.float64), np.float64)
    xx = _c(np.asarray(x, np.complex128).view(np.float64), np.float64)
    out = np.zeros(2 * n) if y is None else _c(np.asarray(y, np.complex128).view(np.float64),
                                                np.float64).copy()
    a = np.array([complex(alpha).real, complex(alpha).imag])
    b = np.array([complex(beta).real, complex(beta).imag])
    lib().orc_spmv_csr_z(int(n), _p(rp), _p(ci), _p(v), _p(xx), _p(a), _p(b), _p(out))
    return out.view(np.complex128)


def absrow_z(n, rowptr, col, val, x):
    rp = _c(rowptr, np.int32)
    ci = _c(col, np.int32)
    v = _c(np.asarray(val, np.complex128).view(np.float64), np.float64)
    xx = _c(np.asarray(x, np.complex128).view(np.float64), np.float64)
    out = np.zeros(int(n))
    lib().orc_absrow_z(int(n), _p(rp), _p(ci), _p(v), _p(xx), _p(out))
    return out


def spmv_coo(n, row, col, val, x, alpha=1.0, beta=0.0, y=None):
    r = _c(row, np.int32)
    c = _c(col, np.int32)
    v = _c(val, np.float64)
    xx = _c(x, np.float64)
    out = _y(n, y, beta)
    lib().orc_spmv_coo(n, len(r), _p(r), _p(c), _p(v), _p(xx), alpha, beta, _p(out))
    return out


def spmv_ell(E: ELL, x, alpha=1.0, beta=0.0, y=None):
    c = _c(E.col, np.int32)
    v = _c(E.val, np.float64)
    xx = _c(x, np.float64)
    out = _y(E.n, y, beta)
    lib().orc_spmv_ell(E.n, E.K, E.stride, _p(c), _p(v), _p(xx), alpha, beta, _p(out))
    return out


def spmv_hyb(Hm: HYB, x, alpha=1.0, beta=0.0, y=None):
    ec = _c(Hm.ecol, np.int32)
    ev = _c(Hm.eval, np.float64)
    cr = _c(Hm.crow, np.int32)
    cc = _c(Hm.ccol, np.int32)
    cv = _c(Hm.cval, np.float64)
    xx = _c(x, np.float64)
    out = _y(Hm.n, y, beta)
    lib().orc_spmv_hyb(Hm.n, Hm.K, Hm.stride, _p(ec), _p(ev), len(cr), _p(cr), _p(cc),
                       _p(cv), _p(xx), alpha, beta, _p(out))
    return out


def spmv_csr_f16(A, h, scale, x, alpha=1.0, beta=0.0, y=None):
    n, rp, ci, _ = _csr(A)
    hh = _c(h, np.uint16)
    ss = _c(scale, np.float32)
    xx = _c(x, np.float64)
    out = _y(n, y, beta)
    lib().orc_spmv_csr_f16(n, _p(rp), _p(ci), _p(hh), _p(ss), _p(xx), alpha, beta, _p(out))
    return out


def absrow(A, x):
    n, rp, ci, v = _csr(A)
    xx = _c(x, np.float64)
    out = np.empty(n, np.float64)
    lib().orc_absrow(n, _p(rp), _p(ci), _p(v), _p(xx), _p(out))
    return out


# ---------------------------------------------------------------------------
# dense
# ---------------------------------------------------------------------------
def dense_matvec(M, x):
    M = _c(M, np.float64)
    xx = _c(x, np.float64)
    y = np.empty(M.shape[0], np.float64)
    lib().orc_dense_matvec(M.shape[0], M.shape[1], _p(M), _p(xx), _p(y))
    return y


def lu_solve(M, b):
    M = _c(M, np.float64)
    bb = _c(b, np.float64)
    x = np.empty(M.shape[0], np.float64)
    st = lib().orc_dense_lu_solve(M.shape[0], _p(M), _p(bb), _p(x))
    return st, x


# ---------------------------------------------------------------------------
# solvers
# ---------------------------------------------------------------------------
def _stop(tol, maxit, abs_tol=0.0, baseline=0, max_replacements=3):
    return Stop(int(maxit), float(tol), float(abs_tol), int(baseline), int(max_replacements))


@dataclass
class SolveResult:
    status: int
    x: np.ndarray
    iters: int
    relres_true: float
    relres_recurrence: float
    replacements: int
    restarts: int
    hist: np.ndarray | None = None


def _result(st, x, info, hist=None):
    return SolveResult(st, x, info.iters, info.relres_true, info.relres_recurrence,
                       info.replacements, info.restarts, hist)


def cg(A, b, x0=None, tol=1e-10, maxit=20000, abs_tol=0.0, hist=False, baseline=0):
    n, rp, ci, v = _csr(A)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64, copy=True)
    info = Info()
    st_ = _stop(tol, maxit, abs_tol, baseline)
    h = np.zeros(2 * maxit if hist else 0, np.float64)
    st = lib().orc_cg(n, _p(rp), _p(ci), _p(v), _p(bb), _p(x), C.byref(st_), C.byref(info),
                      _p(h) if hist else None, len(h))
    return _result(st, x, info, h[: 2 * info.iters].reshape(-1, 2) if hist else None)


PRECONDS = {"jacobi": 1, "block_jacobi": 2}


@dataclass
class Precond:
    kind: int
    bs: int
    minv: np.ndarray   # Jacobi: 1/a_ii; block Jacobi: column-major bs x bs inverses


def jacobi(A) -> tuple[int, Precond]:
    n, rp, ci, v = _csr(A)
    d = np.zeros(n)
    st = lib().orc_jacobi(n, _p(rp), _p(ci), _p(v), _p(d))
    return st, Precond(1, 1, d)


def block_jacobi(A, bs) -> tuple[int, Precond]:
    n, rp, ci, v = _csr(A)
    nb = -(-n // bs)
    m = np.zeros(nb * bs * bs)
    st = lib().orc_block_jacobi(n, _p(rp), _p(ci), _p(v), int(bs), _p(m))
    return st, Precond(2, int(bs), m)


def prec_apply(M: Precond, r):
    rr = _c(r, np.float64)
    z = np.zeros_like(rr)
    lib().orc_prec_apply(len(rr), M.kind, M.bs, _p(_c(M.minv, np.float64)), _p(rr), _p(z))
    return z


def pcg(A, b, M: Precond, x0=None, tol=1e-10, maxit=20000, abs_tol=0.0, baseline=0):
    n, rp, ci, v = _csr(A)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64, copy=True)
    info = Info()
    mv = _c(M.minv, np.float64)
    st = lib().orc_pcg(n, _p(rp), _p(ci), _p(v), M.kind, M.bs, _p(mv), _p(bb), _p(x),
                       C.byref(_stop(tol, maxit, abs_tol, baseline)), C.byref(info))
    return _result(st, x, info)


def pagerank(G, damping=0.85, tol=1e-10, maxit=1000):
    """(status, x, iters, delta) for the in-link CSR pattern of G."""
    rp = _c(G.rowptr, np.int32)
    ci = _c(G.col, np.int32)
    x = np.zeros(int(G.n))
    it = _I64()
    dl = _D()
    st = lib().orc_pagerank(int(G.n), _p(rp), _p(ci), float(damping), float(tol), int(maxit),
                            _p(x), C.byref(it), C.byref(dl))
    return st, x, it.value, dl.value


def pipecg(A, b, x0=None, tol=1e-10, maxit=20000, abs_tol=0.0):
    n, rp, ci, v = _csr(A)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64, copy=True)
    info = Info()
    st = lib().orc_pipecg(n, _p(rp), _p(ci), _p(v), _p(bb), _p(x),
                          C.byref(_stop(tol, maxit, abs_tol)), C.byref(info))
    return _result(st, x, info)


def cgs(A, b, x0=None, tol=1e-10, maxit=10000, abs_tol=0.0):
    n, rp, ci, v = _csr(A)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64, copy=True)
    info = Info()
    st = lib().orc_cgs(n, _p(rp), _p(ci), _p(v), _p(bb), _p(x),
                       C.byref(_stop(tol, maxit, abs_tol)), C.byref(info))
    return _result(st, x, info)


def bicgstab(A, b, x0=None, tol=1e-10, maxit=10000, abs_tol=0.0):
    n, rp, ci, v = _csr(A)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64, copy=True)
    info = Info()
    st = lib().orc_bicgstab(n, _p(rp), _p(ci), _p(v), _p(bb), _p(x),
                            C.byref(_stop(tol, maxit, abs_tol)), C.byref(info))
    return _result(st, x, info)


def gmres(A, b, m=30, x0=None, tol=1e-10, maxit=20000, abs_tol=0.0, hist=False):
    n, rp, ci, v = _csr(A)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64, copy=True)
    info = Info()
    h = np.zeros(maxit if hist else 0, np.float64)
    st = lib().orc_gmres(n, _p(rp), _p(ci), _p(v), _p(bb), _p(x), m,
                         C.byref(_stop(tol, maxit, abs_tol)), C.byref(info),
                         _p(h) if hist else None, len(h))
    return _result(st, x, info, h[: info.iters] if hist else None)


@dataclass
class IRResult:
    status: int
    x: np.ndarray
    outer_iters: int
    inner_iters_total: int
    relres_true: float


def ir(A, b, low="f32", x0=None, tol=1e-10, outer_max=50, inner_tol=1e-4,
       inner_max=20000, last_step_variant=False, val32=None, h16=None, scale=None,
       precond: Precond | None = None, carry_direction=False):
    """Iterative refinement; the low-precision copy is built by the oracle's
    own conversions unless passed in.  `precond` (from jacobi/block_jacobi)
    preconditions the inner CG with its values rounded to FP32.
    `carry_direction` keeps the inner CG's last direction across refinement
    steps (ORC_IR_CARRY) instead of restarting it."""
    flags = (1 if last_step_variant else 0) | (2 if carry_direction else 0)
    n, rp, ci, v = _csr(A)
    bb = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, np.float64, copy=True)
    if low == "f32":
        if val32 is None:
            st, val32 = cast_f32(v)
            assert st == OK
        kind = 0
        v32 = _c(val32, np.float32)
        hh, ss = None, None
    else:
        if h16 is None:
            st, h16, scale = rowscale_f16(A)
            assert st == OK
        kind = 1
        v32 = None
        hh = _c(h16, np.uint16)
        ss = _c(scale, np.float32)
    info = IRInfo()
    if precond is None:
        st = lib().orc_ir(n, _p(rp), _p(ci), _p(v), kind, _p(v32), _p(hh), _p(ss), _p(bb),
                          _p(x), tol, outer_max, inner_tol, inner_max,
                          flags, C.byref(info))
    else:
        st_c, m32 = cast_f32(precond.minv)
        assert st_c == OK
        m32 = _c(m32, np.float32)
        st = lib().orc_ir_pc(n, _p(rp), _p(ci), _p(v), kind, _p(v32), _p(hh), _p(ss), _p(bb),
                             _p(x), tol, outer_max, inner_tol, inner_max,
                             flags, precond.kind, precond.bs,
                             _p(m32), C.byref(info))
    return IRResult(st, x, info.outer_iters, info.inner_iters_total, info.relres_true)


def true_relres(A, b, x):
    """||b - A x||_2 / ||b||_2 with each residual entry accumulated accurately."""
    bb = _c(b, np.float64)
    r = spmv_csr(A, x, alpha=-1.0, beta=1.0, y=bb)
    nb = float(np.sqrt(np.dot(bb, bb)))
    return float(np.sqrt(np.dot(r, r))) / (nb if nb > 0 else 1.0)
