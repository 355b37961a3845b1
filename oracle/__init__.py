"""FP64 CPU oracle for preconditioned s-step CG (arXiv 2501.03743).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product path never does.  It shares no code with
the HIP library.  The arithmetic lives in ``sstep_oracle.c`` (plain C, FP64,
no fast-math, no FMA contraction); this module only compiles and binds it.
``exact.py`` holds a rational-arithmetic version for tiny problems.

Functions follow the paper's algorithms:
  pcg         -- Alg. 1 (PCG-HS)
  pfcg        -- Alg. 2 (PFCG)
  sstep       -- Alg. 3 with Alg. 4 (pMPK), Alg. 5 (cvm) and Alg. 6 (SW)
  sstep_cheb  -- Alg. 3 on a Chebyshev basis with an explicit block Gram
                 product (the stabilised bases of the related work, Sec. IV)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sstep_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OP_CSR, OP_2D5, OP_3D7, OP_3D27, OP_3D7_VARK = 0, 1, 2, 3, 4
PREC_NONE, PREC_JACOBI = 0, 1
OK, NOT_CONVERGED, BREAKDOWN, EINVAL, ENOMEM = 0, 1, 2, -1, -2


def build(force: bool = False) -> str:
    """Compiles the C oracle into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Op(C.Structure):
    _fields_ = [("kind", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("n", C.c_int64), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("val", C.c_void_p), ("k", C.c_void_p), ("diag", C.c_double),
                ("off", C.c_double)]


class _Res(C.Structure):
    _fields_ = [("status", C.c_int), ("outer", C.c_int), ("cg_equiv", C.c_int),
                ("true_rel", C.c_double), ("hist", C.c_void_p), ("hist_cap", C.c_int),
                ("hist_len", C.c_int)]


class _Trace(C.Structure):
    _fields_ = [("cap", C.c_int), ("len", C.c_int), ("vm", C.c_void_p),
                ("alpha", C.c_void_p), ("beta", C.c_void_p), ("W", C.c_void_p),
                ("P", C.c_void_p)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            _lib = C.CDLL(build())
            _lib.orc_dot.restype = C.c_double
            _lib.orc_dot.argtypes = [C.c_int64, C.c_void_p, C.c_void_p]
            _lib.orc_stencil_nnz.restype = C.c_int64
            _lib.orc_stencil_nnz.argtypes = [C.c_int] * 4
            _lib.orc_csr_from_stencil.restype = C.c_int64
            _lib.orc_csr_from_stencil.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                                  C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                                  C.c_void_p]
            _lib.orc_apply.argtypes = [C.POINTER(_Op), C.c_void_p, C.c_void_p]
            _lib.orc_diag.argtypes = [C.POINTER(_Op), C.c_void_p]
            _lib.orc_pcg.restype = C.c_int
            _lib.orc_pcg.argtypes = [C.POINTER(_Op), C.c_int, C.c_void_p, C.c_void_p, C.c_double,
                                     C.c_int, C.POINTER(_Res)]
            _lib.orc_pfcg.restype = C.c_int
            _lib.orc_pfcg.argtypes = _lib.orc_pcg.argtypes
            _lib.orc_sstep.restype = C.c_int
            _lib.orc_sstep.argtypes = [C.POINTER(_Op), C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                       C.c_double, C.c_int, C.c_int, C.POINTER(_Res),
                                       C.POINTER(_Trace)]
            _lib.orc_spd_solve.restype = C.c_int
            _lib.orc_spd_solve.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
            _lib.orc_smax.restype = C.c_int
            _lib.orc_sw.restype = C.c_int
            _lib.orc_mpk_cvm.restype = C.c_int
            _lib.orc_mpk_cvm.argtypes = [C.POINTER(_Op), C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                         C.c_void_p]
            _lib.orc_sw.argtypes = [C.c_int] + [C.c_void_p] * 6
            _lib.orc_sstep_cheb.restype = C.c_int
            _lib.orc_sstep_cheb.argtypes = [C.POINTER(_Op), C.c_int, C.c_void_p, C.c_void_p,
                                            C.c_int, C.c_double, C.c_double, C.c_double,
                                            C.c_int, C.c_int, C.POINTER(_Res),
                                            C.POINTER(_Trace)]
            _lib.orc_cheb_basis.restype = C.c_int
            _lib.orc_cheb_basis.argtypes = [C.POINTER(_Op), C.c_int, C.c_void_p, C.c_int,
                                            C.c_double, C.c_double, C.c_void_p]
            _lib.orc_max_diag.restype = C.c_double
            _lib.orc_max_diag.argtypes = [C.POINTER(_Op)]
            _lib.orc_set_threads.restype = C.c_int
            _lib.orc_set_threads.argtypes = [C.c_int]
        return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class Operator:
    """An operator the oracle can apply: CSR arrays, or a matrix-free stencil.

    Stencil kinds: ``"2d5"`` (4/-1), ``"3d7"`` (6/-1), ``"3d27"`` (26/-1), all
    unscaled with Dirichlet zero outside the grid, and ``"3d7_vark"`` (the
    variable-coefficient 7-point operator of -div(k grad u) with harmonic-mean
    face weights and weight k_p on faces to the boundary).
    """

    KINDS = {"2d5": OP_2D5, "3d7": OP_3D7, "3d27": OP_3D27, "3d7_vark": OP_3D7_VARK}
    DEFAULT_COEF = {"2d5": (4.0, -1.0), "3d7": (6.0, -1.0), "3d27": (26.0, -1.0)}

    def __init__(self, kind, shape=None, csr=None, k=None, coef=None):
        self.kind = kind
        self._keep = []
        op = _Op()
        if kind == "csr":
            rowptr, colind, val = csr
            rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
            colind = np.ascontiguousarray(colind, dtype=np.int32)
            val = np.ascontiguousarray(val, dtype=np.float64)
            self._keep += [rowptr, colind, val]
            op.kind = OP_CSR
            op.n = len(rowptr) - 1
            op.rowptr, op.colind, op.val = _ptr(rowptr), _ptr(colind), _ptr(val)
            op.nx = op.ny = op.nz = 0
            self.n = op.n
            self.csr = (rowptr, colind, val)
        else:
            nx, ny, nz = (tuple(shape) + (1,))[:3] if len(shape) == 2 else tuple(shape)
            op.kind = self.KINDS[kind]
            op.nx, op.ny, op.nz = nx, ny, nz
            op.n = nx * ny * nz
            d, o = coef if coef is not None else self.DEFAULT_COEF.get(kind, (0.0, 0.0))
            op.diag, op.off = d, o
            if kind == "3d7_vark":
                k = np.ascontiguousarray(k, dtype=np.float64).reshape(-1)
                assert k.size == op.n
                self._keep.append(k)
                op.k = _ptr(k)
            self.n = op.n
            self.shape = (nx, ny, nz)
        self._op = op

    def apply(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        lib().orc_apply(C.byref(self._op), _ptr(x), _ptr(y))
        return y

    def diag(self):
        d = np.empty(self.n, dtype=np.float64)
        lib().orc_diag(C.byref(self._op), _ptr(d))
        return d


def stencil_csr(kind, shape, k=None, coef=None):
    """CSR arrays (rowptr, colind, val) of a stencil operator, built by the oracle."""
    nx, ny, nz = (tuple(shape) + (1,))[:3] if len(shape) == 2 else tuple(shape)
    kd = Operator.KINDS[kind]
    nnz = lib().orc_stencil_nnz(kd, nx, ny, nz)
    rowptr = np.empty(nx * ny * nz + 1, dtype=np.int32)
    colind = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    d, o = coef if coef is not None else Operator.DEFAULT_COEF.get(kind, (0.0, 0.0))
    kk = None
    if kind == "3d7_vark":
        kk = np.ascontiguousarray(k, dtype=np.float64).reshape(-1)
    got = lib().orc_csr_from_stencil(kd, nx, ny, nz, d, o, _ptr(kk), _ptr(rowptr), _ptr(colind),
                                     _ptr(val))
    assert got == nnz, (got, nnz)
    return rowptr, colind, val


def stencil_nnz(kind, shape):
    nx, ny, nz = (tuple(shape) + (1,))[:3] if len(shape) == 2 else tuple(shape)
    return int(lib().orc_stencil_nnz(Operator.KINDS[kind], nx, ny, nz))


def dot(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return float(lib().orc_dot(a.size, _ptr(a), _ptr(b)))


def spd_solve(W, c):
    """Solves W y = c with the solver's own Cholesky; returns (status, y)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    y = np.array(c, dtype=np.float64, copy=True)
    st = lib().orc_spd_solve(W.shape[0], _ptr(W), _ptr(y))
    return st, y


def mpk_cvm(op: "Operator", r, s, prec=PREC_JACOBI):
    """Alg. 4 then Alg. 5: returns (P as (2s, n), vm (2s,))."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    P = np.zeros((2 * s, op.n))
    vm = np.zeros(2 * s)
    st = lib().orc_mpk_cvm(C.byref(op._op), prec, _ptr(r), s, _ptr(P), _ptr(vm))
    assert st == OK, st
    return P, vm


def sw(vm, alpha_prev, W_prev):
    """Alg. 6 alone: returns (status, beta, W, alpha) for the given moments,
    previous alpha and previous W."""
    vm = np.ascontiguousarray(vm, dtype=np.float64)
    s = vm.size // 2
    ap = np.ascontiguousarray(alpha_prev, dtype=np.float64)
    Wp = np.ascontiguousarray(W_prev, dtype=np.float64)
    beta = np.zeros((s, s))
    W = np.zeros((s, s))
    alpha = np.zeros(s)
    st = lib().orc_sw(s, _ptr(vm), _ptr(ap), _ptr(Wp), _ptr(beta), _ptr(W), _ptr(alpha))
    return st, beta, W, alpha


class Result(dict):
    __getattr__ = dict.__getitem__


def _result(res, hist, x, trace=None):
    out = Result(status=res.status, outer=res.outer, cg_equiv=res.cg_equiv,
                 true_rel=res.true_rel, hist=hist[:min(res.hist_len, hist.size)].copy(), x=x)
    if trace is not None:
        out.update(trace)
    return out


def _restarted(run, x0, rtol, maxit, s, restarts):
    """Residual replacement by restart: while the recursive stopping test held
    but the true residual ||b - A x|| exceeds rtol ||b||, run the method again
    from the current x (its first residual is the true one), at most
    `restarts` times and within the budget of maxit CG-equivalent steps.
    Iteration counts add up and the histories are concatenated."""
    r = run(x0, maxit)
    used, outer, hists = 0, r.outer, [r.hist]
    while r.status == OK and used < restarts and r.true_rel > rtol:
        left = maxit - outer * s
        if left <= 0:
            break
        r = run(r.x, left)
        used += 1
        outer += r.outer
        hists.append(r.hist)
    r.outer, r.cg_equiv, r.restarts = outer, outer * s, used
    r.hist = np.concatenate(hists)
    return r


def pcg(op: Operator, b, x0=None, rtol=1e-8, maxit=10000, prec=PREC_JACOBI, restarts=0):
    """Alg. 1 on the oracle operator; returns a Result with x and history.
    restarts > 0: residual replacement by restart (_restarted)."""
    if restarts > 0:
        return _restarted(lambda x, m: pcg(op, b, x, rtol, m, prec), x0, rtol, maxit, 1, restarts)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    hist = np.zeros(maxit + 2)
    res = _Res(hist=_ptr(hist), hist_cap=hist.size)
    lib().orc_pcg(C.byref(op._op), prec, _ptr(b), _ptr(x), rtol, maxit, C.byref(res))
    return _result(res, hist, x)


def pfcg(op: Operator, b, x0=None, rtol=1e-8, maxit=10000, prec=PREC_JACOBI, restarts=0):
    """Alg. 2 (PFCG) on the oracle operator; returns a Result with x and history.
    maxit counts every step, the one before the loop included.  restarts > 0:
    residual replacement by restart (_restarted)."""
    if restarts > 0:
        return _restarted(lambda x, m: pfcg(op, b, x, rtol, m, prec), x0, rtol, maxit, 1, restarts)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    hist = np.zeros(maxit + 2)
    res = _Res(hist=_ptr(hist), hist_cap=hist.size)
    lib().orc_pfcg(C.byref(op._op), prec, _ptr(b), _ptr(x), rtol, maxit, C.byref(res))
    return _result(res, hist, x)


def sstep(op: Operator, b, s, x0=None, rtol=1e-8, maxit=10000, prec=PREC_JACOBI,
          fixed_outer=0, trace_cap=0, trace_P=False, restarts=0):
    """Alg. 3 (with Alg. 4-6) on the oracle operator.

    ``fixed_outer`` > 0 runs exactly that many outer iterations.  With
    ``trace_cap`` > 0 the per-iteration moments vm, alpha, beta and W (and with
    ``trace_P`` the block [P_i | A P_i] after the update) are returned.
    ``restarts`` > 0: residual replacement by restart (_restarted).
    """
    if restarts > 0:
        return _restarted(lambda x, m: sstep(op, b, s, x, rtol, m, prec), x0, rtol, maxit, s,
                          restarts)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    outer_cap = fixed_outer if fixed_outer > 0 else (maxit + max(s, 1) - 1) // max(s, 1)
    hist = np.zeros(outer_cap + 2)
    res = _Res(hist=_ptr(hist), hist_cap=hist.size)
    tr = None
    trace = None
    if trace_cap > 0:
        n = op.n
        trace = dict(vm=np.zeros((trace_cap, 2 * s)), alpha=np.zeros((trace_cap, s)),
                     beta=np.zeros((trace_cap, s, s)), W=np.zeros((trace_cap, s, s)))
        if trace_P:
            trace["P"] = np.zeros((trace_cap, 2 * s, n))
        tr = _Trace(cap=trace_cap, len=0, vm=_ptr(trace["vm"]), alpha=_ptr(trace["alpha"]),
                    beta=_ptr(trace["beta"]), W=_ptr(trace["W"]),
                    P=_ptr(trace["P"]) if trace_P else None)
    lib().orc_sstep(C.byref(op._op), prec, _ptr(b), _ptr(x), s, rtol, maxit, fixed_outer,
                    C.byref(res), C.byref(tr) if tr is not None else None)
    if trace is not None:
        ln = tr.len
        trace = {k: v[:ln] for k, v in trace.items()}
        trace = {"trace": trace}
    return _result(res, hist, x, trace)


def basis_interval(op: Operator, prec=PREC_JACOBI):
    """Default interval [lo, hi] enclosing the spectrum of K = B^-1 A for the
    Chebyshev basis: [0, 2] with the Jacobi preconditioner, [0, 2 max a_ii]
    without one (Gershgorin, for weakly diagonally dominant SPD matrices)."""
    if prec == PREC_JACOBI:
        return 0.0, 2.0
    return 0.0, 2.0 * lib().orc_max_diag(C.byref(op._op))


def cheb_basis(op: Operator, r, s, lo, hi, prec=PREC_JACOBI):
    """The Chebyshev basis block of one outer iteration: (2s, n) array
    [z_1 .. z_s, A z_1 .. A z_s] for z_1 = B^-1 r."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    P = np.zeros((2 * s, op.n))
    rc = lib().orc_cheb_basis(C.byref(op._op), prec, _ptr(r), s, lo, hi, _ptr(P))
    if rc:
        raise ValueError("orc_cheb_basis: %d" % rc)
    return P


def sstep_cheb(op: Operator, b, s, x0=None, rtol=1e-8, maxit=10000, prec=PREC_JACOBI,
               interval=None, fixed_outer=0, trace_cap=0, trace_P=False, restarts=0):
    """Alg. 3 on a Chebyshev basis with the block Gram product taken directly
    (``orc_sstep_cheb``).  ``interval`` = (lo, hi) encloses the spectrum of
    B^-1 A (default: ``basis_interval``).  The trace's ``vm`` holds m(1..s)
    then the diagonal of Z^T A Z.  Other arguments as for ``sstep``."""
    lo, hi = basis_interval(op, prec) if interval is None else interval
    if restarts > 0:
        return _restarted(lambda x, m: sstep_cheb(op, b, s, x, rtol, m, prec, (lo, hi)), x0,
                          rtol, maxit, s, restarts)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    outer_cap = fixed_outer if fixed_outer > 0 else (maxit + max(s, 1) - 1) // max(s, 1)
    hist = np.zeros(outer_cap + 2)
    res = _Res(hist=_ptr(hist), hist_cap=hist.size)
    tr = trace = None
    if trace_cap > 0:
        trace = dict(vm=np.zeros((trace_cap, 2 * s)), alpha=np.zeros((trace_cap, s)),
                     beta=np.zeros((trace_cap, s, s)), W=np.zeros((trace_cap, s, s)))
        if trace_P:
            trace["P"] = np.zeros((trace_cap, 2 * s, op.n))
        tr = _Trace(cap=trace_cap, len=0, vm=_ptr(trace["vm"]), alpha=_ptr(trace["alpha"]),
                    beta=_ptr(trace["beta"]), W=_ptr(trace["W"]),
                    P=_ptr(trace["P"]) if trace_P else None)
    lib().orc_sstep_cheb(C.byref(op._op), prec, _ptr(b), _ptr(x), s, lo, hi, rtol, maxit,
                         fixed_outer, C.byref(res), C.byref(tr) if tr is not None else None)
    if trace is not None:
        trace = {"trace": {k: v[:tr.len] for k, v in trace.items()}}
    return _result(res, hist, x, trace)


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's OpenMP loops from now on (n <= 0: unchanged);
    returns the number in use."""
    return lib().orc_set_threads(int(n))
