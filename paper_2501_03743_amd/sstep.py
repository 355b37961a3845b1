"""Thin ctypes binding of libsstep.so (include/sstep.h).

Argument marshalling only: torch tensors supply device memory and the
stream, and every step of a solve runs in the library's HIP kernels.  There
is no fallback: if the library is missing or no GPU is present, the calls
raise.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsstep.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
EINVAL, ENOMEM, EHIP, EUNSUPPORTED = -1, -2, -3, -4
SMAX = 16
STENCIL = {"2d5": 1, "3d7": 2, "3d27": 3, "3d7_vark": 4}
BORROW, COPY, VALIDATE = 0, 1, 2
PREC = {"none": 0, "jacobi": 1, "amg": 2}
AMG_MAX_LEVELS = 16
METHOD = {"sstep": 0, "pcg": 1, "pfcg": 2}
PRECISION = {"fp64": 0, "mixed_ir": 1}
BASIS = {"monomial": 0, "chebyshev": 1}
PROFILE_CLASSES = 5

# C symbols declared in include/sstep.h (checked by the CPU tests)
EXPORTS = (
    "ssp_create", "ssp_destroy", "ssp_matrix_csr", "ssp_matrix_stencil",
    "ssp_matrix_csr_from_stencil", "ssp_matrix_info", "ssp_matrix_csr_arrays",
    "ssp_matrix_destroy", "ssp_set_preconditioner", "ssp_spmv", "ssp_mpk", "ssp_solve",
    "ssp_get_iterations", "ssp_get_residual_history", "ssp_get_true_residual",
    "ssp_get_profile", "ssp_status_string", "ssp_last_error", "ssp_solve_batch",
    "ssp_autotune_batch", "ssp_net_create", "ssp_net_destroy", "ssp_net_params",
    "ssp_net_forward", "ssp_net_predict", "ssp_net_zero_grad", "ssp_net_backward", "ssp_net_loss",
    "ssp_net_adam_step", "ssp_net_get_state", "ssp_net_set_state", "ssp_conv3d",
    "ssp_conv3d_wgrad", "ssp_net_mfma_selftest", "ssp_get_warm_start", "ssp_get_restarts",
    "ssp_net_loss_h1", "ssp_matrix_csr_form", "ssp_mpk_noalloc", "ssp_cheb_basis",
    "ssp_stream_probe", "ssp_set_amg", "ssp_amg_levels", "ssp_amg_apply",
)


class SspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (status_string(code), code, msg))
        self.code = code


class Tune(C.Structure):
    """Batched-solver tuning (ssp_tune): tile_rows, grid, order, spin_limit,
    schedule (0 persistent launch, 1 stepped), run (tiles per claim)."""
    _fields_ = [("tile_rows", C.c_int), ("grid", C.c_int), ("order", C.c_int),
                ("spin_limit", C.c_int), ("schedule", C.c_int), ("run", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AmgOpts(C.Structure):
    """AMG hierarchy options (ssp_amg_opts; 0 = default)."""
    _fields_ = [("theta", C.c_double), ("omega", C.c_double), ("sweeps", C.c_int),
                ("max_coarse", C.c_int), ("max_levels", C.c_int)]


class _Opts(C.Structure):
    _fields_ = [("method", C.c_int), ("precision", C.c_int), ("inner_rtol", C.c_double),
                ("max_refine", C.c_int), ("check_every", C.c_int), ("fixed_outer", C.c_int),
                ("profile", C.c_int), ("trace_cap", C.c_int),
                ("trace_vm", C.c_void_p), ("trace_alpha", C.c_void_p),
                ("trace_beta", C.c_void_p), ("trace_W", C.c_void_p),
                ("warm_start", C.c_int), ("warm_sweeps", C.c_int),
                ("warm_omega", C.c_double), ("restarts", C.c_int),
                ("basis", C.c_int), ("basis_lo", C.c_double), ("basis_hi", C.c_double)]


_lib = None
_live_handles = weakref.WeakSet()


@atexit.register
def _close_all():
    # release library objects before the HIP runtime is torn down
    for h in list(_live_handles):
        try:
            h.close()
        except Exception:
            pass


def load():
    """Loads libsstep.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsstep.so is not built: run `python -m paper_2501_03743_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "ssp_create": (i32, [C.POINTER(vp), i32, vp]),
        "ssp_destroy": (i32, [vp]),
        "ssp_matrix_csr": (i32, [vp, i64, i64, vp, vp, vp, C.c_uint, C.POINTER(vp)]),
        "ssp_matrix_stencil": (i32, [vp, i32, i32, i32, i32, vp, C.POINTER(vp)]),
        "ssp_matrix_csr_from_stencil": (i32, [vp, i32, i32, i32, i32, vp, C.POINTER(vp)]),
        "ssp_matrix_info": (i32, [vp, C.POINTER(i64), C.POINTER(i64)]),
        "ssp_matrix_csr_arrays": (i32, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]),
        "ssp_matrix_destroy": (i32, [vp]),
        "ssp_matrix_csr_form": (i32, [vp, C.POINTER(i32)]),
        "ssp_set_preconditioner": (i32, [vp, i32]),
        "ssp_spmv": (i32, [vp, vp, vp, vp]),
        "ssp_mpk": (i32, [vp, vp, vp, i32, vp, i64, vp]),
        "ssp_mpk_noalloc": (i32, [vp, vp, vp, i32, vp, i64, vp]),
        "ssp_cheb_basis": (i32, [vp, vp, vp, i32, dbl, dbl, vp, i64, vp]),
        "ssp_stream_probe": (i32, [vp, i32, vp, vp, i64, i32, C.POINTER(dbl)]),
        "ssp_solve": (i32, [vp, vp, vp, vp, i32, dbl, i32, C.POINTER(_Opts)]),
        "ssp_get_iterations": (i32, [vp, C.POINTER(i32), C.POINTER(i32)]),
        "ssp_get_residual_history": (i32, [vp, vp, i32, C.POINTER(i32)]),
        "ssp_get_true_residual": (i32, [vp, C.POINTER(dbl)]),
        "ssp_get_warm_start": (i32, [vp, C.POINTER(i32), C.POINTER(dbl)]),
        "ssp_get_restarts": (i32, [vp, C.POINTER(i32)]),
        "ssp_get_profile": (i32, [vp, vp, vp]),
        "ssp_solve_batch": (i32, [vp, i32, vp, vp, vp, i32, dbl, i32, C.POINTER(_Opts),
                                  C.POINTER(Tune), vp, vp, vp]),
        "ssp_autotune_batch": (i32, [vp, i32, vp, vp, i32, C.c_char_p, C.POINTER(Tune)]),
        "ssp_net_create": (i32, [vp, i32, i32, i32, i32, C.c_uint64, C.POINTER(vp)]),
        "ssp_net_destroy": (i32, [vp]),
        "ssp_net_params": (i32, [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(i64)]),
        "ssp_net_forward": (i32, [vp, vp, i32, vp]),
        "ssp_net_predict": (i32, [vp, vp, vp, dbl, vp]),
        "ssp_net_zero_grad": (i32, [vp]),
        "ssp_net_backward": (i32, [vp, vp]),
        "ssp_net_loss": (i32, [vp, vp, vp, vp, C.POINTER(dbl)]),
        "ssp_net_loss_h1": (i32, [vp, vp, vp, C.c_float, vp, C.POINTER(dbl)]),
        "ssp_net_adam_step": (i32, [vp, C.c_float, C.c_float, C.c_float, C.c_float, i32]),
        "ssp_net_get_state": (i32, [vp, vp, i64]),
        "ssp_net_set_state": (i32, [vp, vp, i64]),
        "ssp_conv3d": (i32, [vp, i32, vp, i32, i32, i32, i32, i32, vp, i32, i32, vp]),
        "ssp_conv3d_wgrad": (i32, [vp, vp, i32, i32, i32, i32, i32, vp, i32, i32, vp, vp]),
        "ssp_net_mfma_selftest": (i32, [vp, vp, vp, vp]),
        "ssp_set_amg": (i32, [vp, vp, C.POINTER(AmgOpts)]),
        "ssp_amg_levels": (i32, [vp, C.POINTER(i32), vp]),
        "ssp_amg_apply": (i32, [vp, vp, vp, vp]),
        "ssp_status_string": (C.c_char_p, [i32]),
        "ssp_last_error": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().ssp_status_string(code).decode()


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _check_dev(t, dtype, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if n is not None and t.numel() < n:
        raise ValueError("%s has %d entries, needs %d" % (name, t.numel(), n))


@dataclass
class SolveResult:
    status: int
    outer: int
    cg_equiv: int
    true_rel: float
    hist: np.ndarray
    trace: Optional[dict] = None
    profile: Optional[dict] = None
    warm_kept: int = -1          # 1 warm start used, 0 fell back to x0 = 0, -1 none
    warm_rel0: float = float("nan")
    restarts: int = 0            # residual-replacement restarts made

    @property
    def ok(self):
        return self.status == OK


class Matrix:
    def __init__(self, handle, ptr, n, nnz, keep):
        self.handle = handle
        self._p = ptr
        self.n = n
        self.nnz = nnz
        self._keep = keep       # tensors the library borrows
        handle._matrices.add(self)

    @property
    def csr_form(self) -> int:
        """CSR kernel form in use (0 staged, 1 row, 2 sliced ELL; -1 matrix-free)."""
        f = C.c_int()
        load().ssp_matrix_csr_form(self._p, C.byref(f))
        return f.value

    def set_preconditioner(self, kind: str):
        rc = load().ssp_set_preconditioner(self._p, PREC[kind])
        if rc:
            raise SspError(rc, "set_preconditioner")

    def csr_arrays(self):
        """(rowptr, colind, val) as torch tensors viewing the library's device arrays."""
        import torch
        lib = load()
        rp, ci, va = C.c_void_p(), C.c_void_p(), C.c_void_p()
        rc = lib.ssp_matrix_csr_arrays(self._p, C.byref(rp), C.byref(ci), C.byref(va))
        if rc:
            raise SspError(rc, "not a CSR matrix")
        dev = "cuda:%d" % self.handle.device
        torch.cuda.synchronize()
        out = []
        for ptr, cnt, ts in ((rp.value, self.n + 1, "<i4"), (ci.value, self.nnz, "<i4"),
                             (va.value, self.nnz, "<f8")):
            view = torch.as_tensor(_DeviceArray(ptr, cnt, ts), device=dev)
            out.append(view.clone())
        return tuple(out)

    def close(self):
        # a matrix must be destroyed before its handle; Handle.close() does it
        if self._p and self.handle._h:
            load().ssp_matrix_destroy(self._p)
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    """Exposes a library-owned device array to torch (zero-copy view)."""

    def __init__(self, ptr, count, typestr):
        self.__cuda_array_interface__ = {"shape": (count,), "typestr": typestr,
                                         "data": (ptr, False), "version": 2, "strides": None}


class Handle:
    """A library handle bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the s-step solver runs only on the GPU")
        lib = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self._h = C.c_void_p()
        self._matrices = weakref.WeakSet()
        self._nets = weakref.WeakSet()
        rc = lib.ssp_create(C.byref(self._h), device, C.c_void_p(stream.cuda_stream))
        if rc:
            raise SspError(rc, "ssp_create")
        _live_handles.add(self)

    # ---------------------------------------------------------------- util
    def _err(self, rc, what):
        msg = load().ssp_last_error(self._h).decode()
        raise SspError(rc, "%s: %s" % (what, msg))

    def close(self):
        if self._h:
            for m in list(self._matrices):
                m.close()
            for m in list(self._nets):
                m.close()
            load().ssp_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- matrices
    def matrix_csr(self, rowptr, colind, val, flags: int = BORROW) -> Matrix:
        import torch
        n = rowptr.numel() - 1
        nnz = colind.numel()
        _check_dev(rowptr, torch.int32, name="rowptr")
        _check_dev(colind, torch.int32, name="colind")
        _check_dev(val, torch.float64, nnz, name="val")
        out = C.c_void_p()
        rc = load().ssp_matrix_csr(self._h, n, nnz, _ptr(rowptr), _ptr(colind), _ptr(val), flags,
                                   C.byref(out))
        if rc:
            self._err(rc, "ssp_matrix_csr")
        keep = [] if flags & COPY else [rowptr, colind, val]
        return Matrix(self, out.value, n, nnz, keep)

    def _stencil(self, fn, kind, shape, coef=None, k=None):
        import torch
        nx, ny, nz = (tuple(shape) + (1,))[:3] if len(shape) == 2 else tuple(shape)
        kd = STENCIL[kind]
        keep = []
        if kind == "3d7_vark":
            _check_dev(k, torch.float64, nx * ny * nz, name="k")
            cptr = C.c_void_p(_ptr(k))
            keep.append(k)
        elif coef is not None:
            carr = (C.c_double * 2)(*coef)
            cptr = C.cast(carr, C.c_void_p)
            keep.append(carr)
        else:
            cptr = None
        out = C.c_void_p()
        rc = fn(self._h, kd, nx, ny, nz, cptr, C.byref(out))
        if rc:
            self._err(rc, fn.__name__)
        n, nnz = C.c_int64(), C.c_int64()
        load().ssp_matrix_info(out.value, C.byref(n), C.byref(nnz))
        return Matrix(self, out.value, n.value, nnz.value, keep)

    def matrix_stencil(self, kind: str, shape, coef=None, k=None) -> Matrix:
        return self._stencil(load().ssp_matrix_stencil, kind, shape, coef, k)

    def matrix_csr_from_stencil(self, kind: str, shape, coef=None, k=None) -> Matrix:
        return self._stencil(load().ssp_matrix_csr_from_stencil, kind, shape, coef, k)

    # ---------------------------------------------------------------- AMG
    def set_amg(self, A: Matrix, theta: float = 0.0, omega: float = 0.0, sweeps: int = 0,
                max_coarse: int = 0, max_levels: int = 0):
        """Builds A's aggregation-AMG hierarchy and makes it A's preconditioner
        (0 = the library default for each option)."""
        o = AmgOpts(theta=theta, omega=omega, sweeps=sweeps, max_coarse=max_coarse,
                    max_levels=max_levels)
        rc = load().ssp_set_amg(self._h, A._p, C.byref(o))
        if rc:
            self._err(rc, "ssp_set_amg")

    def amg_levels(self, A: Matrix):
        """Rows of each level of A's hierarchy (empty: none)."""
        lv = C.c_int()
        rows = np.zeros(AMG_MAX_LEVELS, dtype=np.int64)
        rc = load().ssp_amg_levels(A._p, C.byref(lv), rows.ctypes.data_as(C.c_void_p))
        if rc:
            self._err(rc, "ssp_amg_levels")
        return [int(v) for v in rows[:lv.value]]

    def amg_apply(self, A: Matrix, y, z):
        """z = B^-1 y (one V-cycle)."""
        import torch
        _check_dev(y, torch.float64, A.n, "y")
        _check_dev(z, torch.float64, A.n, "z")
        rc = load().ssp_amg_apply(self._h, A._p, _ptr(y), _ptr(z))
        if rc:
            self._err(rc, "ssp_amg_apply")

    # ---------------------------------------------------------------- building blocks
    def spmv(self, A: Matrix, x, y):
        import torch
        _check_dev(x, torch.float64, A.n, "x")
        _check_dev(y, torch.float64, A.n, "y")
        rc = load().ssp_spmv(self._h, A._p, _ptr(x), _ptr(y))
        if rc:
            self._err(rc, "ssp_spmv")

    def mpk(self, A: Matrix, r, s: int, P=None, noalloc: bool = False):
        """Alg. 4 + Alg. 5: returns (P as a (2s, n) view of the block, vm).
        noalloc=True calls ssp_mpk_noalloc (no device allocation in the
        library; P must then be given)."""
        import torch
        _check_dev(r, torch.float64, A.n, "r")
        if P is None:
            if noalloc:
                raise ValueError("mpk(noalloc=True) needs a caller-supplied P")
            P = torch.empty((2 * s, A.n), dtype=torch.float64, device=r.device)
        vm = np.zeros(2 * s)
        fn = load().ssp_mpk_noalloc if noalloc else load().ssp_mpk
        rc = fn(self._h, A._p, _ptr(r), s, _ptr(P), P.stride(0), vm.ctypes.data_as(C.c_void_p))
        if rc:
            self._err(rc, fn.__name__)
        return P, vm

    def cheb_basis(self, A: Matrix, r, s: int, interval=None, P=None):
        """The Chebyshev basis of one outer iteration and its block Gram
        product: returns (P as a (2s, n) view [Z; AZ], gram = Z^T [AZ | r],
        an s x (s+1) array)."""
        import torch
        _check_dev(r, torch.float64, A.n, "r")
        if P is None:
            ld = (A.n + 1) // 2 * 2
            P = torch.empty((2 * s, ld), dtype=torch.float64, device=r.device)[:, :A.n]
        gram = np.zeros((s, s + 1))
        lo, hi = interval if interval else (0.0, 0.0)
        rc = load().ssp_cheb_basis(self._h, A._p, _ptr(r), s, lo, hi, _ptr(P), P.stride(0),
                                   gram.ctypes.data_as(C.c_void_p))
        if rc:
            self._err(rc, "ssp_cheb_basis")
        return P, gram

    def stream_probe(self, src, dst=None, reps: int = 10) -> float:
        """Mean milliseconds of a plain streaming read of src (dst None) or a
        copy src -> dst, timed on the device (the roofline reference)."""
        ms = C.c_double()
        rc = load().ssp_stream_probe(self._h, 0 if dst is None else 1, _ptr(src), _ptr(dst),
                                     src.numel(), reps, C.byref(ms))
        if rc:
            self._err(rc, "ssp_stream_probe")
        return ms.value

    # ---------------------------------------------------------------- batches
    def _batch_arrays(self, mats, bs, xs=None):
        import torch
        m = len(mats)
        A = (C.c_void_p * m)(*[M._p for M in mats])
        for t in bs:
            _check_dev(t, torch.float64, name="b")
        B = (C.c_void_p * m)(*[_ptr(t) for t in bs])
        X = None
        if xs is not None:
            for M, t in zip(mats, xs):
                _check_dev(t, torch.float64, M.n, name="x")
            X = (C.c_void_p * m)(*[_ptr(t) for t in xs])
        return m, A, B, X

    def solve_batch(self, mats, bs, xs, s=4, rtol=1e-8, maxit=10000, inner_rtol=1e-5,
                    max_refine=10, tune=None):
        """One persistent launch over all systems (mixed-precision s-step).
        Returns (worst status, per-system status, inner outer iterations,
        true relative residuals)."""
        m, A, B, X = self._batch_arrays(mats, bs, xs)
        o = _Opts(method=0, precision=PRECISION["mixed_ir"], inner_rtol=inner_rtol,
                  max_refine=max_refine)
        st = np.zeros(m, dtype=np.int32)
        it = np.zeros(m, dtype=np.int32)
        tr = np.zeros(m)
        rc = load().ssp_solve_batch(self._h, m, A, B, X, s, rtol, maxit, C.byref(o),
                                    C.byref(tune) if tune is not None else None,
                                    st.ctypes.data_as(C.c_void_p), it.ctypes.data_as(C.c_void_p),
                                    tr.ctypes.data_as(C.c_void_p))
        if rc < 0:
            self._err(rc, "ssp_solve_batch")
        return rc, st, it, tr

    def autotune_batch(self, mats, bs, s=4, cache_path=None) -> Tune:
        m, A, B, _ = self._batch_arrays(mats, bs)
        out = Tune()
        rc = load().ssp_autotune_batch(self._h, m, A, B, s,
                                       cache_path.encode() if cache_path else None,
                                       C.byref(out))
        if rc < 0:
            self._err(rc, "ssp_autotune_batch")
        return out

    # ---------------------------------------------------------------- solve
    def solve(self, A: Matrix, b, x, s: int = 4, rtol: float = 1e-8, maxit: int = 10000,
              method: str = "sstep", precision: str = "fp64", inner_rtol: float = 1e-5,
              max_refine: int = 10, check_every: int = 0, fixed_outer: int = 0,
              profile: bool = False, trace_cap: int = 0,
              warm_start: bool = False, warm_sweeps: int = 0,
              warm_omega: float = 0.0, restarts: int = 0, basis: str = "monomial",
              interval=None) -> SolveResult:
        """ssp_solve: A x = b on the device (x holds x0 on entry, the solution on
        return).  method: "sstep" (Alg. 3-6, block size s), "pcg" (Alg. 1) or
        "pfcg" (Alg. 2); precision: "fp64" or "mixed_ir" (s-step only: FP32
        inner solves to inner_rtol inside FP64 refinement); fixed_outer > 0
        runs exactly that many outer iterations; restarts > 0 re-runs an FP64
        method from x while its true residual misses rtol; warm_start judges
        the given x (after warm_sweeps damped Jacobi sweeps) and falls back to
        x = 0 when ||b - A x|| >= ||b||; basis "chebyshev" (s-step only) uses
        the Chebyshev basis over `interval` = (lo, hi) (default: the library's
        Gershgorin interval).  Returns the status (0 converged,
        1 not converged, 2 breakdown), iteration counts, residual history and
        true residual; raises SspError on invalid arguments."""
        import torch
        _check_dev(b, torch.float64, A.n, "b")
        _check_dev(x, torch.float64, A.n, "x")
        o = _Opts(method=METHOD[method], precision=PRECISION[precision], inner_rtol=inner_rtol,
                  max_refine=max_refine, check_every=check_every, fixed_outer=fixed_outer,
                  profile=1 if profile else 0, trace_cap=0,
                  warm_start=1 if warm_start else 0, warm_sweeps=warm_sweeps,
                  warm_omega=warm_omega, restarts=restarts, basis=BASIS[basis],
                  basis_lo=interval[0] if interval else 0.0,
                  basis_hi=interval[1] if interval else 0.0)
        trace = None
        if trace_cap > 0:
            trace = dict(vm=np.zeros((trace_cap, 2 * s)), alpha=np.zeros((trace_cap, s)),
                         beta=np.zeros((trace_cap, s, s)), W=np.zeros((trace_cap, s, s)))
            o.trace_cap = trace_cap
            o.trace_vm = trace["vm"].ctypes.data
            o.trace_alpha = trace["alpha"].ctypes.data
            o.trace_beta = trace["beta"].ctypes.data
            o.trace_W = trace["W"].ctypes.data
        lib = load()
        rc = lib.ssp_solve(self._h, A._p, _ptr(b), _ptr(x), s, rtol, maxit, C.byref(o))
        if rc < 0:
            self._err(rc, "ssp_solve")
        outer, cge = C.c_int(), C.c_int()
        lib.ssp_get_iterations(self._h, C.byref(outer), C.byref(cge))
        ln = C.c_int()
        lib.ssp_get_residual_history(self._h, None, 0, C.byref(ln))
        hist = np.zeros(ln.value)
        lib.ssp_get_residual_history(self._h, hist.ctypes.data_as(C.c_void_p), ln.value,
                                     C.byref(ln))
        tr = C.c_double()
        lib.ssp_get_true_residual(self._h, C.byref(tr))
        prof = None
        if profile:
            launches = (C.c_int * PROFILE_CLASSES)()
            ms = (C.c_double * PROFILE_CLASSES)()
            lib.ssp_get_profile(self._h, launches, ms)
            prof = dict(launches=list(launches), ms=list(ms))
        if trace is not None:
            trace = {k: v[:outer.value] for k, v in trace.items()}
        kept, rel0 = C.c_int(), C.c_double()
        lib.ssp_get_warm_start(self._h, C.byref(kept), C.byref(rel0))
        nrs = C.c_int()
        lib.ssp_get_restarts(self._h, C.byref(nrs))
        return SolveResult(status=rc, outer=outer.value, cg_equiv=cge.value, true_rel=tr.value,
                           hist=hist, trace=trace, profile=prof, warm_kept=kept.value,
                           warm_rel0=rel0.value, restarts=nrs.value)

    # ---------------------------------------------------------------- network
    def net(self, shape, max_batch: int = 1, seed: int = 0) -> "Net":
        """The warm-start network for grids of `shape` (D, H, W)."""
        D, H, W = shape
        out = C.c_void_p()
        rc = load().ssp_net_create(self._h, D, H, W, max_batch, seed, C.byref(out))
        if rc:
            self._err(rc, "ssp_net_create")
        return Net(self, out, tuple(shape), max_batch)

    def conv3d(self, x, w, stride=1, mode=0):
        """One 3x3x3 convolution (mode 0) or its input gradient (mode 1) on the
        matrix cores.  x: float32 [B, D, H, W, C]; w: float32 [27, Ci, Co]."""
        import torch
        w = w.contiguous()
        _, ci, co = w.shape
        B, D, H, W, C_ = x.shape
        if mode == 0:
            assert C_ == ci
            shp = (B,) + tuple((n - 1) // stride + 1 for n in (D, H, W)) + (co,)
            grid = (D, H, W)
        else:
            raise ValueError("use conv3d_input_grad")
        out = torch.empty(shp, device=x.device, dtype=torch.float32)
        _check_dev(x, torch.float32, name="x")
        _check_dev(w, torch.float32, name="w")
        rc = load().ssp_conv3d(self._h, 0, _ptr(x), B, *grid, ci, _ptr(w), co, stride, _ptr(out))
        if rc:
            self._err(rc, "ssp_conv3d")
        return out

    def conv3d_input_grad(self, dy, w, in_shape, stride=1):
        """Input gradient of conv3d for the output gradient dy [B, Do, Ho, Wo, Co];
        in_shape = (D, H, W) of the convolution's input."""
        import torch
        w = w.contiguous()
        _, ci, co = w.shape
        B = dy.shape[0]
        out = torch.empty((B,) + tuple(in_shape) + (ci,), device=dy.device, dtype=torch.float32)
        _check_dev(dy, torch.float32, name="dy")
        _check_dev(w, torch.float32, name="w")
        rc = load().ssp_conv3d(self._h, 1, _ptr(dy), B, *in_shape, ci, _ptr(w), co, stride,
                               _ptr(out))
        if rc:
            self._err(rc, "ssp_conv3d")
        return out

    def conv3d_wgrad(self, x, dy, stride=1):
        """(dw [27, Ci, Co], db [Co]) of conv3d for input x and output gradient dy."""
        import torch
        B, D, H, W, ci = x.shape
        co = dy.shape[-1]
        dw = torch.empty((27, ci, co), device=x.device, dtype=torch.float32)
        db = torch.empty((co,), device=x.device, dtype=torch.float32)
        _check_dev(x, torch.float32, name="x")
        _check_dev(dy, torch.float32, name="dy")
        rc = load().ssp_conv3d_wgrad(self._h, _ptr(x), B, D, H, W, ci, _ptr(dy), co, stride,
                                     _ptr(dw), _ptr(db))
        if rc:
            self._err(rc, "ssp_conv3d_wgrad")
        return dw, db

    def mfma_selftest(self, A, B):
        """D = A B (16x32 by 32x16, BF16 operands) with one matrix-core instruction."""
        import torch
        D = torch.empty((16, 16), device=A.device, dtype=torch.float32)
        _check_dev(A, torch.float32, 512, "A")
        _check_dev(B, torch.float32, 512, "B")
        rc = load().ssp_net_mfma_selftest(self._h, _ptr(A), _ptr(B), _ptr(D))
        if rc:
            self._err(rc, "ssp_net_mfma_selftest")
        return D


class Net:
    """The warm-start U-Net (ssp_net_*): parameters, forward, backward, Adam."""

    def __init__(self, handle, ptr, shape, max_batch):
        self.handle = handle
        self._p = ptr
        self.shape = shape
        self.max_batch = max_batch
        handle._nets.add(self)
        pp, gp, cnt = C.c_void_p(), C.c_void_p(), C.c_int64()
        load().ssp_net_params(self._p, C.byref(pp), C.byref(gp), C.byref(cnt))
        self.count = cnt.value
        self._pp, self._gp = pp.value, gp.value
        self.step = 0

    def _rc(self, rc, what):
        if rc:
            self.handle._err(rc, what)

    def params(self):
        """Zero-copy float32 views of the parameters and their gradients."""
        import torch
        dev = "cuda:%d" % self.handle.device
        p = torch.as_tensor(_DeviceArray(self._pp, self.count, "<f4"), device=dev)
        g = torch.as_tensor(_DeviceArray(self._gp, self.count, "<f4"), device=dev)
        return p, g

    def forward(self, inp, out=None):
        """inp: float32 [B, D, H, W, 2] (log k, f) -> float32 [B, D, H, W]."""
        import torch
        B = inp.shape[0]
        if tuple(inp.shape[1:]) != self.shape + (2,):
            raise ValueError("input must be [B, %d, %d, %d, 2]" % self.shape)
        _check_dev(inp, torch.float32, name="inp")
        if out is None:
            out = torch.empty((B,) + self.shape, device=inp.device, dtype=torch.float32)
        _check_dev(out, torch.float32, inp.numel() // 2, "out")
        self._rc(load().ssp_net_forward(self._p, _ptr(inp), B, _ptr(out)), "ssp_net_forward")
        return out

    def predict(self, logk, f, out_scale, out=None):
        """x0 = net(log k, f / rms(f)) rms(f) out_scale for one problem, all on
        the device: logk, f float64 [D*H*W] -> float64 [D*H*W]."""
        import torch
        n = self.shape[0] * self.shape[1] * self.shape[2]
        _check_dev(logk, torch.float64, n, "logk")
        _check_dev(f, torch.float64, n, "f")
        if out is None:
            out = torch.empty(n, device=logk.device, dtype=torch.float64)
        _check_dev(out, torch.float64, n, "out")
        self._rc(load().ssp_net_predict(self._p, _ptr(logk), _ptr(f), float(out_scale), _ptr(out)),
                 "ssp_net_predict")
        return out

    def loss(self, y, target, dy=None):
        """Mean squared error of the last forward's output; returns (loss, dy)."""
        import torch
        if dy is None:
            dy = torch.empty_like(y)
        _check_dev(y, torch.float32, name="y")
        _check_dev(target, torch.float32, y.numel(), "target")
        v = C.c_double()
        self._rc(load().ssp_net_loss(self._p, _ptr(y), _ptr(target), _ptr(dy), C.byref(v)),
                 "ssp_net_loss")
        return v.value, dy

    def loss_h1(self, y, target, lam, dy=None):
        """Energy-type loss e^T (L + lam I) e / N (L: 7-point Laplacian); returns (loss, dy)."""
        import torch
        if dy is None:
            dy = torch.empty_like(y)
        _check_dev(y, torch.float32, name="y")
        _check_dev(target, torch.float32, y.numel(), "target")
        v = C.c_double()
        self._rc(load().ssp_net_loss_h1(self._p, _ptr(y), _ptr(target), float(lam), _ptr(dy),
                                        C.byref(v)), "ssp_net_loss_h1")
        return v.value, dy

    def zero_grad(self):
        self._rc(load().ssp_net_zero_grad(self._p), "ssp_net_zero_grad")

    def backward(self, dy):
        import torch
        _check_dev(dy, torch.float32, name="dy")
        self._rc(load().ssp_net_backward(self._p, _ptr(dy)), "ssp_net_backward")

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        self._rc(load().ssp_net_adam_step(self._p, lr, b1, b2, eps, self.step), "ssp_net_adam_step")

    def get_state(self) -> np.ndarray:
        """Parameters and Adam moments, float32 [3, count]."""
        out = np.zeros(3 * self.count, dtype=np.float32)
        self._rc(load().ssp_net_get_state(self._p, out.ctypes.data_as(C.c_void_p), out.size),
                 "ssp_net_get_state")
        return out.reshape(3, self.count)

    def set_state(self, state):
        arr = np.ascontiguousarray(np.asarray(state, dtype=np.float32).reshape(-1))
        self._rc(load().ssp_net_set_state(self._p, arr.ctypes.data_as(C.c_void_p), arr.size),
                 "ssp_net_set_state")

    def close(self):
        if self._p and self.handle._h:
            load().ssp_net_destroy(self._p)
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
