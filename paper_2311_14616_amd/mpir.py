"""Python binding of libmpir.so (ctypes): argument marshalling only.

Every step of the solve runs in the library's HIP kernels; torch supplies the
device memory and the stream.  Loading fails loudly when the library is not
built -- there is no fallback.

Storage convention: a matrix is passed as a 2-D tensor ``At`` of shape
``(n, lda)`` holding A in column-major order (``At[j, i] == A[i, j]``), the
layout of the C ABI.  For a symmetric A this is A itself.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpir.so")

F64, F32, F16, BF16 = 0, 1, 2, 3
OK, ERR_SINGULAR, ERR_ARG, ERR_ALLOC, ERR_HIP, ERR_NONFINITE, ERR_RANGE, ERR_STATE, ERR_DEVICE = \
    0, 1, -1, -2, -3, -4, -5, -6, -7
STOP_NAMES = {0: "converged", 1: "stagnated", 2: "dstagnated", 3: "litmax", 4: "nonfinite"}
HIST_MAX = 64
PROF_GEMM, PROF_PANEL, PROF_TRSV, PROF_GEMV, PROF_DOWNCAST = 0, 1, 2, 3, 4
BATCH_PHASES = ("downcast", "panel", "interchanges", "u_rows", "update", "solves", "residual")

EXPORTS = [
    "mpir_term_default", "mpir_factor", "mpir_refactor", "mpir_solve", "mpir_ir_solve",
    "mpir_gmres_ir_solve", "mpir_ir_solve_multi", "mpir_bicgstab_ir_solve",
    "mpir_ir_solve_batched", "mpir_destroy", "mpir_status_str", "mpir_downcast",
    "mpir_get_factors", "mpir_residual", "mpir_residual_noalloc", "mpir_prof_enable", "mpir_prof_reset", "mpir_prof_get",
    "mpir_batch_create", "mpir_batch_run", "mpir_batch_destroy",
    "mpir_batch_get_tuning", "mpir_batch_set_tuning", "mpir_batch_autotune",
    "mpir_batch_phase_times",
]


class MpirError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})" if what else status_str(status))


class Term(C.Structure):
    _fields_ = [("Cr", C.c_double), ("Ce", C.c_double), ("Rmax", C.c_double),
                ("litmax", C.c_int32), ("residterm", C.c_int32), ("tol_rel", C.c_double),
                ("onthefly", C.c_int32), ("reserved", C.c_int32)]


TUNE_CLASSES = 8


class Tuning(C.Structure):
    """mpir_batch_tuning: per size class (n <= nmax[k]) the panel width and
    the trailing-update form of the batched kernel."""
    _fields_ = [("nclass", C.c_int32), ("from_cache", C.c_int32),
                ("nmax", C.c_int32 * TUNE_CLASSES), ("panel", C.c_int32 * TUNE_CLASSES),
                ("update", C.c_int32 * TUNE_CLASSES), ("ms", C.c_double * TUNE_CLASSES)]

    def as_dict(self):
        k = self.nclass
        return {"from_cache": bool(self.from_cache),
                "classes": [{"nmax": self.nmax[i], "panel": self.panel[i], "update": self.update[i],
                             "ms": round(self.ms[i], 4)} for i in range(k)]}


class Report(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("stop", C.c_int32), ("n_hist", C.c_int32),
                ("reserved", C.c_int32), ("rhist", C.c_double * HIST_MAX),
                ("dhist", C.c_double * HIST_MAX), ("relres", C.c_double),
                ("bwd_err", C.c_double), ("anorm_inf", C.c_double), ("bnorm_inf", C.c_double),
                ("xnorm_inf", C.c_double), ("info", C.c_int64), ("t_factor_ms", C.c_double),
                ("t_ir_ms", C.c_double)]

    @property
    def stop_name(self) -> str:
        return STOP_NAMES.get(self.stop, str(self.stop))

    def history(self):
        k = self.n_iter
        return np.array(self.rhist[:k + 1]), np.array(self.dhist[:k])


_lib = None


def lib():
    """Load libmpir.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        i64, i32, vp, d = C.c_int64, C.c_int32, C.c_void_p, C.c_double
        P = C.POINTER
        L.mpir_term_default.argtypes = [P(Term)]
        L.mpir_factor.restype = C.c_int
        L.mpir_factor.argtypes = [i64, vp, i64, C.c_int, C.c_int, C.c_int, vp, P(vp), P(i64)]
        L.mpir_refactor.restype = C.c_int
        L.mpir_refactor.argtypes = [vp, vp, i64, P(i64)]
        L.mpir_solve.restype = C.c_int
        L.mpir_solve.argtypes = [vp, vp, vp]
        L.mpir_ir_solve.restype = C.c_int
        L.mpir_ir_solve.argtypes = [vp, vp, vp, P(Term), P(Report)]
        L.mpir_bicgstab_ir_solve.restype = C.c_int
        L.mpir_bicgstab_ir_solve.argtypes = [vp, vp, vp, P(Term), i32, C.c_double, P(Report), P(i32)]
        L.mpir_ir_solve_multi.restype = C.c_int
        L.mpir_ir_solve_multi.argtypes = [vp, i32, vp, i64, vp, i64, P(Term), P(Report)]
        L.mpir_gmres_ir_solve.restype = C.c_int
        L.mpir_gmres_ir_solve.argtypes = [vp, vp, vp, P(Term), i32, C.c_double, P(Report), P(i32)]
        L.mpir_ir_solve_batched.restype = C.c_int
        L.mpir_ir_solve_batched.argtypes = [i32, P(i64), P(vp), P(i64), P(vp), P(vp), C.c_int,
                                            C.c_int, C.c_int, P(Term), P(Report), vp]
        L.mpir_destroy.argtypes = [vp]
        L.mpir_status_str.restype = C.c_char_p
        L.mpir_status_str.argtypes = [C.c_int]
        L.mpir_downcast.restype = C.c_int
        L.mpir_downcast.argtypes = [i64, vp, i64, C.c_int, C.c_int, vp, P(d), vp]
        L.mpir_get_factors.restype = C.c_int
        L.mpir_get_factors.argtypes = [vp, vp, vp]
        L.mpir_residual.restype = C.c_int
        L.mpir_residual.argtypes = [i64, vp, i64, C.c_int, C.c_int, vp, vp, vp, P(d), vp]
        L.mpir_residual_noalloc.restype = C.c_int
        L.mpir_residual_noalloc.argtypes = [i64, vp, i64, C.c_int, C.c_int, vp, vp, vp, P(d), vp]
        L.mpir_batch_create.restype = C.c_int
        L.mpir_batch_create.argtypes = [i32, P(i64), P(vp), P(i64), P(vp), P(vp), C.c_int, C.c_int,
                                        C.c_int, P(Term), i32, vp, P(vp)]
        L.mpir_batch_run.restype = C.c_int
        L.mpir_batch_run.argtypes = [vp, vp]
        L.mpir_batch_destroy.argtypes = [vp]
        L.mpir_batch_get_tuning.restype = C.c_int
        L.mpir_batch_get_tuning.argtypes = [C.c_int, C.c_int, P(Tuning)]
        L.mpir_batch_set_tuning.restype = C.c_int
        L.mpir_batch_set_tuning.argtypes = [C.c_int, C.c_int, P(Tuning)]
        L.mpir_batch_autotune.restype = C.c_int
        L.mpir_batch_autotune.argtypes = [C.c_int, C.c_int, C.c_char_p, vp, P(Tuning)]
        L.mpir_prof_enable.argtypes = [i32]
        L.mpir_prof_get.restype = C.c_int
        L.mpir_prof_get.argtypes = [i32, P(d), P(i64), P(d)]
        L.mpir_batch_phase_times.restype = C.c_int
        L.mpir_batch_phase_times.argtypes = [P(d), i32]
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().mpir_status_str(status).decode()


def _check(status: int, what: str, allow=(OK,)):
    if status not in allow:
        raise MpirError(status, what)
    return status


# ------------------------------------------------------------------ torch glue
def _torch():
    import torch
    return torch


def _prec_of_dtype(dt) -> int:
    torch = _torch()
    if dt == torch.float64:
        return F64
    if dt == torch.float32:
        return F32
    if dt == torch.float16:
        return F16
    if dt == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported dtype {dt}")


def _dtype_of_prec(p: int):
    torch = _torch()
    return {F64: torch.float64, F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}[p]


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t) -> C.c_void_p:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def term(Cr=1.0, Ce=1.0, Rmax=0.5, litmax=10, residterm=True, tol_rel=0.0,
         onthefly=False) -> Term:
    """The paper's TERM parameters (defaults = term_parms_default) and the
    solve form (onthefly: MPS instead of LPS)."""
    return Term(Cr, Ce, Rmax, litmax, 1 if residterm else 0, tol_rel, 1 if onthefly else 0, 0)


class Factorization:
    """A multiprecision factorization (the paper's MPF object).

    Borrows ``At`` (kept referenced here so it stays alive); owns the TF copy."""

    def __init__(self, At, tf: int, tr: int | None = None, stream=None):
        n, lda = At.shape[0], At.shape[1]
        if lda < n:
            raise ValueError("At must have shape (n, lda) with lda >= n")
        self.At = At
        self.n = n
        self.tw = _prec_of_dtype(At.dtype)
        self.tf = tf
        self.tr = self.tw if tr is None else tr
        self.stream = stream
        h = C.c_void_p(0)
        info = C.c_int64(0)
        st = lib().mpir_factor(n, _dev_ptr(At), lda, self.tw, tf, self.tr, _stream_ptr(stream),
                               C.byref(h), C.byref(info))
        self.status = st
        self.info = info.value
        _check(st, "mpir_factor", allow=(OK, ERR_SINGULAR))
        self._h = h

    def refactor(self, At):
        """mplu!(MPF, A): factor At into this handle.  On failure (other than a
        zero pivot) the handle holds no factorization and every solve raises
        (MPIR_ERR_STATE) until a refactor succeeds."""
        if At.shape != self.At.shape or _prec_of_dtype(At.dtype) != self.tw:
            raise ValueError("refactor needs the same size and precision")
        info = C.c_int64(0)
        st = lib().mpir_refactor(self._h, _dev_ptr(At), At.shape[1], C.byref(info))
        # the library now borrows At (also after a failure): keep it alive
        self.At, self.status, self.info = At, st, info.value
        _check(st, "mpir_refactor", allow=(OK, ERR_SINGULAR))
        return self

    def _vec(self, v, name):
        """Device pointer of a contiguous vector of n entries in TW."""
        if v.numel() != self.n or _prec_of_dtype(v.dtype) != self.tw:
            raise ValueError(f"{name} must hold n = {self.n} entries in the working precision")
        return _dev_ptr(v)

    def solve(self, b, x=None):
        torch = _torch()
        x = torch.empty_like(b) if x is None else x
        _check(lib().mpir_solve(self._h, self._vec(b, "b"), self._vec(x, "x")), "mpir_solve")
        return x

    def ir_solve(self, b, x=None, term_parms: Term | None = None):
        torch = _torch()
        x = torch.empty_like(b) if x is None else x
        rep = Report()
        tp = C.byref(term_parms) if term_parms is not None else None
        _check(lib().mpir_ir_solve(self._h, self._vec(b, "b"), self._vec(x, "x"), tp, C.byref(rep)),
               "mpir_ir_solve")
        return x, rep

    def ir_solve_multi(self, B, X=None, term_parms: Term | None = None, allow=(OK,)):
        """Several right-hand sides: B is (nrhs, n), row c = right-hand side c
        (column-major n x nrhs with ldb = B.stride(0)); returns (X, reports)."""
        torch = _torch()
        nrhs, n = B.shape
        if n != self.n or B.stride(1) != 1 or not B.is_cuda or _prec_of_dtype(B.dtype) != self.tw:
            raise ValueError("B must be a device tensor (nrhs, n) in TW with unit stride along n")
        X = torch.empty_like(B) if X is None else X
        if tuple(X.shape) != (nrhs, n) or X.stride(1) != 1 or X.dtype != B.dtype or not X.is_cuda:
            raise ValueError("X must be a device tensor (nrhs, n) of B's dtype with unit stride along n")
        reps = (Report * nrhs)()
        tp = C.byref(term_parms) if term_parms is not None else None
        # rows may be strided (ldb, ldx >= n): pass the base pointers as is
        _check(lib().mpir_ir_solve_multi(self._h, nrhs, C.c_void_p(B.data_ptr()), B.stride(0),
                                         C.c_void_p(X.data_ptr()), X.stride(0), tp, reps),
               "mpir_ir_solve_multi", allow)
        return X, list(reps)

    def bicgstab_ir_solve(self, b, x=None, term_parms: Term | None = None, maxit: int = 10,
                          inner_tol: float = 0.0):
        """BiCGSTAB-IR (the package's mpblu); returns (x, report, khist)."""
        torch = _torch()
        x = torch.empty_like(b) if x is None else x
        rep = Report()
        tp = C.byref(term_parms) if term_parms is not None else None
        litmax = term_parms.litmax if term_parms is not None else 10
        kh = (C.c_int32 * max(litmax, 1))()
        _check(lib().mpir_bicgstab_ir_solve(self._h, self._vec(b, "b"), self._vec(x, "x"), tp, int(maxit),
                                            float(inner_tol), C.byref(rep), kh),
               "mpir_bicgstab_ir_solve")
        return x, rep, [int(kh[i]) for i in range(rep.n_iter)]

    def gmres_ir_solve(self, b, x=None, term_parms: Term | None = None, basissize: int = 10,
                       gmres_tol: float = 0.0):
        """GMRES-IR (the package's mpglu); returns (x, report, khist)."""
        torch = _torch()
        x = torch.empty_like(b) if x is None else x
        rep = Report()
        tp = C.byref(term_parms) if term_parms is not None else None
        litmax = term_parms.litmax if term_parms is not None else 10
        kh = (C.c_int32 * max(litmax, 1))()
        _check(lib().mpir_gmres_ir_solve(self._h, self._vec(b, "b"), self._vec(x, "x"), tp, int(basissize),
                                         float(gmres_tol), C.byref(rep), kh),
               "mpir_gmres_ir_solve")
        return x, rep, [int(kh[i]) for i in range(rep.n_iter)]

    def factors(self):
        """(LU row-major tensor in TF, ipiv numpy int32)."""
        torch = _torch()
        lu = torch.empty((self.n, self.n), dtype=_dtype_of_prec(self.tf), device=self.At.device)
        ipiv = np.zeros(self.n, dtype=np.int32)
        _check(lib().mpir_get_factors(self._h, _dev_ptr(lu), ipiv.ctypes.data_as(C.c_void_p)),
               "mpir_get_factors")
        return lu, ipiv

    def destroy(self):
        if getattr(self, "_h", None):
            lib().mpir_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def factor(At, tf: int, tr: int | None = None, stream=None) -> Factorization:
    return Factorization(At, tf, tr, stream)


def ir_solve(At, b, tf: int, tr: int | None = None, term_parms: Term | None = None, stream=None):
    f = Factorization(At, tf, tr, stream)
    try:
        return f.ir_solve(b, term_parms=term_parms)
    finally:
        f.destroy()


def gmres_ir_solve(At, b, tf: int, term_parms: Term | None = None, basissize: int = 10,
                   gmres_tol: float = 0.0, stream=None):
    """GMRES-IR with TR = F64 (TW from At's dtype); returns (x, report, khist)."""
    f = Factorization(At, tf, F64, stream)
    try:
        return f.gmres_ir_solve(b, term_parms=term_parms, basissize=basissize, gmres_tol=gmres_tol)
    finally:
        f.destroy()


def bicgstab_ir_solve(At, b, tf: int, term_parms: Term | None = None, maxit: int = 10,
                      inner_tol: float = 0.0, stream=None):
    """BiCGSTAB-IR with TR = F64 (TW from At's dtype); returns (x, report, khist)."""
    f = Factorization(At, tf, F64, stream)
    try:
        return f.bicgstab_ir_solve(b, term_parms=term_parms, maxit=maxit, inner_tol=inner_tol)
    finally:
        f.destroy()


def downcast(At, tf: int, stream=None):
    """A_F = I_W^F(A) as a row-major (n, n) tensor in TF, and ||A||_inf."""
    torch = _torch()
    n, lda = At.shape
    out = torch.empty((n, n), dtype=_dtype_of_prec(tf), device=At.device)
    an = C.c_double(0.0)
    st = lib().mpir_downcast(n, _dev_ptr(At), lda, _prec_of_dtype(At.dtype), tf, _dev_ptr(out),
                             C.byref(an), _stream_ptr(stream))
    return out, an.value, st


def residual(At, b, x, tr: int = F64, stream=None):
    """r = b - A x in precision tr (eq. xferrule) and ||r||_inf."""
    torch = _torch()
    n, lda = At.shape
    r = torch.empty(n, dtype=_dtype_of_prec(tr), device=At.device)
    rn = C.c_double(0.0)
    _check(lib().mpir_residual(n, _dev_ptr(At), lda, _prec_of_dtype(At.dtype), tr, _dev_ptr(b),
                               _dev_ptr(x), _dev_ptr(r), C.byref(rn), _stream_ptr(stream)),
           "mpir_residual")
    return r, rn.value


RESIDUAL_NOALLOC_MAX_N = 16384


def residual_noalloc(At, b, x, r, tr: int = F64, stream=None):
    """mpir_residual_noalloc: r = b - A x in precision tr into the caller's r,
    with the library's fixed device scratch (no device allocation); returns
    ||r||_inf."""
    n, lda = At.shape
    if r.numel() != n or _prec_of_dtype(r.dtype) != tr:
        raise ValueError("r must hold n entries in precision tr")
    rn = C.c_double(0.0)
    _check(lib().mpir_residual_noalloc(n, _dev_ptr(At), lda, _prec_of_dtype(At.dtype), tr, _dev_ptr(b),
                                       _dev_ptr(x), _dev_ptr(r), C.byref(rn), _stream_ptr(stream)),
           "mpir_residual_noalloc")
    return rn.value


class Batch:
    """A batch of independent systems solved in one persistent launch
    (mpir_batch_*): the workspace is allocated once and, with use_graph, the
    launch sequence is captured in a hipGraph and replayed by run()."""

    def __init__(self, As, bs, xs, tf: int, tr: int = F64, term_parms: Term | None = None,
                 use_graph: bool = True, stream=None):
        k = len(As)
        self.keep = (As, bs, xs)
        self.k = k
        tw = _prec_of_dtype(As[0].dtype)
        ns = (C.c_int64 * k)(*[a.shape[0] for a in As])
        ldas = (C.c_int64 * k)(*[a.shape[1] for a in As])
        pa = (C.c_void_p * k)(*[_dev_ptr(a).value for a in As])
        pb = (C.c_void_p * k)(*[_dev_ptr(b).value for b in bs])
        px = (C.c_void_p * k)(*[_dev_ptr(x).value for x in xs])
        h = C.c_void_p(0)
        tp = C.byref(term_parms) if term_parms is not None else None
        _check(lib().mpir_batch_create(k, ns, pa, ldas, pb, px, tw, tf, tr, tp, 1 if use_graph else 0,
                                       _stream_ptr(stream), C.byref(h)), "mpir_batch_create")
        self._h = h

    def run(self):
        reps = (Report * self.k)()
        st = lib().mpir_batch_run(self._h, reps)
        if st not in (OK, ERR_SINGULAR, ERR_NONFINITE, ERR_RANGE):
            raise MpirError(st, "mpir_batch_run")
        return st, list(reps)

    def destroy(self):
        if getattr(self, "_h", None):
            lib().mpir_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def ir_solve_batched(As, bs, xs, tf: int, tr: int | None = None, term_parms: Term | None = None,
                     stream=None):
    """Batched IR over lists of column-major matrices / vectors (same TW)."""
    k = len(As)
    tw = _prec_of_dtype(As[0].dtype)
    tr = F64 if tr is None else tr
    ns = (C.c_int64 * k)(*[a.shape[0] for a in As])
    ldas = (C.c_int64 * k)(*[a.shape[1] for a in As])
    pa = (C.c_void_p * k)(*[a.data_ptr() for a in As])
    pb = (C.c_void_p * k)(*[b.data_ptr() for b in bs])
    px = (C.c_void_p * k)(*[x.data_ptr() for x in xs])
    reps = (Report * k)()
    tp = C.byref(term_parms) if term_parms is not None else None
    st = lib().mpir_ir_solve_batched(k, ns, pa, ldas, pb, px, tw, tf, tr, tp, reps,
                                     _stream_ptr(stream))
    return st, list(reps)


def batch_get_tuning(tw: int, tf: int) -> Tuning:
    t = Tuning()
    _check(lib().mpir_batch_get_tuning(tw, tf, C.byref(t)), "mpir_batch_get_tuning")
    return t


def batch_set_tuning(tw: int, tf: int, t: Tuning | None):
    _check(lib().mpir_batch_set_tuning(tw, tf, C.byref(t) if t is not None else None),
           "mpir_batch_set_tuning")


def batch_autotune(tw: int, tf: int, cache_path: str | None = None, stream=None) -> Tuning:
    """Measure (or read from cache_path) the batched kernel's configuration
    per size class and install it for (tw, tf)."""
    t = Tuning()
    cp = cache_path.encode() if cache_path else None
    _check(lib().mpir_batch_autotune(tw, tf, cp, _stream_ptr(stream), C.byref(t)), "mpir_batch_autotune")
    return t


def prof_enable(on: bool = True):
    lib().mpir_prof_enable(1 if on else 0)


def prof_reset():
    lib().mpir_prof_reset()


def prof_get(kind: int):
    ms, cnt, work = C.c_double(0), C.c_int64(0), C.c_double(0)
    _check(lib().mpir_prof_get(kind, C.byref(ms), C.byref(cnt), C.byref(work)), "mpir_prof_get")
    return ms.value, cnt.value, work.value


def batch_phase_times(reset: bool = False) -> dict:
    """Workgroup milliseconds of each phase of the batched kernel since the
    last reset, summed over workgroups and launches on the current device."""
    ms = (C.c_double * len(BATCH_PHASES))()
    _check(lib().mpir_batch_phase_times(ms, 1 if reset else 0), "mpir_batch_phase_times")
    return dict(zip(BATCH_PHASES, list(ms)))
