"""MI355X (gfx950) BOSP eigensolver for the linear response eigenvalue problem.

Thin Python binding of the C ABI in ``include/lrep.h``: every function has
the C name and only marshals arguments (pointers, sizes, structs); all
arithmetic runs in the HIP kernels of ``liblrep.so``.  PyTorch tensors (or
NumPy arrays for host buffers) provide the memory.

Matrices are column-major: an n x k argument is a tensor/array whose
element (i, j) is at offset i + j * ld, e.g. ``torch.empty(k, n).T`` or a
Fortran-ordered NumPy array.  ``colmajor(x)`` returns (pointer, ld, on_device).

The library must be built first (``python -m paper_2506_08355_amd.build`` or
``__graft_entry__.build()``); importing works without it, but the first call
raises ``LibraryNotBuilt`` -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrep.so")
HEADERS = [os.path.join(os.path.dirname(HERE), "include", h) for h in ("lrep.h", "lrep_testing.h")]

LREP_OK = 0
LREP_EINVAL = -1
LREP_ENOMEM = -2
LREP_ENOTCONV = -3
LREP_EBREAKDOWN = -4
LREP_ENOTSPD = -5
LREP_ENUMERIC = -6
LREP_EDEVICE = -7
LREP_EAGAIN = -8
LREP_ECANCELED = -9

LREP_DEVICE_PTR = 0x1
LREP_BORROW = 0x2
LREP_INPUT_AB = 0x4
LREP_NULL_ON_M = 0x8


class LibraryNotBuilt(RuntimeError):
    pass


class LrepError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class lrep_solve_opts_t(ctypes.Structure):
    _fields_ = [
        ("window", ctypes.c_int64),
        ("maxit", ctypes.c_int64),
        ("ngs", ctypes.c_int32),
        ("cg_maxit", ctypes.c_int32),
        ("cg_tol", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("init_U", ctypes.c_void_p),
        ("ld_init", ctypes.c_int64),
        ("init_on_device", ctypes.c_int32),
        ("result_on_device", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("rebiorth_tol", ctypes.c_double),
        ("refresh", ctypes.c_int32),
        ("graphs", ctypes.c_int32),
        ("fused_cg", ctypes.c_int32),
        ("serve_batch", ctypes.c_int32),
    ]


class lrep_stats_t(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int64),
        ("n_converged", ctypes.c_int64),
        ("applies_K", ctypes.c_int64),
        ("applies_M", ctypes.c_int64),
        ("mgs_drops", ctypes.c_int64),
        ("locks", ctypes.c_int64),
        ("rebiorth", ctypes.c_int64),
        ("max_eps", ctypes.c_double),
        ("time_ms", ctypes.c_double),
        ("phase_ms", ctypes.c_double * 5),
        ("prof_launches", ctypes.c_int64),
        ("prof_ms", ctypes.c_double),
        ("prof_bytes", ctypes.c_double),
        ("prof_flops", ctypes.c_double),
        ("cg_batched", ctypes.c_int64),
        ("cg_batch_columns", ctypes.c_int64),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "phase_ms"}
        d["phase_ms"] = list(self.phase_ms)
        return d


class lrep_request_t(ctypes.Structure):
    _fields_ = [
        ("nev", ctypes.c_int64),
        ("block", ctypes.c_int64),
        ("tol", ctypes.c_double),
        ("opts", lrep_solve_opts_t),
        ("lambda_", ctypes.c_void_p),
        ("X", ctypes.c_void_p),
        ("Y", ctypes.c_void_p),
        ("ldxy", ctypes.c_int64),
    ]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double

_SIGS = {
    "lrep_init": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_size_t, _P]),
    "lrep_finalize": (ctypes.c_int, [_P]),
    "lrep_create_dense": (ctypes.c_int, [_P, _I64, _P, _P, _I64, ctypes.c_uint32, ctypes.POINTER(_P)]),
    "lrep_create_lowrank": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _I64, ctypes.c_uint32, ctypes.POINTER(_P)]),
    "lrep_create_callback": (ctypes.c_int, [_P, _I64, _P, _P, ctypes.c_uint32, ctypes.POINTER(_P)]),
    "lrep_set_nullspace": (ctypes.c_int, [_P, _I64, _P, _I64, _I32]),
    "lrep_set_metric": (ctypes.c_int, [_P, _I64, _P, ctypes.c_uint32]),
    "lrep_xy_to_uv": (ctypes.c_int, [_P, _I64, _I64, _P, _P, _I64, _P, _P, _I64]),
    "lrep_set_metric_dense": (ctypes.c_int, [_P, _I64, _P, _I64, ctypes.c_uint32]),
    "lrep_find_nullspace": (ctypes.c_int, [_P, _I64, _D, ctypes.c_uint64, ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    "lrep_destroy_op": (ctypes.c_int, [_P]),
    "lrep_solve": (ctypes.c_int, [_P, _I64, _I64, _I64, _D, ctypes.POINTER(lrep_solve_opts_t), _P, _P, _P, _I64,
                                  ctypes.POINTER(lrep_stats_t)]),
    "lrep_submit": (ctypes.c_int, [_P, _P, ctypes.POINTER(lrep_request_t), ctypes.POINTER(ctypes.c_uint64)]),
    "lrep_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(lrep_stats_t)]),
    "lrep_cancel": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "lrep_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lrep_last_error": (ctypes.c_char_p, [_P]),
    "lrep_version": (ctypes.c_int, []),
    "lrep_test_gemm_nn": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _I64, _P, _I64, _P, _I64,
                                         _D, _D, ctypes.c_int]),
    "lrep_test_gemm_tn": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _I64, _P, _I64, _P, _I64,
                                         ctypes.c_int]),
    "lrep_test_small_lrep": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _I64, _P, _P, _P]),
    "lrep_test_block_mgs": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P, ctypes.POINTER(ctypes.c_int)]),
    "lrep_test_apply": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "lrep_apply_noalloc": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P]),
    "lrep_test_cg": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P, _D, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(_I64)]),
    "lrep_test_convert16": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _I64, _P]),
    "lrep_test_apply16": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P]),
    "lrep_test_read": (ctypes.c_int, [_P, _P, _I64, ctypes.c_int, ctypes.c_int, _P, ctypes.POINTER(ctypes.c_double)]),
    "lrep_test_copy": (ctypes.c_int, [_P, _P, _P, _I64]),
}


def lib():
    """The loaded ``liblrep.so`` (raises LibraryNotBuilt if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryNotBuilt(f"{LIB_PATH} not found: build it with python -m paper_2506_08355_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    """Function names declared in the public headers."""
    names = []
    for h in HEADERS:
        with open(h) as fh:
            txt = fh.read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"\b(lrep_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


def _check(rc, ctx=None, what=""):
    if rc != LREP_OK:
        detail = ""
        if ctx is not None:
            detail = lib().lrep_last_error(ctx).decode()
        raise LrepError(rc, f"{what}: {lib().lrep_strerror(rc).decode()} {detail}".strip())
    return rc


def _ready(x):
    """The library does not order its streams after torch's: wait for the
    work torch has queued on a device tensor's current stream, so that the
    data behind the pointer is complete when the library reads it."""
    if x.is_cuda:
        import torch
        torch.cuda.current_stream(x.device).synchronize()


def colmajor(x):
    """(pointer, leading dimension, on_device) of a column-major matrix/vector
    (for a device tensor, after torch's queued work on it has finished)."""
    try:
        import torch
        if isinstance(x, torch.Tensor):
            if x.dtype != torch.float64:
                raise TypeError("FP64 tensors required")
            _ready(x)
            if x.dim() == 1:
                if x.stride(0) != 1:
                    raise ValueError("vector must be contiguous")
                return x.data_ptr(), x.shape[0], x.is_cuda
            if x.stride(0) != 1:
                raise ValueError("matrix must be column-major (stride(0) == 1), e.g. torch.empty(k, n).T")
            return x.data_ptr(), max(x.stride(1), x.shape[0]), x.is_cuda
    except ImportError:
        pass
    import numpy as np
    if not isinstance(x, np.ndarray) or x.dtype != np.float64:
        raise TypeError("expected a float64 torch tensor or numpy array")
    if x.ndim == 1:
        if not x.flags.c_contiguous:
            raise ValueError("vector must be contiguous")
        return x.ctypes.data, x.shape[0], False
    if x.strides[0] != 8:
        raise ValueError("matrix must be column-major (Fortran order)")
    return x.ctypes.data, max(x.strides[1] // 8, x.shape[0]), False


# ---------------------------------------------------------------- C names
def lrep_init(device: int = 0, hbm_budget_bytes: int = 0, hip_stream: Optional[int] = None):
    h = _P()
    _check(lib().lrep_init(ctypes.byref(h), device, hbm_budget_bytes, hip_stream), what="lrep_init")
    return h


def lrep_finalize(ctx):
    return _check(lib().lrep_finalize(ctx), what="lrep_finalize")


def lrep_create_dense(ctx, K, M, flags: int = 0):
    pk, ldk, dk = colmajor(K)
    pm, ldm, dm = colmajor(M)
    if ldk != ldm or dk != dm or K.shape != M.shape or K.shape[0] != K.shape[1]:
        raise ValueError("K and M must be square, same shape, layout and location")
    if dk:
        flags |= LREP_DEVICE_PTR
    op = _P()
    _check(lib().lrep_create_dense(ctx, K.shape[0], pk, pm, ldk, flags, ctypes.byref(op)), ctx, "lrep_create_dense")
    return op


# C type of the operator product callback (lrep_apply_fn)
APPLY_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p)
_callbacks = {}   # op handle -> the ctypes callback, kept alive while the operator exists


def lrep_create_callback(ctx, n, apply, flags: int = 0):
    """Matrix-free operator: apply(which, cols, X_ptr, ldx, Y_ptr, ldy, stream)
    makes Y = K X (which 0) or M X (which 1) on the device (raw pointers,
    column-major) and returns 0; see lrep_apply_fn in lrep.h."""
    def tramp(user, which, cols, X, ldx, Y, ldy, stream):
        try:
            return int(apply(which, cols, X, ldx, Y, ldy, stream))
        except Exception:   # an exception must not cross the C boundary
            return -1
    cb = APPLY_FN(tramp)
    op = _P()
    _check(lib().lrep_create_callback(ctx, n, ctypes.cast(cb, ctypes.c_void_p), None, flags, ctypes.byref(op)), ctx,
           "lrep_create_callback")
    _callbacks[op.value] = cb
    return op


def lrep_create_lowrank(ctx, delta, L, flags: int = 0):
    pd, n, dd = colmajor(delta)
    pl, ldl, dl = colmajor(L)
    if dd != dl or L.shape[0] != n:
        raise ValueError("delta and L must share n and location")
    if dd:
        flags |= LREP_DEVICE_PTR
    op = _P()
    _check(lib().lrep_create_lowrank(ctx, n, L.shape[1], pd, pl, ldl, flags, ctypes.byref(op)), ctx,
           "lrep_create_lowrank")
    return op


def lrep_set_nullspace(op, X0, ctx=None):
    if X0 is None:
        return _check(lib().lrep_set_nullspace(op, 0, None, 1, 0), ctx, "lrep_set_nullspace")
    p, ld, dev = colmajor(X0)
    return _check(lib().lrep_set_nullspace(op, X0.shape[1], p, ld, int(dev)), ctx, "lrep_set_nullspace")


def lrep_find_nullspace(op, rmax, tol=1e-10, seed=0, ctx=None):
    """Compute and declare the null space of the semidefinite operator;
    returns (r, residual) -- see lrep_find_nullspace in lrep.h."""
    r = ctypes.c_int64(0)
    res = ctypes.c_double(0.0)
    _check(lib().lrep_find_nullspace(op, rmax, tol, seed, ctypes.byref(r), ctypes.byref(res)), ctx,
           "lrep_find_nullspace")
    return r.value, res.value


def lrep_set_metric(op, b, ctx=None):
    """Diagonal metric B = diag(b) of a generalized LREP (b: n positive
    values, a NumPy array or a device tensor)."""
    if b.ndim != 1:
        raise ValueError("b must be a vector")
    p, _, dev = colmajor(b)
    return _check(lib().lrep_set_metric(op, b.shape[0], p, LREP_DEVICE_PTR if dev else 0), ctx, "lrep_set_metric")


def lrep_xy_to_uv(ctx, X, Y, U, V):
    """U = Y + X, V = Y - X for column-major device tensors (n x nev): the
    eigenvectors of [[A, B], [-B, -A]] from those of H."""
    px, ldx, dx = colmajor(X)
    py, ldy, dy = colmajor(Y)
    pu, ldu, du = colmajor(U)
    pv, ldv, dv = colmajor(V)
    if not (dx and dy and du and dv) or ldx != ldy or ldu != ldv or X.shape != Y.shape or U.shape != X.shape \
            or V.shape != X.shape:
        raise ValueError("X, Y, U, V must be device tensors of one shape, X/Y and U/V with equal leading dimensions")
    return _check(lib().lrep_xy_to_uv(ctx, X.shape[0], X.shape[1], px, py, ldx, pu, pv, ldu), ctx, "lrep_xy_to_uv")


def lrep_set_metric_dense(op, B, ctx=None):
    """Dense SPD metric B (n x n, column-major NumPy array or device tensor;
    its lower triangle is read) of a generalized LREP, for dense operators."""
    if B.ndim != 2 or B.shape[0] != B.shape[1]:
        raise ValueError("B must be square")
    p, ld, dev = colmajor(B)
    return _check(lib().lrep_set_metric_dense(op, B.shape[0], p, ld, LREP_DEVICE_PTR if dev else 0), ctx,
                  "lrep_set_metric_dense")


def lrep_destroy_op(op):
    rc = _check(lib().lrep_destroy_op(op), what="lrep_destroy_op")
    _callbacks.pop(op.value if isinstance(op, _P) else op, None)
    return rc


def make_opts(window=0, maxit=0, ngs=0, cg_maxit=0, cg_tol=0.0, seed=0, init=None, result_on_device=False,
              rebiorth_tol=0.0, profile=False, refresh=0, precision=0, graphs=0, fused_cg=0, serve_batch=0):
    o = lrep_solve_opts_t()
    o.graphs = graphs
    o.fused_cg = fused_cg
    o.serve_batch = serve_batch
    o.window, o.maxit, o.ngs, o.cg_maxit, o.cg_tol, o.seed = window, maxit, ngs, cg_maxit, cg_tol, seed
    if init is not None:
        p, ld, dev = colmajor(init)
        o.init_U, o.ld_init, o.init_on_device = p, ld, int(dev)
    o.result_on_device = int(result_on_device)
    o.rebiorth_tol = rebiorth_tol
    o.profile = int(profile)
    o.refresh = int(refresh)
    o.precision = int(precision)
    return o


def lrep_solve(op, n, nev, block, tol, opts, lam, X, Y, ctx=None, check=True):
    """Returns (rc, stats).  lam (nev), X, Y (n x nev column-major) are filled."""
    pl, _, dl = colmajor(lam)
    px, ldx, dx = colmajor(X)
    py, ldy, dy = colmajor(Y)
    if ldx != ldy or not (dl == dx == dy):
        raise ValueError("X and Y must share layout and location with lambda")
    if opts is None:
        opts = make_opts()
    opts.result_on_device = int(dx)
    st = lrep_stats_t()
    rc = lib().lrep_solve(op, n, nev, block, tol, ctypes.byref(opts), pl, px, py, ldx, ctypes.byref(st))
    if check and rc not in (LREP_OK,):
        _check(rc, ctx, "lrep_solve")
    return rc, st


def lrep_submit(ctx, op, nev, block, tol, opts, lam, X, Y):
    pl, _, dl = colmajor(lam)
    px, ldx, dx = colmajor(X)
    py, ldy, dy = colmajor(Y)
    r = lrep_request_t()
    r.nev, r.block, r.tol = nev, block, tol
    if opts is None:
        opts = make_opts()
    opts.result_on_device = int(dx)
    r.opts = opts
    r.lambda_, r.X, r.Y, r.ldxy = pl, px, py, ldx
    t = ctypes.c_uint64()
    _check(lib().lrep_submit(ctx, op, ctypes.byref(r), ctypes.byref(t)), ctx, "lrep_submit")
    return t.value


def lrep_poll(ctx, ticket):
    st = lrep_stats_t()
    rc = lib().lrep_poll(ctx, ticket, ctypes.byref(st))
    return rc, st


def lrep_cancel(ctx, ticket):
    return lib().lrep_cancel(ctx, ticket)


def lrep_strerror(code):
    return lib().lrep_strerror(code).decode()


def lrep_last_error(ctx):
    return lib().lrep_last_error(ctx).decode()


def lrep_version():
    return lib().lrep_version()


# ------------------------------------------------------------- test hooks
def lrep_test_gemm_nn(ctx, A, B, C, alpha=1.0, beta=0.0, ksplit=0):
    pa, lda, _ = colmajor(A)
    pb, ldb, _ = colmajor(B)
    pc, ldc, _ = colmajor(C)
    m, p = A.shape
    q = B.shape[1]
    return _check(lib().lrep_test_gemm_nn(ctx, m, q, p, pa, lda, pb, ldb, pc, ldc, alpha, beta, ksplit), ctx,
                  "lrep_test_gemm_nn")


def lrep_test_gemm_tn(ctx, A, B, C, symmetrize=False):
    pa, lda, _ = colmajor(A)
    pb, ldb, _ = colmajor(B)
    pc, ldc, _ = colmajor(C)
    return _check(lib().lrep_test_gemm_tn(ctx, A.shape[0], A.shape[1], B.shape[1], pa, lda, pb, ldb, pc, ldc,
                                          int(symmetrize)), ctx, "lrep_test_gemm_tn")


def lrep_test_small_lrep(ctx, Kh, Mh, lam, Xh, Yh):
    pk, ldh, _ = colmajor(Kh)
    pm, _, _ = colmajor(Mh)
    return lib().lrep_test_small_lrep(ctx, Kh.shape[0], pk, pm, ldh, colmajor(lam)[0], colmajor(Xh)[0],
                                      colmajor(Yh)[0])


def lrep_test_block_mgs(ctx, X, Y):
    px, ld, _ = colmajor(X)
    py, _, _ = colmajor(Y)
    k = ctypes.c_int()
    _check(lib().lrep_test_block_mgs(ctx, X.shape[0], X.shape[1], px, py, ctypes.byref(k)), ctx,
           "lrep_test_block_mgs")
    return k.value


def lrep_apply_noalloc(op, which, X, Y, ctx=None):
    """Y = K X (which 0) or M X (which 1) through the allocation-free entry
    point; X, Y device tensors of n x cols in column-major layout."""
    px, ldx, _ = colmajor(X)
    py, ldy, _ = colmajor(Y)
    if ldx != X.shape[0] or ldy != Y.shape[0] or X.shape != Y.shape:
        raise ValueError("X and Y must be n x cols with leading dimension n")
    return _check(lib().lrep_apply_noalloc(op, which, X.shape[1], px, py), ctx, "lrep_apply_noalloc")


def lrep_test_cg(op, which, B, X, tol=1e-2, maxit=20, fused=0):
    """One Step-6 CG solve A X = B (A = K for which 0, M for 1) on device
    tensors (n x nw, ld n); returns the number of column applies."""
    k = _I64()
    _check(lib().lrep_test_cg(op, which, B.shape[1], colmajor(B)[0], colmajor(X)[0], tol, maxit, fused,
                              ctypes.byref(k)), what="lrep_test_cg")
    return k.value


def lrep_test_apply(op, which, X, Y):
    return _check(lib().lrep_test_apply(op, which, X.shape[1], colmajor(X)[0], colmajor(Y)[0]),
                  what="lrep_test_apply")


def lrep_test_convert16(ctx, precision, A, out):
    """out (n * n 16-bit device tensor, column-major n x n; 3 n * n, the hi,
    mid and lo parts, for precision 3) = the 16-bit copy of the column-major
    FP64 device matrix A."""
    p, ld, _ = colmajor(A)
    n = A.shape[0]
    parts = 3 if precision == 3 else 1
    if out.numel() != parts * n * n or out.element_size() != 2:
        raise ValueError("out must hold %d n * n 16-bit values" % parts)
    _ready(out)
    return _check(lib().lrep_test_convert16(ctx, precision, n, p, ld, ctypes.c_void_p(out.data_ptr())), ctx,
                  "lrep_test_convert16")


def lrep_test_apply16(ctx, precision, A16, X, rr, Y):
    """Y = A16 X on a 16-bit copy (X, Y column-major device n x cols, rr the
    device vector of squared column norms of X)."""
    n, cols = X.shape
    parts = 3 if precision == 3 else 1
    if A16.numel() != parts * n * n or A16.element_size() != 2:
        raise ValueError("A16 must hold %d n * n 16-bit values" % parts)
    _ready(A16)
    return _check(lib().lrep_test_apply16(ctx, precision, n, cols, ctypes.c_void_p(A16.data_ptr()),
                                          colmajor(X)[0], ctypes.c_void_p(rr.data_ptr()), colmajor(Y)[0]),
                  ctx, "lrep_test_apply16")


def lrep_test_read(ctx, src, out, iters=1):
    """out[b] = block b's share of the sum of the contiguous FP64 device
    tensor src (a plain streaming read), len(out) blocks, `iters` launches;
    returns their total time in ms (HIP events on the library's stream)."""
    _ready(src)
    ms = ctypes.c_double(0.0)
    _check(lib().lrep_test_read(ctx, ctypes.c_void_p(src.data_ptr()), src.numel(), out.numel(), iters,
                                ctypes.c_void_p(out.data_ptr()), ctypes.byref(ms)), ctx, "lrep_test_read")
    return ms.value


def lrep_test_copy(ctx, src, dst):
    """dst = src for two contiguous FP64 device tensors of the same even length."""
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in size")
    _ready(src)
    return _check(lib().lrep_test_copy(ctx, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                       src.numel()), ctx, "lrep_test_copy")
