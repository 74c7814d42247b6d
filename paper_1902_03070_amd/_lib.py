"""ctypes binding of libtsvdmi (include/tsvdmi.h).  Argument marshalling only.

Tensors are torch tensors on a ROCm device with logical shape (n1, n2, n3) in
column-major layout (strides (1, n1, n1*n2)), the layout of the C interface.
``fortran(x)`` makes such a view; outputs are allocated in that layout.
Every computation runs in the HIP library; if it is not built, importing this
module raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsvdmi.so")

FP64, FP32, MIXED = 0, 1, 2
OK, WARN_NOCONV, EINVAL, ENOMEM, EHIP, ENONFINITE, EBUSY, ETIMEOUT, ECANCELED = 0, 1, -1, -2, -3, -4, -5, -6, -7
OPT_MAX_SWEEPS, OPT_SYNC_STATUS, OPT_TEAM_SIZE, OPT_SPIN_LIMIT, OPT_PROFILE, OPT_GRAPHS = 0, 1, 2, 3, 4, 5
OPT_AUTOTUNE, OPT_GROUP_LANES, OPT_GROUP_COLUMNS, OPT_WARM_START, OPT_COOPERATIVE, OPT_GRAM = 6, 7, 8, 9, 10, 11
OPT_LONG_TUBES = 12
OPT_TEAM_SLOTS = 13
OPT_KEPT_COLUMNS = 14
PHASES = ("forward_transform", "jacobi", "threshold_rebuild", "inverse_transform", "warm_start", "certificate")
TRANSFORM_DOMAIN, FULL = 1, 2
REQ_TSVT, REQ_COMPLETE = 0, 1

EXPORTED = [
    "tsvd_create", "tsvd_destroy", "tsvd_last_error", "tsvd_set_option", "tsvd_get_option", "tsvd_sync_status",
    "tsvd_get_stats", "tsvd_get_tile",
    "tprod_dct", "tsvd_dct", "tsvt_dct", "tsvt_dct_noalloc", "tsvt_transform", "tsvt_dft", "tnn_c", "tnn_f",
    "complete_tensor", "tsvt_dct_batched", "tsvd_server_create",
    "tsvd_server_submit", "tsvd_server_cancel", "tsvd_server_poll", "tsvd_server_now", "tsvd_server_stats",
    "tsvd_server_destroy",
]

if not os.path.exists(LIB_PATH):
    raise ImportError("libtsvdmi.so is not built (run __graft_entry__.build() or python -m paper_1902_03070_amd.build)")

lib = C.CDLL(LIB_PATH)

_vp, _i64, _i32, _d = C.c_void_p, C.c_int64, C.c_int, C.c_double


class CompleteOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("tol", C.c_double), ("beta", C.c_double),
                ("tau_schedule", C.POINTER(C.c_double)), ("check_every", C.c_int), ("start_iter", C.c_int),
                ("M_init", C.c_void_p), ("M_out", C.c_void_p), ("init_observed", C.c_int)]


class CompleteInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("rel_change", C.c_double), ("status", C.c_int), ("max_sweeps", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("slice_sweeps", C.c_int64), ("ms", C.c_double * 6), ("launches", C.c_int64 * 6),
                ("pairs", C.c_int64), ("fallback_slices", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("kind", C.c_int), ("n1", C.c_int64), ("n2", C.c_int64), ("n3", C.c_int64),
                ("input", C.POINTER(C.c_float)), ("mask", C.POINTER(C.c_uint8)), ("tau", C.c_double),
                ("iters", C.c_int), ("tau0", C.c_double), ("tau1", C.c_double), ("deadline_s", C.c_double)]


lib.tsvd_create.argtypes = [C.POINTER(_vp), _i32]
lib.tsvd_destroy.argtypes = [_vp]
lib.tsvd_destroy.restype = None
lib.tsvd_last_error.argtypes = [_vp]
lib.tsvd_last_error.restype = C.c_char_p
lib.tsvd_set_option.argtypes = [_vp, _i32, _d]
lib.tsvd_get_option.argtypes = [_vp, _i32]
lib.tsvd_get_option.restype = _d
lib.tsvd_sync_status.argtypes = [_vp, _vp, C.POINTER(C.c_int)]
lib.tsvd_get_stats.argtypes = [_vp, _vp, C.POINTER(Stats), _i32]
lib.tsvd_get_tile.argtypes = [_vp, _i32, _i64, _i64, _i64, _i32, _i32, C.POINTER(C.c_int32)]
lib.tprod_dct.argtypes = [_vp, _i32, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp]
lib.tsvd_dct.argtypes = [_vp, _i32, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _i32, _vp]
lib.tsvt_dct.argtypes = [_vp, _i32, _i64, _i64, _i64, _vp, _vp, _d, C.POINTER(C.c_int32), _vp]
lib.tsvt_dct_noalloc.argtypes = [_vp, _i32, _i64, _i64, _i64, _vp, _vp, _d, C.POINTER(C.c_int32), _vp]
lib.tsvt_transform.argtypes = [_vp, _i32, _i64, _i64, _i64, C.POINTER(_d), _vp, _vp, _d, C.POINTER(C.c_int32), _vp]
lib.tsvt_dft.argtypes = [_vp, _i32, _i64, _i64, _i64, _vp, _vp, _d, C.POINTER(C.c_int32), _vp]
lib.tnn_c.argtypes = [_vp, _i32, _i64, _i64, _i64, _vp, C.POINTER(_d), _vp]
lib.tnn_f.argtypes = [_vp, _i32, _i64, _i64, _i64, _vp, C.POINTER(_d), _vp]
lib.complete_tensor.argtypes = [_vp, _i32, _i64, _i64, _i64, _vp, _vp, _vp, C.POINTER(CompleteOpts),
                                C.POINTER(CompleteInfo), _vp]
lib.tsvt_dct_batched.argtypes = [_vp, _i32, _i32, C.POINTER(C.c_int64), C.POINTER(_vp), C.POINTER(_vp),
                                 C.POINTER(C.c_double), C.POINTER(C.c_int32), _vp]
lib.tsvd_server_create.argtypes = [C.POINTER(_vp), _vp, _i32, _i64, _i32]
lib.tsvd_server_submit.argtypes = [_vp, C.POINTER(Request)]
lib.tsvd_server_submit.restype = _i64
lib.tsvd_server_cancel.argtypes = [_vp, _i64]
lib.tsvd_server_poll.argtypes = [_vp, _i64, C.POINTER(C.c_float), C.POINTER(_d), C.POINTER(_d), C.POINTER(_d)]
lib.tsvd_server_now.argtypes = [_vp]
lib.tsvd_server_now.restype = _d
lib.tsvd_server_stats.argtypes = [_vp] + [C.POINTER(C.c_int64)] * 4
lib.tsvd_server_destroy.argtypes = [_vp]
lib.tsvd_server_destroy.restype = None


class TsvdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("tsvdmi error %d: %s" % (code, msg))
        self.code = code


class Context:
    """Owns a tsvd_ctx (device workspace, transform matrices, options)."""

    def __init__(self, device: int = 0):
        h = _vp()
        rc = lib.tsvd_create(C.byref(h), device)
        if rc != OK:
            raise TsvdError(rc, "tsvd_create(%d) failed" % device)
        self.h = h
        self.device = device
        _register(self)

    def close(self):
        if self.h:
            lib.tsvd_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP call while the interpreter shuts down: contexts still open
        # then were closed by the exit hook below, before the runtime's own
        # teardown; anything left is reclaimed by the process exit (the check
        # is bound at definition time: module globals may already be gone)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int, allow_warn: bool = True) -> int:
        if rc < 0 or (rc > 0 and not allow_warn):
            raise TsvdError(rc, lib.tsvd_last_error(self.h).decode())
        return rc

    def set_option(self, opt: int, value: float):
        self.check(lib.tsvd_set_option(self.h, opt, float(value)))

    def get_option(self, opt: int) -> float:
        return lib.tsvd_get_option(self.h, opt)

    def stats(self, reset: bool = True, stream=None) -> dict:
        st = Stats()
        self.check(lib.tsvd_get_stats(self.h, _stream(stream, self.device), C.byref(st), int(reset)))
        return {"slice_sweeps": st.slice_sweeps,
                "pairs": st.pairs, "fallback_slices": st.fallback_slices,
                "ms": {PHASES[i]: st.ms[i] for i in range(6)},
                "launches": {PHASES[i]: st.launches[i] for i in range(6)}}

    def tile(self, prec: int, n1: int, n2: int, n3: int, batched: bool = False, with_v: bool = False) -> dict:
        """Jacobi tile this context uses for the shape (tunes it if needed)."""
        out = (C.c_int32 * 6)()
        self.check(lib.tsvd_get_tile(self.h, prec, n1, n2, n3, int(batched), int(with_v), out))
        return dict(zip(("team", "G", "W", "threads", "source", "K"), list(out)))

    def sync_status(self, stream=None):
        ms = C.c_int(0)
        rc = lib.tsvd_sync_status(self.h, _stream(stream, self.device), C.byref(ms))
        return rc, ms.value


_contexts = {}
_open = []  # weak references to every context and server, closed at exit


def default_context(device: int = 0) -> Context:
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


def _register(obj):
    import weakref

    _open[:] = [r for r in _open if r() is not None]
    _open.append(weakref.ref(obj))


def close_all():
    """Close every server and context this process opened (servers first).

    Runs at interpreter exit, before module teardown, so that no device object
    of the library outlives the HIP runtime or a profiler attached to it."""
    objs = [r() for r in _open]
    for o in objs:
        if isinstance(o, Server):
            o.close()
    for o in objs:
        if isinstance(o, Context):
            o.close()
    _open.clear()
    _contexts.clear()


atexit.register(close_all)


def _stream(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return _vp(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def fortran(x: torch.Tensor) -> torch.Tensor:
    """Column-major view (strides 1, n1, n1*n2) of a 3-D tensor, copying if needed."""
    if x.dim() == 2:
        x = x.unsqueeze(2)
    if x.dim() != 3:
        raise ValueError("expected a 3-D tensor")
    n1, n2, n3 = x.shape
    if x.stride() == (1, n1, n1 * n2) or x.numel() == 0:
        return x
    return x.permute(2, 1, 0).contiguous().permute(2, 1, 0)


def empty_f(n1: int, n2: int, n3: int, dtype, device) -> torch.Tensor:
    return torch.empty((n3, n2, n1), dtype=dtype, device=device).permute(2, 1, 0)


def _prec_of(t: torch.Tensor, prec: Optional[int]) -> int:
    if prec is None:
        prec = FP64 if t.dtype == torch.float64 else FP32
    want = torch.float64 if prec == FP64 else torch.float32
    if t.dtype != want:
        raise TypeError("precision %d needs %s data, got %s" % (prec, want, t.dtype))
    return prec


def _dev(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("tensors must be on a ROCm device")
    return t.device.index or 0


def tsvt_dct(Z: torch.Tensor, tau: float, Y: Optional[torch.Tensor] = None, prec: Optional[int] = None,
             return_ranks: bool = False, ctx: Optional[Context] = None, stream=None):
    """t-SVT with threshold tau (Theorem 5).  Returns Y (and per-slice ranks)."""
    Z = fortran(Z)
    d = _dev(Z)
    prec = _prec_of(Z, prec)
    ctx = ctx or default_context(d)
    n1, n2, n3 = Z.shape
    if Y is None:
        Y = empty_f(n1, n2, n3, Z.dtype, Z.device)
    ranks = (C.c_int32 * n3)() if return_ranks else None
    rc = lib.tsvt_dct(ctx.h, prec, n1, n2, n3, Z.data_ptr(), Y.data_ptr(), float(tau), ranks,
                      _stream(stream, d))
    ctx.check(rc)
    if return_ranks:
        return Y, [int(r) for r in ranks]
    return Y


def tsvt_transform(Z: torch.Tensor, tau: float, L, Y: Optional[torch.Tensor] = None, prec: Optional[int] = None,
                   return_ranks: bool = False, ctx: Optional[Context] = None, stream=None):
    """t-SVT under an invertible transform L (n3 x n3, host, row-major
    L[k][t]) along the tubes in place of the DCT."""
    Z = fortran(Z)
    d = _dev(Z)
    prec = _prec_of(Z, prec)
    ctx = ctx or default_context(d)
    n1, n2, n3 = Z.shape
    Lf = [float(v) for row in L for v in row] if not hasattr(L, "ravel") else [float(v) for v in L.ravel()]
    if len(Lf) != n3 * n3:
        raise ValueError("L must be n3 x n3")
    Lc = (C.c_double * (n3 * n3))(*Lf)
    if Y is None:
        Y = empty_f(n1, n2, n3, Z.dtype, Z.device)
    ranks = (C.c_int32 * n3)() if return_ranks else None
    ctx.check(lib.tsvt_transform(ctx.h, prec, n1, n2, n3, Lc, Z.data_ptr(), Y.data_ptr(), float(tau), ranks,
                                 _stream(stream, d)))
    if return_ranks:
        return Y, [int(r) for r in ranks]
    return Y


def tsvt_dft(Z: torch.Tensor, tau: float, Y: Optional[torch.Tensor] = None, prec: Optional[int] = None,
             return_ranks: bool = False, ctx: Optional[Context] = None, stream=None):
    """Fourier-domain t-SVT (the prox of tau * TNN-F).  Returns Y (and the
    rank of every Fourier slice)."""
    Z = fortran(Z)
    d = _dev(Z)
    prec = _prec_of(Z, prec)
    ctx = ctx or default_context(d)
    n1, n2, n3 = Z.shape
    if Y is None:
        Y = empty_f(n1, n2, n3, Z.dtype, Z.device)
    ranks = (C.c_int32 * n3)() if return_ranks else None
    ctx.check(lib.tsvt_dft(ctx.h, prec, n1, n2, n3, Z.data_ptr(), Y.data_ptr(), float(tau), ranks,
                           _stream(stream, d)))
    if return_ranks:
        return Y, [int(r) for r in ranks]
    return Y


def _tnn(fn, X, prec, ctx, stream):
    X = fortran(X)
    d = _dev(X)
    prec = _prec_of(X, prec)
    ctx = ctx or default_context(d)
    out = C.c_double(0.0)
    ctx.check(fn(ctx.h, prec, *X.shape, X.data_ptr(), C.byref(out), _stream(stream, d)))
    return out.value


def tnn_c(X: torch.Tensor, prec: Optional[int] = None, ctx: Optional[Context] = None, stream=None) -> float:
    """TNN-C (equation (equTNN1)) of X."""
    return _tnn(lib.tnn_c, X, prec, ctx, stream)


def tnn_f(X: torch.Tensor, prec: Optional[int] = None, ctx: Optional[Context] = None, stream=None) -> float:
    """TNN-F (equation (tnn)) of X."""
    return _tnn(lib.tnn_f, X, prec, ctx, stream)


NOALLOC_MAX_BYTES = 128 << 20


def tsvt_dct_noalloc(Z: torch.Tensor, tau: float, Y: torch.Tensor, prec: Optional[int] = None,
                     return_ranks: bool = False, ctx: Optional[Context] = None, stream=None):
    """t-SVT (Theorem 5) through the entry point that makes no device
    allocation: the caller passes the output Y (column-major, Z's shape and
    type) and the library works in its fixed per-GPU scratch."""
    Z, Y = fortran(Z), fortran(Y)
    d = _dev(Z)
    prec = _prec_of(Z, prec)
    ctx = ctx or default_context(d)
    n1, n2, n3 = Z.shape
    if tuple(Y.shape) != (n1, n2, n3) or Y.dtype != Z.dtype:
        raise ValueError("Y must have Z's shape and type")
    ranks = (C.c_int32 * n3)() if return_ranks else None
    rc = lib.tsvt_dct_noalloc(ctx.h, prec, n1, n2, n3, Z.data_ptr(), Y.data_ptr(), float(tau), ranks,
                              _stream(stream, d))
    ctx.check(rc)
    if return_ranks:
        return Y, [int(r) for r in ranks]
    return Y


def tprod_dct(X: torch.Tensor, Yt: torch.Tensor, prec: Optional[int] = None, ctx: Optional[Context] = None,
              stream=None) -> torch.Tensor:
    """DCT t-product Z = X * Y (equation (tproduct dct))."""
    X, Yt = fortran(X), fortran(Yt)
    d = _dev(X)
    prec = _prec_of(X, prec)
    ctx = ctx or default_context(d)
    n1, n2, n3 = X.shape
    if Yt.shape[0] != n2 or Yt.shape[2] != n3:
        raise ValueError("shape mismatch")
    n4 = Yt.shape[1]
    Z = empty_f(n1, n4, n3, X.dtype, X.device)
    ctx.check(lib.tprod_dct(ctx.h, prec, n1, n2, n4, n3, X.data_ptr(), Yt.data_ptr(), Z.data_ptr(),
                            _stream(stream, d)))
    return Z


def tsvd_dct(X: torch.Tensor, prec: Optional[int] = None, transform_domain: bool = False, full: bool = False,
             ctx: Optional[Context] = None, stream=None):
    """DCT t-SVD (Theorem 4).  Returns U (n1,p,n3), S (p,n3), V (n2,p,n3); with
    full=True U (n1,n1,n3) and V (n2,n2,n3)."""
    X = fortran(X)
    d = _dev(X)
    prec = _prec_of(X, prec)
    ctx = ctx or default_context(d)
    n1, n2, n3 = X.shape
    p = min(n1, n2)
    U = empty_f(n1, n1 if full else p, n3, X.dtype, X.device)
    V = empty_f(n2, n2 if full else p, n3, X.dtype, X.device)
    S = torch.empty((n3, p), dtype=X.dtype, device=X.device).t()
    flags = (TRANSFORM_DOMAIN if transform_domain else 0) | (FULL if full else 0)
    ctx.check(lib.tsvd_dct(ctx.h, prec, n1, n2, n3, X.data_ptr(), U.data_ptr(), S.data_ptr(), V.data_ptr(),
                           flags, _stream(stream, d)))
    return U, S, V


def complete_tensor(B: torch.Tensor, mask: torch.Tensor, X: Optional[torch.Tensor] = None, max_iter: int = 500,
                    tol: float = 1e-8, beta: float = 1e-2, tau_schedule: Optional[Sequence[float]] = None,
                    check_every: int = 10, start_iter: int = 0, M_init: Optional[torch.Tensor] = None,
                    return_M: bool = False, prec: Optional[int] = None, ctx: Optional[Context] = None,
                    stream=None):
    """Algorithm 1 (ADMM for TNN-C completion).  Returns (X, info[, M])."""
    B = fortran(B)
    d = _dev(B)
    prec = _prec_of(B, prec)
    ctx = ctx or default_context(d)
    n1, n2, n3 = B.shape
    mask = fortran(mask.to(torch.uint8))
    init_observed = X is None  # the library forms Algorithm 1's initial iterate B on the observed set
    if X is None:
        X = empty_f(n1, n2, n3, B.dtype, B.device)
    else:
        X = fortran(X.clone())
    M_out = empty_f(n1, n2, n3, B.dtype, B.device) if return_M else None
    sched = None
    if tau_schedule is not None:
        sched = (C.c_double * len(tau_schedule))(*[float(t) for t in tau_schedule])
        if start_iter + max_iter > len(tau_schedule):
            raise ValueError("tau_schedule shorter than start_iter + max_iter")
    opts = CompleteOpts(max_iter, float(tol), float(beta),
                        C.cast(sched, C.POINTER(C.c_double)) if sched is not None else None, check_every,
                        start_iter, fortran(M_init).data_ptr() if M_init is not None else None,
                        M_out.data_ptr() if M_out is not None else None, int(init_observed))
    info = CompleteInfo()
    rc = lib.complete_tensor(ctx.h, prec, n1, n2, n3, B.data_ptr(), mask.data_ptr(), X.data_ptr(),
                             C.byref(opts), C.byref(info), _stream(stream, d))
    ctx.check(rc)
    out = {"iters": info.iters, "rel_change": info.rel_change, "status": info.status,
           "max_sweeps": info.max_sweeps}
    if return_M:
        return X, out, M_out
    return X, out


def tsvt_dct_batched(Zs: Sequence[torch.Tensor], taus: Sequence[float], Ys: Optional[Sequence[torch.Tensor]] = None,
                     prec: Optional[int] = None, ctx: Optional[Context] = None, stream=None,
                     return_status: bool = False):
    """Batched t-SVT of tensors of independent shapes.  Returns the list of Y
    (and, with return_status, each tensor's own status code)."""
    Zs = [fortran(z) for z in Zs]
    d = _dev(Zs[0])
    prec = _prec_of(Zs[0], prec)
    ctx = ctx or default_context(d)
    count = len(Zs)
    if Ys is None:
        Ys = [empty_f(*z.shape, z.dtype, z.device) for z in Zs]
    dims = (C.c_int64 * (3 * count))(*[int(v) for z in Zs for v in z.shape])
    zp = (_vp * count)(*[z.data_ptr() for z in Zs])
    yp = (_vp * count)(*[y.data_ptr() for y in Ys])
    tp = (C.c_double * count)(*[float(t) for t in taus])
    st = (C.c_int32 * count)() if return_status else None
    ctx.check(lib.tsvt_dct_batched(ctx.h, prec, count, dims, zp, yp, tp, st, _stream(stream, d)))
    if return_status:
        return list(Ys), [int(v) for v in st]
    return list(Ys)


class Server:
    """Continuous-batching server over a context (tsvd_server_* in the header).

    Host arrays are float32, shape (n1, n2, n3), any layout (copied in
    column-major order at submit)."""

    def __init__(self, budget_bytes: int, max_active: int, prec: int = FP32, ctx: Optional[Context] = None,
                 device: int = 0):
        import numpy as np  # noqa: F401

        self.ctx = ctx or Context(device)
        self._own_ctx = ctx is None
        h = _vp()
        rc = lib.tsvd_server_create(C.byref(h), self.ctx.h, prec, int(budget_bytes), int(max_active))
        if rc != OK:
            raise TsvdError(rc, "tsvd_server_create failed")
        self.h = h
        self.shapes = {}
        _register(self)

    @staticmethod
    def _host(a):
        import numpy as np

        return np.asfortranarray(np.asarray(a, dtype=np.float32))

    def _submit(self, req: "Request", shape) -> int:
        rid = lib.tsvd_server_submit(self.h, C.byref(req))
        if rid < 0:
            raise TsvdError(int(rid), "submit refused")
        self.shapes[rid] = shape
        return rid

    def submit_tsvt(self, Z, tau: float, deadline_s: float = 0.0) -> int:
        Z = self._host(Z)
        n1, n2, n3 = Z.shape
        req = Request(REQ_TSVT, n1, n2, n3, Z.ctypes.data_as(C.POINTER(C.c_float)), None, float(tau), 0, 0.0, 0.0,
                      float(deadline_s))
        return self._submit(req, Z.shape)

    def submit_complete(self, B, mask, iters: int, tau0: float, tau1: float, deadline_s: float = 0.0) -> int:
        import numpy as np

        B = self._host(B)
        mk = np.asfortranarray(np.asarray(mask, dtype=np.uint8))
        n1, n2, n3 = B.shape
        req = Request(REQ_COMPLETE, n1, n2, n3, B.ctypes.data_as(C.POINTER(C.c_float)),
                      mk.ctypes.data_as(C.POINTER(C.c_uint8)), 0.0, int(iters), float(tau0), float(tau1),
                      float(deadline_s))
        return self._submit(req, B.shape)

    def cancel(self, rid: int) -> int:
        """0 if cancelled (polls as ECANCELED), 1 if it had already ended."""
        rc = lib.tsvd_server_cancel(self.h, rid)
        if rc < 0:
            raise TsvdError(rc, "cancel of request %d failed" % rid)
        return rc

    def poll(self, rid: int):
        """None while running; else (result array, (t_submit, t_admit, t_done)).
        A failed request raises TsvdError with its own code."""
        import numpy as np

        shape = self.shapes[rid]
        out = np.empty(shape, dtype=np.float32, order="F")
        ts, ta, td = C.c_double(), C.c_double(), C.c_double()
        rc = lib.tsvd_server_poll(self.h, rid, out.ctypes.data_as(C.POINTER(C.c_float)), C.byref(ts), C.byref(ta),
                                  C.byref(td))
        if rc == 0:
            return None
        del self.shapes[rid]
        if rc < 0:
            raise TsvdError(rc, "request %d failed" % rid)
        return out, (ts.value, ta.value, td.value)

    def now(self) -> float:
        return lib.tsvd_server_now(self.h)

    def stats(self) -> dict:
        v = [C.c_int64() for _ in range(4)]
        lib.tsvd_server_stats(self.h, *[C.byref(x) for x in v])
        return dict(zip(("admitted", "completed", "ticks", "peak_bytes"), [x.value for x in v]))

    def close(self):
        if self.h:
            lib.tsvd_server_destroy(self.h)
            self.h = None
        if self._own_ctx and self.ctx:
            self.ctx.close()
            self.ctx = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
