"""ctypes front end of the plain C FP64 oracle (``tsvd_oracle.c``).

TEST INFRASTRUCTURE ONLY: see the package docstring.  Every function takes and
returns numpy float64 arrays in column-major (Fortran) order, so that a tensor
of shape (n1, n2, n3) has X(i,j,k) at flat index i + n1*j + n1*n2*k, the layout
the paper's MATLAB notation implies.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsvd_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT_DIR, "libtsvd_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_i64 = C.c_int64


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vendor math, no BLAS)."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = C.CDLL(_LIB)
    lib.or_dct_matrix.argtypes = [C.c_int, _dp]
    lib.or_set_threads.argtypes = [C.c_int]
    lib.or_get_threads.restype = C.c_int
    for name in ("or_dct_tubes", "or_idct_tubes", "or_split_shift", "or_bt", "or_bh", "or_btph",
                 "or_unfold", "or_fold"):
        getattr(lib, name).argtypes = [_i64, _i64, _i64, _dp, _dp]
    lib.or_btph_product.argtypes = [_i64, _i64, _i64, _i64, _dp, _dp, _dp]
    lib.or_tprod_dct.argtypes = [_i64, _i64, _i64, _i64, _dp, _dp, _dp]
    lib.or_jacobi_svd.argtypes = [_i64, _i64, _dp, _i64, _dp, _dp, _dp, C.c_int]
    lib.or_jacobi_svd.restype = C.c_int
    lib.or_tsvd_dct.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, _dp, C.c_int]
    lib.or_tsvd_dct.restype = C.c_int
    lib.or_tsvd_dct_full.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, _dp, C.c_int]
    lib.or_tsvd_dct_full.restype = C.c_int
    lib.or_tsvt_dct.argtypes = [_i64, _i64, _i64, _dp, C.c_double, _dp, C.POINTER(C.c_int32), C.c_int]
    lib.or_tsvt_dct.restype = C.c_int
    lib.or_tnn_c.argtypes = [_i64, _i64, _i64, _dp, C.c_int]
    lib.or_tnn_c.restype = C.c_double
    lib.or_complete.argtypes = [_i64, _i64, _i64, _dp, C.POINTER(C.c_uint8), C.c_int, _dp, _dp, C.c_double,
                                C.c_int, _dp, _dp, _dp]
    lib.or_complete.restype = C.c_int
    lib.or_tsvt_transform.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, C.c_double, _dp, C.POINTER(C.c_int32),
                                      C.c_int]
    lib.or_tsvt_transform.restype = C.c_int
    lib.or_dft_tubes.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp]
    lib.or_idft_tubes.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, _dp]
    lib.or_bcirc.argtypes = [_i64, _i64, _i64, _dp, _dp]
    lib.or_jacobi_svt_c.argtypes = [_i64, _i64, _dp, _dp, C.c_double, _dp, _dp, _dp, C.POINTER(C.c_int32), C.c_int]
    lib.or_jacobi_svt_c.restype = C.c_int
    lib.or_tsvt_dft.argtypes = [_i64, _i64, _i64, _dp, C.c_double, _dp, C.POINTER(C.c_int32), _dp, C.c_int]
    lib.or_tsvt_dft.restype = C.c_int
    lib.or_tnn_f.argtypes = [_i64, _i64, _i64, _dp, C.c_int]
    lib.or_tnn_f.restype = C.c_double
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _as3(a) -> np.ndarray:
    a = _f64(a)
    if a.ndim == 2:
        a = a.reshape(a.shape[0], a.shape[1], 1, order="F")
    assert a.ndim == 3
    return a


MAX_SWEEPS = 100


def set_threads(n: int) -> int:
    """Split independent work (slices, tubes) over n host threads; results
    are bitwise the same for every n.  Returns the previous count."""
    lib = _load()
    old = lib.or_get_threads()
    lib.or_set_threads(int(n))
    return old


def host_threads() -> int:
    """Threads this process may run on (its CPU affinity)."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def dct_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II matrix, C[k, t] (row = frequency)."""
    out = np.empty(n * n)
    _load().or_dct_matrix(n, _p(out))
    return out.reshape(n, n)  # stored row-major C[k*n+t]


def _tube_op(name, X):
    X = _as3(X)
    out = np.empty_like(X, order="F")
    getattr(_load(), name)(*X.shape, _p(X), _p(out))
    return out


def dct_tubes(X):
    """Xbar = dct(X,[],3): orthonormal DCT-II along every mode-3 tube."""
    return _tube_op("or_dct_tubes", X)


def idct_tubes(Xbar):
    """Inverse of dct_tubes."""
    return _tube_op("or_idct_tubes", Xbar)


def split_shift(X):
    """A with X = A + sigma(A) (Section 3)."""
    return _tube_op("or_split_shift", X)


def _block_matrix(name, A):
    A = _as3(A)
    n1, n2, n3 = A.shape
    out = np.empty((n1 * n3, n2 * n3), order="F")
    getattr(_load(), name)(n1, n2, n3, _p(A), _p(out))
    return out


def bt(A):
    """Block Toeplitz matrix of the slices of A (Section 3)."""
    return _block_matrix("or_bt", A)


def bh(A):
    """Block Hankel matrix of the slices of A (Section 3)."""
    return _block_matrix("or_bh", A)


def btph(A):
    """Block Toeplitz-plus-Hankel matrix bt(A) + bh(A) (Section 3)."""
    return _block_matrix("or_btph", A)


def unfold(X):
    X = _as3(X)
    n1, n2, n3 = X.shape
    out = np.empty((n1 * n3, n2), order="F")
    _load().or_unfold(n1, n2, n3, _p(X), _p(out))
    return out


def fold(U, n1, n2, n3):
    U = _f64(U)
    out = np.empty((n1, n2, n3), order="F")
    _load().or_fold(n1, n2, n3, _p(U), _p(out))
    return out


def btph_product(X, Y):
    """Z = fold(btph(A) unfold(Y)), the definition-level DCT t-product."""
    X, Y = _as3(X), _as3(Y)
    n1, n2, n3 = X.shape
    assert Y.shape[0] == n2 and Y.shape[2] == n3
    n4 = Y.shape[1]
    out = np.empty((n1, n4, n3), order="F")
    _load().or_btph_product(n1, n2, n4, n3, _p(X), _p(Y), _p(out))
    return out


def tprod_dct(X, Y):
    """Z = idct(slice-wise Xbar^(k) Ybar^(k)), the transform-domain t-product."""
    X, Y = _as3(X), _as3(Y)
    n1, n2, n3 = X.shape
    assert Y.shape[0] == n2 and Y.shape[2] == n3
    n4 = Y.shape[1]
    out = np.empty((n1, n4, n3), order="F")
    _load().or_tprod_dct(n1, n2, n4, n3, _p(X), _p(Y), _p(out))
    return out


def jacobi_svd(A, max_sweeps: int = MAX_SWEEPS):
    """Thin SVD of one matrix by one-sided Jacobi.  Returns (U, s, V, sweeps)."""
    A = _f64(A)
    m, n = A.shape
    p = min(m, n)
    U = np.empty((m, p), order="F")
    V = np.empty((n, p), order="F")
    s = np.empty(p)
    sw = _load().or_jacobi_svd(m, n, _p(A), m, _p(U), _p(s), _p(V), max_sweeps)
    return U, s, V, sw


def tsvd_dct(X, max_sweeps: int = MAX_SWEEPS):
    """DCT t-SVD, transform-domain thin factors (Ubar, Sbar, Vbar, sweeps).

    Ubar: n1 x p x n3, Sbar: p x n3 (descending per column), Vbar: n2 x p x n3.
    """
    X = _as3(X)
    n1, n2, n3 = X.shape
    p = min(n1, n2)
    U = np.empty((n1, p, n3), order="F")
    V = np.empty((n2, p, n3), order="F")
    S = np.empty((p, n3), order="F")
    sw = _load().or_tsvd_dct(n1, n2, n3, _p(X), _p(U), _p(S), _p(V), max_sweeps)
    return U, S, V, sw


def tsvd_dct_full(X, max_sweeps: int = MAX_SWEEPS):
    """DCT t-SVD with full factors (Theorem 4): Ubar n1 x n1 x n3 and Vbar
    n2 x n2 x n3 orthogonal per slice, Sbar p x n3.  The first p columns are
    tsvd_dct's; the rest complete the longer side's basis (see the C source)."""
    X = _as3(X)
    n1, n2, n3 = X.shape
    p = min(n1, n2)
    U = np.empty((n1, n1, n3), order="F")
    V = np.empty((n2, n2, n3), order="F")
    S = np.empty((p, n3), order="F")
    sw = _load().or_tsvd_dct_full(n1, n2, n3, _p(X), _p(U), _p(S), _p(V), max_sweeps)
    return U, S, V, sw


def tsvt_dct(Z, tau: float, max_sweeps: int = MAX_SWEEPS, return_ranks: bool = False):
    """t-SVT (Theorem 5) with threshold tau on the orthonormal-DCT slices."""
    Z = _as3(Z)
    n1, n2, n3 = Z.shape
    Y = np.empty_like(Z, order="F")
    ranks = np.empty(n3, dtype=np.int32)
    sw = _load().or_tsvt_dct(n1, n2, n3, _p(Z), float(tau), _p(Y), ranks.ctypes.data_as(C.POINTER(C.c_int32)),
                             max_sweeps)
    if return_ranks:
        return Y, ranks, sw
    return Y


def tnn_c(X, max_sweeps: int = MAX_SWEEPS) -> float:
    """TNN-C: (1/n3) * sum of nuclear norms of the DCT-domain slices."""
    X = _as3(X)
    return float(_load().or_tnn_c(*X.shape, _p(X), max_sweeps))


def complete(B, mask, betas, taus=None, tol: float = 0.0, X0=None, M0=None, max_sweeps: int = MAX_SWEEPS):
    """Algorithm 1 (ADMM for TNN-C completion) with a per-iteration penalty.

    betas: length-L array of beta_l; taus: thresholds (default 1/beta_l, as in
    Algorithm 1).  X0 defaults to B on the observed set, M0 to zero.
    Returns (X, M, iters, relchange).
    """
    B = _as3(B)
    n1, n2, n3 = B.shape
    mask = np.asfortranarray(np.asarray(mask, dtype=np.uint8).reshape(B.shape, order="F"))
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    L = betas.shape[0]
    taus = 1.0 / betas if taus is None else np.ascontiguousarray(taus, dtype=np.float64)
    X = _f64(np.where(mask != 0, B, 0.0)) if X0 is None else _as3(X0).copy(order="F")
    M = np.zeros_like(B, order="F") if M0 is None else _as3(M0).copy(order="F")
    rc = C.c_double(0.0)
    it = _load().or_complete(n1, n2, n3, _p(B), mask.ctypes.data_as(C.POINTER(C.c_uint8)), L, _p(betas), _p(taus),
                             float(tol), max_sweeps, _p(X), _p(M), C.byref(rc))
    return X, M, it, rc.value


def tsvt_transform(Z, tau: float, L, Linv=None, max_sweeps: int = MAX_SWEEPS, return_ranks: bool = False):
    """t-SVT under an invertible transform L along the tubes (Section 6: other
    transforms in place of the DCT): slices of L applied along the tubes are
    thresholded, then Linv (default: numpy's inverse of L) maps back."""
    Z = _as3(Z)
    n1, n2, n3 = Z.shape
    L = np.ascontiguousarray(L, dtype=np.float64).reshape(n3, n3)
    Linv = np.ascontiguousarray(np.linalg.inv(L) if Linv is None else Linv, dtype=np.float64).reshape(n3, n3)
    Y = np.empty_like(Z, order="F")
    ranks = np.empty(n3, dtype=np.int32)
    sw = _load().or_tsvt_transform(n1, n2, n3, _p(L), _p(Linv), _p(Z), float(tau), _p(Y),
                                   ranks.ctypes.data_as(C.POINTER(C.c_int32)), max_sweeps)
    if return_ranks:
        return Y, ranks, sw
    return Y


def dft_tubes(X):
    """fft(X,[],3) from the definition (unnormalized), as a complex array."""
    X = _as3(X)
    Xr = np.empty_like(X, order="F")
    Xi = np.empty_like(X, order="F")
    _load().or_dft_tubes(*X.shape, _p(X), _p(Xr), _p(Xi))
    return Xr + 1j * Xi


def idft_tubes(Xt):
    """ifft(Xt,[],3) from the definition, as a complex array."""
    Xt = np.asarray(Xt)
    if Xt.ndim == 2:
        Xt = Xt.reshape(Xt.shape[0], Xt.shape[1], 1)
    Xr, Xi = _f64(Xt.real), _f64(Xt.imag)
    Yr = np.empty_like(Xr, order="F")
    Yi = np.empty_like(Xr, order="F")
    _load().or_idft_tubes(*Xr.shape, _p(Xr), _p(Xi), _p(Yr), _p(Yi))
    return Yr + 1j * Yi


def bcirc(X):
    """Block circulant matrix of the slices of X (equation (bcirc))."""
    return _block_matrix("or_bcirc", X)


def svt_complex(A, tau: float, max_sweeps: int = MAX_SWEEPS):
    """Matrix SVT of a complex matrix by complex one-sided Jacobi: returns
    (U (S - tau)_+ V^H, singular values descending, rank, sweeps)."""
    A = np.asarray(A, dtype=np.complex128)
    m, n = A.shape
    Ar, Ai = _f64(A.real), _f64(A.imag)
    s = np.empty(min(m, n))
    Yr = np.empty((m, n), order="F")
    Yi = np.empty((m, n), order="F")
    rk = C.c_int32(0)
    sw = _load().or_jacobi_svt_c(m, n, _p(Ar), _p(Ai), float(tau), _p(s), _p(Yr), _p(Yi), C.byref(rk), max_sweeps)
    return Yr + 1j * Yi, s, int(rk.value), sw


def tsvt_dft(Z, tau: float, max_sweeps: int = MAX_SWEEPS, return_ranks: bool = False, return_imag: bool = False):
    """DFT t-SVT (the TNN-F counterpart of Theorem 5): every slice of the
    unnormalized fft(Z,[],3) thresholded at tau, then ifft; real output."""
    Z = _as3(Z)
    n1, n2, n3 = Z.shape
    Y = np.empty_like(Z, order="F")
    ranks = np.empty(n3, dtype=np.int32)
    mi = C.c_double(0.0)
    sw = _load().or_tsvt_dft(n1, n2, n3, _p(Z), float(tau), _p(Y), ranks.ctypes.data_as(C.POINTER(C.c_int32)),
                             C.byref(mi), max_sweeps)
    out = [Y]
    if return_ranks:
        out += [ranks, sw]
    if return_imag:
        out.append(mi.value)
    return out[0] if len(out) == 1 else tuple(out)


def tnn_f(X, max_sweeps: int = MAX_SWEEPS) -> float:
    """TNN-F: (1/n3) * sum of nuclear norms of the unnormalized DFT slices."""
    X = _as3(X)
    return float(_load().or_tnn_f(*X.shape, _p(X), max_sweeps))
