"""Stated error bounds of the reduced-precision paths, shared by the GPU tests.

Per result:  ||Y - Y*||_F <= c_path * u_eff * ||Z||_F, with Y* the FP64 oracle
on the same float-rounded input Z, u_eff = 2^-24 for FP32 (FP32 matrix-core
transforms, FP32 Jacobi sweeps) and 2^-16 for MIXED (bfloat16 hi+lo
transforms, which drop the lo*lo term).  A check of one transformed slice uses
that slice's own norm: ||Ybar_k - Ybar*_k||_F <= c_path * u_eff * ||Zbar_k||_F.
A completion of L iterations is allowed L times the single-t-SVT bound (each
iteration's t-SVT is nonexpansive, so errors add at most linearly).

c_path is calibrated on the oracle: twice the largest ratio observed over the
calibration cases of test_gpu_precision.py and test_gpu_fullsize.py, rounded
up to a power of two (observed maxima recorded next to each constant).
"""
import numpy as np

U_EFF = {1: 2.0 ** -24, 2: 2.0 ** -16}
# largest observed c: FP32 170.5 (one slice of the 256 x 256 x 31 t-SVT at
# tau = 0.1, whole tensor 149.5); MIXED ~0.3.  The FP32 floor is set by the
# rotation threshold 2 sqrt(m) u of the FP32 sweeps (pairs whose cosine is
# below it stay unrotated): 32 u at m = 256, times a small factor.
C_PATH = {1: 512.0, 2: 1.0}
FP64_TOL = 1e-10


def ratio(Y, Ystar, Z, prec):
    return float(np.linalg.norm(np.asarray(Y) - np.asarray(Ystar)) / (U_EFF[prec] * np.linalg.norm(Z)))


def within(Y, Ystar, Z, prec, iters=1):
    return ratio(Y, Ystar, Z, prec) <= iters * C_PATH[prec]


def within_completion(X, Xo, zmax, prec, iters):
    """Completion bound: iters * c_path * u_eff * max_l ||Z_l||."""
    return float(np.linalg.norm(np.asarray(X) - np.asarray(Xo))) <= iters * C_PATH[prec] * U_EFF[prec] * zmax


def oracle_iterates(B, mask, taus, L):
    """The oracle's completion one iteration at a time (Algorithm 1 with
    beta_l = 1/tau_l, from X = B on the observed set and M = 0): final X, M
    and the largest norm of a t-SVT input Z_l = X_l - M_l / beta_l."""
    import oracle

    X = np.asfortranarray(np.where(mask != 0, B, 0.0))
    M = np.zeros_like(B, order="F")
    zmax = 0.0
    for l in range(L):
        zmax = max(zmax, float(np.linalg.norm(X - M * taus[l])))
        X, M, _, _ = oracle.complete(B, mask, np.array([1.0 / taus[l]]), np.array([taus[l]]), X0=X, M0=M)
    return X, M, zmax
