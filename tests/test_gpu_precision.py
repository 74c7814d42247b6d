"""Tube transforms on the matrix cores, and the error bounds of the reduced-precision paths.

Stated bound (per result): ||Y - Y*||_F / ||Y*||_F <= c * u_eff * ||Z||_F / ||Y*||_F, with
Y* the FP64 oracle on the same (float-rounded) input, u_eff = 2^-24 for FP32 and
2^-16 for MIXED (bfloat16 hi+lo transforms), and c = C_BOUND below.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu

U_EFF = {1: 2.0 ** -24, 2: 2.0 ** -16}
C_BOUND = 128.0  # calibrated: largest observed c is about 60 (FP32, 256 x 256 slices)


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def rnd(seed, *shape):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape))


@pytest.mark.parametrize("n3", [1, 2, 3, 4, 5, 16, 17, 31, 32, 33, 64, 100, 128, 129, 200])
def test_tube_transform_lengths_fp64(tm, n3):
    announce("tube_fp64", n3=n3)
    X, Y = rnd(n3, 37, 6, n3), rnd(n3 + 1, 6, 5, n3)
    Z = tm.tprod_dct(to_dev(X), to_dev(Y))
    assert rel(to_np(Z), oracle.tprod_dct(X, Y)) <= 1e-12


@pytest.mark.parametrize("prec,tol", [(1, 2e-6), (2, 2e-4)])
@pytest.mark.parametrize("n3", [3, 31, 100, 128])
def test_tube_transform_reduced(tm, prec, tol, n3):
    announce("tube_reduced", prec=prec, n3=n3)
    X, Y = rnd(n3, 40, 7, n3), rnd(n3 + 1, 7, 9, n3)
    Xf, Yf = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    Z = tm.tprod_dct(to_dev(Xf, torch.float32), to_dev(Yf, torch.float32), prec=prec)
    assert rel(to_np(Z), oracle.tprod_dct(Xf, Yf)) <= tol


def bound_ratio(Y, Ystar, Z, prec):
    err = np.linalg.norm(Y - Ystar)
    return err / (U_EFF[prec] * np.linalg.norm(Z))


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("shape", [(64, 64, 16), (48, 80, 31), (256, 256, 3)])
def test_tsvt_reduced_precision_bound(tm, prec, shape):
    announce("tsvt_bound", prec=prec, shape=shape)
    n1, n2, n3 = shape
    c = synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, max(2, min(n1, n2) // 10), 0.01,
                        0.1 * (np.sqrt(n1) + np.sqrt(n2)), seed=99)
    Zf = c.Z.astype(np.float32).astype(np.float64)
    Ystar = oracle.tsvt_dct(Zf, c.tau)
    Y = to_np(tm.tsvt_dct(to_dev(Zf, torch.float32), c.tau, prec=prec))
    ratio = bound_ratio(Y, Ystar, Zf, prec)
    print("bound ratio c = %.3f (prec %d, shape %s, rel err %.3e)" % (ratio, prec, shape, rel(Y, Ystar)))
    assert ratio <= C_BOUND


def test_complete_mixed_tracks_fp64(tm):
    announce("complete_mixed")
    cc = synth.completion_case(oracle.tprod_dct, 40, 36, 8, 3, 0.5, 20, 7, tau0=2.0, tau1=0.05)
    Bf = cc.B.astype(np.float32).astype(np.float64)
    Xo, _, _, _ = oracle.complete(Bf, cc.mask, cc.betas, cc.taus)
    for prec in (1, 2):
        X, info = tm.complete_tensor(to_dev(Bf, torch.float32), to_dev(cc.mask, torch.uint8), max_iter=20, tol=0.0,
                                     tau_schedule=cc.taus, prec=prec)
        err = rel(to_np(X), Xo)
        print("completion prec %d rel err vs FP64 oracle %.3e" % (prec, err))
        # 20 iterations, each within the single-t-SVT bound: at most linear growth
        assert err <= 20 * C_BOUND * U_EFF[prec] * np.linalg.norm(Bf) / np.linalg.norm(Xo)


def test_video_shaped_mixed_sampled_slices(tm):
    # 144 x 176 x 100 (rank 15, observed 20%), MIXED, at full size: sampled
    # transformed slices of the result against the oracle's matrix SVT of the
    # same slice of the (float-rounded) input, within the stated bound
    import scipy.fft

    announce("video_shaped_mixed")

    def lib_tprod(A, B):
        Ab = scipy.fft.dct(A, type=2, norm="ortho", axis=2)
        Bb = scipy.fft.dct(B, type=2, norm="ortho", axis=2)
        Zb = np.matmul(Ab.transpose(2, 0, 1), Bb.transpose(2, 0, 1)).transpose(1, 2, 0)
        return np.asfortranarray(scipy.fft.idct(Zb, type=2, norm="ortho", axis=2))

    cc = synth.completion_case(lib_tprod, 144, 176, 100, 15, 0.2, 100, synth.SEED_BASE + 3)
    Zf = cc.B.astype(np.float32).astype(np.float64)
    tau = float(cc.taus[0])
    Y = to_np(tm.tsvt_dct(to_dev(Zf, torch.float32), tau, prec=2))
    Yb = scipy.fft.dct(Y, type=2, norm="ortho", axis=2)
    Zb = oracle.dct_tubes(Zf)
    zn = np.linalg.norm(Zf)
    for k in (0, 1, 37, 99):
        want = oracle.tsvt_dct(np.asfortranarray(Zb[:, :, k:k + 1]), tau)[:, :, 0]
        err = np.linalg.norm(Yb[:, :, k] - want)
        print("slice %d: |Y - Y*| / (u_eff |Z|) = %.2f" % (k, err / (U_EFF[2] * zn)))
        assert err <= C_BOUND * U_EFF[2] * zn
