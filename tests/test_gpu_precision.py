"""Tube transforms on the matrix cores, and the error bounds of the reduced-precision paths.

Stated bound (per result, constants in bounds.py): ||Y - Y*||_F <= c_path * u_eff * ||Z||_F,
with Y* the FP64 oracle on the same (float-rounded) input, u_eff = 2^-24 for FP32
and 2^-16 for MIXED (bfloat16 hi+lo transforms); one transformed slice against
its own norm.  The ratios these tests print are the calibration data of c_path.
"""
import numpy as np
import pytest

import oracle
import synth
from bounds import C_PATH, U_EFF, oracle_iterates, ratio
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu


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
    c = ratio(Y, Ystar, Zf, prec)
    print("bound ratio c = %.3f (prec %d, shape %s, rel err %.3e)" % (c, prec, shape, rel(Y, Ystar)))
    assert c <= C_PATH[prec]


def test_complete_mixed_tracks_fp64(tm):
    announce("complete_mixed")
    cc = synth.completion_case(oracle.tprod_dct, 40, 36, 8, 3, 0.5, 20, 7, tau0=2.0, tau1=0.05)
    Bf = cc.B.astype(np.float32).astype(np.float64)
    Xo, _, zmax = oracle_iterates(Bf, cc.mask, cc.taus, 20)
    for prec in (1, 2):
        X, info = tm.complete_tensor(to_dev(Bf, torch.float32), to_dev(cc.mask, torch.uint8), max_iter=20, tol=0.0,
                                     tau_schedule=cc.taus, prec=prec)
        c = np.linalg.norm(to_np(X) - Xo) / (U_EFF[prec] * zmax)
        print("completion prec %d rel err vs FP64 oracle %.3e, c per iteration %.3f" % (prec, rel(to_np(X), Xo), c / 20))
        # 20 iterations, each within the single-t-SVT bound: at most linear growth
        assert c <= 20 * C_PATH[prec]


def test_video_shaped_mixed_every_slice(tm):
    # 144 x 176 x 100 (rank 15, observed 20%), MIXED, at full size: the whole
    # result against the FP64 oracle on the float-rounded input, and every
    # transformed slice against the oracle's within that slice's own norm
    import scipy.fft

    announce("video_shaped_mixed")

    def lib_tprod(A, B):
        Ab = scipy.fft.dct(A, type=2, norm="ortho", axis=2)
        Bb = scipy.fft.dct(B, type=2, norm="ortho", axis=2)
        Zb = np.matmul(Ab.transpose(2, 0, 1), Bb.transpose(2, 0, 1)).transpose(1, 2, 0)
        return np.asfortranarray(scipy.fft.idct(Zb, type=2, norm="ortho", axis=2))

    cc = synth.completion_case(lib_tprod, 144, 176, 100, 15, 0.2, 100, synth.SEED_BASE + 3)
    Zf = cc.B.astype(np.float32).astype(np.float64)
    oracle.set_threads(min(16, oracle.host_threads()))
    for tau in (float(cc.taus[0]), 1.0):
        Y = to_np(tm.tsvt_dct(to_dev(Zf, torch.float32), tau, prec=2))
        Yo = oracle.tsvt_dct(Zf, tau)
        c = ratio(Y, Yo, Zf, 2)
        Yb, Yob, Zb = oracle.dct_tubes(Y), oracle.dct_tubes(Yo), oracle.dct_tubes(Zf)
        ck = [np.linalg.norm(Yb[:, :, k] - Yob[:, :, k]) / (U_EFF[2] * np.linalg.norm(Zb[:, :, k]))
              for k in range(100)]
        print("tau %.3g: c = %.3f, worst slice c = %.3f (slice %d), rel err %.3e" % (
            tau, c, max(ck), int(np.argmax(ck)), rel(Y, Yo)))
        assert c <= C_PATH[2]
        assert max(ck) <= C_PATH[2]
