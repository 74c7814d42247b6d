"""GPU parity of the other transforms along the tubes against the FP64 oracle
(through the C-ABI):
  * tsvt_transform: the t-SVT under a caller-given invertible transform
    (concluding remarks), including L = the DCT matrix (equals tsvt_dct),
    orthogonal and non-orthogonal L, tubes longer than the matrix-core limit;
  * tsvt_dft: the Fourier-domain t-SVT (Section 2, TNN-F), odd and even n3;
  * tnn_c and tnn_f.
FP64 bar: relative Frobenius error <= 1e-10; FP32 / MIXED: the stated
per-result bound (orthogonal transforms, whose scale equals the DCT's).
"""
import numpy as np
import pytest

import oracle
import synth
from bounds import C_PATH, FP64_TOL, ratio
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def _case(shape, seed, r=3, tau=None):
    n1, n2, n3 = shape
    if tau is None:
        tau = 0.1 * (np.sqrt(n1) + np.sqrt(n2))
    return synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, r, 0.01, tau, seed)


def _orthogonal(n, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return q


@pytest.mark.parametrize("shape", [(40, 30, 8), (256, 256, 3), (33, 70, 31)])
def test_transform_dct_matrix_equals_tsvt_dct(tm, shape):
    announce("transform_dct", shape=shape)
    c = _case(shape, 31)
    Z = to_dev(c.Z)
    C = oracle.dct_matrix(shape[2])
    Y1 = tm.tsvt_transform(Z, c.tau, C)
    Y0 = tm.tsvt_dct(Z, c.tau)
    assert rel(to_np(Y1), to_np(Y0)) <= FP64_TOL


@pytest.mark.parametrize("shape,kind", [((48, 36, 6), "orth"), ((48, 36, 6), "general"), ((20, 25, 150), "orth"),
                                        ((256, 200, 4), "general"), ((7, 5, 1), "general")])
def test_transform_fp64_against_oracle(tm, shape, kind):
    announce("transform_fp64", shape=shape, kind=kind)
    n3 = shape[2]
    L = _orthogonal(n3, 40 + n3) if kind == "orth" else \
        np.eye(n3) + 0.2 * np.random.default_rng(41).standard_normal((n3, n3))
    c = _case(shape, 32)
    Y, ranks = tm.tsvt_transform(to_dev(c.Z), c.tau, L, return_ranks=True)
    Yo, ro, _ = oracle.tsvt_transform(c.Z, c.tau, L, return_ranks=True)
    err = rel(to_np(Y), Yo)
    print("transform %s %s: rel err %.3e" % (kind, shape, err))
    assert err <= FP64_TOL
    assert ranks == [int(x) for x in ro]


@pytest.mark.parametrize("prec", [1, 2])
def test_transform_reduced_against_oracle(tm, prec):
    announce("transform_reduced", prec=prec)
    shape = (64, 48, 12)
    L = _orthogonal(12, 42)
    c = _case(shape, 33)
    Zf = c.Z.astype(np.float32).astype(np.float64)
    Y = tm.tsvt_transform(to_dev(Zf, torch.float32), c.tau, L, prec=prec)
    Yo = oracle.tsvt_transform(Zf, c.tau, L)
    cr = ratio(to_np(Y), Yo, Zf, prec)
    print("transform prec %d: c = %.3f" % (prec, cr))
    assert cr <= C_PATH[prec]


def test_transform_matrix_change_between_calls(tm):
    # the device form of L is cached by content: a new L with the same shape is used
    announce("transform_change")
    c = _case((30, 24, 5), 34)
    Z = to_dev(c.Z)
    ctx = tm.Context(0)
    try:
        for seed in (50, 51, 50):
            L = _orthogonal(5, seed)
            Y = tm.tsvt_transform(Z, c.tau, L, ctx=ctx)
            assert rel(to_np(Y), oracle.tsvt_transform(c.Z, c.tau, L)) <= FP64_TOL
    finally:
        ctx.close()


def test_transform_rejects_singular_and_nonfinite_matrices(tm):
    announce("transform_invalid")
    Z = to_dev(np.ones((4, 3, 3)))
    L = np.eye(3)
    L[2] = L[1]
    with pytest.raises(tm.TsvdError) as ei:
        tm.tsvt_transform(Z, 0.5, L)
    assert ei.value.code == tm.EINVAL
    L = np.eye(3)
    L[0, 1] = np.nan
    with pytest.raises(tm.TsvdError) as ei:
        tm.tsvt_transform(Z, 0.5, L)
    assert ei.value.code == tm.EINVAL


@pytest.mark.parametrize("shape", [(7, 5, 1), (6, 4, 2), (24, 20, 5), (40, 36, 8), (64, 64, 16), (100, 60, 31),
                                   (130, 90, 6)])
def test_tsvt_dft_fp64_against_oracle(tm, shape):
    announce("tsvt_dft_fp64", shape=shape)
    c = _case(shape, 35, tau=0.15 * (np.sqrt(shape[0]) + np.sqrt(shape[1])) * np.sqrt(shape[2]))
    Y, ranks = tm.tsvt_dft(to_dev(c.Z), c.tau, return_ranks=True)
    Yo, ro, _ = oracle.tsvt_dft(c.Z, c.tau, return_ranks=True)
    err = rel(to_np(Y), Yo)
    print("tsvt_dft %s: rel err %.3e ranks %s" % (shape, err, ranks[:6]))
    assert err <= FP64_TOL
    assert ranks == [int(x) for x in ro]


@pytest.mark.parametrize("prec", [1, 2])
def test_tsvt_dft_reduced_against_oracle(tm, prec):
    # the real Fourier transform is sqrt(n3) (DC, Nyquist) or sqrt(n3 / 2) times an
    # orthogonal one: condition number sqrt(2), so the bound is twice the DCT path's
    announce("tsvt_dft_reduced", prec=prec)
    shape = (64, 48, 9)
    c = _case(shape, 36, tau=1.0)
    Zf = c.Z.astype(np.float32).astype(np.float64)
    Y = tm.tsvt_dft(to_dev(Zf, torch.float32), c.tau, prec=prec)
    Yo = oracle.tsvt_dft(Zf, c.tau)
    cr = ratio(to_np(Y), Yo, Zf, prec)
    print("tsvt_dft prec %d: c = %.3f" % (prec, cr))
    assert cr <= 2 * C_PATH[prec]


@pytest.mark.parametrize("tau", [10.0, 0.5])
def test_tsvt_dft_bench_shape_fp64(tm, tau):
    # the multispectral-shaped workload's first iterate; thresholds scaled by sqrt(n3)
    # to the unnormalized Fourier slices
    announce("tsvt_dft_256", tau=tau)
    cc = synth.completion_case(oracle.tprod_dct, 256, 256, 31, 10, 0.3, 100, synth.SEED_BASE + 2)
    tau = tau * np.sqrt(31)
    oracle.set_threads(min(16, oracle.host_threads()))
    Yo, ro, _ = oracle.tsvt_dft(cc.B, tau, return_ranks=True)
    Y, ranks = tm.tsvt_dft(to_dev(cc.B), tau, return_ranks=True)
    err = rel(to_np(Y), Yo)
    print("tsvt_dft 256x256x31 tau %.3g: rel err %.3e, ranks %s" % (tau, err, ranks[:4]))
    assert err <= FP64_TOL
    assert ranks == [int(x) for x in ro]


@pytest.mark.parametrize("shape", [(24, 20, 5), (50, 64, 8), (256, 256, 3)])
def test_tnn_c_and_tnn_f(tm, shape):
    announce("tnn", shape=shape)
    X = _case(shape, 37).Z
    a, b = tm.tnn_c(to_dev(X)), tm.tnn_f(to_dev(X))
    ao, bo = oracle.tnn_c(X), oracle.tnn_f(X)
    print("TNN-C %.12g (oracle %.12g), TNN-F %.12g (oracle %.12g)" % (a, ao, b, bo))
    assert abs(a - ao) <= FP64_TOL * ao
    assert abs(b - bo) <= FP64_TOL * bo
