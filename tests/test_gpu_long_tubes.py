"""Tubes longer than the matrix-core limit of 128: the fast O(n3 log n3)
transforms along the tubes (the orthonormal DCT-II of Section 3 by Makhoul's
reordering, and the real form of the DFT of Section 2, both by Bluestein's
chirp with radix-2 FFTs) against the FP64 oracle, through the C-ABI:
  * forward and inverse DCT inside tprod_dct, lengths around the FFT sizes
    (129, 255/256/257, 511/512) and odd/even;
  * t-SVT, the t-SVD factors, and the completion loop (the fused prologue
    and epilogue, replayed graph and direct launches);
  * the Fourier path (tsvt_dft, tnn_f) and tnn_c;
  * the dense kernel's limits: FP64 tubes longer than 512 are rejected before
    any launch; float data up to 608 still runs there.
FP64 bar: relative Frobenius error <= 1e-10 (1e-12 for the linear tprod);
reduced precisions: the stated per-result bound.
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


def rnd(seed, *shape):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape))


def tsvt_case(shape, seed, r=3):
    n1, n2, n3 = shape
    return synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, r, 0.01, 0.1 * (np.sqrt(n1) + np.sqrt(n2)), seed)


@pytest.mark.parametrize("n3", [129, 130, 150, 200, 255, 256, 257, 300, 400, 511, 512])
def test_tprod_long_tubes_fp64(tm, n3):
    announce("tprod_long", n3=n3)
    X, Y = rnd(n3, 37, 6, n3), rnd(n3 + 1, 6, 5, n3)
    Z = tm.tprod_dct(to_dev(X), to_dev(Y))
    err = rel(to_np(Z), oracle.tprod_dct(X, Y))
    print("tprod n3 %d: rel err %.3e" % (n3, err))
    assert err <= 1e-12


@pytest.mark.parametrize("prec,tol", [(1, 2e-6), (2, 2e-4)])
@pytest.mark.parametrize("n3", [150, 400])
def test_tprod_long_tubes_reduced(tm, prec, tol, n3):
    announce("tprod_long_reduced", prec=prec, n3=n3)
    X, Y = rnd(n3, 40, 7, n3), rnd(n3 + 1, 7, 9, n3)
    Xf, Yf = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    Z = tm.tprod_dct(to_dev(Xf, torch.float32), to_dev(Yf, torch.float32), prec=prec)
    assert rel(to_np(Z), oracle.tprod_dct(Xf, Yf)) <= tol


@pytest.mark.parametrize("shape", [(64, 48, 129), (40, 30, 400), (100, 100, 400), (20, 25, 512)])
def test_tsvt_long_tubes_fp64(tm, shape):
    announce("tsvt_long", shape=shape)
    c = tsvt_case(shape, 60)
    Y, ranks = tm.tsvt_dct(to_dev(c.Z), c.tau, return_ranks=True)
    Yo, ro, _ = oracle.tsvt_dct(c.Z, c.tau, return_ranks=True)
    err = rel(to_np(Y), Yo)
    print("tsvt %s: rel err %.3e" % (shape, err))
    assert err <= FP64_TOL
    assert ranks == [int(x) for x in ro]


@pytest.mark.parametrize("prec", [1, 2])
def test_tsvt_long_tubes_reduced(tm, prec):
    announce("tsvt_long_reduced", prec=prec)
    c = tsvt_case((64, 48, 300), 61)
    Zf = c.Z.astype(np.float32).astype(np.float64)
    Y = tm.tsvt_dct(to_dev(Zf, torch.float32), c.tau, prec=prec)
    cr = ratio(to_np(Y), oracle.tsvt_dct(Zf, c.tau), Zf, prec)
    print("tsvt long prec %d: c = %.3f" % (prec, cr))
    assert cr <= C_PATH[prec]


def test_tsvd_long_tubes_reconstruction(tm):
    # spatial-domain factors: U * S * V^T (DCT t-products) gives X back
    announce("tsvd_long")
    n1, n2, n3 = 20, 14, 300
    X = rnd(62, n1, n2, n3)
    _, Sb, _ = tm.tsvd_dct(to_dev(X), transform_domain=True)
    _, So, _, _ = oracle.tsvd_dct(X)
    assert rel(to_np(Sb), So) <= 1e-12
    U, S, V = tm.tsvd_dct(to_dev(X))
    p = min(n1, n2)
    Sd = torch.zeros((p, p, n3), dtype=torch.float64, device="cuda:0")
    for k in range(n3):
        Sd[:, :, k] = torch.diag(S[:, k])
    R = tm.tprod_dct(tm.tprod_dct(U, Sd), V.permute(1, 0, 2))
    assert rel(to_np(R), X) <= 1e-12


@pytest.mark.parametrize("shape", [(20, 18, 300), (60, 50, 200)])
def test_complete_long_tubes_fp64(tm, shape):
    # the fused completion prologue/epilogue on the fast transform, in a replayed
    # graph and in direct launches (same bits), against the oracle's iterates
    announce("complete_long", shape=shape)
    cc = synth.completion_case(oracle.tprod_dct, *shape, 3, 0.5, 6, 90, tau0=1.0, tau1=0.01)
    Xo, Mo, _, _ = oracle.complete(cc.B, cc.mask, cc.betas, cc.taus)
    B, mk = to_dev(cc.B), to_dev(cc.mask, torch.uint8)
    outs = []
    for graphs in (1, 0):
        ctx = tm.Context(0)
        ctx.set_option(tm.OPT_GRAPHS, graphs)
        try:
            X, info, M = tm.complete_tensor(B, mk, max_iter=6, tol=0.0, tau_schedule=cc.taus, return_M=True, ctx=ctx)
            outs.append((to_np(X), to_np(M)))
        finally:
            ctx.close()
        assert info["status"] == 0
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    err = rel(outs[0][0], Xo)
    print("completion %s: rel err %.3e" % (shape, err))
    assert err <= FP64_TOL
    assert rel(outs[0][1], Mo) <= FP64_TOL


@pytest.mark.parametrize("shape", [(30, 20, 129), (24, 20, 256), (40, 30, 401)])
def test_tsvt_dft_long_tubes(tm, shape):
    announce("tsvt_dft_long", shape=shape)
    n1, n2, n3 = shape
    c = synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, 3, 0.01, 0.15 * (np.sqrt(n1) + np.sqrt(n2)) * np.sqrt(n3), 63)
    Y, ranks = tm.tsvt_dft(to_dev(c.Z), c.tau, return_ranks=True)
    Yo, ro, _ = oracle.tsvt_dft(c.Z, c.tau, return_ranks=True)
    err = rel(to_np(Y), Yo)
    print("tsvt_dft %s: rel err %.3e" % (shape, err))
    assert err <= FP64_TOL
    assert ranks == [int(x) for x in ro]


def test_tnn_long_tubes(tm):
    announce("tnn_long")
    X = tsvt_case((40, 30, 400), 64).Z
    a, b = tm.tnn_c(to_dev(X)), tm.tnn_f(to_dev(X))
    ao, bo = oracle.tnn_c(X), oracle.tnn_f(X)
    print("TNN-C %.12g (oracle %.12g), TNN-F %.12g (oracle %.12g)" % (a, ao, b, bo))
    assert abs(a - ao) <= FP64_TOL * ao
    assert abs(b - bo) <= FP64_TOL * bo


def test_dense_kernel_limits(tm):
    # FP64 tubes past the fast transform's 512 need the dense kernel, whose LDS
    # tile holds 304 of them: rejected on the host.  Float data fits up to 608.
    announce("dense_limits")
    with pytest.raises(tm.TsvdError) as ei:
        tm.tsvt_dct(to_dev(np.ones((4, 3, 600))), 0.5)
    assert ei.value.code == tm.EINVAL
    c = tsvt_case((8, 6, 600), 65, r=2)
    Zf = c.Z.astype(np.float32).astype(np.float64)
    Y = tm.tsvt_dct(to_dev(Zf, torch.float32), c.tau, prec=1)
    cr = ratio(to_np(Y), oracle.tsvt_dct(Zf, c.tau), Zf, 1)
    print("dense FP32 n3 600: c = %.3f" % cr)
    assert cr <= C_PATH[1]


@pytest.mark.parametrize("shape", [(7, 5, 300), (1, 1, 129), (3, 1, 512), (17, 1, 200)])
def test_tsvt_long_tubes_odd_and_tiny_tube_counts(tm, shape):
    # an odd number of tubes leaves the last pair of a workgroup half empty;
    # fewer than 16 tubes leave most of the only workgroup empty
    announce("tsvt_long_odd", shape=shape)
    c = tsvt_case(shape, 66, r=1)
    Y, ranks = tm.tsvt_dct(to_dev(c.Z), c.tau, return_ranks=True)
    Yo, ro, _ = oracle.tsvt_dct(c.Z, c.tau, return_ranks=True)
    assert rel(to_np(Y), Yo) <= FP64_TOL
    assert ranks == [int(x) for x in ro]
    Yd = tm.tsvt_dft(to_dev(c.Z), c.tau * np.sqrt(shape[2]))
    assert rel(to_np(Yd), oracle.tsvt_dft(c.Z, c.tau * np.sqrt(shape[2]))) <= FP64_TOL


@pytest.mark.parametrize("prec", [1, 2])
def test_complete_long_tubes_reduced(tm, prec):
    # FP32 / MIXED completion on the fast transform against the oracle's iterates
    # on the float-rounded input, within the per-iteration bound
    from bounds import U_EFF, oracle_iterates

    announce("complete_long_reduced", prec=prec)
    L = 6
    cc = synth.completion_case(oracle.tprod_dct, 20, 18, 300, 3, 0.5, L, 91, tau0=1.0, tau1=0.01)
    Bf = cc.B.astype(np.float32).astype(np.float64)
    Xo, _, zmax = oracle_iterates(Bf, cc.mask, cc.taus, L)
    X, info = tm.complete_tensor(to_dev(Bf, torch.float32), to_dev(cc.mask, torch.uint8), max_iter=L, tol=0.0,
                                 tau_schedule=cc.taus, prec=prec)
    assert info["status"] == 0
    cr = np.linalg.norm(to_np(X) - Xo) / (U_EFF[prec] * zmax)
    print("completion long tubes prec %d: c per iteration %.3f" % (prec, cr / L))
    assert cr <= L * C_PATH[prec]


@pytest.mark.parametrize("prec", [1, 2])
def test_tsvt_dft_long_tubes_reduced(tm, prec):
    # the FP32 fast transform on the Fourier path; the real DFT has condition
    # number sqrt(2) relative to an orthogonal transform, so the bound is twice
    # the DCT path's
    announce("tsvt_dft_long_reduced", prec=prec)
    n1, n2, n3 = 48, 36, 300
    c = synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, 3, 0.01, 0.15 * (np.sqrt(n1) + np.sqrt(n2)) * np.sqrt(n3), 67)
    Zf = c.Z.astype(np.float32).astype(np.float64)
    Y = tm.tsvt_dft(to_dev(Zf, torch.float32), c.tau, prec=prec)
    cr = ratio(to_np(Y), oracle.tsvt_dft(Zf, c.tau), Zf, prec)
    print("tsvt_dft long prec %d: c = %.3f" % (prec, cr))
    assert cr <= 2 * C_PATH[prec]
