"""Full t-SVD factors (Theorem 4) on the GPU against the oracle, and the
completion of zero singular values' vectors (both forms)."""
import numpy as np
import pytest

import oracle
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def rnd(seed, *shape):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape))


@pytest.mark.parametrize("shape", [(12, 5, 4), (5, 12, 3), (90, 40, 3), (40, 90, 2), (300, 170, 2), (170, 300, 2),
                                   (64, 64, 3)])
def test_tsvd_full_fp64_matches_oracle(tm, shape):
    announce("tsvd_full", shape=shape)
    n1, n2, n3 = shape
    X = rnd(7 + n1, *shape)
    U, S, V = tm.tsvd_dct(to_dev(X), transform_domain=True, full=True)
    Uo, So, Vo, _ = oracle.tsvd_dct_full(X)
    Ug, Sg, Vg = to_np(U), to_np(S), to_np(V)
    assert Ug.shape == (n1, n1, n3) and Vg.shape == (n2, n2, n3)
    assert rel(Sg, So) <= 1e-12
    eu, ev = rel(Ug, Uo), rel(Vg, Vo)
    print("full t-SVD %s: U rel %.3e, V rel %.3e" % (shape, eu, ev))
    assert eu <= 1e-9 and ev <= 1e-9
    Xb = oracle.dct_tubes(X)
    p = min(n1, n2)
    for k in range(n3):
        assert np.abs(Ug[:, :, k].T @ Ug[:, :, k] - np.eye(n1)).max() <= 1e-12
        assert np.abs(Vg[:, :, k].T @ Vg[:, :, k] - np.eye(n2)).max() <= 1e-12
        Sk = np.zeros((n1, n2))
        Sk[:p, :p] = np.diag(Sg[:, k])
        assert np.abs(Ug[:, :, k] @ Sk @ Vg[:, :, k].T - Xb[:, :, k]).max() <= 1e-12 * max(1.0, np.abs(Xb).max())


def test_tsvd_full_spatial_factorization(tm):
    # Theorem 4 in the spatial domain: X = U * S * V^T with the library's t-product
    announce("tsvd_full_spatial")
    n1, n2, n3 = 14, 6, 5
    X = rnd(21, n1, n2, n3)
    U, S, V = tm.tsvd_dct(to_dev(X), full=True)
    Sbar = np.zeros((n1, n2, n3))
    Sg = oracle.dct_tubes(np.asfortranarray(to_np(S).reshape(n2, 1, n3)))[:, 0, :]  # spatial -> transform
    for k in range(n3):
        Sbar[:n2, :n2, k] = np.diag(Sg[:, k])
    Ssp = to_dev(oracle.idct_tubes(Sbar))
    Vt = tm.fortran(V.permute(1, 0, 2))
    R = tm.tprod_dct(tm.tprod_dct(U, Ssp), Vt)
    assert rel(to_np(R), X) <= 1e-12


@pytest.mark.parametrize("full", [False, True])
@pytest.mark.parametrize("shape", [(30, 12, 3), (12, 30, 3)])
def test_tsvd_zero_singular_values_completed(tm, shape, full):
    # slices of rank 4 < p: the zero singular values' vectors are completed as in the oracle
    announce("tsvd_zero_sigma", shape=shape, full=full)
    n1, n2, n3 = shape
    g = np.random.default_rng(31)
    A, B = g.standard_normal((n1, 4, n3)), g.standard_normal((4, n2, n3))
    X = oracle.tprod_dct(np.asfortranarray(A), np.asfortranarray(B))
    U, S, V = tm.tsvd_dct(to_dev(X), transform_domain=True, full=full)
    Uo, So, Vo, _ = (oracle.tsvd_dct_full if full else oracle.tsvd_dct)(X)
    Ug, Sg, Vg = to_np(U), to_np(S), to_np(V)
    # the nonzero part agrees; the completed columns are orthonormal like the oracle's
    p = min(n1, n2)
    for k in range(n3):
        assert np.abs(Ug[:, :, k].T @ Ug[:, :, k] - np.eye(Ug.shape[1])).max() <= 1e-10
        assert np.abs(Vg[:, :, k].T @ Vg[:, :, k] - np.eye(Vg.shape[1])).max() <= 1e-10
    assert np.abs(Sg[:4] - So[:4]).max() <= 1e-12 * So.max()
    assert rel(Ug[:, :4], Uo[:, :4]) <= 1e-9 and rel(Vg[:, :4], Vo[:, :4]) <= 1e-9
    Xb = oracle.dct_tubes(X)
    for k in range(n3):
        Sk = np.zeros((Ug.shape[1], Vg.shape[1]))
        Sk[:p, :p] = np.diag(Sg[:, k])
        assert np.abs(Ug[:, :, k] @ Sk @ Vg[:, :, k].T - Xb[:, :, k]).max() <= 1e-11 * np.abs(Xb).max()


@pytest.mark.parametrize("prec", [1, 2])
def test_tsvd_full_reduced_precision(tm, prec):
    announce("tsvd_full_reduced", prec=prec)
    n1, n2, n3 = 120, 50, 3
    X = rnd(41, n1, n2, n3).astype(np.float32).astype(np.float64)
    U, S, V = tm.tsvd_dct(to_dev(X, torch.float32), prec=prec, transform_domain=True, full=True)
    Ug, Sg, Vg = to_np(U), to_np(S), to_np(V)
    Xb = oracle.dct_tubes(X)
    for k in range(n3):
        assert np.abs(Ug[:, :, k].T @ Ug[:, :, k] - np.eye(n1)).max() <= 1e-5
        Sk = np.zeros((n1, n2))
        Sk[:n2, :n2] = np.diag(Sg[:, k])
        assert np.linalg.norm(Ug[:, :, k] @ Sk @ Vg[:, :, k].T - Xb[:, :, k]) <= 1e-4 * np.linalg.norm(Xb[:, :, k])
