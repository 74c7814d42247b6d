"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is either
printed in the paper (Example 1 fixture), a closed form, an invariant, or a
special case that reduces to an independent library routine (scipy's FFT-based
DCT, LAPACK's SVD through numpy).  These run on the CPU only.
"""
import json
import os

import numpy as np
import pytest
import scipy.fft

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def F(a):
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def rnd(seed, *shape):
    return F(np.random.default_rng(seed).standard_normal(shape))


def lib_dct(X):
    return scipy.fft.dct(X, type=2, norm="ortho", axis=2)


def lib_idct(X):
    return scipy.fft.idct(X, type=2, norm="ortho", axis=2)


# ----------------------------------------------------------------------------
# DCT matrix and tube transforms (Section 3: Xbar = dct(X,[],3), orthonormal)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 31, 64, 100, 128])
def test_dct_matrix_orthonormal(orc, n):
    C = orc.dct_matrix(n)
    assert np.abs(C @ C.T - np.eye(n)).max() <= 4e-15 * max(1, np.sqrt(n))


def test_dct_matrix_closed_forms(orc):
    assert np.array_equal(orc.dct_matrix(1), [[1.0]])
    h = 1.0 / np.sqrt(2.0)
    assert np.abs(orc.dct_matrix(2) - np.array([[h, h], [h, -h]])).max() <= 2.3e-16


def test_dct_constant_tube_maps_to_dc(orc):
    n3 = 9
    X = F(np.full((2, 3, n3), 1.5))
    Xb = orc.dct_tubes(X)
    assert np.abs(Xb[:, :, 0] - 1.5 * np.sqrt(n3)).max() < 1e-14
    assert np.abs(Xb[:, :, 1:]).max() < 1e-14


@pytest.mark.parametrize("k0", [1, 3, 10])
def test_dct_pure_cosine_tube(orc, k0):
    # x_t = cos(pi (2t+1) k0 / (2n)) is row k0 of C up to the factor sqrt(2/n):
    # its transform is sqrt(n/2) at k0 and zero elsewhere.
    n = 12
    t = np.arange(n)
    x = np.cos(np.pi * (2 * t + 1) * k0 / (2 * n))
    Xb = orc.dct_tubes(F(x.reshape(1, 1, n)))[0, 0]
    want = np.zeros(n)
    want[k0] = np.sqrt(n / 2.0)
    assert np.abs(Xb - want).max() < 1e-14


def test_dct_matches_fft_based_library(orc):
    X = rnd(1, 5, 4, 13)
    assert np.abs(orc.dct_tubes(X) - lib_dct(X)).max() < 1e-14
    assert np.abs(orc.idct_tubes(X) - lib_idct(X)).max() < 1e-14


def test_idct_inverts_dct(orc):
    X = rnd(2, 6, 3, 11)
    assert np.abs(orc.idct_tubes(orc.dct_tubes(X)) - X).max() < 1e-14


def test_frobenius_norm_preserved(orc):
    # ||X||_F^2 is the sum over slices (Section 2); the transform is orthonormal.
    X = rnd(3, 7, 5, 10)
    assert abs(np.linalg.norm(orc.dct_tubes(X)) - np.linalg.norm(X)) < 1e-13


# ----------------------------------------------------------------------------
# Example 1 (Section 3): printed values, exact
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def ex1():
    with open(os.path.join(GOLDEN, "example1.json")) as f:
        g = json.load(f)
    return {k: (np.array(v, dtype=np.float64) if isinstance(v, list) else v) for k, v in g.items()}


def ex1_tensor(ex1):
    X = np.zeros((2, 2, 2), order="F")
    X[:, :, 0] = ex1["X1"]
    X[:, :, 1] = ex1["X2"]
    return X


def test_example1_split(orc, ex1):
    A = orc.split_shift(ex1_tensor(ex1))
    assert np.array_equal(A[:, :, 0], ex1["A1"])
    assert np.array_equal(A[:, :, 1], ex1["A2"])


def test_example1_block_matrices(orc, ex1):
    A = orc.split_shift(ex1_tensor(ex1))
    assert np.array_equal(orc.bt(A), ex1["bt"])
    assert np.array_equal(orc.bh(A), ex1["bh"])
    assert np.array_equal(orc.btph(A), ex1["btph"])
    P = ex1["P"]
    assert np.array_equal(P @ orc.btph(A) @ P, ex1["PbtphP"])


def test_example1_transformed(orc, ex1):
    A = orc.split_shift(ex1_tensor(ex1))
    C2 = orc.dct_matrix(2)
    K = np.kron(C2, np.eye(2))
    got = K @ orc.btph(A) @ np.kron(C2.T, np.eye(2))
    assert np.abs(got - ex1["transformed"]).max() < 1e-13
    # The orthonormal dct gives the printed slices divided by sqrt(2) = 1/C[k][0].
    Xb = orc.dct_tubes(ex1_tensor(ex1))
    assert np.abs(Xb[:, :, 0] - ex1["transformed"][:2, :2] / np.sqrt(2)).max() < 1e-13
    assert np.abs(Xb[:, :, 1] - ex1["transformed"][2:, 2:] / np.sqrt(2)).max() < 1e-13


# ----------------------------------------------------------------------------
# Theorem 3 (read with the per-slice factor 1/C[k][0]) and the t-product
# ----------------------------------------------------------------------------
def bdiag(X):
    n1, n2, n3 = X.shape
    out = np.zeros((n1 * n3, n2 * n3))
    for k in range(n3):
        out[k * n1:(k + 1) * n1, k * n2:(k + 1) * n2] = X[:, :, k]
    return out


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 6), (4, 2, 7), (1, 1, 3)])
def test_theorem3_corrected(orc, shape):
    n1, n2, n3 = shape
    X = rnd(10 + n3, *shape)
    A = orc.split_shift(X)
    C = orc.dct_matrix(n3)
    lhs = np.kron(C, np.eye(n1)) @ orc.btph(A) @ np.kron(C.T, np.eye(n2))
    Xhat = lib_dct(X) / C[:, 0][None, None, :]
    assert np.abs(lhs - bdiag(Xhat)).max() < 1e-12 * max(1.0, np.abs(lhs).max())
    # The statement without the factor does not hold for n3 > 1 with the
    # orthonormal transform (documented reading).
    if n3 > 1:
        assert np.abs(lhs - bdiag(lib_dct(X))).max() > 1e-3


def test_unfold_fold_roundtrip(orc):
    X = rnd(4, 3, 5, 4)
    U = orc.unfold(X)
    assert U.shape == (12, 5)
    assert np.array_equal(U[3:6, :], X[:, :, 1])
    assert np.array_equal(orc.fold(U, 3, 5, 4), X)


@pytest.mark.parametrize("shape", [(3, 4, 2, 5), (2, 2, 3, 6), (4, 3, 1, 3)])
def test_btph_product_equals_scaled_transform_product(orc, shape):
    n1, n2, n4, n3 = shape
    X, Y = rnd(20, n1, n2, n3), rnd(21, n2, n4, n3)
    C = orc.dct_matrix(n3)
    Xt = F(lib_idct(lib_dct(X) / C[:, 0][None, None, :]))
    assert np.abs(orc.btph_product(X, Y) - orc.tprod_dct(Xt, Y)).max() < 1e-12


def test_tprod_matches_library_slicewise(orc):
    X, Y = rnd(30, 4, 3, 6), rnd(31, 3, 5, 6)
    Xb, Yb = lib_dct(X), lib_dct(Y)
    Zb = np.einsum("ijk,jlk->ilk", Xb, Yb)
    assert np.abs(orc.tprod_dct(X, Y) - lib_idct(Zb)).max() < 1e-13


def test_tprod_n3_one_is_matmul(orc):
    X, Y = rnd(32, 5, 4, 1), rnd(33, 4, 3, 1)
    assert np.abs(orc.tprod_dct(X, Y)[:, :, 0] - X[:, :, 0] @ Y[:, :, 0]).max() < 1e-13
    assert np.abs(orc.btph_product(X, Y)[:, :, 0] - X[:, :, 0] @ Y[:, :, 0]).max() < 1e-13


def test_identity_tensors(orc):
    n1, n3 = 3, 4
    E = np.zeros((n1, n1, n3), order="F")
    E[:, :, 0] = np.eye(n1)
    # The identity of the definition-level product: btph(e1 (x) I) = I.
    assert np.array_equal(orc.btph(orc.split_shift(E)), np.eye(n1 * n3))
    Y = rnd(34, n1, 2, n3)
    assert np.abs(orc.btph_product(E, Y) - Y).max() < 1e-13
    # The identity of the transform-domain product: every transformed slice is I.
    Ib = np.zeros((n1, n1, n3), order="F")
    Ib[:, :, :] = np.eye(n1)[:, :, None]
    I = F(lib_idct(Ib))
    assert np.abs(orc.tprod_dct(I, Y) - Y).max() < 1e-13


# ----------------------------------------------------------------------------
# One-sided Jacobi SVD and the DCT t-SVD (Theorem 4)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("m,n", [(7, 5), (5, 7), (16, 16), (33, 9), (1, 6), (6, 1), (40, 40)])
def test_jacobi_svd_against_lapack(orc, m, n):
    A = rnd(m * 100 + n, m, n)
    U, s, V, sw = orc.jacobi_svd(A)
    p = min(m, n)
    assert sw > 0
    assert np.abs(U @ np.diag(s) @ V.T - A).max() < 1e-13 * max(1, s[0])
    assert np.abs(U.T @ U - np.eye(p)).max() < 1e-13
    assert np.abs(V.T @ V - np.eye(p)).max() < 1e-13
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.abs(s - ref).max() < 1e-13 * ref[0]
    assert np.all(np.diff(s) <= 0)
    for j in range(p):  # sign convention: largest-magnitude entry of u_j positive
        assert U[np.argmax(np.abs(U[:, j])), j] > 0


def test_jacobi_svd_rank_deficient_and_zero(orc):
    g = np.random.default_rng(5)
    A = F(g.standard_normal((9, 2)) @ g.standard_normal((2, 6)))
    U, s, V, _ = orc.jacobi_svd(A)
    assert np.abs(U @ np.diag(s) @ V.T - A).max() < 1e-13 * s[0]
    assert np.abs(s[2:]).max() < 1e-13 * s[0]
    assert np.abs(U.T @ U - np.eye(6)).max() < 1e-12
    U, s, V, _ = orc.jacobi_svd(np.zeros((4, 3)))
    assert np.array_equal(s, np.zeros(3))
    assert np.abs(U.T @ U - np.eye(3)).max() < 1e-15


def test_jacobi_svd_repeated_singular_values(orc):
    g = np.random.default_rng(6)
    Q1, _ = np.linalg.qr(g.standard_normal((8, 8)))
    Q2, _ = np.linalg.qr(g.standard_normal((5, 5)))
    A = F(Q1[:, :5] @ np.diag([3.0, 3.0, 3.0, 1.0, 1.0]) @ Q2.T)
    U, s, V, _ = orc.jacobi_svd(A)
    assert np.abs(s - [3, 3, 3, 1, 1]).max() < 1e-14
    assert np.abs(U @ np.diag(s) @ V.T - A).max() < 1e-14


def spatial_tsvd_product(orc, Ub, Sb, Vb):
    """U * S * V^T (t-products) with the transform-domain factors mapped back."""
    n1, p, n3 = Ub.shape
    n2 = Vb.shape[0]
    Sd = np.zeros((p, p, n3), order="F")
    for k in range(n3):
        Sd[:, :, k] = np.diag(Sb[:, k])
    U = orc.idct_tubes(Ub)
    S = orc.idct_tubes(F(Sd))
    Vt = orc.idct_tubes(F(np.transpose(Vb, (1, 0, 2))))
    return orc.tprod_dct(orc.tprod_dct(U, S), Vt)


@pytest.mark.parametrize("shape", [(6, 4, 5), (4, 6, 3), (8, 8, 1), (5, 5, 7)])
def test_tsvd_dct_reconstruction(orc, shape):
    X = rnd(40 + shape[2], *shape)
    Ub, Sb, Vb, sw = orc.tsvd_dct(X)
    assert sw > 0
    R = spatial_tsvd_product(orc, Ub, Sb, Vb)
    assert np.linalg.norm(R - X) / np.linalg.norm(X) < 1e-13
    Xb = lib_dct(X)
    for k in range(shape[2]):
        assert np.abs(Ub[:, :, k].T @ Ub[:, :, k] - np.eye(min(shape[:2]))).max() < 1e-13
        ref = np.linalg.svd(Xb[:, :, k], compute_uv=False)
        assert np.abs(Sb[:, k] - ref).max() < 1e-13 * max(1, ref[0])


def test_tnn_c(orc):
    X = rnd(50, 5, 4, 6)
    Xb = lib_dct(X)
    want = sum(np.linalg.svd(Xb[:, :, k], compute_uv=False).sum() for k in range(6)) / 6
    assert abs(orc.tnn_c(X) - want) < 1e-12 * want


# ----------------------------------------------------------------------------
# t-SVT (Theorem 5): optimality conditions, special cases, equivariances
# ----------------------------------------------------------------------------
def svt_objective(Y, Z, tau):
    Yb = lib_dct(Y)
    nuc = sum(np.linalg.svd(Yb[:, :, k], compute_uv=False).sum() for k in range(Y.shape[2]))
    return tau * nuc + 0.5 * np.linalg.norm(Y - Z) ** 2


def lowrank_noisy(orc, seed, n1, n2, n3, r, sigma):
    g = np.random.default_rng(seed)
    A, B = F(g.standard_normal((n1, r, n3))), F(g.standard_normal((r, n2, n3)))
    return F(orc.tprod_dct(A, B) + sigma * g.standard_normal((n1, n2, n3)))


@pytest.mark.parametrize("shape,tau", [((8, 6, 5), 1.0), ((6, 9, 4), 2.5), ((12, 12, 3), 0.5)])
def test_tsvt_optimality_conditions(orc, shape, tau):
    Z = lowrank_noisy(orc, 60, *shape, 2, 0.3)
    Y, ranks, sw = orc.tsvt_dct(Z, tau, return_ranks=True)
    Zb, Yb = lib_dct(Z), lib_dct(Y)
    inner, nuc = 0.0, 0.0
    for k in range(shape[2]):
        D = Zb[:, :, k] - Yb[:, :, k]
        assert np.linalg.norm(D, 2) <= tau * (1 + 1e-12)
        inner += np.sum(D * Yb[:, :, k])
        sv = np.linalg.svd(Yb[:, :, k], compute_uv=False)
        nuc += sv.sum()
        zs = np.linalg.svd(Zb[:, :, k], compute_uv=False)
        assert ranks[k] == np.sum(zs > tau)
    assert abs(inner - tau * nuc) < 1e-11 * max(1.0, tau * nuc)


def test_tsvt_brute_force_tiny(orc):
    Z = lowrank_noisy(orc, 61, 4, 3, 3, 1, 0.5)
    tau = 0.7
    Y = orc.tsvt_dct(Z, tau)
    f0 = svt_objective(Y, Z, tau)
    g = np.random.default_rng(62)
    for _ in range(500):
        P = g.standard_normal(Z.shape) * g.choice([1e-1, 1e-3, 1e-5])
        assert svt_objective(Y + P, Z, tau) >= f0 - 1e-12


def test_tsvt_tau_zero_is_identity(orc):
    Z = rnd(63, 7, 5, 4)
    assert np.abs(orc.tsvt_dct(Z, 0.0) - Z).max() < 1e-13


def test_tsvt_large_tau_is_zero(orc):
    Z = rnd(64, 7, 5, 4)
    Zb = lib_dct(Z)
    smax = max(np.linalg.norm(Zb[:, :, k], 2) for k in range(4))
    Y, ranks, _ = orc.tsvt_dct(Z, smax * 1.0000001, return_ranks=True)
    assert np.abs(Y).max() == 0.0
    assert np.all(ranks == 0)


def test_tsvt_n3_one_is_matrix_svt(orc):
    Z = rnd(65, 9, 6, 1)
    U, s, Vt = np.linalg.svd(Z[:, :, 0], full_matrices=False)
    want = U @ np.diag(np.maximum(s - 1.2, 0)) @ Vt
    assert np.abs(orc.tsvt_dct(Z, 1.2)[:, :, 0] - want).max() < 1e-13


def test_tsvt_single_row_is_group_shrinkage(orc):
    Z = rnd(66, 1, 7, 6)
    tau = 1.1
    Zb = lib_dct(Z)
    Yb = np.zeros_like(Zb)
    for k in range(6):
        z = Zb[0, :, k]
        nz = np.linalg.norm(z)
        Yb[0, :, k] = max(1 - tau / nz, 0.0) * z
    assert np.abs(orc.tsvt_dct(Z, tau) - lib_idct(Yb)).max() < 1e-13


def test_tsvt_slice_diagonal_is_elementwise_shrink(orc):
    g = np.random.default_rng(67)
    n, n3, tau = 5, 4, 0.8
    Zb = np.zeros((n, n, n3))
    for k in range(n3):
        Zb[:, :, k] = np.diag(g.standard_normal(n) * 2)
    Z = F(lib_idct(Zb))
    Yb = np.sign(Zb) * np.maximum(np.abs(Zb) - tau, 0.0)
    assert np.abs(orc.tsvt_dct(Z, tau) - lib_idct(Yb)).max() < 1e-13


def test_tsvt_scaling_and_transpose(orc):
    Z = lowrank_noisy(orc, 68, 7, 5, 4, 2, 0.2)
    tau, a = 0.9, 3.5
    Y = orc.tsvt_dct(Z, tau)
    assert np.abs(orc.tsvt_dct(a * Z, a * tau) - a * Y).max() < 1e-12 * a * np.abs(Y).max()
    Zt = F(np.transpose(Z, (1, 0, 2)))
    assert np.abs(orc.tsvt_dct(Zt, tau) - np.transpose(Y, (1, 0, 2))).max() < 1e-13


def test_tsvt_nonexpansive(orc):
    Z1 = lowrank_noisy(orc, 69, 6, 6, 5, 2, 0.3)
    Z2 = F(Z1 + 0.05 * np.random.default_rng(70).standard_normal(Z1.shape))
    d = np.linalg.norm(orc.tsvt_dct(Z1, 0.5) - orc.tsvt_dct(Z2, 0.5))
    assert d <= np.linalg.norm(Z1 - Z2) * (1 + 1e-12)


# ----------------------------------------------------------------------------
# Algorithm 1 (ADMM completion)
# ----------------------------------------------------------------------------
def small_completion(orc, seed=80, shape=(12, 10, 5), r=2, sr=0.6, L=30):
    import synth

    return synth.completion_case(orc.tprod_dct, *shape, r, sr, L, seed, tau0=1.0, tau1=0.01)


def test_complete_keeps_observed_entries(orc):
    case = small_completion(orc)
    for L in (1, 2, 7):
        X, M, it, _ = orc.complete(case.B, case.mask, case.betas[:L], case.taus[:L])
        assert it == L
        obs = case.mask != 0
        assert np.array_equal(X[obs], case.B[obs])
        # Steps 2 and 3 together leave the multiplier supported on the observed
        # set: off it, M + beta (Y - (Y + M/beta)) = 0 up to rounding.
        assert np.abs(M[~obs]).max() <= 1e-12 * max(1.0, np.abs(M).max())


def test_complete_multiplier_support_from_warm_start(orc):
    # From any warm start (X0, M0), one iteration leaves M zero off the observed
    # set and X equal to B on it (Algorithm 1, X-update and multiplier update).
    case = small_completion(orc)
    g = np.random.default_rng(81)
    X0 = F(g.standard_normal(case.B.shape))
    M0 = F(g.standard_normal(case.B.shape))
    X, M, _, _ = orc.complete(case.B, case.mask, case.betas[:1], case.taus[:1], X0=X0, M0=M0)
    obs = case.mask != 0
    assert np.abs(M[~obs]).max() <= 1e-12 * np.abs(M).max()
    assert np.array_equal(X[obs], case.B[obs])


def test_complete_all_observed_is_fixed_point(orc):
    case = small_completion(orc)
    ones = np.ones_like(case.mask)
    X, M, it, rc = orc.complete(case.T, ones, case.betas[:5], case.taus[:5])
    assert np.array_equal(X, case.T)
    assert rc == 0.0


def test_complete_first_iteration_against_library(orc):
    # One iteration from X = B, M = 0 written with LAPACK's SVD and scipy's DCT.
    case = small_completion(orc)
    b, tau = case.betas[0], case.taus[0]
    Zb = lib_dct(case.B)
    Yb = np.zeros_like(Zb)
    for k in range(Zb.shape[2]):
        U, s, Vt = np.linalg.svd(Zb[:, :, k], full_matrices=False)
        Yb[:, :, k] = U @ np.diag(np.maximum(s - tau, 0)) @ Vt
    Y = lib_idct(Yb)
    Xw = np.where(case.mask != 0, case.B, Y)
    Mw = b * (Y - Xw)
    X, M, _, _ = orc.complete(case.B, case.mask, case.betas[:1], case.taus[:1])
    assert np.abs(X - Xw).max() < 1e-12
    assert np.abs(M - Mw).max() < 1e-12 * max(1, np.abs(Mw).max())


def test_complete_iterations_from_warm_start_against_library(orc):
    # Four iterations of Algorithm 1 from a random (X0, M0), each written with
    # LAPACK's SVD and scipy's DCT: Z = X - M/beta, Y = t-SVT(Z, 1/beta),
    # X = B on the observed set and Y + M/beta off it, M = M + beta (Y - X).
    # A nonzero M exercises both multiplier terms and their signs.
    case = small_completion(orc)
    g = np.random.default_rng(82)
    X = F(g.standard_normal(case.B.shape))
    M = F(g.standard_normal(case.B.shape))
    obs = case.mask != 0
    L = 4
    Xo, Mo, _, _ = orc.complete(case.B, case.mask, case.betas[:L], case.taus[:L], X0=X, M0=M)
    for b, tau in zip(case.betas[:L], case.taus[:L]):
        Zb = lib_dct(X - M / b)
        Yb = np.zeros_like(Zb)
        for k in range(Zb.shape[2]):
            U, s, Vt = np.linalg.svd(Zb[:, :, k], full_matrices=False)
            Yb[:, :, k] = U @ np.diag(np.maximum(s - tau, 0)) @ Vt
        Y = lib_idct(Yb)
        X = np.where(obs, case.B, Y + M / b)
        M = M + b * (Y - X)
    assert np.abs(Xo - X).max() <= 1e-11 * np.abs(X).max()
    assert np.abs(Mo - M).max() <= 1e-11 * np.abs(M).max()


def test_complete_resume_equals_straight_run(orc):
    case = small_completion(orc)
    X, M, _, _ = orc.complete(case.B, case.mask, case.betas[:10], case.taus[:10])
    X1, M1, _, _ = orc.complete(case.B, case.mask, case.betas[:5], case.taus[:5])
    X2, M2, _, _ = orc.complete(case.B, case.mask, case.betas[5:10], case.taus[5:10], X0=X1, M0=M1)
    assert np.array_equal(X, X2) and np.array_equal(M, M2)


def test_complete_recovers_low_rank(orc):
    case = small_completion(orc, shape=(20, 18, 6), r=2, sr=0.7, L=60)
    X, _, _, _ = orc.complete(case.B, case.mask, case.betas, case.taus)
    err = np.linalg.norm(X - case.T) / np.linalg.norm(case.T)
    err0 = np.linalg.norm(case.B - case.T) / np.linalg.norm(case.T)
    assert err < 0.05 * err0


def test_complete_tolerance_stops_early(orc):
    case = small_completion(orc, L=200)
    betas = np.full(200, 10.0)
    X, M, it, rc = orc.complete(case.B, case.mask, betas, tol=1e-6)
    assert it < 200 and rc <= 1e-6
