"""Pins of the oracle's general-transform t-SVT (Section 6: other transforms
along the tubes) and of its DFT path (Section 2: fft(X,[],3), bcirc, the DFT
t-product, TNN-F and the Fourier-domain t-SVT).

Expected values come from independent routines (numpy's FFT and LAPACK SVD),
from theorems the paper states (the block diagonalization of bcirc), from
closed forms and from the optimality conditions of the proximal problem.
"""
import numpy as np
import pytest
import scipy.fft



def F(a):
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def rnd(seed, *shape):
    return F(np.random.default_rng(seed).standard_normal(shape))


def lib_svt(A, tau):
    U, s, Vh = np.linalg.svd(A, full_matrices=False)
    return (U * np.maximum(s - tau, 0.0)) @ Vh


def apply_tubes(M, X):
    """out(:,:,k) = sum_t M[k,t] X(:,:,t) (numpy, for the checks)."""
    return F(np.einsum("kt,ijt->ijk", M, X))


# ----------------------------------------------------------------------------
# General invertible transform (Section 6)
# ----------------------------------------------------------------------------
def test_transform_dct_matrix_equals_tsvt_dct(orc):
    Z = rnd(70, 9, 7, 6)
    C = orc.dct_matrix(6)
    want = orc.tsvt_dct(Z, 0.8)
    got = orc.tsvt_transform(Z, 0.8, C, C.T.copy())
    assert np.abs(got - want).max() < 1e-14


def test_transform_identity_is_slicewise_matrix_svt(orc):
    Z = rnd(71, 8, 5, 4)
    got = orc.tsvt_transform(Z, 0.6, np.eye(4))
    for k in range(4):
        assert np.abs(got[:, :, k] - lib_svt(Z[:, :, k], 0.6)).max() < 1e-13


def test_transform_diagonal_scaling_closed_form(orc):
    # L = diag(d): slice k is SVT(d_k Z_k, tau) / d_k = SVT(Z_k, tau / |d_k|)
    Z = rnd(72, 7, 6, 5)
    d = np.array([2.0, -0.5, 1.0, 3.0, -1.5])
    got = orc.tsvt_transform(Z, 0.9, np.diag(d))
    for k in range(5):
        assert np.abs(got[:, :, k] - lib_svt(Z[:, :, k], 0.9 / abs(d[k]))).max() < 1e-13


def test_transform_slice_permutation_equivariance(orc):
    Z = rnd(73, 6, 6, 4)
    P = np.eye(4)[[2, 0, 3, 1]]
    got = orc.tsvt_transform(Z, 0.7, P)
    for k in range(4):
        assert np.abs(got[:, :, k] - lib_svt(Z[:, :, k], 0.7)).max() < 1e-13


def test_transform_orthogonal_optimality_conditions(orc):
    # orthogonal L: Y is the prox of tau * sum_k ||(L Y)_k||_* (per transformed slice)
    g = np.random.default_rng(74)
    Q, _ = np.linalg.qr(g.standard_normal((5, 5)))
    Z = rnd(75, 8, 6, 5)
    tau = 1.1
    Y = orc.tsvt_transform(Z, tau, Q)
    Zb, Yb = apply_tubes(Q, Z), apply_tubes(Q, Y)
    inner = nuc = 0.0
    for k in range(5):
        D = Zb[:, :, k] - Yb[:, :, k]
        assert np.linalg.norm(D, 2) <= tau * (1 + 1e-12)
        inner += np.sum(D * Yb[:, :, k])
        nuc += np.linalg.svd(Yb[:, :, k], compute_uv=False).sum()
    assert abs(inner - tau * nuc) < 1e-11 * max(1.0, tau * nuc)


def test_transform_general_invertible_against_library(orc):
    # a non-orthogonal, well-conditioned L: transform, slice SVT, inverse, all from numpy/LAPACK
    g = np.random.default_rng(76)
    L = np.eye(6) + 0.3 * g.standard_normal((6, 6))
    Z = rnd(77, 7, 9, 6)
    Zb = apply_tubes(L, Z)
    Yb = F(np.stack([lib_svt(Zb[:, :, k], 0.5) for k in range(6)], axis=2))
    want = apply_tubes(np.linalg.inv(L), Yb)
    got, ranks, _ = orc.tsvt_transform(Z, 0.5, L, return_ranks=True)
    assert np.abs(got - want).max() < 1e-12 * max(1.0, np.abs(want).max())
    for k in range(6):
        assert ranks[k] == np.sum(np.linalg.svd(Zb[:, :, k], compute_uv=False) > 0.5)


# ----------------------------------------------------------------------------
# DFT path (Section 2)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n3", [1, 2, 5, 8, 31])
def test_dft_tubes_match_library_fft(orc, n3):
    X = rnd(80, 4, 3, n3)
    got = orc.dft_tubes(X)
    assert np.abs(got - np.fft.fft(X, axis=2)).max() < 1e-13 * max(1, n3)
    assert np.abs(orc.idft_tubes(got) - X).max() < 1e-14 * max(1, n3)


def test_dft_conjugate_symmetry_of_real_tubes(orc):
    X = rnd(81, 3, 4, 7)
    Xt = orc.dft_tubes(X)
    for k in range(1, 7):
        assert np.abs(Xt[:, :, k] - np.conj(Xt[:, :, 7 - k])).max() < 1e-13


def test_bcirc_structure(orc):
    X = rnd(82, 2, 3, 4)
    M = orc.bcirc(X)
    assert M.shape == (8, 12)
    # first block column = unfold(X); block (r, c) = X^((r - c) mod n3)
    for r in range(4):
        for c in range(4):
            assert np.array_equal(M[2 * r:2 * r + 2, 3 * c:3 * c + 3], X[:, :, (r - c) % 4])


@pytest.mark.parametrize("shape", [(2, 3, 4), (3, 2, 5), (1, 1, 6)])
def test_bcirc_block_diagonalized_by_unitary_dft(orc, shape):
    # Theorem 1 (block diagonalization), with F the unitary DFT matrix
    n1, n2, n3 = shape
    X = rnd(83, *shape)
    Fu = np.fft.fft(np.eye(n3)) / np.sqrt(n3)
    D = np.kron(Fu, np.eye(n1)) @ orc.bcirc(X) @ np.kron(Fu.conj().T, np.eye(n2))
    Xt = np.fft.fft(X, axis=2)
    want = np.zeros_like(D)
    for k in range(n3):
        want[k * n1:(k + 1) * n1, k * n2:(k + 1) * n2] = Xt[:, :, k]
    assert np.abs(D - want).max() < 1e-13


def test_dft_tproduct_definition_and_fourier_form(orc):
    # equation (tproduct): fold(bcirc(X) unfold(Y)) equals ifft of slice products (t-product DFT)
    X, Y = rnd(84, 3, 4, 5), rnd(85, 4, 2, 5)
    spatial = orc.fold(orc.bcirc(X) @ orc.unfold(Y), 3, 2, 5)
    Xt, Yt = orc.dft_tubes(X), orc.dft_tubes(Y)
    Zt = np.stack([Xt[:, :, k] @ Yt[:, :, k] for k in range(5)], axis=2)
    fourier = orc.idft_tubes(Zt)
    assert np.abs(fourier.imag).max() < 1e-13
    assert np.abs(spatial - fourier.real).max() < 1e-13


@pytest.mark.parametrize("m,n", [(6, 4), (4, 7), (5, 5), (1, 3), (3, 1)])
def test_complex_jacobi_against_lapack(orc, m, n):
    g = np.random.default_rng(86 + m * n)
    A = g.standard_normal((m, n)) + 1j * g.standard_normal((m, n))
    Y, s, r, sw = orc.svt_complex(A, 0.0)
    assert sw > 0
    assert np.abs(s - np.linalg.svd(A, compute_uv=False)).max() < 1e-13 * max(1, s[0])
    assert np.abs(Y - A).max() < 1e-13
    Y, s, r, _ = orc.svt_complex(A, 0.9)
    assert np.abs(Y - lib_svt(A, 0.9)).max() < 1e-13
    assert r == np.sum(np.linalg.svd(A, compute_uv=False) > 0.9)


def test_complex_jacobi_rank_deficient(orc):
    g = np.random.default_rng(90)
    u = g.standard_normal((6, 1)) + 1j * g.standard_normal((6, 1))
    v = g.standard_normal((1, 4)) + 1j * g.standard_normal((1, 4))
    A = u @ v
    Y, s, r, _ = orc.svt_complex(A, 0.1)
    assert r == 1
    assert np.abs(s[1:]).max() < 1e-13 * s[0]
    assert np.abs(Y - lib_svt(A, 0.1)).max() < 1e-13 * s[0]


def tnn_f_objective(Y, Z, tau):
    n3 = Z.shape[2]
    Yt = np.fft.fft(Y, axis=2)
    nuc = sum(np.linalg.svd(Yt[:, :, k], compute_uv=False).sum() for k in range(n3)) / n3
    return tau * nuc + 0.5 * np.sum((Y - Z) ** 2)


@pytest.mark.parametrize("shape,tau", [((6, 5, 4), 1.0), ((5, 7, 5), 2.0), ((8, 8, 3), 0.5)])
def test_tsvt_dft_optimality_conditions(orc, shape, tau):
    # the Fourier-domain t-SVT at tau is the prox of tau * TNN-F: per unnormalized
    # slice ||Zt_k - Yt_k||_2 <= tau and sum_k Re<Zt_k - Yt_k, Yt_k> = tau sum_k ||Yt_k||_*
    Z = rnd(91, *shape)
    Y, ranks, _, mi = orc.tsvt_dft(Z, tau, return_ranks=True, return_imag=True)
    assert mi < 1e-13
    Zt, Yt = np.fft.fft(Z, axis=2), np.fft.fft(Y, axis=2)
    inner = nuc = 0.0
    for k in range(shape[2]):
        D = Zt[:, :, k] - Yt[:, :, k]
        assert np.linalg.norm(D, 2) <= tau * (1 + 1e-12)
        inner += np.real(np.vdot(Yt[:, :, k], D))
        nuc += np.linalg.svd(Yt[:, :, k], compute_uv=False).sum()
        assert ranks[k] == np.sum(np.linalg.svd(Zt[:, :, k], compute_uv=False) > tau)
    assert abs(inner - tau * nuc) < 1e-11 * max(1.0, tau * nuc)


def test_tsvt_dft_brute_force_tiny(orc):
    Z = rnd(92, 4, 3, 4)
    tau = 1.3
    Y = orc.tsvt_dft(Z, tau)
    f0 = tnn_f_objective(Y, Z, tau)
    g = np.random.default_rng(93)
    for _ in range(400):
        P = g.standard_normal(Z.shape) * g.choice([1e-1, 1e-3, 1e-5])
        assert tnn_f_objective(Y + P, Z, tau) >= f0 - 1e-12


def test_tsvt_dft_special_cases(orc):
    Z = rnd(94, 6, 4, 5)
    assert np.abs(orc.tsvt_dft(Z, 0.0) - Z).max() < 1e-13
    Zt = np.fft.fft(Z, axis=2)
    smax = max(np.linalg.norm(Zt[:, :, k], 2) for k in range(5))
    assert np.abs(orc.tsvt_dft(Z, smax * 1.0000001)).max() == 0.0
    Z1 = rnd(95, 7, 5, 1)  # n3 = 1: matrix SVT
    assert np.abs(orc.tsvt_dft(Z1, 0.8)[:, :, 0] - lib_svt(Z1[:, :, 0], 0.8)).max() < 1e-13


def test_tsvt_dft_against_library_route(orc):
    # numpy FFT + LAPACK complex SVD, slice by slice
    Z = rnd(96, 9, 6, 7)
    tau = 1.5
    Zt = np.fft.fft(Z, axis=2)
    Yt = np.stack([lib_svt(Zt[:, :, k], tau) for k in range(7)], axis=2)
    want = np.fft.ifft(Yt, axis=2).real
    assert np.abs(orc.tsvt_dft(Z, tau) - want).max() < 1e-13


def test_tnn_f_against_library(orc):
    X = rnd(97, 6, 5, 6)
    Xt = np.fft.fft(X, axis=2)
    want = sum(np.linalg.svd(Xt[:, :, k], compute_uv=False).sum() for k in range(6)) / 6
    assert abs(orc.tnn_f(X) - want) < 1e-12 * want


def test_tnn_c_and_tnn_f_relation_constant_tubes(orc):
    # a tensor constant along the tubes: only frequency 0 is nonzero in both transforms;
    # the DCT slice is sqrt(n3) X^(1), the DFT slice n3 X^(1), so TNN-C = ||X^(1)||_* / sqrt(n3)
    # and TNN-F = ||X^(1)||_*
    A = rnd(98, 5, 4, 1)[:, :, 0]
    X = F(np.repeat(A[:, :, None], 6, axis=2))
    nuc = np.linalg.svd(A, compute_uv=False).sum()
    assert abs(orc.tnn_f(X) - nuc) < 1e-12 * nuc
    assert abs(orc.tnn_c(X) - nuc / np.sqrt(6)) < 1e-12 * nuc


# ----------------------------------------------------------------------------
# Full (non-thin) t-SVD factors (Theorem 4: U is m1 x m1, V is m2 x m2)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(9, 5, 3), (5, 9, 4), (6, 6, 2), (12, 3, 4), (1, 4, 2)])
def test_tsvd_full_orthogonal_and_reconstructs(orc, shape):
    n1, n2, n3 = shape
    X = rnd(100 + n1, *shape)
    U, S, V, sw = orc.tsvd_dct_full(X)
    p = min(n1, n2)
    Xb = scipy.fft.dct(X, type=2, norm="ortho", axis=2)
    for k in range(n3):
        assert np.abs(U[:, :, k].T @ U[:, :, k] - np.eye(n1)).max() < 1e-13
        assert np.abs(V[:, :, k].T @ V[:, :, k] - np.eye(n2)).max() < 1e-13
        Sk = np.zeros((n1, n2))
        Sk[:p, :p] = np.diag(S[:, k])
        assert np.abs(U[:, :, k] @ Sk @ V[:, :, k].T - Xb[:, :, k]).max() < 1e-13
        # the completed columns span the complement of the range (LAPACK's full factors)
        Ul, sl, Vlt = np.linalg.svd(Xb[:, :, k])
        if n1 > p:
            P1 = U[:, p:, k] @ U[:, p:, k].T
            P2 = Ul[:, p:] @ Ul[:, p:].T
            assert np.abs(P1 - P2).max() < 1e-12
        if n2 > p:
            P1 = V[:, p:, k] @ V[:, p:, k].T
            P2 = Vlt[p:, :].T @ Vlt[p:, :]
            assert np.abs(P1 - P2).max() < 1e-12


def test_tsvd_full_theorem4_tensor_factorization(orc):
    # X = U * S * V^T with the DCT t-product, S the f-diagonal n1 x n2 x n3 tensor
    n1, n2, n3 = 7, 4, 5
    X = rnd(110, n1, n2, n3)
    U, S, V, _ = orc.tsvd_dct_full(X)
    Sb = np.zeros((n1, n2, n3))
    for k in range(n3):
        Sb[:4, :4, k] = np.diag(S[:, k])
    Ut, St, Vt = (scipy.fft.idct(A, type=2, norm="ortho", axis=2) for A in (U, Sb, V))
    VtT = F(np.transpose(Vt, (1, 0, 2)))
    R = orc.tprod_dct(orc.tprod_dct(F(Ut), F(St)), VtT)
    assert np.abs(R - X).max() < 1e-13


def test_tsvd_full_completion_rule_closed_form(orc):
    # slices whose range is spanned by e_1..e_p: the completion takes e_{p+1}, ..., e_m
    n1, n2, n3 = 7, 3, 2
    X = np.zeros((n1, n2, n3))
    X[:3, :3, 0] = np.diag([3.0, 2.0, 1.0])  # every DCT slice: a multiple of diag(3,2,1) padded
    X[:, :, 1] = X[:, :, 0]
    U, S, V, _ = orc.tsvd_dct_full(F(X))
    for k in range(n3):
        if S[0, k] == 0.0:
            continue
        assert np.array_equal(np.abs(U[:, 3:, k]), np.eye(n1)[:, 3:])


@pytest.mark.parametrize("shape,rank", [((30, 30, 2), 29), ((20, 12, 2), 5), ((12, 20, 2), 11), ((90, 40, 2), 40)])
def test_tsvd_zero_sigma_and_full_completion_orthogonal(orc, shape, rank):
    # rank-deficient square and rectangular slices, and a tall full factor whose
    # last columns span a small complement: every completed basis is orthonormal
    n1, n2, n3 = shape
    g = np.random.default_rng(120 + n1)
    Xb = np.stack([g.standard_normal((n1, rank)) @ g.standard_normal((rank, n2)) for _ in range(n3)], axis=2)
    X = F(scipy.fft.idct(Xb, type=2, norm="ortho", axis=2))
    for full in (False, True):
        U, S, V, _ = (orc.tsvd_dct_full if full else orc.tsvd_dct)(X)
        for k in range(n3):
            assert np.abs(U[:, :, k].T @ U[:, :, k] - np.eye(U.shape[1])).max() < 1e-12
            assert np.abs(V[:, :, k].T @ V[:, :, k] - np.eye(V.shape[1])).max() < 1e-12
            Sk = np.zeros((U.shape[1], V.shape[1]))
            p = min(n1, n2)
            Sk[:p, :p] = np.diag(S[:, k])
            assert np.abs(U[:, :, k] @ Sk @ V[:, :, k].T - Xb[:, :, k]).max() < 1e-11 * np.abs(Xb).max()
