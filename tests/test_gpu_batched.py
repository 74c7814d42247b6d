"""Batched t-SVT of tensors of uneven shapes: parity with the oracle, and each
result independent of the rest of the batch."""
import numpy as np
import pytest
import scipy.fft

import oracle
import synth
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def lib_tprod(A, B):
    # t-product through scipy's FFT-based DCT and batched matmul: a fast input
    # generator for large shapes that shares nothing with the HIP library
    Ab = scipy.fft.dct(A, type=2, norm="ortho", axis=2)
    Bb = scipy.fft.dct(B, type=2, norm="ortho", axis=2)
    Zb = np.matmul(Ab.transpose(2, 0, 1), Bb.transpose(2, 0, 1)).transpose(1, 2, 0)
    return np.asfortranarray(scipy.fft.idct(Zb, type=2, norm="ortho", axis=2))


SHAPES = [(20, 30, 4), (64, 48, 9), (130, 70, 3), (300, 260, 2), (17, 5, 7), (256, 256, 2), (40, 520 - 8, 2)]


def batch_cases(shapes, seed0=500):
    out = []
    for i, (n1, n2, n3) in enumerate(shapes):
        out.append(synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, max(1, min(n1, n2) // 10), 0.01,
                                   0.1 * (np.sqrt(n1) + np.sqrt(n2)), seed0 + i))
    return out


def test_batched_fp64_matches_oracle(tm):
    announce("batched_fp64")
    cases = batch_cases(SHAPES)
    Ys = tm.tsvt_dct_batched([to_dev(c.Z) for c in cases], [c.tau for c in cases])
    for c, Y in zip(cases, Ys):
        assert rel(to_np(Y), oracle.tsvt_dct(c.Z, c.tau)) <= 1e-10, c.Z.shape


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batched_result_independent_of_batch(tm, prec):
    announce("batched_alone_vs_mix", prec=prec)
    dt = torch.float64 if prec == 0 else torch.float32
    cases = batch_cases(SHAPES, seed0=600)
    Zs = [to_dev(c.Z, dt) for c in cases]
    taus = [c.tau for c in cases]
    mix = tm.tsvt_dct_batched(Zs, taus, prec=prec)
    for i in (0, 3, 6):
        alone = tm.tsvt_dct_batched([Zs[i]], [taus[i]], prec=prec)[0]
        assert torch.equal(alone, mix[i]), (prec, i)
    # and the batched path agrees with the single-tensor call to the path's tolerance
    tol = {0: 1e-10, 1: 1e-4, 2: 1e-3}[prec]
    for i in (1, 4):
        single = tm.tsvt_dct(Zs[i], taus[i], prec=prec)
        assert rel(to_np(single), to_np(mix[i])) <= tol


def test_batched_uneven_full_size_sampled(tm):
    # 64 tensors, n1, n2 uniform in [32, 512], n3 in [8, 128], rank min(n1,n2)/10,
    # Gaussian t-product + N(0, 0.01), FP32; sampled slices against the oracle.
    announce("batched_uneven_64")
    shapes = synth.batch_shapes(64, synth.SEED_BASE + 4)
    Zs, taus, Zhost = [], [], []
    for s in shapes:
        Z = synth.tsvt_case(lib_tprod, s.n1, s.n2, s.n3, s.r, 0.01, s.tau, s.seed).Z
        Zf = Z.astype(np.float32).astype(np.float64)
        Zhost.append(Zf)
        Zs.append(to_dev(Zf, torch.float32))
        taus.append(s.tau)
    Ys = tm.tsvt_dct_batched(Zs, taus, prec=1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for j in rng.choice(64, size=4, replace=False):
        Yb = scipy.fft.dct(to_np(Ys[j]), type=2, norm="ortho", axis=2)
        Zb = oracle.dct_tubes(Zhost[j])
        k = int(rng.integers(0, Zhost[j].shape[2]))
        want = oracle.tsvt_dct(Zb[:, :, k:k + 1], taus[j])[:, :, 0]
        err = rel(Yb[:, :, k], want)
        print("tensor %d %s slice %d rel err %.2e" % (j, Zhost[j].shape, k, err))
        assert err <= 1e-4
