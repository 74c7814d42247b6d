"""Batched t-SVT of tensors of uneven shapes: parity with the oracle, and each
result independent of the rest of the batch."""
import numpy as np
import pytest
import scipy.fft

import oracle
import synth
from bounds import C_PATH, FP64_TOL, U_EFF, ratio, within
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
    # and the batched path agrees with the single-tensor call to the path's
    # tolerance (each within the stated bound of the oracle, so within twice it of each other)
    for i in (1, 4):
        single = tm.tsvt_dct(Zs[i], taus[i], prec=prec)
        if prec == 0:
            assert rel(to_np(single), to_np(mix[i])) <= 2 * FP64_TOL
        else:
            assert ratio(to_np(single), to_np(mix[i]), to_np(Zs[i]), prec) <= 2 * C_PATH[prec]


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
    Ys, status = tm.tsvt_dct_batched(Zs, taus, prec=1, return_status=True)
    torch.cuda.synchronize()
    assert status == [0] * 64
    # whole tensors against the oracle (on all host threads): the largest job
    # and the ten cheapest, within the stated FP32 bound
    oracle.set_threads(min(16, oracle.host_threads()))
    cost = [s.n1 * s.n2 * min(s.n1, s.n2) * s.n3 for s in shapes]
    order = list(np.argsort(cost))
    for j in [order[-1]] + order[:10]:
        want = oracle.tsvt_dct(Zhost[j], taus[j])
        c = ratio(to_np(Ys[j]), want, Zhost[j], 1)
        print("tensor %d %s: c = %.2f, rel err %.2e" % (j, Zhost[j].shape, c, rel(to_np(Ys[j]), want)))
        assert c <= C_PATH[1]


@pytest.mark.parametrize("prec", [0, 2])
def test_batched_nonfinite_tensor_fails_alone(tm, prec):
    # one tensor holds a NaN: only its status says so; the others are
    # bitwise the results they get alone
    announce("batched_nonfinite_alone", prec=prec)
    dt = torch.float64 if prec == 0 else torch.float32
    cases = batch_cases(SHAPES[:4], seed0=640)
    Zh = [c.Z.copy() for c in cases]
    Zh[1][5, 3, 1] = np.nan
    Zs = [to_dev(z, dt) for z in Zh]
    taus = [c.tau for c in cases]
    Ys, status = tm.tsvt_dct_batched(Zs, taus, prec=prec, return_status=True)
    assert status[1] == tm.ENONFINITE
    assert [status[i] for i in (0, 2, 3)] == [0, 0, 0]
    for i in (0, 2, 3):
        alone = tm.tsvt_dct_batched([Zs[i]], [taus[i]], prec=prec)[0]
        assert torch.equal(alone, Ys[i]), i
    # without per-tensor statuses the call reports the failure
    with pytest.raises(tm.TsvdError) as ei:
        tm.tsvt_dct_batched(Zs, taus, prec=prec)
    assert ei.value.code == tm.ENONFINITE
