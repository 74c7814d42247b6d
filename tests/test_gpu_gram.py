"""The block-Gram multi-workgroup Jacobi kernel (TSVD_OPT_GRAM = 1 forces it)
against the FP64 oracle: FP64 (<= 1e-10), FP32 and MIXED (stated bounds), on
shapes with several blocks and ragged edges (p not a multiple of 16, wide
slices read transposed, m not a multiple of 64), team sizes from one
workgroup to one per block pair, with V (t-SVD factors, completion warm
start), degenerate spectra, and the benchmarked 256 x 256 x 31 workload.
"""
import numpy as np
import pytest

import oracle
import synth
from bounds import C_PATH, FP64_TOL, U_EFF, oracle_iterates, ratio
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def case(shape, seed, tau=None):
    n1, n2, n3 = shape
    if tau is None:
        tau = 0.1 * (np.sqrt(n1) + np.sqrt(n2))
    return synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, max(1, min(n1, n2) // 10), 0.01, tau, seed)


def gram_ctx(tm, W=0):
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_GRAM, 1)
    if W:
        ctx.set_option(tm.OPT_TEAM_SIZE, W)
    return ctx


SHAPES = [((256, 256, 3), (0, 1, 8)), ((250, 230, 2), (3,)), ((200, 300, 2), (4,)), ((300, 170, 2), (2, 6)),
          ((512, 512, 1), (16,)), ((300, 130, 3), (1,))]


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("shape,teams", SHAPES)
def test_gram_kernel_tsvt_matches_oracle(tm, shape, teams, prec):
    c = case(shape, 800 + shape[0] + shape[2])
    dt = torch.float64 if prec == 0 else torch.float32
    Zh = c.Z if prec == 0 else c.Z.astype(np.float32).astype(np.float64)
    want = oracle.tsvt_dct(Zh, c.tau)
    Z = to_dev(Zh, dt)
    for W in teams:
        announce("gram_tsvt", shape=shape, W=W, prec=prec)
        ctx = gram_ctx(tm, W)
        try:
            t = ctx.tile(prec, *shape)
            assert t["team"] == 2 and t["source"] == 2
            Y, ranks = tm.tsvt_dct(Z, c.tau, prec=prec, ctx=ctx, return_ranks=True)
            Yg = to_np(Y)
            if prec == 0:
                err = rel(Yg, want)
                print("gram %s W %d FP64: rel err %.3e tile %s" % (shape, W, err, t))
                assert err <= FP64_TOL
            else:
                cr = ratio(Yg, want, Zh, prec)
                print("gram %s W %d prec %d: c = %.3f tile %s" % (shape, W, prec, cr, t))
                assert cr <= C_PATH[prec]
        finally:
            ctx.close()


@pytest.mark.parametrize("prec", [0, 2])
def test_gram_kernel_tsvd_factors(tm, prec):
    # with V: U S V^T reconstructs every transformed slice; sigma matches the oracle
    shape = (220, 160, 3)
    announce("gram_tsvd", prec=prec)
    c = case(shape, 810)
    dt = torch.float64 if prec == 0 else torch.float32
    Zh = c.Z if prec == 0 else c.Z.astype(np.float32).astype(np.float64)
    ctx = gram_ctx(tm, 2)
    try:
        U, S, V = tm.tsvd_dct(to_dev(Zh, dt), prec=prec, transform_domain=True, ctx=ctx)
        Uo, So, Vo, _ = oracle.tsvd_dct(Zh)
        Ug, Sg, Vg = to_np(U), to_np(S), to_np(V)
        Zb = oracle.dct_tubes(Zh)
        tol = FP64_TOL if prec == 0 else 64 * U_EFF[prec]
        for k in range(shape[2]):
            R = (Ug[:, :, k] * Sg[:, k]) @ Vg[:, :, k].T
            assert np.linalg.norm(R - Zb[:, :, k]) <= tol * np.linalg.norm(Zb[:, :, k])
            assert np.abs(Sg[:, k] - So[:, k]).max() <= tol * So[0, k]
            assert np.abs(Vg[:, :, k].T @ Vg[:, :, k] - np.eye(160)).max() <= (1e-12 if prec == 0 else 1e-4)
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", [0, 2])
def test_gram_kernel_completion_warm_start(tm, prec):
    # completion with V carried between iterations (warm start) on the block-Gram kernel
    announce("gram_complete", prec=prec)
    L = 6
    cc = synth.completion_case(oracle.tprod_dct, 256, 256, 31, 10, 0.3, 100, synth.SEED_BASE + 2)
    Bh = cc.B if prec == 0 else cc.B.astype(np.float32).astype(np.float64)
    dt = torch.float64 if prec == 0 else torch.float32
    ctx = gram_ctx(tm)
    try:
        X, info = tm.complete_tensor(to_dev(Bh, dt), to_dev(cc.mask, torch.uint8), max_iter=L, tol=0.0,
                                     tau_schedule=cc.taus, prec=prec, ctx=ctx)
        assert ctx.tile(prec, 256, 256, 31, with_v=True)["team"] == 2
    finally:
        ctx.close()
    oracle.set_threads(min(16, oracle.host_threads()))
    Xo, _, zmax = oracle_iterates(Bh, cc.mask, cc.taus, L)
    Xg = to_np(X)
    if prec == 0:
        err = rel(Xg, Xo)
        print("gram completion FP64: rel err %.3e" % err)
        assert err <= FP64_TOL
    else:
        cr = np.linalg.norm(Xg - Xo) / (U_EFF[prec] * zmax)
        print("gram completion prec %d: c per iteration %.3f" % (prec, cr / L))
        assert cr <= L * C_PATH[prec]
    assert info["status"] == 0


@pytest.mark.parametrize("prec", [0, 2])
@pytest.mark.parametrize("kind", ["zero", "equal_columns", "repeated"])
def test_gram_kernel_degenerate_spectra(tm, prec, kind):
    announce("gram_degenerate", prec=prec, kind=kind)
    n1, n2, n3 = 240, 200, 2
    g = np.random.default_rng(820)
    if kind == "zero":
        Z = np.zeros((n1, n2, n3))
    elif kind == "equal_columns":
        col = g.standard_normal((n1, 1, n3))
        Z = np.repeat(col, n2, axis=1)
    else:
        Q1, _ = np.linalg.qr(g.standard_normal((n1, n2)))
        Q2, _ = np.linalg.qr(g.standard_normal((n2, n2)))
        s = np.repeat([3.0, 2.0, 1.0, 0.5], n2 // 4)
        Z = np.stack([(Q1 * s) @ Q2.T] * n3, axis=2)
    Z = np.asfortranarray(Z)
    dt = torch.float64 if prec == 0 else torch.float32
    Zh = Z if prec == 0 else Z.astype(np.float32).astype(np.float64)
    tau = 0.7
    ctx = gram_ctx(tm, 3)
    try:
        Y = to_np(tm.tsvt_dct(to_dev(Zh, dt), tau, prec=prec, ctx=ctx))
    finally:
        ctx.close()
    want = oracle.tsvt_dct(Zh, tau)
    assert np.isfinite(Y).all()
    if prec == 0:
        assert np.linalg.norm(Y - want) <= FP64_TOL * max(1.0, np.linalg.norm(want))
    else:
        assert np.linalg.norm(Y - want) <= C_PATH[prec] * U_EFF[prec] * max(1.0, np.linalg.norm(Zh))


@pytest.mark.parametrize("prec", [0, 2])
def test_gram_kernel_bench_workload(tm, prec):
    # the benchmarked t-SVT inputs' first iterate, every slice
    announce("gram_bench", prec=prec)
    cc = synth.completion_case(oracle.tprod_dct, 256, 256, 31, 10, 0.3, 100, synth.SEED_BASE + 2)
    Zh = cc.B if prec == 0 else cc.B.astype(np.float32).astype(np.float64)
    dt = torch.float64 if prec == 0 else torch.float32
    oracle.set_threads(min(16, oracle.host_threads()))
    for tau in (float(cc.taus[0]), float(cc.taus[-1])):
        ctx = gram_ctx(tm)
        try:
            Y = to_np(tm.tsvt_dct(to_dev(Zh, dt), tau, prec=prec, ctx=ctx))
            st = ctx.stats()
        finally:
            ctx.close()
        want = oracle.tsvt_dct(Zh, tau)
        if prec == 0:
            err = rel(Y, want)
            print("gram bench FP64 tau %.3g: rel err %.3e, slice-sweeps %d" % (tau, err, st["slice_sweeps"]))
            assert err <= FP64_TOL
        else:
            cr = ratio(Y, want, Zh, prec)
            print("gram bench prec %d tau %.3g: c = %.3f, slice-sweeps %d" % (prec, tau, cr, st["slice_sweeps"]))
            assert cr <= C_PATH[prec]
