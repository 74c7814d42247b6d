"""Oracle parity of the benchmarked configurations at full size.

256 x 256 x 31 (multispectral-shaped; tubal rank 10, [0, 1], 30% observed):
  * the isolated t-SVT, every slice, FP64 (<= 1e-10) and MIXED (stated bound),
    at the schedule's first and last thresholds;
  * the isolated t-SVT of a late iterate of the schedule (the oracle's 30th),
    where the kept-column Jacobi certifies every slice, every slice checked;
  * the completion (Algorithm 1) on the path the benchmark times: the
    multi-workgroup Jacobi kernel carrying V (warm start), FP64 and MIXED,
    whole tensor, against the oracle's iterations;
  * a MIXED and an FP32 completion long enough to cross the reset of the
    warm-start vectors (every 64 iterations).
The oracle runs on all host threads (slices split across threads; its
arithmetic per slice is unchanged, so its results do not depend on the count).
"""
import numpy as np
import pytest

import oracle
import synth
from bounds import C_PATH, FP64_TOL, U_EFF, oracle_iterates, ratio
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu

N1, N2, N3 = 256, 256, 31


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    oracle.set_threads(min(16, oracle.host_threads()))
    return tm


@pytest.fixture(scope="module")
def cc():
    return synth.completion_case(oracle.tprod_dct, N1, N2, N3, 10, 0.3, 100, synth.SEED_BASE + 2)


@pytest.mark.parametrize("which", ["first", "last"])
def test_tsvt_fullsize_every_slice_fp64(tm, cc, which):
    tau = float(cc.taus[0] if which == "first" else cc.taus[-1])
    announce("tsvt_full_fp64", tau=tau)
    Yo, ro, _ = oracle.tsvt_dct(cc.B, tau, return_ranks=True)
    Y, ranks = tm.tsvt_dct(to_dev(cc.B), tau, return_ranks=True)
    err = rel(to_np(Y), Yo)
    print("FP64 t-SVT 256x256x31 tau %.3g: rel err %.3e, ranks %s" % (tau, err, ranks))
    assert list(ranks) == [int(r) for r in ro]
    assert err <= FP64_TOL


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("which", ["first", "last"])
def test_tsvt_fullsize_every_slice_reduced(tm, cc, prec, which):
    tau = float(cc.taus[0] if which == "first" else cc.taus[-1])
    announce("tsvt_full_reduced", prec=prec, tau=tau)
    Zf = cc.B.astype(np.float32).astype(np.float64)
    Yo = oracle.tsvt_dct(Zf, tau)
    Y = to_np(tm.tsvt_dct(to_dev(Zf, torch.float32), tau, prec=prec))
    c = ratio(Y, Yo, Zf, prec)
    # per slice, against each slice's own norm
    Yb, Yob, Zb = oracle.dct_tubes(Y), oracle.dct_tubes(Yo), oracle.dct_tubes(Zf)
    ck = max(np.linalg.norm(Yb[:, :, k] - Yob[:, :, k]) / (U_EFF[prec] * np.linalg.norm(Zb[:, :, k]))
             for k in range(N3))
    print("prec %d t-SVT 256x256x31 tau %.3g: c = %.3f, worst slice c = %.3f, rel err vs FP64 oracle %.3e, "
          "vs FP64 input %.3e" % (prec, tau, c, ck, rel(Y, Yo), rel(Y, oracle.tsvt_dct(cc.B, tau))))
    assert c <= C_PATH[prec]
    assert ck <= C_PATH[prec]


@pytest.fixture(scope="module")
def late_iterate(cc):
    # a late t-SVT input of the benchmark's schedule, Z_L = X_L - M_L / beta_L,
    # from L iterations of the oracle's Algorithm 1 (a rank-10 part far above
    # tau_L, the rest well below: the kept-column mode's fast path)
    L = 30
    X, M, _, _ = oracle.complete(cc.B, cc.mask, cc.betas[:L], cc.taus[:L])
    return np.asfortranarray(X - M / cc.betas[L]), float(cc.taus[L])


@pytest.mark.parametrize("prec", [0, 2])
def test_tsvt_fullsize_late_iterate_kept_columns(tm, late_iterate, prec):
    Z, tau = late_iterate
    announce("tsvt_full_late", prec=prec, tau=tau)
    Zi = Z if prec == 0 else Z.astype(np.float32).astype(np.float64)
    Yo, ro, _ = oracle.tsvt_dct(Zi, tau, return_ranks=True)
    ctx = tm.Context(0)
    try:
        ctx.stats(reset=True)
        Y, ranks = tm.tsvt_dct(to_dev(Zi, torch.float32 if prec else torch.float64), tau, prec=prec,
                               return_ranks=True, ctx=ctx)
        st = ctx.stats(reset=True)
    finally:
        ctx.close()
    Y = to_np(Y)
    print("late iterate prec %d tau %.3g: ranks %s, pairs %d, fallback %d, sweeps per slice %.2f" % (
        prec, tau, list(ranks), st["pairs"], st["fallback_slices"], st["slice_sweeps"] / N3))
    assert list(ranks) == [int(r) for r in ro]
    assert st["pairs"] > 0 and st["fallback_slices"] == 0
    if prec == 0:
        Yb, Yob = oracle.dct_tubes(Y), oracle.dct_tubes(Yo)
        worst = max(np.linalg.norm(Yb[:, :, k] - Yob[:, :, k]) / max(np.linalg.norm(Yob[:, :, k]), 1e-300)
                    for k in range(N3) if ro[k] > 0)
        print("  FP64 rel err %.3e, worst kept slice %.3e" % (rel(Y, Yo), worst))
        assert rel(Y, Yo) <= FP64_TOL
        assert worst <= FP64_TOL
    else:
        Yb, Yob, Zb = oracle.dct_tubes(Y), oracle.dct_tubes(Yo), oracle.dct_tubes(Zi)
        ck = max(np.linalg.norm(Yb[:, :, k] - Yob[:, :, k]) / (U_EFF[prec] * np.linalg.norm(Zb[:, :, k]))
                 for k in range(N3))
        c = ratio(Y, Yo, Zi, prec)
        print("  MIXED c = %.3f, worst slice c = %.3f" % (c, ck))
        assert c <= C_PATH[prec] and ck <= C_PATH[prec]


def test_complete_fullsize_fp64_bench_path(tm, cc):
    L = 6
    announce("complete_full_fp64", L=L)
    ctx = tm.Context(0)
    X, info, M = tm.complete_tensor(to_dev(cc.B), to_dev(cc.mask, torch.uint8), max_iter=L, tol=0.0,
                                    tau_schedule=cc.taus, ctx=ctx, return_M=True)
    tile = ctx.tile(tm.FP64, N1, N2, N3, with_v=True)
    ctx.close()
    Xo, Mo, _ = oracle_iterates(cc.B, cc.mask, cc.taus, L)
    ex, em = rel(to_np(X), Xo), rel(to_np(M), Mo)
    print("FP64 completion 256x256x31, %d iterations, tile %s: X rel err %.3e, M rel err %.3e" % (L, tile, ex, em))
    assert info["iters"] == L and info["status"] == 0
    assert tile["team"] == 1  # the multi-workgroup kernel, as in the benchmark
    assert ex <= FP64_TOL and em <= FP64_TOL


@pytest.mark.parametrize("prec", [2, 1])
def test_complete_fullsize_reduced_bench_path(tm, cc, prec):
    L = 8
    announce("complete_full_reduced", prec=prec, L=L)
    Bf = cc.B.astype(np.float32).astype(np.float64)
    ctx = tm.Context(0)
    X, info = tm.complete_tensor(to_dev(Bf, torch.float32), to_dev(cc.mask, torch.uint8), max_iter=L, tol=0.0,
                                 tau_schedule=cc.taus, prec=prec, ctx=ctx)
    tile = ctx.tile(prec, N1, N2, N3, with_v=True)
    ctx.close()
    Xo, _, zmax = oracle_iterates(Bf, cc.mask, cc.taus, L)
    Xg = to_np(X)
    err = np.linalg.norm(Xg - Xo)
    c = err / (U_EFF[prec] * zmax)
    print("prec %d completion 256x256x31, %d iterations, tile %s: rel err %.3e, c per iteration %.3f" % (
        prec, L, tile, rel(Xg, Xo), c / L))
    assert info["iters"] == L and info["status"] == 0
    assert tile["team"] == 1
    # observed entries stay exactly B
    obs = cc.mask != 0
    assert np.array_equal(Xg[obs], Bf[obs].astype(np.float32).astype(np.float64))
    assert c <= L * C_PATH[prec]


@pytest.mark.parametrize("prec", [2, 1])
def test_complete_crosses_warm_start_reset(tm, prec):
    # 70 iterations: the warm-start vectors are reset to the identity at
    # iteration 64, so both sides of the reset are checked against the oracle
    L = 70
    announce("complete_warm_reset", prec=prec, L=L)
    c0 = synth.completion_case(oracle.tprod_dct, 40, 36, 8, 3, 0.5, L, 7, tau0=2.0, tau1=0.05)
    Bf = c0.B.astype(np.float32).astype(np.float64)
    X, info = tm.complete_tensor(to_dev(Bf, torch.float32), to_dev(c0.mask, torch.uint8), max_iter=L, tol=0.0,
                                 tau_schedule=c0.taus, prec=prec)
    Xo, _, zmax = oracle_iterates(Bf, c0.mask, c0.taus, L)
    err = np.linalg.norm(to_np(X) - Xo)
    c = err / (U_EFF[prec] * zmax)
    print("prec %d completion 40x36x8, %d iterations: rel err %.3e, c per iteration %.3f" % (
        prec, L, rel(to_np(X), Xo), c / L))
    assert info["iters"] == L
    assert c <= L * C_PATH[prec]


def test_complete_nonfinite_input(tm):
    announce("complete_nonfinite")
    c0 = synth.completion_case(oracle.tprod_dct, 24, 20, 5, 2, 0.5, 4, 11)
    X0 = np.where(c0.mask != 0, c0.B, 0.0)
    X0[3, 4, 2] = np.nan
    with pytest.raises(tm.TsvdError) as ei:
        tm.complete_tensor(to_dev(c0.B), to_dev(c0.mask, torch.uint8), X=to_dev(X0), max_iter=3, tol=0.0,
                           tau_schedule=c0.taus)
    assert ei.value.code == tm.ENONFINITE
    # an infinite observed value reaches Z through the X-update of the first iteration
    B = c0.B.copy()
    idx = tuple(np.argwhere(c0.mask != 0)[0])
    B[idx] = np.inf
    with pytest.raises(tm.TsvdError) as ei:
        tm.complete_tensor(to_dev(B), to_dev(c0.mask, torch.uint8), max_iter=3, tol=0.0, tau_schedule=c0.taus)
    assert ei.value.code == tm.ENONFINITE
    # the context is usable afterwards
    X, info = tm.complete_tensor(to_dev(c0.B), to_dev(c0.mask, torch.uint8), max_iter=3, tol=0.0,
                                 tau_schedule=c0.taus)
    assert info["status"] == 0 and np.isfinite(to_np(X)).all()


def test_complete_initial_iterate_formed_on_device(tm):
    # X omitted: the library starts from B on the observed set; the same as passing it
    announce("complete_init_observed")
    c0 = synth.completion_case(oracle.tprod_dct, 30, 26, 6, 3, 0.4, 5, 12)
    B = c0.B.copy()
    B[c0.mask == 0] = 7.0  # unobserved entries of B must not be read
    Xa, _ = tm.complete_tensor(to_dev(B), to_dev(c0.mask, torch.uint8), max_iter=5, tol=0.0, tau_schedule=c0.taus)
    Xb, _ = tm.complete_tensor(to_dev(B), to_dev(c0.mask, torch.uint8), X=to_dev(np.where(c0.mask != 0, B, 0.0)),
                               max_iter=5, tol=0.0, tau_schedule=c0.taus)
    assert torch.equal(Xa, Xb)
    Xo, _, _, _ = oracle.complete(c0.B, c0.mask, c0.betas)
    assert rel(to_np(Xa), Xo) <= FP64_TOL


def test_complete_beyond_history_ring(tm):
    # more iterations than the device's 4096 history slots, with the stopping
    # test every iteration: the relative change read back is the last one
    announce("complete_history_ring")
    c0 = synth.completion_case(oracle.tprod_dct, 6, 5, 2, 1, 0.5, 2, 13, tau0=1.0, tau1=0.5)
    taus = [1.0, 0.25] * 2050  # alternating thresholds: the iterates never settle
    args = (to_dev(c0.B), to_dev(c0.mask, torch.uint8))
    Xa, ia = tm.complete_tensor(*args, max_iter=4100, tol=1e-300, check_every=1, tau_schedule=taus)
    Xb, ib = tm.complete_tensor(*args, max_iter=4100, tol=1e-300, check_every=4100, tau_schedule=taus)
    assert ia["iters"] == ib["iters"] == 4100
    assert torch.equal(Xa, Xb)
    assert ia["rel_change"] == ib["rel_change"] and np.isfinite(ia["rel_change"]) and ia["rel_change"] > 0.0
