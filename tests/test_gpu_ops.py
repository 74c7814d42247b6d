"""GPU parity of tprod_dct, tsvd_dct and complete_tensor against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def rnd(seed, *shape):
    return np.asfortranarray(np.random.default_rng(seed).standard_normal(shape))


@pytest.mark.parametrize("shape", [(4, 3, 5, 6), (33, 17, 9, 5), (64, 64, 64, 16), (7, 1, 3, 1), (100, 20, 70, 31)])
def test_tprod_fp64(tm, shape):
    n1, n2, n4, n3 = shape
    announce("tprod", shape=shape)
    X, Y = rnd(1, n1, n2, n3), rnd(2, n2, n4, n3)
    Z = tm.tprod_dct(to_dev(X), to_dev(Y))
    assert rel(to_np(Z), oracle.tprod_dct(X, Y)) <= 1e-12


# (130, 75, 90, 7): several 64-wide output tiles and 32-deep K chunks, each with a ragged tail
@pytest.mark.parametrize("shape", [(20, 10, 12, 8), (130, 75, 90, 7)])
def test_tprod_fp32(tm, shape):
    n1, n2, n4, n3 = shape
    announce("tprod_fp32", shape=shape)
    X, Y = rnd(3, n1, n2, n3), rnd(4, n2, n4, n3)
    Z = tm.tprod_dct(to_dev(X, torch.float32), to_dev(Y, torch.float32))
    assert rel(to_np(Z), oracle.tprod_dct(X, Y)) <= 1e-5


@pytest.mark.parametrize("shape", [(12, 8, 5), (8, 12, 4), (64, 64, 16), (200, 150, 3), (96, 300, 2)])
def test_tsvd_fp64(tm, shape):
    announce("tsvd", shape=shape)
    X = rnd(5, *shape)
    U, S, V = tm.tsvd_dct(to_dev(X), transform_domain=True)
    Uo, So, Vo, _ = oracle.tsvd_dct(X)
    assert rel(to_np(S)[:, :], So) <= 1e-12
    # singular vectors are unique up to the sign convention when the gaps are clear
    assert rel(to_np(U), Uo) <= 1e-9
    assert rel(to_np(V), Vo) <= 1e-9


def test_tsvd_spatial_reconstruction(tm):
    announce("tsvd_spatial")
    n1, n2, n3 = 20, 14, 6
    X = rnd(6, n1, n2, n3)
    U, S, V = tm.tsvd_dct(to_dev(X))
    p = min(n1, n2)
    Sd = torch.zeros((p, p, n3), dtype=torch.float64, device="cuda:0")
    for k in range(n3):
        Sd[:, :, k] = torch.diag(S[:, k])
    Vt = V.permute(1, 0, 2)
    R = tm.tprod_dct(tm.tprod_dct(U, Sd), Vt)
    assert rel(to_np(R), X) <= 1e-12


def small_case(L=30, shape=(20, 18, 6), r=2, sr=0.6, seed=80):
    return synth.completion_case(oracle.tprod_dct, *shape, r, sr, L, seed, tau0=1.0, tau1=0.01)


# warm start of the Jacobi SVDs: automatic period, cold starts, and a reset every
# other iteration (exercises the reset inside the captured iteration)
WARM = [-1, 0, 2]


@pytest.mark.parametrize("warm", WARM)
def test_complete_fp64_matches_oracle(tm, warm):
    announce("complete_fp64", warm=warm)
    cc = small_case()
    Xo, Mo, it, _ = oracle.complete(cc.B, cc.mask, cc.betas, cc.taus)
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_WARM_START, warm)
    X, info, M = tm.complete_tensor(to_dev(cc.B), to_dev(cc.mask, torch.uint8), max_iter=len(cc.taus), tol=0.0,
                                    tau_schedule=cc.taus, return_M=True, ctx=ctx)
    ctx.close()
    assert info["iters"] == it
    assert rel(to_np(X), Xo) <= 1e-10
    assert rel(to_np(M), Mo) <= 1e-10
    obs = cc.mask != 0
    assert np.array_equal(to_np(X)[obs], cc.B[obs])


@pytest.mark.parametrize("warm", WARM)
@pytest.mark.parametrize("shape", [(180, 160, 3), (150, 280, 2)])
def test_complete_fp64_team_shape_matches_oracle(tm, warm, shape):
    announce("complete_fp64_team", warm=warm, shape=shape)
    cc = small_case(L=6, shape=shape, r=4, sr=0.5)
    Xo, _, _, _ = oracle.complete(cc.B, cc.mask, cc.betas, cc.taus)
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_WARM_START, warm)
    X, info = tm.complete_tensor(to_dev(cc.B), to_dev(cc.mask, torch.uint8), max_iter=6, tol=0.0,
                                 tau_schedule=cc.taus, ctx=ctx)
    ctx.close()
    assert rel(to_np(X), Xo) <= 1e-10


def test_complete_warm_start_needs_fewer_sweeps(tm):
    # same iterates to rounding; the warm-started SVDs take fewer sweeps
    announce("complete_warm_sweeps")
    cc = small_case(L=12, shape=(120, 100, 4), r=3, sr=0.5)
    out = {}
    for warm in (0, -1):
        ctx = tm.Context(0)
        ctx.set_option(tm.OPT_WARM_START, warm)
        ctx.stats(reset=True)
        X, _ = tm.complete_tensor(to_dev(cc.B), to_dev(cc.mask, torch.uint8), max_iter=12, tol=0.0,
                                  tau_schedule=cc.taus, ctx=ctx)
        out[warm] = (to_np(X), ctx.stats(reset=True)["slice_sweeps"])
        ctx.close()
    print("slice sweeps cold %d warm %d" % (out[0][1], out[-1][1]))
    assert rel(out[-1][0], out[0][0]) <= 1e-12
    assert out[-1][1] < 0.8 * out[0][1]


def test_complete_resume(tm):
    announce("complete_resume")
    cc = small_case(L=10)
    B, mk = to_dev(cc.B), to_dev(cc.mask, torch.uint8)
    X, _ = tm.complete_tensor(B, mk, max_iter=10, tol=0.0, tau_schedule=cc.taus)
    X1, _, M1 = tm.complete_tensor(B, mk, max_iter=5, tol=0.0, tau_schedule=cc.taus, return_M=True)
    X2, _ = tm.complete_tensor(B, mk, X=X1, M_init=M1, max_iter=5, start_iter=5, tol=0.0, tau_schedule=cc.taus)
    assert rel(to_np(X2), to_np(X)) <= 1e-13


def test_complete_tolerance_stop(tm):
    announce("complete_tol")
    cc = small_case(L=200)
    X, info = tm.complete_tensor(to_dev(cc.B), to_dev(cc.mask, torch.uint8), max_iter=200, tol=1e-6, beta=10.0,
                                 check_every=1)
    assert info["iters"] < 200 and info["rel_change"] <= 1e-6
    Xo, _, it, _ = oracle.complete(cc.B, cc.mask, np.full(200, 10.0), tol=1e-6)
    assert info["iters"] == it
    assert rel(to_np(X), Xo) <= 1e-10


@pytest.mark.parametrize("shape", [(20, 18, 6), (260, 200, 3)])
def test_complete_graph_replays_match_direct_launches(tm, shape):
    # The captured iteration is replayed L times with a host synchronization
    # between replays (check_every = 1); every L must give the same bits as
    # direct launches of the same kernels.
    announce("complete_graph", shape=shape)
    cc = small_case(L=5, shape=shape, r=3, sr=0.5)
    B, mk = to_dev(cc.B), to_dev(cc.mask, torch.uint8)
    for L in (1, 2, 3, 5):
        outs = []
        for graphs in (1, 0):
            ctx = tm.Context(0)
            ctx.set_option(tm.OPT_GRAPHS, graphs)
            X, info, M = tm.complete_tensor(B, mk, max_iter=L, tol=1e-300, check_every=1, tau_schedule=cc.taus,
                                            return_M=True, ctx=ctx)
            torch.cuda.synchronize()
            outs.append((to_np(X), to_np(M), info["iters"]))
            ctx.close()
        assert outs[0][2] == outs[1][2] == L
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_profile_levels(tm):
    # level 1 times every phase, level 2 the Jacobi launches only; results are unchanged
    announce("profile_levels")
    cc = small_case(L=4)
    B, mk = to_dev(cc.B), to_dev(cc.mask, torch.uint8)
    out = {}
    for level in (0, 1, 2):
        ctx = tm.Context(0)
        ctx.set_option(tm.OPT_PROFILE, level)
        ctx.stats(reset=True)
        X, _ = tm.complete_tensor(B, mk, max_iter=4, tol=0.0, tau_schedule=cc.taus, ctx=ctx)
        st = ctx.stats(reset=True)
        out[level] = to_np(X)
        if level == 0:
            assert all(v == 0 for v in st["launches"].values())
        elif level == 1:
            assert st["launches"]["jacobi"] == 4 and st["launches"]["forward_transform"] == 4
        else:
            assert st["launches"]["jacobi"] == 4 and st["launches"]["forward_transform"] == 0
            assert st["ms"]["jacobi"] > 0.0
        ctx.close()
    assert rel(out[1], out[0]) <= 1e-13 and rel(out[2], out[0]) <= 1e-13
    ctx = tm.Context(0)
    with pytest.raises(tm.TsvdError):
        ctx.set_option(tm.OPT_PROFILE, 3)
    ctx.close()
