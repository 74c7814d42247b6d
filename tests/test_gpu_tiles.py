"""Jacobi tiles: every tile the tuner may pick gives the oracle's result, and the
tuned choice is stable within a process."""
import numpy as np
import pytest

import oracle
import synth
from bounds import FP64_TOL, oracle_iterates, ratio, within, within_completion
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def case(shape, seed):
    n1, n2, n3 = shape
    return synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, max(1, min(n1, n2) // 10), 0.01,
                           0.1 * (np.sqrt(n1) + np.sqrt(n2)), seed)


# (shape, group widths, team sizes, group columns): resident slices, team
# slices with both group widths and one or two columns per group, a wide
# tensor whose 300-row slices need 32-lane groups, and large teams
FORCED = [
    ((64, 48, 9), (16, 32), (0,), (1,)),
    ((256, 200, 3), (16, 32), (1, 2, 3, 4), (1, 2)),
    ((130, 300, 2), (32,), (1, 2, 4), (1, 2)),
    ((257, 190, 2), (32,), (1, 3, 8), (2,)),
    # teams of 12 and 16 workgroups: 4-column blocks, 32 of them, handed over point to point
    ((300, 128, 2), (32,), (12, 16), (1,)),
    # one column pair per wavefront (64-lane groups, up to 1024 threads)
    ((256, 200, 3), (64,), (2, 4, 8), (1,)),
    ((300, 128, 2), (64,), (3, 16), (1,)),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape,widths,teams,cols", FORCED)
def test_forced_tiles_match_oracle(tm, shape, widths, teams, cols, prec):
    c = case(shape, 700 + shape[0])
    dt = torch.float64 if prec == 0 else torch.float32
    Zh = c.Z if prec == 0 else c.Z.astype(np.float32).astype(np.float64)
    want = oracle.tsvt_dct(Zh, c.tau)
    Z = to_dev(Zh, dt)
    for G in widths:
        for W in teams:
            for K in cols:
                announce("forced_tile", shape=shape, G=G, W=W, K=K, prec=prec)
                ctx = tm.Context(0)
                ctx.set_option(tm.OPT_GROUP_LANES, G)
                ctx.set_option(tm.OPT_TEAM_SIZE, W)
                ctx.set_option(tm.OPT_GROUP_COLUMNS, K)
                t = ctx.tile(prec, *shape)
                assert t["source"] == 2 and t["G"] == G
                assert t["K"] == (K if t["team"] else 0)
                Y = tm.tsvt_dct(Z, c.tau, prec=prec, ctx=ctx)
                err = rel(to_np(Y), want)
                print("shape %s prec %d G %d W %d K %d tile %s rel err %.2e" % (shape, prec, G, W, K, t, err))
                if prec == 0:
                    assert err <= FP64_TOL
                else:
                    assert within(to_np(Y), want, Zh, prec), ratio(to_np(Y), want, Zh, prec)
                ctx.close()


@pytest.mark.parametrize("shape", [(64, 48, 9), (256, 200, 3), (200, 256, 5)])
@pytest.mark.parametrize("prec", [0, 1])
def test_tuned_tile_matches_oracle_and_is_stable(tm, shape, prec):
    announce("tuned_tile", shape=shape, prec=prec)
    c = case(shape, 720 + shape[2])
    ctx1, ctx2 = tm.Context(0), tm.Context(0)
    t1 = ctx1.tile(prec, *shape)
    t2 = ctx2.tile(prec, *shape)
    print("tuned tile", shape, prec, t1)
    assert t1 == t2 and t1["source"] in (0, 1)
    dt = torch.float64 if prec == 0 else torch.float32
    Zf = c.Z if prec == 0 else c.Z.astype(np.float32).astype(np.float64)
    Y = tm.tsvt_dct(to_dev(Zf, dt), c.tau, prec=prec, ctx=ctx1)
    want = oracle.tsvt_dct(Zf, c.tau)
    if prec == 0:
        assert rel(to_np(Y), want) <= FP64_TOL
    else:
        assert within(to_np(Y), want, Zf, prec), ratio(to_np(Y), want, Zf, prec)
    ctx1.close()
    ctx2.close()


def test_batched_tiles_are_per_shape(tm):
    # the batched tile of a shape is the same whichever context or batch asks
    announce("batched_tiles")
    ctx = tm.Context(0)
    shapes = [(100, 90, 7), (256, 256, 3), (300, 40, 4)]
    tiles = [ctx.tile(1, *s, batched=True) for s in shapes]
    ctx2 = tm.Context(0)
    assert tiles == [ctx2.tile(1, *s, batched=True) for s in shapes]
    for t in tiles:
        assert t["threads"] == 512
    ctx.close()
    ctx2.close()


def test_team_residency_with_six_wavefront_workgroups(tm):
    # 200 x 144 x 48 FP32 completion (V carried), forced 32-lane groups and teams
    # of 6: 12-column blocks give 384-thread workgroups (6 wavefronts) whose
    # registers allow one workgroup per CU, although the occupancy query allows
    # two.  The launch must size the grid so that every team member is resident
    # (otherwise a team waits until its bounded spin gives up).
    announce("team_residency", shape=(200, 144, 48))
    cc = synth.completion_case(oracle.tprod_dct, 200, 144, 48, 4, 0.5, 2, 812, tau0=1.0, tau1=0.5)
    Bf = cc.B.astype(np.float32).astype(np.float64)
    Xo, _, zmax = oracle_iterates(Bf, cc.mask, cc.taus, 2)
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_GROUP_LANES, 32)
    ctx.set_option(tm.OPT_TEAM_SIZE, 6)
    t = ctx.tile(1, 200, 144, 48, with_v=True)
    assert t["threads"] == 384 and t["W"] == 6
    X, info = tm.complete_tensor(to_dev(Bf, torch.float32), to_dev(cc.mask, torch.uint8), max_iter=2, tol=0.0,
                                 tau_schedule=cc.taus, prec=1, ctx=ctx)
    ctx.close()
    assert info["status"] == 0
    assert within_completion(to_np(X), Xo, zmax, 1, 2)


@pytest.mark.parametrize("slots,W", [(1, 8), (3, 16), (2, 4)])
def test_team_slots_forced_completion_fp64(tm, slots, W):
    # fewer slices in flight per XCD than the tensor has slices per XCD: teams
    # take several slices in turn (the tuner's L2-fitting candidates).  FP64
    # completion with V at 256 x 256 x 31 against the oracle's iterates.
    announce("team_slots", slots=slots, W=W)
    cc = synth.completion_case(oracle.tprod_dct, 256, 256, 31, 10, 0.3, 3, synth.SEED_BASE + 2)
    oracle.set_threads(min(16, oracle.host_threads()))
    Xo, _, _ = oracle_iterates(cc.B, cc.mask, cc.taus, 3)
    ctx = tm.Context(0)
    try:
        ctx.set_option(tm.OPT_TEAM_SLOTS, slots)
        ctx.set_option(tm.OPT_TEAM_SIZE, W)
        assert ctx.get_option(tm.OPT_TEAM_SLOTS) == slots
        t = ctx.tile(0, 256, 256, 31, with_v=True)
        assert t["team"] == 1 and t["source"] == 2
        X, info = tm.complete_tensor(to_dev(cc.B), to_dev(cc.mask, torch.uint8), max_iter=3, tol=0.0,
                                     tau_schedule=cc.taus, ctx=ctx)
    finally:
        ctx.close()
    assert info["status"] == 0
    err = rel(to_np(X), Xo)
    print("slots %d W %d: rel err %.3e" % (slots, W, err))
    assert err <= FP64_TOL
