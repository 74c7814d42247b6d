"""GPU parity of the t-SVT hot path against the FP64 oracle (through the C-ABI).

FP64 bar: relative Frobenius error <= 1e-10 against the oracle on the same input.
"""
import numpy as np
import pytest

import oracle
import synth
from bounds import within
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def case(shape, r=3, noise=0.01, tau=None, seed=11):
    n1, n2, n3 = shape
    if tau is None:
        tau = 0.1 * (np.sqrt(n1) + np.sqrt(n2))
    return synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, r, noise, tau, seed)


SMALL = [(7, 5, 3), (5, 7, 4), (33, 17, 9), (17, 33, 2), (1, 6, 5), (6, 1, 5), (64, 64, 16), (100, 80, 7),
         (80, 100, 3), (130, 70, 5), (65, 64, 1), (2, 2, 2), (150, 150, 2)]


@pytest.mark.parametrize("shape", SMALL)
def test_tsvt_fp64_small(tm, shape):
    announce("tsvt_fp64_small", shape=shape)
    c = case(shape, r=max(1, min(shape[:2]) // 4))
    Y, ranks = tm.tsvt_dct(to_dev(c.Z), c.tau, return_ranks=True)
    Yo, ro, _ = oracle.tsvt_dct(c.Z, c.tau, return_ranks=True)
    err = rel(to_np(Y), Yo)
    assert err <= TOL64, err
    assert list(ranks) == [int(x) for x in ro]


def test_tsvt_fp64_config_small_case(tm):
    # 64 x 64 x 16, tubal rank 5 Gaussian factors + N(0, 0.01) noise, tau = 1.0
    announce("tsvt_fp64_64x64x16")
    c = synth.tsvt_case(oracle.tprod_dct, 64, 64, 16, 5, 0.01, 1.0, synth.SEED_BASE + 1)
    Y, ranks = tm.tsvt_dct(to_dev(c.Z), c.tau, return_ranks=True)
    Yo, ro, _ = oracle.tsvt_dct(c.Z, c.tau, return_ranks=True)
    assert rel(to_np(Y), Yo) <= TOL64
    assert list(ranks) == [int(x) for x in ro]


@pytest.mark.parametrize("shape", [(256, 256, 3), (200, 300, 2), (300, 170, 2), (512, 512, 1)])
def test_tsvt_fp64_team_kernel(tm, shape):
    # slices larger than one workgroup's LDS: block-pair team kernel
    announce("tsvt_fp64_team", shape=shape)
    c = case(shape, r=10)
    Y = tm.tsvt_dct(to_dev(c.Z), c.tau)
    Yo = oracle.tsvt_dct(c.Z, c.tau)
    assert rel(to_np(Y), Yo) <= TOL64


@pytest.mark.parametrize("team", [1, 2, 5])
def test_tsvt_fp64_team_sizes_agree(tm, team):
    announce("tsvt_team_sizes", team=team)
    c = case((256, 192, 2), r=8)
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_TEAM_SIZE, team)
    Y = tm.tsvt_dct(to_dev(c.Z), c.tau, ctx=ctx)
    Yo = oracle.tsvt_dct(c.Z, c.tau)
    assert rel(to_np(Y), Yo) <= TOL64
    ctx.close()


def test_tsvt_special_cases(tm):
    announce("tsvt_special")
    c = case((20, 12, 5))
    Z = to_dev(c.Z)
    assert rel(to_np(tm.tsvt_dct(Z, 0.0)), c.Z) <= 1e-12
    Y = tm.tsvt_dct(Z, 1e6)
    assert float(torch.abs(Y).max()) == 0.0


def test_tsvt_fp32(tm):
    announce("tsvt_fp32")
    c = case((48, 40, 8), r=5)
    Y = tm.tsvt_dct(to_dev(c.Z, torch.float32), c.tau)
    Yo = oracle.tsvt_dct(c.Z, c.tau)
    assert rel(to_np(Y), Yo) <= 1e-5


def test_tsvt_nonfinite_input_is_an_error(tm):
    announce("tsvt_nan")
    c = case((10, 8, 3))
    Z = c.Z.copy(order="F")
    Z[3, 2, 1] = np.nan
    with pytest.raises(tm.TsvdError) as ei:
        tm.tsvt_dct(to_dev(Z), c.tau)
    assert ei.value.code == tm.ENONFINITE


def test_tsvt_sweep_limit_warns(tm):
    announce("tsvt_sweep_limit")
    c = case((40, 30, 3), r=6)
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_MAX_SWEEPS, 1)
    rc = tm.lib.tsvt_dct(ctx.h, 0, 40, 30, 3, to_dev(c.Z).data_ptr(), to_dev(c.Z).data_ptr(), c.tau, None, None)
    torch.cuda.synchronize()
    assert rc == tm.WARN_NOCONV
    ctx.close()


def test_tsvt_invalid_arguments(tm):
    announce("tsvt_invalid")
    ctx = tm.default_context(0)
    Z = to_dev(np.zeros((4, 4, 2)))
    assert tm.lib.tsvt_dct(ctx.h, 0, 0, 4, 2, Z.data_ptr(), Z.data_ptr(), 1.0, None, None) == tm.EINVAL
    assert tm.lib.tsvt_dct(ctx.h, 0, 4, 4, 2, Z.data_ptr(), Z.data_ptr(), -1.0, None, None) == tm.EINVAL
    assert tm.lib.tsvt_dct(ctx.h, 7, 4, 4, 2, Z.data_ptr(), Z.data_ptr(), 1.0, None, None) == tm.EINVAL
    assert tm.lib.tsvt_dct(ctx.h, 0, 4, 4, 2, None, Z.data_ptr(), 1.0, None, None) == tm.EINVAL


def degenerate_tensor(kind, shape, seed):
    """Frontal slices all equal to one matrix M, so the transformed tensor has
    sqrt(n3) M as slice 0 and exact zeros elsewhere.  kind: 'zero' (M = 0),
    'repeated' (singular values 3, 3, 3, 1, 1, 1) or 'equal_columns' (every
    column of M the same vector: pairs of equal norm and cosine 1)."""
    n1, n2, n3 = shape
    g = synth.rng(seed)
    if kind == "zero":
        M = np.zeros((n1, n2))
    elif kind == "repeated":
        q1, _ = np.linalg.qr(synth.gaussian(g, (n1, 6)))
        q2, _ = np.linalg.qr(synth.gaussian(g, (n2, 6)))
        M = q1 @ np.diag([3.0, 3.0, 3.0, 1.0, 1.0, 1.0]) @ q2.T
    else:
        M = np.outer(synth.gaussian(g, (n1,)), np.ones(n2)) / np.sqrt(n2)
    return np.asfortranarray(np.repeat(M[:, :, None], n3, axis=2))


# resident slices and team slices; tau between the two repeated groups (scaled
# by sqrt(n3)), and below the single singular value of the equal-columns case
@pytest.mark.parametrize("shape", [(24, 16, 3), (260, 200, 2)])
@pytest.mark.parametrize("kind", ["zero", "repeated", "equal_columns"])
@pytest.mark.parametrize("prec", [0, 2])
def test_tsvt_degenerate_spectra(tm, shape, kind, prec):
    announce("tsvt_degenerate", shape=shape, kind=kind, prec=prec)
    Z = degenerate_tensor(kind, shape, 31 + shape[0])
    tau = 2.0 * np.sqrt(shape[2])
    Yo, ro, _ = oracle.tsvt_dct(Z, tau, return_ranks=True)
    dt = torch.float64 if prec == 0 else torch.float32
    Y, ranks = tm.tsvt_dct(to_dev(Z, dt), tau, prec=prec, return_ranks=True)
    Yg = to_np(Y)
    assert np.isfinite(Yg).all()
    assert list(ranks) == [int(x) for x in ro]
    if kind == "zero":
        assert float(np.abs(Yg).max()) == 0.0
    else:
        if prec == 0:
            assert rel(Yg, Yo) <= TOL64
        else:
            assert within(Yg, oracle.tsvt_dct(Z.astype(np.float32).astype(np.float64), tau),
                          Z.astype(np.float32).astype(np.float64), prec)


def test_team_kernel_ordinary_and_cooperative_launches_agree(tm):
    # the multi-workgroup Jacobi kernel: ordinary launches (default) and
    # cooperative ones give bitwise the same result
    announce("tsvt_launch_kinds")
    c = case((256, 256, 3), r=8, seed=5)
    Z = to_dev(c.Z)
    a = tm.Context(0)
    b = tm.Context(0)
    try:
        assert a.get_option(tm.OPT_COOPERATIVE) == 0
        b.set_option(tm.OPT_COOPERATIVE, 1)
        assert a.tile(tm.FP64, 256, 256, 3)["team"] == 1
        Ya = tm.tsvt_dct(Z, c.tau, ctx=a)
        Yb = tm.tsvt_dct(Z, c.tau, ctx=b)
        torch.cuda.synchronize()
        assert torch.equal(Ya, Yb)
        assert rel(to_np(Ya), oracle.tsvt_dct(c.Z, c.tau)) <= TOL64
    finally:
        a.close()
        b.close()
