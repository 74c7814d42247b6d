"""Kept-column Jacobi with the threshold certificate (TSVD_OPT_KEPT_COLUMNS).

A t-SVT (Theorem 5) needs only the singular values above tau and their
vectors.  In this mode the multi-workgroup Jacobi kernel evaluates only the
column pairs that touch a column of norm > tau; each slice is then certified
(the kept columns orthogonal to all others, the remaining columns of spectral
norm <= tau) or sent through the full iteration; a slice that shows a
remaining column near tau (no gap below it) turns into the full iteration at
once.  Checked through the C-ABI against the FP64 oracle and against the full
iteration:
  * several shapes (tall and wide slices) on the multi-workgroup kernel in the
    three precisions, with tau twice the noise's largest singular value (a gap
    below tau): values within the bar, ranks exact, the mode in use and every
    slice certified;
  * tau at the noise's largest singular value (no gap): the slices turn into
    the full iteration, which must give the oracle's result;
  * a slice whose columns are all below tau while its spectral norm is 3 tau:
    the mode never rotates it, so the certificate must reject it and the full
    iteration must follow;
  * slices with nothing above tau (rank 0);
  * the mode against the full iteration on the same input.
"""
import numpy as np
import pytest

import oracle
import synth
from bounds import C_PATH, FP64_TOL, ratio
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def team_ctx(tm, W, kept=1):
    ctx = tm.Context(0)
    ctx.set_option(tm.OPT_TEAM_SIZE, W)
    ctx.set_option(tm.OPT_GROUP_COLUMNS, 1)
    ctx.set_option(tm.OPT_KEPT_COLUMNS, kept)
    return ctx


def case(shape, seed, r=4, gap=True):
    # rank-r signal (singular values ~ sqrt(n1 n2)) plus N(0, 0.01) noise, whose
    # largest singular value is about 0.1 (sqrt(n1) + sqrt(n2)); tau twice that
    # (gap) or equal to it
    n1, n2, n3 = shape
    tau = (0.2 if gap else 0.1) * (np.sqrt(n1) + np.sqrt(n2))
    return synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, r, 0.01, tau, seed)


# slices too large for one workgroup's LDS, so that the multi-workgroup kernel runs them
SHAPES = [((200, 150, 3), 4), ((150, 200, 4), 2), ((256, 256, 3), 8), ((180, 140, 5), 3)]
SHAPES_F32 = [((200, 150, 3), 4), ((256, 200, 3), 4), ((200, 256, 2), 2)]


@pytest.mark.parametrize("shape,W", SHAPES)
def test_kept_columns_fp64(tm, shape, W):
    announce("kept_fp64", shape=shape, W=W)
    c = case(shape, 70)
    ctx = team_ctx(tm, W)
    try:
        ctx.stats(reset=True)
        Y, ranks = tm.tsvt_dct(to_dev(c.Z), c.tau, return_ranks=True, ctx=ctx)
        st = ctx.stats(reset=True)
    finally:
        ctx.close()
    Yo, ro, _ = oracle.tsvt_dct(c.Z, c.tau, return_ranks=True)
    err = rel(to_np(Y), Yo)
    print("kept FP64 %s W %d: rel err %.3e, ranks %s, pairs %d, fallback %d, sweeps %d" % (
        shape, W, err, list(ranks), st["pairs"], st["fallback_slices"], st["slice_sweeps"]))
    assert list(ranks) == [int(x) for x in ro]
    assert err <= FP64_TOL
    assert st["pairs"] > 0
    assert st["fallback_slices"] == 0


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("shape,W", SHAPES_F32)
def test_kept_columns_reduced(tm, shape, W, prec):
    announce("kept_reduced", shape=shape, W=W, prec=prec)
    c = case(shape, 71)
    Zf = c.Z.astype(np.float32).astype(np.float64)
    ctx = team_ctx(tm, W)
    try:
        ctx.stats(reset=True)
        Y, ranks = tm.tsvt_dct(to_dev(Zf, torch.float32), c.tau, prec=prec, return_ranks=True, ctx=ctx)
        st = ctx.stats(reset=True)
    finally:
        ctx.close()
    Yo, ro, _ = oracle.tsvt_dct(Zf, c.tau, return_ranks=True)
    cr = ratio(to_np(Y), Yo, Zf, prec)
    print("kept prec %d %s: c = %.3f, pairs %d, fallback %d" % (prec, shape, cr, st["pairs"], st["fallback_slices"]))
    assert list(ranks) == [int(x) for x in ro]
    assert cr <= C_PATH[prec]
    assert st["pairs"] > 0
    assert st["fallback_slices"] == 0


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_kept_columns_noise_edge(tm, prec):
    announce("kept_edge", prec=prec)
    c = case((200, 150, 4), 75, gap=False)
    Z = c.Z if prec == 0 else c.Z.astype(np.float32).astype(np.float64)
    ctx = team_ctx(tm, 4)
    try:
        ctx.stats(reset=True)
        Y, ranks = tm.tsvt_dct(to_dev(Z, torch.float32 if prec else torch.float64), c.tau, prec=prec,
                               return_ranks=True, ctx=ctx)
        st = ctx.stats(reset=True)
    finally:
        ctx.close()
    Yo, ro, _ = oracle.tsvt_dct(Z, c.tau, return_ranks=True)
    print("noise edge prec %d: ranks %s, fallback %d, sweeps %d, pairs %d" % (
        prec, list(ranks), st["fallback_slices"], st["slice_sweeps"], st["pairs"]))
    assert list(ranks) == [int(x) for x in ro]
    if prec == 0:
        assert rel(to_np(Y), Yo) <= FP64_TOL
    else:
        assert ratio(to_np(Y), Yo, Z, prec) <= C_PATH[prec]


def hidden_norm_tensor(n1, n2, n3, tau, seed):
    # transform-domain slices: slice 1 is 3 tau u v^T with v spread evenly over
    # the columns (every column has norm 3 tau / sqrt(n2) < tau) plus a little
    # noise; the others are small noise.  Back to the spatial domain by the
    # inverse DCT along the tubes.
    g = np.random.default_rng(seed)
    Zb = 1e-3 * tau * g.standard_normal((n1, n2, n3))
    u = g.standard_normal(n1)
    u /= np.linalg.norm(u)
    v = np.ones(n2) / np.sqrt(n2)
    Zb[:, :, 1] += 3.0 * tau * np.outer(u, v)
    return np.asfortranarray(oracle.idct_tubes(Zb))


@pytest.mark.parametrize("prec", [0, 2])
def test_kept_columns_hidden_norm(tm, prec):
    announce("kept_hidden", prec=prec)
    n1, n2, n3, tau = 200, 160, 4, 1.0
    Z = hidden_norm_tensor(n1, n2, n3, tau, 72)
    if prec:
        Z = Z.astype(np.float32).astype(np.float64)
    ctx = team_ctx(tm, 2)
    try:
        ctx.stats(reset=True)
        Y, ranks = tm.tsvt_dct(to_dev(Z, torch.float32 if prec else torch.float64), tau, prec=prec,
                               return_ranks=True, ctx=ctx)
        st = ctx.stats(reset=True)
    finally:
        ctx.close()
    Yo, ro, _ = oracle.tsvt_dct(Z, tau, return_ranks=True)
    print("hidden norm prec %d: ranks %s (oracle %s), fallback %d" % (prec, list(ranks), list(ro), st["fallback_slices"]))
    assert list(ranks) == [int(x) for x in ro]
    assert ro[1] == 1
    assert st["fallback_slices"] >= 1
    if prec == 0:
        assert rel(to_np(Y), Yo) <= FP64_TOL
    else:
        assert ratio(to_np(Y), Yo, Z, prec) <= C_PATH[prec]


@pytest.mark.parametrize("factor", [1.5, 1.01])
def test_kept_columns_rank_zero(tm, factor):
    # tau above every singular value: no column is ever above it, so the
    # iteration stops at once and the certificate alone decides.  At 1.5 sigma_1
    # its bound holds; at 1.01 sigma_1 it cannot tell, and the full iteration
    # must give the same (zero) result.
    announce("kept_rank0", factor=factor)
    c = case((200, 150, 5), 73)
    s1 = max(np.linalg.norm(oracle.dct_tubes(c.Z)[:, :, k], 2) for k in range(5))
    tau = factor * s1
    ctx = team_ctx(tm, 2)
    try:
        ctx.stats(reset=True)
        Y, ranks = tm.tsvt_dct(to_dev(c.Z), tau, return_ranks=True, ctx=ctx)
        st = ctx.stats(reset=True)
    finally:
        ctx.close()
    print("rank 0 at %.2f sigma_1: fallback %d, sweeps %d" % (factor, st["fallback_slices"], st["slice_sweeps"]))
    assert list(ranks) == [0] * 5
    assert float(torch.abs(Y).max()) == 0.0
    if factor > 1.2:
        assert st["fallback_slices"] == 0


@pytest.mark.parametrize("prec", [0, 2])
def test_kept_columns_against_full_iteration(tm, prec):
    announce("kept_vs_full", prec=prec)
    c = case((240, 200, 6), 74)
    Z = to_dev(c.Z) if prec == 0 else to_dev(c.Z.astype(np.float32), torch.float32)
    out = {}
    for kept in (1, 0):
        ctx = team_ctx(tm, 4, kept)
        try:
            ctx.stats(reset=True)
            Y, ranks = tm.tsvt_dct(Z, c.tau, prec=prec, return_ranks=True, ctx=ctx)
            out[kept] = (to_np(Y), list(ranks), ctx.stats(reset=True))
        finally:
            ctx.close()
    print("kept vs full prec %d: sweeps %d vs %d, pairs %d, fallback %d" % (
        prec, out[1][2]["slice_sweeps"], out[0][2]["slice_sweeps"], out[1][2]["pairs"],
        out[1][2]["fallback_slices"]))
    assert out[1][1] == out[0][1]
    assert out[0][2]["pairs"] == 0
    assert out[1][2]["fallback_slices"] == 0
    assert out[1][2]["slice_sweeps"] < out[0][2]["slice_sweeps"]
    Zn = c.Z if prec == 0 else c.Z.astype(np.float32).astype(np.float64)
    if prec == 0:
        assert rel(out[1][0], out[0][0]) <= FP64_TOL
    else:
        assert ratio(out[1][0], out[0][0], Zn, prec) <= 2 * C_PATH[prec]


def test_kept_columns_transform(tm):
    # the t-SVT under a caller-given orthogonal transform along the tubes
    announce("kept_transform")
    n1, n2, n3 = 200, 150, 4
    c = case((n1, n2, n3), 76)
    L, _ = np.linalg.qr(np.random.default_rng(77).standard_normal((n3, n3)))
    ctx = team_ctx(tm, 4)
    try:
        ctx.stats(reset=True)
        Y, ranks = tm.tsvt_transform(to_dev(c.Z), c.tau, L, return_ranks=True, ctx=ctx)
        st = ctx.stats(reset=True)
    finally:
        ctx.close()
    Yo, ro, _ = oracle.tsvt_transform(c.Z, c.tau, L, return_ranks=True)
    err = rel(to_np(Y), Yo)
    print("kept transform: rel err %.3e, ranks %s, pairs %d, fallback %d" % (err, list(ranks), st["pairs"],
                                                                           st["fallback_slices"]))
    assert list(ranks) == [int(x) for x in ro]
    assert err <= FP64_TOL
    assert st["pairs"] > 0
    assert st["fallback_slices"] == 0


@pytest.mark.parametrize("prec", [0, 2])
def test_kept_columns_dft(tm, prec):
    # the Fourier path: complex slices thresholded through their 2 n1 x 2 n2 real
    # forms (every singular value twice), real slices as they are; its slices
    # carry sqrt(n3) times the orthonormal transform's scale
    announce("kept_dft", prec=prec)
    n1, n2, n3 = 120, 100, 5
    c = case((n1, n2, n3), 78)
    tau = c.tau * np.sqrt(n3)
    Z = c.Z if prec == 0 else c.Z.astype(np.float32).astype(np.float64)
    ctx = team_ctx(tm, 4)
    try:
        ctx.stats(reset=True)
        Y, ranks = tm.tsvt_dft(to_dev(Z, torch.float32 if prec else torch.float64), tau, prec=prec,
                               return_ranks=True, ctx=ctx)
        st = ctx.stats(reset=True)
    finally:
        ctx.close()
    Yo, ro, _ = oracle.tsvt_dft(Z, tau, return_ranks=True)
    print("kept dft prec %d: ranks %s (oracle %s), pairs %d, fallback %d" % (
        prec, list(ranks), [int(x) for x in ro], st["pairs"], st["fallback_slices"]))
    assert list(ranks) == [int(x) for x in ro]
    assert st["pairs"] > 0
    assert st["fallback_slices"] == 0
    if prec == 0:
        assert rel(to_np(Y), Yo) <= FP64_TOL
    else:
        assert ratio(to_np(Y), Yo, Z, prec) <= 2 * C_PATH[prec]


def test_kept_columns_graph_replays(tm):
    # a kept-column t-SVT captured in a HIP graph (the library's workspace and
    # tile already set up by an eager call): every replay, with other eager
    # work on the same workspace between replays, gives the eager result bitwise
    announce("kept_graph")
    n1, n2, n3 = 200, 150, 4
    c = case((n1, n2, n3), 79)
    ctx = team_ctx(tm, 4)
    ctx.set_option(tm.OPT_SYNC_STATUS, 0)  # no host synchronization inside the capture
    try:
        Z, Z2 = to_dev(c.Z), to_dev(2.0 * c.Z)
        Y, Y2 = tm.empty_f(n1, n2, n3, torch.float64, "cuda:0"), tm.empty_f(n1, n2, n3, torch.float64, "cuda:0")
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            tm.tsvt_dct(Z, c.tau, Y=Y, ctx=ctx, stream=s)
        torch.cuda.synchronize()
        ref = Y.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
            tm.tsvt_dct(Z, c.tau, Y=Y, ctx=ctx, stream=s)
        torch.cuda.synchronize()
        for rep in range(3):
            tm.tsvt_dct(Z2, c.tau, Y=Y2, ctx=ctx)  # eager work on the same workspace
            Y.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(Y, ref), "replay %d differs from the eager result" % rep
        status, _ = ctx.sync_status()
        st = ctx.stats(reset=True)
    finally:
        ctx.close()
    assert status == 0
    assert st["pairs"] > 0
    assert rel(to_np(ref), oracle.tsvt_dct(c.Z, c.tau)) <= FP64_TOL


@pytest.mark.parametrize("prec", [0, 2])
def test_kept_columns_nonfinite_input(tm, prec):
    # a NaN in a slice that the kept-column mode would take: every sweep limit
    # still ends the iteration, the certificate rejects the slice, and the call
    # reports the input as non-finite
    announce("kept_nan", prec=prec)
    c = case((200, 150, 4), 80)
    Z = c.Z.copy()
    Z[17, 33, 2] = np.nan
    ctx = team_ctx(tm, 4)
    try:
        with pytest.raises(tm.TsvdError) as ei:
            tm.tsvt_dct(to_dev(Z, torch.float32 if prec else torch.float64), c.tau, prec=prec, ctx=ctx)
        assert ei.value.code == tm.ENONFINITE
        # the context stays usable
        Y = tm.tsvt_dct(to_dev(c.Z), c.tau, ctx=ctx)
    finally:
        ctx.close()
    assert rel(to_np(Y), oracle.tsvt_dct(c.Z, c.tau)) <= FP64_TOL


def test_kept_columns_completion_mixed(tm):
    # the MIXED completion with cold SVDs (no warm start) in the kept-column
    # mode, whose thresholds come from the device-side schedule: the oracle's
    # iterates within the per-iteration bound, the mode in use, and a replayed
    # graph giving the direct launches' result bitwise
    from bounds import U_EFF, oracle_iterates

    announce("kept_completion")
    L = 8
    cc = synth.completion_case(oracle.tprod_dct, 200, 150, 6, 4, 0.5, L, 92, tau0=1.0, tau1=0.01)
    Bf = cc.B.astype(np.float32).astype(np.float64)
    Xo, _, zmax = oracle_iterates(Bf, cc.mask, cc.taus, L)
    outs = []
    for graphs in (1, 0):
        ctx = team_ctx(tm, 4)
        ctx.set_option(tm.OPT_GRAPHS, graphs)
        ctx.set_option(tm.OPT_WARM_START, 0)
        try:
            ctx.stats(reset=True)
            X, info = tm.complete_tensor(to_dev(Bf, torch.float32), to_dev(cc.mask, torch.uint8), max_iter=L,
                                         tol=0.0, tau_schedule=cc.taus, prec=tm.MIXED, ctx=ctx)
            st = ctx.stats(reset=True)
        finally:
            ctx.close()
        assert info["status"] == 0
        assert st["pairs"] > 0
        outs.append(to_np(X))
    assert np.array_equal(outs[0], outs[1])
    cr = np.linalg.norm(outs[0] - Xo) / (U_EFF[2] * zmax)
    print("kept completion MIXED: c per iteration %.3f, pairs %d, fallback %d" % (cr / L, st["pairs"],
                                                                                 st["fallback_slices"]))
    assert cr <= L * C_PATH[2]
