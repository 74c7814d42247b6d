"""Serving loop: continuous batching, admission by device-memory footprint,
results independent of the mix."""
import time

import numpy as np
import pytest

import oracle
import synth
from bounds import C_PATH, oracle_iterates, ratio, within_completion
from gpu_util import announce, need_gpu, rel, to_dev, to_np, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tm():
    need_gpu()
    import paper_1902_03070_amd as tm

    return tm


def wait_all(srv, ids, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(ids):
        for i in ids:
            if i not in out:
                r = srv.poll(i)
                if r is not None:
                    out[i] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.002)
    return out


def requests(seed=0, n=6):
    shapes = [(40, 30, 5), (64, 64, 8), (130, 90, 4), (260, 200, 3), (50, 70, 6), (300, 280, 2)][:n]
    reqs = []
    for i, (n1, n2, n3) in enumerate(shapes):
        if i % 2 == 0:
            c = synth.tsvt_case(oracle.tprod_dct, n1, n2, n3, max(1, min(n1, n2) // 10), 0.01,
                                0.1 * (np.sqrt(n1) + np.sqrt(n2)), seed + i)
            reqs.append(("tsvt", c.Z.astype(np.float32), c.tau))
        else:
            cc = synth.completion_case(oracle.tprod_dct, n1, n2, n3, 3, 0.3, 6, seed + i, tau0=2.0, tau1=0.1)
            reqs.append(("complete", cc.B.astype(np.float32), cc.mask, cc))
    return reqs


def submit(srv, r):
    if r[0] == "tsvt":
        return srv.submit_tsvt(r[1], r[2])
    return srv.submit_complete(r[1], r[2], 6, 2.0, 0.1)


def test_serving_mix_equals_alone(tm):
    announce("serving_mix_vs_alone")
    reqs = requests()
    alone = []
    for r in reqs:
        srv = tm.Server(budget_bytes=4 << 30, max_active=8)
        rid = submit(srv, r)
        alone.append(wait_all(srv, [rid])[rid][0])
        srv.close()
    srv = tm.Server(budget_bytes=4 << 30, max_active=8)
    ids = [submit(srv, r) for r in reqs]
    mixed = wait_all(srv, ids)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs)
    for k, rid in enumerate(ids):
        assert np.array_equal(mixed[rid][0], alone[k]), k


def test_serving_results_match_oracle(tm):
    announce("serving_vs_oracle")
    reqs = requests(seed=10, n=4)
    srv = tm.Server(budget_bytes=4 << 30, max_active=8)
    ids = [submit(srv, r) for r in reqs]
    got = wait_all(srv, ids)
    srv.close()
    for r, rid in zip(reqs, ids):
        Y = got[rid][0].astype(np.float64)
        Zf = r[1].astype(np.float64)
        if r[0] == "tsvt":
            want = oracle.tsvt_dct(Zf, r[2])
            assert ratio(Y, want, Zf, 1) <= C_PATH[1], r[0]
        else:
            cc = r[3]
            want, _, zmax = oracle_iterates(Zf, r[2], cc.taus, 6)
            assert within_completion(Y, want, zmax, 1, 6), r[0]


def test_serving_admission_budget(tm):
    announce("serving_admission")
    reqs = requests(seed=20, n=4)
    srv = tm.Server(budget_bytes=1 << 20, max_active=8)
    with pytest.raises(tm.TsvdError) as ei:
        srv.submit_tsvt(reqs[3][1], 1.0)  # 260 x 200 x 3 cannot fit 1 MiB
    assert ei.value.code == tm.EBUSY
    srv.close()
    # a budget that holds one request at a time still serves them all, in order
    big = 12 << 20
    srv = tm.Server(budget_bytes=big, max_active=8)
    ids = [submit(srv, r) for r in reqs[:3]]
    got = wait_all(srv, ids)
    st = srv.stats()
    srv.close()
    assert st["peak_bytes"] <= big
    t_admit = [got[i][1][1] for i in ids]
    assert t_admit == sorted(t_admit)


def test_serving_poisson_arrivals(tm):
    announce("serving_poisson")
    g = np.random.default_rng(5)
    arrivals = synth.poisson_arrivals(g, 200.0, 12)
    reqs = requests(seed=30) * 2
    srv = tm.Server(budget_bytes=4 << 30, max_active=4)
    t0 = time.time()
    ids = []
    for a, r in zip(arrivals, reqs):
        while time.time() - t0 < a:
            time.sleep(0.0005)
        ids.append(submit(srv, r))
    got = wait_all(srv, ids)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(ids) and st["ticks"] >= 1
    for i in ids:
        ts, ta, td = got[i][1]
        assert 0.0 <= ts <= ta <= td


def wait_codes(srv, ids, timeout=60.0):
    """Poll until every request ended; returns id -> result array or error code."""
    out = {}
    t0 = time.time()
    while len(out) < len(ids):
        for i in ids:
            if i in out:
                continue
            try:
                r = srv.poll(i)
            except Exception as e:  # noqa: BLE001  (a request's own failure)
                out[i] = e.code
                continue
            if r is not None:
                out[i] = r[0]
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.002)
    return out


def test_serving_nonfinite_request_fails_alone(tm):
    # a t-SVT request and a completion request holding a NaN fail with
    # ENONFINITE; every other request of the same ticks gets bitwise its
    # result alone
    announce("serving_nonfinite_alone")
    reqs = requests(seed=40)
    bad_t = ("tsvt", reqs[0][1].copy(), reqs[0][2])
    bad_t[1][2, 3, 1] = np.nan
    bad_c = list(reqs[1])
    bad_c[1] = bad_c[1].copy()
    obs = np.argwhere(bad_c[2] != 0)[0]
    bad_c[1][tuple(obs)] = np.nan
    bad_c = tuple(bad_c)
    alone = []
    for r in reqs[2:]:
        srv = tm.Server(budget_bytes=4 << 30, max_active=8)
        rid = submit(srv, r)
        alone.append(wait_all(srv, [rid])[rid][0])
        srv.close()
    srv = tm.Server(budget_bytes=4 << 30, max_active=8)
    ids = [submit(srv, r) for r in [bad_t, bad_c] + reqs[2:]]
    got = wait_codes(srv, ids)
    srv.close()
    assert got[ids[0]] == tm.ENONFINITE and got[ids[1]] == tm.ENONFINITE
    for k, rid in enumerate(ids[2:]):
        assert not isinstance(got[rid], int), got[rid]
        assert np.array_equal(got[rid], alone[k]), k


def test_serving_cancel_and_deadline(tm):
    announce("serving_cancel_deadline")
    reqs = requests(seed=50, n=4)
    cc = reqs[1][3]
    srv = tm.Server(budget_bytes=4 << 30, max_active=8)
    long_id = srv.submit_complete(reqs[1][1], reqs[1][2], 100000, 2.0, 0.1)        # cancelled while running
    late_id = srv.submit_complete(reqs[3][1], reqs[3][2], 100000, 2.0, 0.1, deadline_s=0.5)
    ok_ids = [submit(srv, r) for r in reqs]
    time.sleep(0.2)
    assert srv.cancel(long_id) == 0
    got = wait_codes(srv, [long_id, late_id] + ok_ids, timeout=120.0)
    srv.close()
    assert got[long_id] == tm.ECANCELED
    assert got[late_id] == tm.ETIMEOUT
    for rid in ok_ids:
        assert not isinstance(got[rid], int), got[rid]
    del cc


def test_serving_rejects_unsupported_shapes(tm):
    announce("serving_shapes")
    srv = tm.Server(budget_bytes=4 << 30, max_active=8)
    with pytest.raises(tm.TsvdError) as ei:
        srv.submit_tsvt(np.zeros((600, 40, 2), np.float32), 1.0)  # 600-row slices
    assert ei.value.code == tm.EINVAL
    with pytest.raises(tm.TsvdError) as ei:
        srv.submit_complete(np.zeros((8, 8, 2), np.float32), np.ones((8, 8, 2), np.uint8), 3, 1.0, float("nan"))
    assert ei.value.code == tm.EINVAL
    # the server still serves a valid request
    rid = srv.submit_tsvt(np.ones((8, 8, 2), np.float32), 0.5)
    assert not isinstance(wait_codes(srv, [rid])[rid], int)
    srv.close()
