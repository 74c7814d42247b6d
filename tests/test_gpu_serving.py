"""Serving loop: continuous batching, admission by device-memory footprint,
results independent of the mix."""
import time

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
        if r[0] == "tsvt":
            want = oracle.tsvt_dct(r[1].astype(np.float64), r[2])
        else:
            cc = r[3]
            want, _, _, _ = oracle.complete(r[1].astype(np.float64), r[2], cc.betas, cc.taus)
        assert rel(Y, want) <= 1e-4, r[0]


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
