"""The serving loop's scheduler (admission by footprint, FIFO order, the cap on
running requests, cancellation, deadlines), driven on the CPU by a simulated
executor: every admitted request runs a fixed number of ticks.  The code under
test is the library's own scheduler header, compiled here with g++."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sched_harness.cpp")
OK, EBUSY, ETIMEOUT, ECANCELED = 0, -5, -6, -7
PENDING, ACTIVE, DONE = 1, 2, 3


@pytest.fixture(scope="module")
def sh():
    out = os.path.join(tempfile.mkdtemp(prefix="sched_"), "libsched_harness.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-I", os.path.join(ROOT, "include"), SRC,
                           "-o", out])
    lib = C.CDLL(out)
    vp, i64, d = C.c_void_p, C.c_int64, C.c_double
    lib.sh_new.restype = vp
    lib.sh_new.argtypes = [i64, C.c_int]
    lib.sh_free.argtypes = [vp]
    lib.sh_submit.restype = i64
    lib.sh_submit.argtypes = [vp, i64, d, d]
    lib.sh_admit.argtypes = [vp, d, C.POINTER(i64), C.c_int]
    lib.sh_expire.argtypes = [vp, d]
    lib.sh_take_stopped.argtypes = [vp, d, C.POINTER(i64), C.POINTER(C.c_int), C.c_int]
    lib.sh_cancel.argtypes = [vp, i64, d]
    lib.sh_finish.argtypes = [vp, i64, C.c_int]
    for n in ("sh_state", "sh_status"):
        getattr(lib, n).argtypes = [vp, i64]
    lib.sh_forget.argtypes = [vp, i64]
    for n in ("sh_held", "sh_peak", "sh_queued", "sh_completed"):
        getattr(lib, n).restype = i64
        getattr(lib, n).argtypes = [vp]
    lib.sh_active.argtypes = [vp]
    return lib


class Sim:
    """The server loop with a fake executor: a request needs `work` ticks."""

    def __init__(self, sh, budget, max_active):
        self.sh, self.s = sh, sh.sh_new(budget, max_active)
        self.work, self.left, self.admit_tick, self.done_tick, self.status = {}, {}, {}, {}, {}
        self.running = []
        self.tick_no = 0

    def submit(self, footprint, work, deadline=0.0):
        rid = self.sh.sh_submit(self.s, footprint, float(self.tick_no), deadline)
        if rid > 0:
            self.work[rid] = work
        return rid

    def tick(self):
        t = float(self.tick_no)
        self.sh.sh_expire(self.s, t)
        ids = (C.c_int64 * 256)()
        n = self.sh.sh_admit(self.s, t, ids, 256)
        for i in range(n):
            self.running.append(ids[i])
            self.left[ids[i]] = self.work[ids[i]]
            self.admit_tick[ids[i]] = self.tick_no
        assert self.sh.sh_held(self.s) <= self.budget_check
        codes = (C.c_int * 256)()
        n = self.sh.sh_take_stopped(self.s, t, ids, codes, 256)
        stopped = {ids[i]: codes[i] for i in range(n)}
        still = []
        for rid in self.running:
            if rid in stopped:
                self.sh.sh_finish(self.s, rid, stopped[rid])
                self.done_tick[rid] = self.tick_no
                continue
            self.left[rid] -= 1
            if self.left[rid] == 0:
                self.sh.sh_finish(self.s, rid, OK)
                self.done_tick[rid] = self.tick_no
            else:
                still.append(rid)
        self.running = still
        self.tick_no += 1

    def state(self, rid):
        return self.sh.sh_state(self.s, rid)

    def run(self, ticks):
        for _ in range(ticks):
            self.tick()


def make(sh, budget, max_active):
    s = Sim(sh, budget, max_active)
    s.budget_check = budget
    return s


def test_fifo_order_and_budget(sh):
    s = make(sh, budget=100, max_active=8)
    ids = [s.submit(40, work=3) for _ in range(5)]
    s.run(20)
    # two fit at a time (80 <= 100), admitted strictly in arrival order
    adm = [s.admit_tick[i] for i in ids]
    assert adm == sorted(adm)
    assert adm[:2] == [0, 0] and adm[2] > 0
    assert sh.sh_peak(s.s) == 80
    assert all(s.state(i) == DONE for i in ids)
    assert sh.sh_completed(s.s) == 5


def test_max_active_cap(sh):
    s = make(sh, budget=10 ** 9, max_active=3)
    ids = [s.submit(1, work=2) for _ in range(7)]
    for _ in range(10):
        s.tick()
        assert sh.sh_active(s.s) <= 3
    assert all(s.state(i) == DONE for i in ids)


def test_large_request_is_not_starved(sh):
    # a large request behind small ones is admitted as soon as memory frees up;
    # small requests that arrive after it wait behind it (no overtaking)
    s = make(sh, budget=100, max_active=16)
    small = [s.submit(30, work=4) for _ in range(3)]
    big = s.submit(90, work=2)
    later = [s.submit(5, work=1) for _ in range(4)]
    s.run(30)
    assert s.admit_tick[big] <= min(s.admit_tick[i] for i in later)
    assert s.admit_tick[big] >= max(s.done_tick[i] for i in small)
    assert all(s.state(i) == DONE for i in small + [big] + later)


def test_over_budget_request_is_refused(sh):
    s = make(sh, budget=100, max_active=4)
    assert s.submit(101, work=1) == EBUSY
    assert s.submit(100, work=1) > 0


def test_cancel_queued_and_running(sh):
    s = make(sh, budget=50, max_active=4)
    a = s.submit(40, work=10)
    b = s.submit(40, work=10)   # waits for memory
    s.tick()
    assert s.state(a) == ACTIVE and s.state(b) == PENDING
    assert sh.sh_cancel(s.s, b, 1.0) == 0
    assert s.state(b) == DONE and sh.sh_status(s.s, b) == ECANCELED
    assert sh.sh_cancel(s.s, a, 1.0) == 0
    assert s.state(a) == ACTIVE  # stops at the next step boundary
    s.tick()
    assert s.state(a) == DONE and sh.sh_status(s.s, a) == ECANCELED
    assert sh.sh_held(s.s) == 0
    assert sh.sh_cancel(s.s, a, 2.0) == 1
    assert sh.sh_cancel(s.s, 999, 2.0) == -1


def test_deadlines_queued_and_running(sh):
    s = make(sh, budget=50, max_active=4)
    a = s.submit(40, work=100, deadline=5.0)   # runs, misses its deadline
    b = s.submit(40, work=1, deadline=3.0)     # never admitted in time
    c = s.submit(10, work=2, deadline=50.0)    # fits beside a, finishes in time
    s.run(12)
    assert sh.sh_status(s.s, a) == ETIMEOUT and s.done_tick[a] == 6
    assert sh.sh_status(s.s, b) == ETIMEOUT and b not in s.admit_tick
    assert sh.sh_status(s.s, c) == OK
    assert sh.sh_held(s.s) == 0


def test_random_stream_invariants(sh):
    # a Poisson-like stream of mixed sizes: memory never exceeds the budget,
    # admission order equals arrival order, every request ends
    g = np.random.default_rng(5)
    s = make(sh, budget=1000, max_active=6)
    ids = []
    for t in range(300):
        for _ in range(g.poisson(0.8)):
            ids.append(s.submit(int(g.integers(10, 600)), work=int(g.integers(1, 8))))
        s.tick()
    s.run(2000)
    assert all(s.state(i) == DONE for i in ids)
    adm = [s.admit_tick[i] for i in ids]
    assert adm == sorted(adm)
    assert sh.sh_held(s.s) == 0 and sh.sh_queued(s.s) == 0
