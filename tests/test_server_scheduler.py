"""The request server's scheduler on the CPU, driven by a host-only executor.

The library's server (bura_server_*) is the scheduler of
paper_1612_04846_amd/csrc/bura_scheduler.h with an executor that runs slot
plans on the GPU.  Here the same scheduler source is compiled with a stub
executor (tests/server_stub/stub_executor.cpp): plans are host records with a
footprint, a request's solve is a countdown of outer steps.  That exercises
the scheduling without a device: continuous batching (a request joins a
running solve), FIFO groups for FP64 keys, term classes, the max_concurrent
limit, HBM-budget eviction, waiting for memory held by busy plans, and
refusing a plan that can never fit.
"""

import ctypes
import os
import subprocess
import time

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
MIXED, FP64 = 1, 0
OK, ENOMEM = 0, -5


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_longlong) for n in
                ("submitted", "completed", "failed", "batches", "plans_created", "plans_evicted")] + [
        ("unknown_pole_solves", ctypes.c_double), ("p50_latency_s", ctypes.c_double),
        ("p99_latency_s", ctypes.c_double), ("mean_batch", ctypes.c_double), ("resident_bytes", ctypes.c_size_t),
        ("joined_running", ctypes.c_longlong)]


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("stub") / "libstub.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread",
                    os.path.join(HERE, "server_stub", "stub_executor.cpp"), "-o", out], check=True)
    L = ctypes.CDLL(out)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.stub_server_create.restype = P
    L.stub_server_create.argtypes = [ctypes.c_size_t, I, I, I]
    L.stub_server_submit.argtypes = [P, I, I, D, I, D, I, P, P, ctypes.POINTER(ctypes.c_uint64)]
    L.stub_server_poll.argtypes = [P, ctypes.c_uint64]
    L.stub_server_wait.argtypes = [P, ctypes.c_uint64]
    L.stub_server_stats.argtypes = [P, ctypes.POINTER(Stats)]
    L.stub_server_counters.argtypes = [P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                       ctypes.POINTER(I)]
    L.stub_plan_bytes.restype = ctypes.c_size_t
    L.stub_plan_bytes.argtypes = [I, I, I, I, I]
    L.stub_server_destroy.argtypes = [P]
    return L


class Server:
    def __init__(self, L, budget=0, max_concurrent=4, max_group=2, step_us=1000):
        self.L = L
        self.h = L.stub_server_create(budget, max_concurrent, max_group, step_us)
        self.bufs = []

    def submit(self, n, k=5, tol=1e-9, precision=MIXED, dim=2, f0=0.0):
        f = (ctypes.c_double * 1)(f0)
        u = (ctypes.c_double * 1)(-1.0)
        tk = ctypes.c_uint64()
        assert self.L.stub_server_submit(self.h, dim, n, 0.5, k, tol, precision, f, u, ctypes.byref(tk)) == OK
        self.bufs.append((f, u))
        return tk.value, u, f0 + (k + 1) * (k + 2) / 2

    def wait(self, tk):
        return self.L.stub_server_wait(self.h, tk)

    def stats(self):
        st = Stats()
        self.L.stub_server_stats(self.h, ctypes.byref(st))
        return st

    def counters(self):
        c, d, m = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
        self.L.stub_server_counters(self.h, ctypes.byref(c), ctypes.byref(d), ctypes.byref(m))
        return c.value, d.value, m.value

    def close(self):
        self.L.stub_server_destroy(self.h)


def test_request_joins_a_running_solve(lib):
    """max_group 2: a request for the same key submitted while another one's
    solve runs is admitted into that solve at a step boundary and finishes
    first (fewer steps), without waiting for the long one."""
    s = Server(lib, max_group=2, step_us=2000)
    t_long, u_long, e_long = s.submit(127, tol=1e-30, f0=1.0)   # 10 outer steps
    while s.stats().batches == 0:   # the long solve has taken its first step
        time.sleep(0.0005)
    t_short, u_short, e_short = s.submit(127, tol=1e-3, f0=2.0)   # 1 outer step
    assert s.wait(t_short) == OK
    assert s.L.stub_server_poll(s.h, t_long) == 1   # still running (BURA_PENDING)
    assert s.wait(t_long) == OK
    st = s.stats()
    s.close()
    assert st.joined_running >= 1 and st.plans_created == 1
    assert u_long[0] == e_long and u_short[0] == e_short


def test_fp64_key_batches_queued_requests(lib):
    """FP64 keys solve up to max_group queued requests per solve."""
    s = Server(lib, max_group=4, step_us=3000)
    reqs = [s.submit(255, k=7, tol=1e-9, precision=FP64, f0=float(i)) for i in range(8)]
    for tk, _, _ in reqs:
        assert s.wait(tk) == OK
    st = s.stats()
    s.close()
    assert all(u[0] == e for _, u, e in reqs)
    assert st.batches <= 4 and st.mean_batch > 1.5


def test_term_classes_share_or_split_plans(lib):
    """k + 1 <= 13 terms share one plan of a grid; larger k gets a 17-slot plan."""
    s = Server(lib, step_us=200)
    tks = [s.submit(63, k=k) for k in (5, 12, 9)]
    for tk, _, _ in tks:
        assert s.wait(tk) == OK
    assert s.stats().plans_created == 1
    tk, u, e = s.submit(63, k=13)
    assert s.wait(tk) == OK and u[0] == e
    st = s.stats()
    s.close()
    assert st.plans_created == 2


def test_max_concurrent_bounds_plans_with_work(lib):
    """Requests on three keys: with max_concurrent 1 never more than one plan
    steps at a time; with 3 they overlap."""
    for mc, lo, hi in ((1, 1, 1), (3, 2, 3)):
        s = Server(lib, max_concurrent=mc, max_group=1, step_us=2000)
        reqs = [s.submit(n, tol=1e-9) for n in (31, 63, 127) for _ in range(2)]
        for tk, u, e in reqs:
            assert s.wait(tk) == OK and u[0] == e
        _, _, busy = s.counters()
        s.close()
        assert lo <= busy <= hi, (mc, busy)


def test_budget_evicts_idle_plans_least_recently_used(lib):
    """A budget that holds two plans: a third key evicts the idle plan used
    longest ago, and the resident bytes stay within the budget."""
    b = lib.stub_plan_bytes(2, 127, 5, MIXED, 2)
    s = Server(lib, budget=int(2.5 * b), step_us=200)
    for n in (127, 125, 127):   # 125 is now the least recently used plan
        tk, u, e = s.submit(n)
        assert s.wait(tk) == OK and u[0] == e
    tk, u, e = s.submit(123)
    assert s.wait(tk) == OK and u[0] == e
    st = s.stats()
    created, destroyed, _ = s.counters()
    s.close()
    assert st.plans_created == 3 and st.plans_evicted == 1 and destroyed == 1
    assert st.resident_bytes <= int(2.5 * b)
    # the evicted plan was 125's (127 was used after it): a new 127 request needs no plan
    s = Server(lib, budget=int(2.5 * b), step_us=200)
    for n in (127, 125, 127, 123, 127):
        tk, _, _ = s.submit(n)
        assert s.wait(tk) == OK
    assert s.stats().plans_created == 3
    s.close()


def test_request_waits_for_memory_held_by_a_busy_plan(lib):
    """A budget for one plan: a request for another key that arrives while the
    first plan is solving waits (the busy plan cannot be evicted), then runs
    once the first plan is idle and evicted."""
    b = lib.stub_plan_bytes(2, 127, 5, MIXED, 2)
    s = Server(lib, budget=int(1.5 * b), step_us=3000)
    t1, u1, e1 = s.submit(127, tol=1e-30)   # 10 steps
    while s.stats().batches == 0:
        time.sleep(0.0005)
    t2, u2, e2 = s.submit(125, tol=1e-3)
    assert s.wait(t2) == OK and s.L.stub_server_poll(s.h, t1) == OK   # t1 finished first
    st = s.stats()
    s.close()
    assert u1[0] == e1 and u2[0] == e2
    assert st.plans_created == 2 and st.plans_evicted == 1 and st.failed == 0


def test_plan_that_can_never_fit_fails_with_enomem(lib):
    """A key whose plan exceeds the whole budget fails its requests with
    BURA_ENOMEM (nothing waits forever); smaller keys are still served."""
    b = lib.stub_plan_bytes(2, 127, 5, MIXED, 2)
    s = Server(lib, budget=int(1.5 * b), step_us=200)
    t_big, u_big, _ = s.submit(1023)
    t_ok, u_ok, e_ok = s.submit(127)
    assert s.wait(t_big) == ENOMEM and u_big[0] == -1.0
    assert s.wait(t_ok) == OK and u_ok[0] == e_ok
    st = s.stats()
    s.close()
    assert st.failed == 1 and st.completed == 2


def test_destroy_waits_for_queued_requests(lib):
    """Destroying the server finishes every queued and running request first."""
    s = Server(lib, max_group=2, step_us=1000)
    reqs = [s.submit(n, tol=1e-9) for n in (63, 63, 63, 127, 127)]
    s.close()
    assert all(u[0] == e for _, u, e in reqs)
