"""Host logic of the serving scheduler (CPU): admission under the budget,
continuous batching, FIFO order, tickets, release, isolation of a request with
invalid keys, shutdown, and a thread-sanitized multi-client stress run.

The scheduler here is the library's own (paper_2405_07122_amd/csrc/
pcf_serve_core.cpp); only the executor is replaced by one over host memory
that sorts each segment with std::stable_sort."""
import ctypes
import subprocess
import time

import numpy as np
import pytest

from tests.serve_mock import build_mock

OK, INVALID_ARGUMENT, INVALID_KEY, OUT_OF_MEMORY = 0, 1, 2, 3
PENDING, UNKNOWN_TICKET, SHUTDOWN = 6, 7, 8


class Res(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_uint64), ("idx", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("latency_ns", ctypes.c_uint64), ("queue_ns", ctypes.c_uint64),
                ("status", ctypes.c_int32), ("batch_requests", ctypes.c_uint32)]


@pytest.fixture(scope="module")
def M():
    lib = ctypes.CDLL(build_mock.build_lib())
    lib.mock_create.restype = ctypes.c_void_p
    lib.mock_create.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                ctypes.c_uint32]
    lib.mock_submit.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                                ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
    lib.mock_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(Res)]
    lib.mock_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                              ctypes.POINTER(Res)]
    lib.mock_release.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    lib.mock_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
    lib.mock_stop.argtypes = [ctypes.c_void_p]
    lib.mock_destroy.argtypes = [ctypes.c_void_p]
    lib.mock_max_batch.restype = ctypes.c_uint64
    lib.mock_batches_started.restype = ctypes.c_uint64
    lib.mock_gate.argtypes = [ctypes.c_int]
    return lib


class Srv:
    def __init__(self, M, budget=1 << 22, slots=2, maxreq=64, maxkeys=1 << 20, delay_us=0):
        self.M = M
        self.h = M.mock_create(budget, slots, maxreq, maxkeys, delay_us)
        assert self.h
        self.keep = {}

    def submit(self, keys: np.ndarray, argsort=False, kt=None):
        t = ctypes.c_uint64()
        kt = (0 if keys.dtype == np.float64 else 1) if kt is None else kt
        keys = np.ascontiguousarray(keys)
        rc = self.M.mock_submit(self.h, kt, keys.ctypes.data if keys.size else None, keys.size,
                                int(argsort), ctypes.byref(t))
        if rc == OK:
            self.keep[t.value] = keys  # the input must outlive the request
        return rc, t.value

    def wait(self, t, ms=20000):
        r = Res()
        rc = self.M.mock_wait(self.h, t, ms, ctypes.byref(r))
        return rc, r

    def poll(self, t):
        r = Res()
        return self.M.mock_poll(self.h, t, ctypes.byref(r)), r

    def result(self, r, dtype):
        if r.n == 0:
            return np.zeros(0, dtype), None
        k = np.ctypeslib.as_array((ctypes.c_uint64 * r.n).from_address(r.keys)).view(dtype).copy()
        i = None
        if r.idx:
            i = np.ctypeslib.as_array((ctypes.c_uint32 * r.n).from_address(r.idx)).copy()
        return k, i

    def release(self, t):
        return self.M.mock_release(self.h, t)

    def stats(self):
        a = (ctypes.c_uint64 * 8)()
        self.M.mock_stats(self.h, a)
        return dict(zip(["submitted", "completed", "released", "batches", "budget", "in_use",
                         "high_water", "queued"], list(a)))

    def close(self):
        self.M.mock_destroy(self.h)


def test_results_and_batching(M):
    s = Srv(M, slots=1, delay_us=20000)
    rng = np.random.default_rng(1)
    arrs = [rng.random(int(rng.integers(0, 3000))) for _ in range(40)]
    ts = []
    for a in arrs:
        rc, t = s.submit(a, argsort=True)
        assert rc == OK
        ts.append(t)
    sizes = []
    for a, t in zip(arrs, ts):
        rc, r = s.wait(t)
        assert rc == OK and r.status == OK and r.n == a.size
        k, i = s.result(r, np.float64)
        np.testing.assert_array_equal(k, np.sort(a, kind="stable"))
        if a.size:
            np.testing.assert_array_equal(i, np.argsort(a, kind="stable"))
        sizes.append(r.batch_requests)
        assert r.latency_ns >= r.queue_ns
        assert s.release(t) == OK
    # requests that arrived while the single slot was busy shared batches
    assert max(sizes) > 1 and M.mock_max_batch() > 1
    st = s.stats()
    assert st["in_use"] == 0 and st["completed"] == 40 and st["released"] == 40
    assert st["batches"] < 40
    s.close()


def test_kinds_never_share_a_batch(M):
    s = Srv(M, slots=1, delay_us=20000)
    rng = np.random.default_rng(2)
    subs = []
    for j in range(12):
        if j % 3 == 0:
            a = rng.random(500)
            subs.append((a, False, s.submit(a)[1]))
        elif j % 3 == 1:
            a = rng.integers(0, 2**63, 700, dtype=np.uint64)
            subs.append((a, False, s.submit(a)[1]))
        else:
            a = rng.random(300)
            subs.append((a, True, s.submit(a, argsort=True)[1]))
    for a, as_, t in subs:
        rc, r = s.wait(t)
        assert rc == OK and r.status == OK
        k, i = s.result(r, a.dtype)
        np.testing.assert_array_equal(k, np.sort(a, kind="stable"))
        assert (i is not None) == as_
        s.release(t)
    s.close()


def test_budget_admission_and_fifo_wait(M):
    budget = 1 << 20
    s = Srv(M, budget=budget, slots=2)
    # mock work = 16 n + 64 nseg + 1024 bytes, outputs 8 n (+ 4 n): alone > budget
    rc, _ = s.submit(np.random.default_rng(3).random(60_000))
    assert rc == OUT_OF_MEMORY
    # hold most of the budget with results that are not released
    a = np.random.default_rng(4).random(40_000)
    rc, t1 = s.submit(a)
    assert rc == OK and s.wait(t1)[0] == OK
    held = s.stats()["in_use"]
    assert 0 < held <= budget
    b = np.random.default_rng(5).random(40_000)
    rc, t2 = s.submit(b)
    assert rc == OK
    time.sleep(0.2)
    assert s.poll(t2)[0] == PENDING  # waits for memory, not rejected
    assert s.stats()["queued"] == 1
    assert s.release(t1) == OK
    rc, r = s.wait(t2)
    assert rc == OK and r.status == OK
    np.testing.assert_array_equal(s.result(r, np.float64)[0], np.sort(b))
    s.release(t2)
    st = s.stats()
    assert st["high_water"] <= budget and st["in_use"] == 0
    s.close()


def test_tickets_and_release(M):
    s = Srv(M, slots=1, delay_us=50000)
    rng = np.random.default_rng(6)
    rc, t1 = s.submit(rng.random(1000))
    rc, t2 = s.submit(rng.random(1000))
    rc, t3 = s.submit(rng.random(1000))
    # release a request that has not run: its ticket disappears
    assert s.release(t3) == OK
    assert s.poll(t3)[0] == UNKNOWN_TICKET
    assert s.release(t3) == UNKNOWN_TICKET
    assert s.poll(123456)[0] == UNKNOWN_TICKET
    assert s.wait(t1)[0] == OK
    assert s.wait(t2)[0] == OK
    assert s.release(t1) == OK and s.release(t2) == OK
    assert s.stats()["in_use"] == 0
    # empty request: done at once, no memory
    rc, t0 = s.submit(np.zeros(0))
    rc, r = s.poll(t0)
    assert rc == OK and r.n == 0 and r.status == OK
    s.release(t0)
    # argument errors
    t = ctypes.c_uint64()
    assert M.mock_submit(s.h, 5, None, 0, 0, ctypes.byref(t)) == INVALID_ARGUMENT
    assert M.mock_submit(s.h, 0, None, 10, 0, ctypes.byref(t)) == INVALID_ARGUMENT
    s.close()


def _until(cond, seconds=20.0):
    t0 = time.monotonic()
    while not cond():
        assert time.monotonic() - t0 < seconds, "condition not reached"
        time.sleep(0.001)


def test_invalid_key_is_isolated(M):
    """A request with a NaN fails alone; the requests batched with it succeed.
    A gate holds the only slot's first batch until the six requests are all
    queued, so they are taken as one batch whatever the thread timing."""
    s = Srv(M, slots=1)
    M.mock_gate(1)
    try:
        rng = np.random.default_rng(7)
        blocker = rng.random(100)
        s.submit(blocker)
        _until(lambda: M.mock_batches_started() >= 1)
        arrs = [rng.random(400) for _ in range(6)]
        arrs[3][17] = np.nan
        ts = [s.submit(a)[1] for a in arrs]
        _until(lambda: s.stats()["queued"] == 6)
    finally:
        M.mock_gate(0)
    for j, (a, t) in enumerate(zip(arrs, ts)):
        rc, r = s.wait(t)
        assert rc == OK
        if j == 3:
            assert r.status == INVALID_KEY
        else:
            assert r.status == OK
            np.testing.assert_array_equal(s.result(r, np.float64)[0], np.sort(a))
        assert r.batch_requests == 6
    s.close()


def test_shutdown(M):
    s = Srv(M, slots=1, maxreq=1, delay_us=100000)  # one request per batch: some stay queued
    rng = np.random.default_rng(8)
    ts = [s.submit(rng.random(100))[1] for _ in range(5)]
    time.sleep(0.02)
    M.mock_stop(s.h)
    codes = [s.wait(t, 1000)[1].status for t in ts]
    # the running batch completes; whatever was still queued is failed
    assert SHUTDOWN in codes and all(c in (OK, SHUTDOWN) for c in codes)
    assert s.submit(rng.random(10))[0] == SHUTDOWN
    s.close()


def test_concurrent_slots_overlap(M):
    s = Srv(M, slots=3, maxreq=1, delay_us=30000)
    rng = np.random.default_rng(9)
    ts = [s.submit(rng.random(100))[1] for _ in range(9)]
    for t in ts:
        assert s.wait(t)[1].status == OK
    assert M.mock_max_running() == 3
    s.close()


def test_stress_thread_sanitizer():
    """Four clients submit, wait, release (some before completion) against
    three worker slots, under ThreadSanitizer: no race, every byte returned."""
    exe = build_mock.build_stress("thread")
    r = subprocess.run([exe, "4", "150"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ThreadSanitizer" not in r.stderr
