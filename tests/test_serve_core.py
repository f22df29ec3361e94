"""CPU tests of the served form's scheduling core (serve_core.cpp) over a
host-only fake device (tests/fake_device/fake_serve.cpp): admission against
the arena budget, continuous batching in arrival order, exclusive and
grouped requests, cancellation, status propagation and latency accounting.
The fake device sleeps for a request's simulated duration and checks every
arena block it is given against the budget and the blocks in use."""
import ctypes as C
import subprocess
import time
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]
SRC = ROOT / "paper_2506_06190_amd" / "csrc"
OUT = ROOT / "_build" / "fake_serve" / "libnat_fake_serve.so"

ST_OK, ST_INVALID, ST_BUDGET, ST_NOCONV, ST_PENDING, ST_CANCELLED = 0, 1, 2, 3, 6, 7


@pytest.fixture(scope="module")
def fs():
    OUT.parent.mkdir(parents=True, exist_ok=True)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-shared", "-fPIC", "-pthread", "-Wall", "-I", str(SRC),
           str(ROOT / "tests" / "fake_device" / "fake_serve.cpp"), str(SRC / "serve_core.cpp"),
           "-o", str(OUT)]
    subprocess.run(cmd, check=True, capture_output=True)
    L = C.CDLL(str(OUT))
    L.fs_create.argtypes = [C.c_int32, C.c_int32, C.c_uint64, C.c_uint64]
    L.fs_create.restype = C.c_void_p
    L.fs_submit.argtypes = [C.c_void_p, C.c_uint64, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                            C.POINTER(C.c_uint64)]
    L.fs_submit.restype = C.c_int32
    L.fs_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_double, C.POINTER(C.c_double)]
    L.fs_wait.restype = C.c_int32
    L.fs_cancel.argtypes = [C.c_void_p, C.c_uint64]
    L.fs_cancel.restype = C.c_int32
    L.fs_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
    L.fs_batch_log.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int64]
    L.fs_batch_log.restype = C.c_int64
    L.fs_destroy.argtypes = [C.c_void_p]
    return L


class Srv:
    def __init__(self, L, n_slots, max_batch, budget, overhead=0):
        self.L = L
        self.h = L.fs_create(n_slots, max_batch, budget, overhead)

    def submit(self, nbytes, run_ms, exclusive=0, group=0, status=ST_OK):
        t = C.c_uint64()
        st = self.L.fs_submit(self.h, nbytes, run_ms, exclusive, group, status, C.byref(t))
        return st, t.value

    def wait(self, ticket, timeout_ms=-1.0):
        out = (C.c_double * 6)()
        st = self.L.fs_wait(self.h, ticket, timeout_ms, out)
        return st, {"latency": out[0], "queue": out[1], "run": out[2], "batch_size": int(out[3]),
                    "slot": int(out[4]), "batch_id": int(out[5])}

    def stats(self):
        o = (C.c_int64 * 8)()
        self.L.fs_stats(self.h, o)
        keys = ["submitted", "completed", "cancelled", "batches", "max_batch", "max_concurrent",
                "peak_bytes", "violations"]
        return dict(zip(keys, list(o)))

    def batches(self):
        buf = (C.c_int64 * 20000)()
        n = self.L.fs_batch_log(self.h, buf, 10000)
        out = {}
        for i in range(min(n, 10000)):
            out.setdefault(buf[2 * i], []).append(buf[2 * i + 1])
        return out

    def close(self):
        self.L.fs_destroy(self.h)


def test_budget_never_exceeded_under_load(fs):
    rng = np.random.default_rng(5)
    budget = 1 << 20
    s = Srv(fs, n_slots=4, max_batch=8, budget=budget, overhead=4096)
    tickets = []
    for _ in range(300):
        st, t = s.submit(int(rng.integers(1, 200_000)), float(rng.uniform(0.1, 2.0)))
        assert st == ST_OK
        tickets.append(t)
        if rng.random() < 0.3:
            time.sleep(0.0005)
    for t in tickets:
        st, r = s.wait(t)
        assert st == ST_OK
        assert abs(r["latency"] - r["queue"] - r["run"]) < 1e-6
        assert r["queue"] >= 0.0 and r["run"] > 0.0 and 1 <= r["batch_size"] <= 8
    stt = s.stats()
    assert stt["violations"] == 0
    assert 0 < stt["peak_bytes"] <= budget
    assert stt["completed"] == 300 and stt["max_batch"] <= 8
    # the load queued work: batches formed and ran side by side
    assert stt["batches"] < 300 and stt["max_concurrent"] >= 2
    s.close()


def test_continuous_batching_in_arrival_order(fs):
    # one worker busy with a long request; the next 10 queue and start as
    # batches of at most 4 in arrival order as soon as the worker is free
    s = Srv(fs, n_slots=1, max_batch=4, budget=1 << 30)
    st, first = s.submit(1000, 60.0)
    time.sleep(0.02)
    rest = [s.submit(1000, 1.0)[1] for _ in range(10)]
    for t in [first] + rest:
        assert s.wait(t)[0] == ST_OK
    b = s.batches()
    order = [b[k] for k in sorted(b)]
    assert order[0] == [first]
    assert order[1:] == [rest[0:4], rest[4:8], rest[8:10]]
    s.close()


def test_exclusive_and_groups_never_share(fs):
    s = Srv(fs, n_slots=1, max_batch=16, budget=1 << 30)
    st, blocker = s.submit(10, 40.0)
    time.sleep(0.01)
    kinds = {}
    for i in range(12):
        exclusive = 1 if i % 5 == 2 else 0
        group = i % 2
        t = s.submit(10, 0.5, exclusive=exclusive, group=group)[1]
        kinds[t] = (exclusive, group)
    for t in [blocker] + list(kinds):
        assert s.wait(t)[0] == ST_OK
    for members in s.batches().values():
        if any(kinds.get(t, (0, 0))[0] for t in members):
            assert len(members) == 1
        assert len({kinds[t][1] for t in members if t in kinds}) <= 1
    s.close()


def test_head_is_not_overtaken_by_later_requests(fs):
    # a request that needs the whole arena waits for the running ones; the
    # small requests submitted after it start only after it
    budget = 1 << 20
    s = Srv(fs, n_slots=4, max_batch=1, budget=budget)
    early = [s.submit(100_000, 30.0)[1] for _ in range(3)]
    time.sleep(0.01)
    big = s.submit(budget, 5.0)[1]
    late = [s.submit(100_000, 1.0)[1] for _ in range(3)]
    res = {t: s.wait(t)[1] for t in early + [big] + late}
    assert all(res[t]["batch_id"] > res[big]["batch_id"] for t in late)
    assert s.stats()["violations"] == 0
    s.close()


def test_budget_rejection_cancellation_and_status(fs):
    s = Srv(fs, n_slots=1, max_batch=1, budget=1 << 16, overhead=1024)
    assert s.submit(1 << 16, 1.0)[0] == ST_BUDGET          # overhead + bytes > budget
    st, running = s.submit(100, 50.0)
    time.sleep(0.01)
    st, queued = s.submit(100, 1.0)
    st, failing = s.submit(100, 1.0, status=ST_NOCONV)
    assert s.L.fs_cancel(s.h, queued) == ST_OK
    assert s.L.fs_cancel(s.h, queued) == ST_INVALID          # already cancelled
    assert s.L.fs_cancel(s.h, running) == ST_INVALID         # already started
    st, r = s.wait(queued)
    assert st == ST_CANCELLED and r["slot"] == -1
    assert s.wait(running)[0] == ST_OK
    assert s.wait(failing)[0] == ST_NOCONV
    assert s.wait(running)[0] == ST_INVALID                  # ticket already collected
    st, pending = s.submit(100, 40.0)
    assert s.wait(pending, timeout_ms=1.0)[0] == ST_PENDING
    assert s.wait(pending)[0] == ST_OK
    stt = s.stats()
    assert stt["cancelled"] == 1 and stt["completed"] == 3
    s.close()


def test_destroy_cancels_queued_and_finishes_running(fs):
    s = Srv(fs, n_slots=1, max_batch=1, budget=1 << 20)
    s.submit(100, 30.0)
    time.sleep(0.005)
    for _ in range(5):
        s.submit(100, 30.0)
    t0 = time.perf_counter()
    s.close()            # returns once the running request has finished
    assert time.perf_counter() - t0 < 1.0
