"""Host-only tests of the continuous-batching scheduler (admission by
workspace footprint, FIFO order, batching per data set, concurrent streams,
latency percentiles, failure isolation) through a mock executor with a
virtual clock.  The scheduler source is the library's own serve_core.cpp."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_07096_amd", "csrc")


@pytest.fixture(scope="module")
def mock(tmp_path_factory):
    out = tmp_path_factory.mktemp("servemock") / "libservemock.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread", "-I", CSRC,
                    os.path.join(CSRC, "serve_core.cpp"), os.path.join(ROOT, "tests", "serve_mock",
                                                                         "mock_executor.cpp"),
                    "-o", str(out)], check=True)
    lib = C.CDLL(str(out))
    lib.mock_create.restype = C.c_void_p
    lib.mock_create.argtypes = [C.c_uint64, C.c_int32, C.c_int64, C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                C.c_int32]
    lib.mock_destroy.argtypes = [C.c_void_p]
    lib.mock_submit.restype = C.c_uint64
    lib.mock_submit.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_int32, C.c_int32]
    lib.mock_advance.argtypes = [C.c_void_p, C.c_double]
    lib.mock_poll.restype = C.c_int32
    lib.mock_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    lib.mock_stats.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
    lib.mock_launches.restype = C.c_int32
    lib.mock_launches.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.c_int32]
    return lib


class Sim:
    def __init__(self, lib, budget, ns, maxb=1 << 30, c0=1.0, c1=0.0, bpq=1, chunk=1 << 40, max_items=1024):
        self.lib = lib
        self.h = lib.mock_create(budget, ns, maxb, c0, c1, bpq, chunk, max_items)

    def submit(self, ds, m, fail=False, key=0):
        t = self.lib.mock_submit(self.h, ds, m, 1 if fail else 0, key)
        return t

    def advance(self, dt):
        self.lib.mock_advance(self.h, dt)

    def poll(self, t):
        st, lat = C.c_int32(), C.c_double()
        done = self.lib.mock_poll(self.h, t, C.byref(st), C.byref(lat))
        return done, st.value, lat.value

    def stats(self):
        out = (C.c_double * 12)()
        self.lib.mock_stats(self.h, out)
        keys = ["submitted", "completed", "failed", "rejected", "batches", "queries", "p50", "p99", "mean", "max",
                "inflight", "peak"]
        return dict(zip(keys, list(out)))

    def launches(self):
        buf = (C.c_int32 * 65536)()
        n = self.lib.mock_launches(self.h, buf, 65536)
        return [tuple(buf[5 * k:5 * k + 4]) for k in range(n)]

    def launch_keys(self):
        buf = (C.c_int32 * 65536)()
        n = self.lib.mock_launches(self.h, buf, 65536)
        return [buf[5 * k + 4] for k in range(n)]

    def close(self):
        self.lib.mock_destroy(self.h)


def test_admission_by_footprint_and_rejection(mock):
    sim = Sim(mock, budget=1000, ns=4, bpq=10, c0=1.0)
    a = sim.submit(0, 60)    # 600 B
    b = sim.submit(0, 60)    # 600 B: does not fit next to a
    big = sim.submit(0, 200)  # 2000 B > budget: rejected
    sim.advance(0.0)
    assert sim.poll(big)[:2] == (1, 5)
    assert sim.stats()["inflight"] == 600
    assert sim.poll(a)[0] == 0 and sim.poll(b)[0] == 0
    sim.advance(1.0)          # a finishes, b admitted and launched
    assert sim.poll(a) == (1, 0, 1.0)
    assert sim.poll(b)[0] == 0
    sim.advance(1.0)
    assert sim.poll(b) == (1, 0, 2.0)
    st = sim.stats()
    assert st["rejected"] == 1 and st["completed"] == 2 and st["peak"] == 600 and st["inflight"] == 0
    sim.close()


def test_fifo_head_of_line(mock):
    sim = Sim(mock, budget=100, ns=4, bpq=1, c0=1.0)
    t1 = sim.submit(0, 80)
    t2 = sim.submit(1, 50)   # does not fit beside t1: waits
    t3 = sim.submit(2, 10)   # would fit, but must not overtake t2
    sim.advance(0.0)
    assert [sim.poll(t)[0] for t in (t1, t2, t3)] == [0, 0, 0]
    assert sim.stats()["inflight"] == 80
    sim.advance(1.0)
    assert sim.poll(t1)[0] == 1
    assert sim.stats()["inflight"] == 60  # t2 and t3 admitted together once t1 left
    sim.advance(1.0)
    assert sim.poll(t2)[:2] == (1, 0) and sim.poll(t3)[:2] == (1, 0)
    sim.close()


def test_batching_per_dataset_and_concurrent_streams(mock):
    sim = Sim(mock, budget=10 ** 9, ns=2, c0=1.0, maxb=100)
    ts = [sim.submit(0, 30) for _ in range(3)] + [sim.submit(1, 5), sim.submit(0, 50)]
    sim.advance(0.0)
    lg = sim.launches()
    # stream 0: the three data-set-0 requests packed (90 queries; the fourth
    # would exceed 100); stream 1: data set 1; then the last one waits
    assert lg[0] == (0, 0, 3, 90)
    assert lg[1] == (1, 1, 1, 5)
    sim.advance(1.0)
    lg = sim.launches()
    assert lg[-1][1:] == (0, 1, 50)
    sim.advance(1.0)
    assert all(sim.poll(t)[:2] == (1, 0) for t in ts)
    assert sim.stats()["batches"] == 3
    sim.close()


def test_latency_percentiles(mock):
    sim = Sim(mock, budget=10 ** 9, ns=1, c0=1.0, c1=0.0, maxb=1)
    ts = [sim.submit(0, 1) for _ in range(10)]  # one stream, one query per batch: done at t = 1..10
    for _ in range(10):
        sim.advance(1.0)
    lats = sorted(sim.poll(t)[2] for t in ts)
    assert lats == [float(k) for k in range(1, 11)]
    st = sim.stats()
    assert st["p50"] == 5.0 and st["p99"] == 10.0 and st["mean"] == 5.5 and st["max"] == 10.0
    sim.close()


def test_failure_isolated_to_request(mock):
    sim = Sim(mock, budget=10 ** 9, ns=2, c0=1.0)
    good1 = sim.submit(0, 4)
    bad = sim.submit(0, 4, fail=True)
    good2 = sim.submit(0, 4)
    other = sim.submit(99, 4)  # launch failure on a data set
    sim.advance(1.0)
    assert sim.poll(good1)[:2] == (1, 0)
    assert sim.poll(good2)[:2] == (1, 0)
    assert sim.poll(bad)[:2] == (1, 3)
    assert sim.poll(other)[:2] == (1, 3)
    later = sim.submit(0, 4)
    sim.advance(1.0)
    assert sim.poll(later)[:2] == (1, 0)  # the loop keeps going
    st = sim.stats()
    assert st["failed"] == 2 and st["completed"] == 3 and st["inflight"] == 0
    sim.close()


def test_batch_item_limit(mock):
    """Many one-query requests of one data set: no batch exceeds the
    executor's item limit, and every request completes."""
    sim = Sim(mock, budget=10 ** 9, ns=2, c0=1.0, maxb=65536, max_items=1024)
    ts = [sim.submit(0, 1) for _ in range(2600)]
    for _ in range(4):
        sim.advance(1.0)
    lg = sim.launches()
    assert max(l[2] for l in lg) <= 1024
    assert sum(l[2] for l in lg) == 2600
    assert all(sim.poll(t)[:2] == (1, 0) for t in ts)
    assert sim.stats()["completed"] == 2600
    sim.close()


def test_chunks_let_small_requests_pass(mock):
    """A large request is served in chunks; a small one that arrives right
    after it rides in the next batch instead of waiting for all its chunks.
    Batch time is proportional to its queries."""
    sim = Sim(mock, budget=10 ** 9, ns=1, c0=0.0, c1=1.0, maxb=1000, chunk=100)
    big = sim.submit(0, 1000)
    sim.advance(0.0)
    small = sim.submit(0, 5)
    sim.advance(100.0)                  # first chunk (100 queries) done
    lg = sim.launches()
    assert lg[0] == (0, 0, 1, 100)      # the big request's first chunk alone
    assert lg[1] == (0, 0, 2, 105)      # its second chunk with the small request
    assert sim.poll(small)[0] == 0
    sim.advance(105.0)
    assert sim.poll(small) == (1, 0, 205.0)
    assert sim.poll(big)[0] == 0
    for _ in range(8):
        sim.advance(100.0)
    done, st, lat = sim.poll(big)
    assert (done, st) == (1, 0) and lat == 1005.0
    st = sim.stats()
    assert st["completed"] == 2 and st["queries"] == 1005
    sim.close()


def test_chunks_over_streams_and_keys(mock):
    """One large request spreads its chunks over the idle streams; a request
    with another key (form or estimator) is never batched with it and, being
    younger, takes the next free stream."""
    sim = Sim(mock, budget=10 ** 9, ns=4, c0=1.0, maxb=10 ** 6, chunk=256)
    big = sim.submit(0, 1024)
    other = sim.submit(0, 10, key=1)
    sim.advance(0.0)
    lg, keys = sim.launches(), sim.launch_keys()
    assert [(l[0], l[3]) for l in lg] == [(0, 256), (1, 256), (2, 256), (3, 256)] and keys == [0, 0, 0, 0]
    sim.advance(1.0)
    assert sim.poll(big) == (1, 0, 1.0)
    lg, keys = sim.launches(), sim.launch_keys()
    assert lg[-1][2:] == (1, 10) and keys[-1] == 1
    sim.advance(1.0)
    assert sim.poll(other) == (1, 0, 2.0)
    sim.close()


def test_chunk_failure_fails_request_once(mock):
    """A failed chunk fails its request (once), the others complete."""
    sim = Sim(mock, budget=10 ** 9, ns=2, c0=1.0, maxb=10 ** 6, chunk=8)
    bad = sim.submit(0, 40, fail=True)
    good = sim.submit(0, 40)
    for _ in range(10):
        sim.advance(1.0)
    assert sim.poll(bad)[:2] == (1, 3)
    assert sim.poll(good)[:2] == (1, 0)
    st = sim.stats()
    assert st["failed"] == 1 and st["completed"] == 1 and st["inflight"] == 0
    sim.close()
