"""Serving logic on the CPU: buddy allocation, memory admission, arrival-order
admission, cancellation, failure isolation and latency statistics, with a fake
executor that computes with the oracle and completes batches after a delay."""
import random
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1005_1497_amd.serve import BuddyAllocator, ConvServer

M = 31065037602817


def test_buddy_allocator_random():
    rng = random.Random(0)
    a = BuddyAllocator(12, 2)
    live = {}
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off, k = live.popitem()
            a.free(off, k)
        else:
            k = rng.randint(2, 9)
            off = a.alloc(k)
            if off is None:
                assert a.capacity - a.used < (1 << 12)
                continue
            assert off % (1 << k) == 0 and off + (1 << k) <= a.capacity
            for o2, k2 in live.items():
                assert off + (1 << k) <= o2 or o2 + (1 << k2) <= off
            live[off] = k
        assert a.used == sum(1 << k for k in live.values())
    for off, k in live.items():
        a.free(off, k)
    assert a.used == 0 and a.free_lists[12] == {0}


class FakeExecutor:
    """Executor double: the work of a batch is the oracle's direct convolution;
    a batch completes `delay` seconds after launch.  Records the peak number of
    arena elements in use by launched-but-incomplete batches."""

    def __init__(self, m, delay=0.002, fail_on=None):
        self.m = m
        self.delay = delay
        self.streams = [0, 1]
        self.fail_on = fail_on
        self.launches = []

    def staging(self, n):
        return (np.zeros(n, np.uint64), np.zeros(n, np.uint64))

    def operand_views(self, staged):
        return staged

    def prepare(self, f, g):
        return (np.array(f, dtype=np.uint64), np.array(g, dtype=np.uint64))

    def launch(self, reqs, sid):
        if self.fail_on is not None and any(r.rid == self.fail_on for r in reqs):
            raise RuntimeError("injected launch failure")
        outs = [oracle.conv_direct(r.staged[0], r.staged[1], self.m) for r in reqs]
        self.launches.append([r.rid for r in reqs])
        return (time.monotonic() + self.delay, outs)

    def poll(self, h):
        return time.monotonic() >= h[0]

    def results(self, h):
        return h[1]


def _reqs(n, seed=0, lo=2, hi=8):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        k = int(rng.integers(lo, hi + 1))
        out.append((rng.integers(0, M, 1 << k, dtype=np.uint64), rng.integers(0, M, 1 << k, dtype=np.uint64)))
    return out


def test_results_equal_alone_and_budget_respected():
    ex = FakeExecutor(M)
    srv = ConvServer(ex, capacity_log2=10, min_log2=0, max_inflight=3)
    reqs = _reqs(120, seed=1)
    # queued before the scheduler starts: its first admissions form batches of
    # several requests whatever the timing
    futs = [srv.submit(f, g) for f, g in reqs]
    srv.start()
    srv.drain()
    srv.stop()
    for (f, g), fu in zip(reqs, futs):
        assert np.array_equal(fu.result(), oracle.conv_direct(f, g, M))
    assert srv.stats.peak_used <= 1 << 10
    assert srv.stats.completed == 120
    assert sorted(srv.admission_log) == list(srv.admission_log)    # arrival order
    assert max(srv.stats.batch_sizes) > 1                      # requests were batched
    assert srv.stats.percentile(50) <= srv.stats.percentile(99)


def test_admission_waits_for_memory():
    # capacity 2^8 elements: two 2^7 requests fill it; the third waits for a completion
    ex = FakeExecutor(M, delay=0.05)
    srv = ConvServer(ex, capacity_log2=8, max_inflight=4)
    reqs = _reqs(3, seed=2, lo=7, hi=7)
    futs = [srv.submit(f, g) for f, g in reqs]   # all queued before the first admission
    srv.start()
    srv.drain()
    srv.stop()
    assert [len(b) for b in ex.launches][0] == 2
    assert ex.launches[1] == [2]
    assert all(f.done() for f in futs)


def test_cancel_before_admission():
    ex = FakeExecutor(M, delay=0.05)
    srv = ConvServer(ex, capacity_log2=7, max_inflight=1).start()
    reqs = _reqs(4, seed=3, lo=7, hi=7)
    futs = [srv.submit(f, g) for f, g in reqs]
    time.sleep(0.01)
    assert srv.cancel(futs[3])
    srv.drain()
    srv.stop()
    assert futs[3].cancelled()
    assert all(3 not in b for b in ex.launches)
    assert all(f.done() for f in futs[:3])


def test_failed_launch_is_isolated():
    ex = FakeExecutor(M, delay=0.001, fail_on=5)
    srv = ConvServer(ex, capacity_log2=3, max_inflight=1).start()   # one 2^3 request per batch
    reqs = _reqs(10, seed=4, lo=3, hi=3)
    futs = [srv.submit(f, g) for f, g in reqs]
    srv.drain()
    srv.stop()
    with pytest.raises(RuntimeError):
        futs[5].result()
    for i, ((f, g), fu) in enumerate(zip(reqs, futs)):
        if i != 5:
            assert np.array_equal(fu.result(), oracle.conv_direct(f, g, M))
    assert srv.alloc.used == 0


def test_concurrent_clients():
    ex = FakeExecutor(M, delay=0.001)
    srv = ConvServer(ex, capacity_log2=11).start()
    reqs = _reqs(80, seed=5)
    futs = [None] * len(reqs)

    def client(idx):
        for i in idx:
            futs[i] = srv.submit(*reqs[i])

    ts = [threading.Thread(target=client, args=(range(k, 80, 4),)) for k in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    srv.drain()
    srv.stop()
    for (f, g), fu in zip(reqs, futs):
        assert np.array_equal(fu.result(), oracle.conv_direct(f, g, M))


def test_rejects_bad_requests():
    srv = ConvServer(FakeExecutor(M), capacity_log2=4)
    with pytest.raises(ValueError):
        srv.submit(np.zeros(6, np.uint64), np.zeros(6, np.uint64))
    with pytest.raises(ValueError):
        srv.submit(np.zeros(64, np.uint64), np.zeros(64, np.uint64))


def test_zero_copy_submission():
    ex = FakeExecutor(M)
    srv = ConvServer(ex, capacity_log2=9).start()
    reqs = _reqs(40, seed=9)
    futs = []
    for f, g in reqs:
        bf, bg, tok = srv.buffers(f.size)
        bf[...] = f
        bg[...] = g
        futs.append(srv.submit_staged(tok))
        with pytest.raises(ValueError):
            srv.submit_staged(tok)          # a token is submitted once
    srv.stop()
    for (f, g), fu in zip(reqs, futs):
        assert np.array_equal(fu.result(), oracle.conv_direct(f, g, M))
    for bad in (0, 12, 1024):
        with pytest.raises(ValueError):
            srv.buffers(bad)


def test_batch_element_cap():
    ex = FakeExecutor(M, delay=0.001)
    srv = ConvServer(ex, capacity_log2=10, max_batch_elems=256)
    reqs = _reqs(60, seed=4, lo=3, hi=9)                 # up to 512 elements: above the cap
    futs = [srv.submit(f, g) for f, g in reqs]
    srv.start()
    srv.stop()
    sizes = {r: f.size for r, (f, _) in enumerate(reqs)}
    for batch in ex.launches:
        total = sum(sizes[r] for r in batch)
        assert total <= 256 or len(batch) == 1
    assert [r for b in ex.launches for r in b] == list(range(60))     # arrival order kept
    for (f, g), fu in zip(reqs, futs):
        assert np.array_equal(fu.result(), oracle.conv_direct(f, g, M))


def test_long_requests_run_alone():
    # requests of 2^solo_log2n words and more close the batch being formed and
    # run as batches of their own; arrival order is kept
    ex = FakeExecutor(M, delay=0.001)
    srv = ConvServer(ex, capacity_log2=12, max_inflight=1, solo_log2n=6)
    rng = np.random.default_rng(9)
    sizes = [3, 6, 3, 3, 7, 3]
    reqs = [(rng.integers(0, M, 1 << k, dtype=np.uint64), rng.integers(0, M, 1 << k, dtype=np.uint64)) for k in sizes]
    futs = [srv.submit(f, g) for f, g in reqs]   # all queued before the first admission
    srv.start()
    srv.drain()
    srv.stop()
    assert ex.launches == [[0], [1], [2, 3], [4], [5]]
    for (f, g), fu in zip(reqs, futs):
        assert np.array_equal(fu.result(), oracle.conv_direct(f, g, M))
    # with the limit off every length shares a batch
    ex0 = FakeExecutor(M, delay=0.001)
    srv0 = ConvServer(ex0, capacity_log2=12, max_inflight=1, solo_log2n=0)
    for f, g in reqs:
        srv0.submit(f, g)
    srv0.start()
    srv0.drain()
    srv0.stop()
    assert ex0.launches == [[0, 1, 2, 3, 4, 5]]
