"""Served form on the GPU: continuous batching over several streams; every
served result equals the same request run alone (bit-exact), and the oracle."""
import time

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bits,m", [(64, si.M_U64), (32, si.M_13631489)])
def test_served_equals_alone(bits, m):
    import paper_1005_1497_amd as nt
    from paper_1005_1497_amd.serve import ConvServer, GpuExecutor
    rng = np.random.default_rng(7)
    lens = si.served_lengths(150, seed=5) if bits == 64 else rng.integers(6, 15, 150)
    dt = np.uint64 if bits == 64 else np.uint32
    reqs = [(rng.integers(0, m, 1 << int(n), dtype=dt), rng.integers(0, m, 1 << int(n), dtype=dt)) for n in lens]
    ex = GpuExecutor(m, capacity_log2=21, elem_bits=bits, streams=2)
    srv = ConvServer(ex, capacity_log2=21, max_inflight=4)
    # the first 16 requests queue before the scheduler starts, so its first
    # admission forms a batch of several whatever the timing of the box
    futs = [srv.submit(f, g) for f, g in reqs[:16]]
    srv.start()
    for i, (f, g) in enumerate(reqs[16:]):
        futs.append(srv.submit(f, g))
        if i % 10 == 9:
            time.sleep(0.0005)      # arrivals while earlier batches run
    srv.drain()
    srv.stop()
    assert srv.stats.completed == len(reqs)
    assert max(srv.stats.batch_sizes) > 1
    for (f, g), fu in zip(reqs, futs):
        alone = host(nt.conv_circular(dev(f), dev(g), m))
        assert np.array_equal(fu.result(), alone)
    for k in (0, len(reqs) // 2, len(reqs) - 1):
        f, g = reqs[k]
        idx = np.array([0, f.size - 1])
        assert np.array_equal(futs[k].result()[idx], oracle.conv_entries(f, g, m, idx).astype(dt))


def test_zero_copy_submission_and_result_lifetime():
    # operands written in place into the executor's pinned staging rows; the
    # results are views of pinned rows and must stay intact after later batches
    import paper_1005_1497_amd as nt
    from paper_1005_1497_amd.serve import ConvServer, GpuExecutor
    m = si.M_U64
    rng = np.random.default_rng(17)
    lens = si.served_lengths(120, seed=8)
    ex = GpuExecutor(m, capacity_log2=21, elem_bits=64, streams=2)
    srv = ConvServer(ex, capacity_log2=21, max_inflight=4).start()
    ops, futs = [], []
    for n in lens:
        N = 1 << int(n)
        bf, bg, tok = srv.buffers(N)
        bf[...] = rng.integers(0, m, N, dtype=np.uint64)
        bg[...] = rng.integers(0, m, N, dtype=np.uint64)
        ops.append((bf.copy(), bg.copy()))
        futs.append(srv.submit_staged(tok))
    first = [fu.result() for fu in futs[:10]]
    snap = [a.copy() for a in first]
    for f, g in ops[:40]:                       # more batches after the first results
        srv.submit(f, g)
    srv.drain()
    srv.stop()
    for a, b in zip(first, snap):
        assert np.array_equal(a, b)
    for (f, g), fu in zip(ops, futs):
        assert np.array_equal(fu.result(), host(nt.conv_circular(dev(f), dev(g), m)))


@pytest.mark.parametrize("host_arenas", [False, True])
@pytest.mark.parametrize("solo", [None, 0])
@pytest.mark.parametrize("bits,m", [(64, si.M_U64), (32, si.M_13631489)])
def test_native_server_equals_alone(bits, m, solo, host_arenas):
    # solo None: the default admission (requests of 2^16 words and more run as
    # batches of their own); 0: every length may share a batch.  host_arenas:
    # the slots are in pinned host arenas that the kernels read and write
    # directly (several chunks here: 200 staged requests exceed one)
    # the library's own scheduler thread: every result equals the request run
    # alone; two client threads submit at once; the oracle checks a few
    # entries.  Operands are staged first and the threads only queue them, so
    # the queue fills faster than a batch launches and batches form whatever
    # the timing of the box.
    import threading

    import paper_1005_1497_amd as nt
    from paper_1005_1497_amd.serve import NativeConvServer
    rng = np.random.default_rng(11)
    lens = si.served_lengths(200, seed=6) if bits == 64 else rng.integers(4, 16, 200)
    dt = np.uint64 if bits == 64 else np.uint32
    reqs = [(rng.integers(0, m, 1 << int(n), dtype=dt), rng.integers(0, m, 1 << int(n), dtype=dt)) for n in lens]
    with NativeConvServer(m, capacity_log2=21, elem_bits=bits, streams=4, max_batch_elems=1 << 19,
                          solo_log2n=solo, host_arenas=host_arenas) as srv:
        tickets = []
        for f, g in reqs:
            bf, bg, t = srv.stage(f.size)
            bf[...] = f
            bg[...] = g
            tickets.append(t)

        def client(part):
            for i in range(part, len(reqs), 2):
                srv.submit_staged(tickets[i])

        ths = [threading.Thread(target=client, args=(k,)) for k in range(2)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        outs = [srv.result(t, timeout=60.0) for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs)
    assert st["mean_batch"] > 1
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    for (f, g), o in zip(reqs, outs):
        assert np.array_equal(o, host(nt.conv_circular(dev(f), dev(g), m)))
    for k in (0, len(reqs) - 1):
        f, g = reqs[k]
        idx = np.array([0, f.size - 1])
        assert np.array_equal(outs[k][idx], oracle.conv_entries(f, g, m, idx).astype(dt))


def test_native_server_admission_and_shutdown():
    # an arena of 2^14 words and requests of 2^12..2^14: admission waits for
    # slots; tickets not waited for are released at shutdown
    import paper_1005_1497_amd as nt
    from paper_1005_1497_amd.serve import NativeConvServer
    m = si.M_13631489
    rng = np.random.default_rng(12)
    reqs = [(rng.integers(0, m, 1 << int(n), dtype=np.uint32), rng.integers(0, m, 1 << int(n), dtype=np.uint32))
            for n in rng.integers(12, 15, 40)]
    srv = NativeConvServer(m, capacity_log2=14, elem_bits=32, streams=2, max_inflight=2)
    tickets = [srv.submit(f, g) for f, g in reqs]
    for (f, g), t in list(zip(reqs, tickets))[:30]:
        assert np.array_equal(srv.result(t, timeout=60.0), host(nt.conv_circular(dev(f), dev(g), m)))
    with pytest.raises(nt.NttError) as e:
        srv.submit(np.zeros(1 << 15, np.uint32), np.zeros(1 << 15, np.uint32))    # larger than the arena
    assert e.value.name == "NTT_E_LENGTH"
    srv.close()                                   # ten tickets still pending


def test_native_server_host_arenas_submit_and_shutdown():
    # host arenas of 2^14-word chunks: every submission takes a slot at once
    # (new chunks as needed), results equal the requests run alone, a slot is
    # reused after its result is read, tickets not waited for are released at
    # shutdown
    import paper_1005_1497_amd as nt
    from paper_1005_1497_amd.serve import NativeConvServer
    m = si.M_13631489
    rng = np.random.default_rng(14)
    reqs = [(rng.integers(0, m, 1 << int(n), dtype=np.uint32), rng.integers(0, m, 1 << int(n), dtype=np.uint32))
            for n in rng.integers(4, 15, 60)]
    srv = NativeConvServer(m, capacity_log2=14, elem_bits=32, streams=2, max_inflight=2, host_arenas=True)
    tickets = [srv.submit(f, g) for f, g in reqs[:40]]
    for (f, g), t in list(zip(reqs, tickets))[:30]:
        assert np.array_equal(srv.result(t, timeout=60.0), host(nt.conv_circular(dev(f), dev(g), m)))
    more = [srv.submit(f, g) for f, g in reqs[40:]]
    for (f, g), t in zip(reqs[40:], more):
        assert np.array_equal(srv.result(t, timeout=60.0), host(nt.conv_circular(dev(f), dev(g), m)))
    with pytest.raises(nt.NttError) as e:
        srv.submit(np.zeros(1 << 15, np.uint32), np.zeros(1 << 15, np.uint32))    # larger than a chunk
    assert e.value.name == "NTT_E_LENGTH"
    bf, bg, t = srv.stage(1 << 10)
    f, g = rng.integers(0, m, 1 << 10, dtype=np.uint32), rng.integers(0, m, 1 << 10, dtype=np.uint32)
    bf[...] = f
    bg[...] = g
    srv.submit_staged(t)
    assert np.array_equal(srv.result(t, timeout=60.0), host(nt.conv_circular(dev(f), dev(g), m)))
    srv.close()                                   # ten tickets still pending


def test_native_server_zero_copy_submission():
    import paper_1005_1497_amd as nt
    from paper_1005_1497_amd.serve import NativeConvServer
    m = si.M_U64
    rng = np.random.default_rng(13)
    lens = si.served_lengths(60, seed=9)
    with NativeConvServer(m, capacity_log2=20, elem_bits=64, streams=2) as srv:
        ops, tickets = [], []
        for n in lens:
            N = 1 << int(n)
            bf, bg, t = srv.stage(N)
            bf[...] = rng.integers(0, m, N, dtype=np.uint64)
            bg[...] = rng.integers(0, m, N, dtype=np.uint64)
            ops.append((bf.copy(), bg.copy()))
            tickets.append(t)
        with pytest.raises(nt.NttError):
            srv.result(tickets[0], timeout=0.0)          # staged, never queued
        for t in tickets:
            srv.submit_staged(t)
        with pytest.raises(nt.NttError):
            srv.submit_staged(tickets[0])                # queued once only
        outs = [srv.result(t, timeout=60.0) for t in tickets]
    for (f, g), o in zip(ops, outs):
        assert np.array_equal(o, host(nt.conv_circular(dev(f), dev(g), m)))


@pytest.mark.parametrize("host_arenas", [False, True])
def test_native_server_cross_thread_waits(host_arenas):
    # four submitting threads and four waiting threads, tickets handed over
    # through a queue: every result equals the same convolution run alone
    # (host arenas: the submitters take slots, and new chunks, concurrently)
    import queue
    import threading

    import paper_1005_1497_amd as nt
    from paper_1005_1497_amd.serve import NativeConvServer
    m = si.M_13631489
    rng = np.random.default_rng(14)
    reqs = [(rng.integers(0, m, 1 << int(n), dtype=np.uint32), rng.integers(0, m, 1 << int(n), dtype=np.uint32))
            for n in rng.integers(4, 15, 240)]
    handoff = queue.Queue()
    results = {}
    with NativeConvServer(m, capacity_log2=19, elem_bits=32, streams=3, max_batch=64,
                          host_arenas=host_arenas) as srv:
        def submitter(k):
            for i in range(k, len(reqs), 4):
                handoff.put((i, srv.submit(*reqs[i])))

        def waiter():
            while True:
                item = handoff.get()
                if item is None:
                    return
                i, t = item
                results[i] = srv.result(t, timeout=60.0)

        subs = [threading.Thread(target=submitter, args=(k,)) for k in range(4)]
        waits = [threading.Thread(target=waiter) for _ in range(4)]
        for t in subs + waits:
            t.start()
        for t in subs:
            t.join()
        for _ in waits:
            handoff.put(None)
        for t in waits:
            t.join()
    assert len(results) == len(reqs)
    for i, (f, g) in enumerate(reqs):
        assert np.array_equal(results[i], host(nt.conv_circular(dev(f), dev(g), m))), i


@pytest.mark.parametrize("host_arenas", [False, True])
def test_native_server_one_waiter_per_ticket_and_timeout(host_arenas):
    # two threads wait for the same ticket: one gets the result, the other
    # NTT_E_ARG (the ticket is taken, or already released); a wait whose time
    # runs out reports NTT_E_TIMEOUT and leaves the ticket valid
    import threading

    import paper_1005_1497_amd as nt
    from paper_1005_1497_amd.serve import NativeConvServer
    m = si.M_13631489
    rng = np.random.default_rng(15)
    f, g = (rng.integers(0, m, 1 << 18, dtype=np.uint32) for _ in range(2))
    want = host(nt.conv_circular(dev(f), dev(g), m))
    with NativeConvServer(m, capacity_log2=19, elem_bits=32, streams=2, host_arenas=host_arenas) as srv:
        t = srv.submit(f, g)
        try:
            got = srv.result(t, timeout=0.0)
        except nt.NttError as e:
            assert e.name == "NTT_E_TIMEOUT"
            got = None
        if got is None:
            outcome = {}

            def waiter(k):
                try:
                    outcome[k] = srv.result(t, timeout=60.0)
                except nt.NttError as e:
                    outcome[k] = e.name
            ths = [threading.Thread(target=waiter, args=(k,)) for k in range(2)]
            for th in ths:
                th.start()
            for th in ths:
                th.join()
            wins = [v for v in outcome.values() if isinstance(v, np.ndarray)]
            assert len(wins) == 1 and sorted(v for v in outcome.values() if isinstance(v, str)) == ["NTT_E_ARG"]
            got = wins[0]
        assert np.array_equal(got, want)
