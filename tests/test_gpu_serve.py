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
    srv = ConvServer(ex, capacity_log2=21, max_inflight=4).start()
    futs = []
    for i, (f, g) in enumerate(reqs):
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
