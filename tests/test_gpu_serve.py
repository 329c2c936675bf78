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
