"""Graph capture of the batched convolution: a conv_batched call captured in a
HIP graph (after a warm-up call on the capture stream has built its plans and
workspaces) replays bit-identically to the eager call, replay after replay,
with eager work and new operand values in between."""
import numpy as np
import pytest
import torch

import seeded_inputs as si
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

M = 13631489


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def _capture(nt, f, g, desc, h, stream):
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        nt.conv_batched(f, g, desc, M, out=h, stream=stream)   # warm-up on the capture stream
    stream.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        nt.conv_batched(f, g, desc, M, out=h, stream=stream)
    return graph


@pytest.mark.parametrize("kind", ["uniform16", "uneven"])
def test_graph_replay_matches_eager(nt, kind):
    if kind == "uniform16":
        lengths = (16,) * 40
    else:
        lengths = tuple(si.uneven_batch(count=50, seed=7).log2n)
    offs = si.offsets(lengths)
    w = si.Workload("graph", M, lengths, 32, M, 21)
    f_h, g_h = si.operands(w)
    f, g = dev(f_h), dev(g_h)
    desc = nt.BatchDesc(lengths, offs)
    ref = host(nt.conv_batched(f, g, desc, M))
    torch.cuda.synchronize()

    stream = torch.cuda.Stream()
    h = torch.zeros_like(f)
    graph = _capture(nt, f, g, desc, h, stream)
    torch.cuda.synchronize()
    for rep in range(4):
        h.fill_(-1)                    # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(h), ref), rep

    # new operand values in the captured buffers: the replay follows them
    w2 = si.Workload("graph2", M, lengths, 32, M, 22)
    f2_h, g2_h = si.operands(w2)
    ref2 = host(nt.conv_batched(dev(f2_h), dev(g2_h), desc, M))
    f.copy_(dev(f2_h))
    g.copy_(dev(g2_h))
    torch.cuda.synchronize()
    for rep in range(2):
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(h), ref2), rep
