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


@pytest.mark.parametrize("kind", ["uniform16", "fused14", "uneven"])
def test_graph_replay_matches_eager(nt, kind):
    if kind == "uniform16":
        lengths = (16,) * 40            # few items: the multi-launch four-step form
    elif kind == "fused14":
        lengths = (14,) * 600           # enough items for the persistent fused kernel
    else:
        lengths = tuple(si.uneven_batch(count=50, seed=7).log2n)
    offs = si.offsets(lengths)
    w = si.Workload("graph", M, lengths, 32, M, 21)
    f_h, g_h = si.operands(w)
    f, g = dev(f_h), dev(g_h)
    desc = nt.BatchDesc(lengths, offs)
    before = nt.launch_counts()
    ref = host(nt.conv_batched(f, g, desc, M))
    torch.cuda.synchronize()
    form = {"uniform16": "fourstep", "fused14": "fused"}.get(kind)
    if form:
        assert nt.launch_counts()[form] == before[form] + 1

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


def test_graph_survives_workspace_growth_and_descriptor_churn(nt):
    # after capture, eager calls on the same stream outgrow the workspace and
    # push more than the descriptor cache's 256 entries through it; the graph's
    # workspace is retired (not freed) and its descriptors are kept, so the
    # replay still reads live memory and reproduces the eager result
    lengths = tuple(si.uneven_batch(count=30, seed=9).log2n) + (16, 9, 16)
    offs = si.offsets(lengths)
    w = si.Workload("graph3", M, lengths, 32, M, 23)
    f_h, g_h = si.operands(w)
    f, g = dev(f_h), dev(g_h)
    desc = nt.BatchDesc(lengths, offs)
    before = nt.launch_counts()
    ref = host(nt.conv_batched(f, g, desc, M))
    # (the two items of 2^16 apart: the multi-length launch and its descriptor)
    assert nt.launch_counts()["multi"] == before["multi"] + 1
    stream = torch.cuda.Stream()
    h = torch.zeros_like(f)
    graph = _capture(nt, f, g, desc, h, stream)
    torch.cuda.synchronize()

    # a larger workspace on the capture stream: 64 items of 2^19 (64 resident
    # workgroups of 4 MB scratch each, above the 30-item batch's)
    big = torch.zeros(64 << 19, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(stream):
        nt.conv_batched(big, big, nt.BatchDesc([19] * 64, si.offsets([19] * 64)), M, out=big.clone(),
                        stream=stream)
    # 300 distinct descriptors through the cache (one length, two items apart:
    # each needs an offset list), more than its 256 entries, so it evicts
    small = torch.zeros(1 << 15, dtype=torch.int32, device="cuda")
    before = nt.launch_counts()
    with torch.cuda.stream(stream):
        for i in range(300):
            nt.conv_batched(small, small, nt.BatchDesc([5, 5], [0, 64 + 64 * i]), M, out=small.clone(),
                            stream=stream)
    torch.cuda.synchronize()
    after = nt.launch_counts()
    assert after["desc_cached"] - before["desc_cached"] == 300
    assert after["desc_evicted"] > before["desc_evicted"]
    for rep in range(2):
        h.fill_(-1)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(h), ref), rep
