"""GPU parity of the multi-launch four-step kernels in the launch shapes where
their row kernels take several row blocks per workgroup (rows of 512 and more
positions in a convolution, 2048 in a natural-order transform, with enough
items that the launch narrows its grid), and of the two workgroup sizes (a
batch whose 512-thread column blocks fill the chip keeps them; one item runs
256-thread blocks), each checked against the one-item launches and the oracle
(Eq. 1 sampled per item; Eq. 2 on sampled bins of every row; Eq. 3 through the
round trip)."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

M = 13631489


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def _delta(nt, before):
    after = nt.launch_counts()
    return {k: after[k] - before[k] for k in after}


@pytest.mark.parametrize("n,count", [(17, 100), (18, 96), (19, 128)])
def test_fourstep_batch_with_row_loops(nt, n, count):
    N = 1 << n
    rng = np.random.default_rng(100 + n)
    f = rng.integers(0, M, count * N, dtype=np.uint32)
    g = rng.integers(0, M, count * N, dtype=np.uint32)
    desc = nt.BatchDesc([n] * count, [i * N for i in range(count)])
    before = nt.launch_counts()
    h = host(nt.conv_batched(dev(f), dev(g), desc, M))
    torch.cuda.synchronize()
    # fewer items than two thirds of the fused kernel's resident workgroups:
    # the multi-launch four-step form ran
    assert _delta(nt, before)["fourstep"] == 1
    h1 = host(nt.conv_batched(dev(f), dev(g), desc, M, flags=nt.FLAG_PER_ITEM))
    assert np.array_equal(h, h1)
    for i in (0, 1, count // 2, count - 1):
        idx = np.unique(np.concatenate([[0, 1, N // 2, N - 1], rng.integers(0, N, 12)])).astype(np.uint64)
        ref = oracle.conv_entries(f[i * N:(i + 1) * N], g[i * N:(i + 1) * N], M, idx)
        assert np.array_equal(h[i * N + idx.astype(np.int64)], ref.astype(np.uint32)), i


def test_ntt_rows_with_row_loops(nt):
    n, rows = 19, 128
    N = 1 << n
    rng = np.random.default_rng(19)
    x = rng.integers(0, M, (rows, N), dtype=np.uint32)
    X = nt.ntt_forward(dev(x), M)
    Xh = host(X)
    root = nt.default_root(M, n)
    bins = rng.integers(0, N, (rows, 4)).astype(np.uint64)
    bins[:, 0] = 0
    bins[:, 1] = N - 1
    ref = oracle.ntt_bins_rows(x, M, root, bins)
    got = np.take_along_axis(Xh, bins.astype(np.int64), axis=1)
    assert np.array_equal(got, ref.astype(np.uint32))
    y = host(nt.ntt_inverse(X, M))
    assert np.array_equal(y, x)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("n,count", [(13, 150), (14, 100), (15, 100), (16, 100)])
def test_fourstep_workgroup_sizes_agree(nt, n, count, bits):
    # count is large enough that the batch's 512-thread column blocks give
    # every CU one, and below two thirds of the fused kernel's residency, so
    # the batch runs the 512-thread four-step kernels; each item alone
    # (FLAG_PER_ITEM) runs the 256-thread ones
    import seeded_inputs as si
    m = M if bits == 32 else si.M_U64
    dt = np.uint32 if bits == 32 else np.uint64
    N = 1 << n
    rng = np.random.default_rng(200 + n + bits)
    f = rng.integers(0, m, count * N, dtype=dt)
    g = rng.integers(0, m, count * N, dtype=dt)
    f[:N] = m - 1                      # item 0 at the top of the canonical range
    desc = nt.BatchDesc([n] * count, [i * N for i in range(count)])
    before = nt.launch_counts()
    h = host(nt.conv_batched(dev(f), dev(g), desc, m))
    assert _delta(nt, before)["fourstep"] == 1
    h1 = host(nt.conv_batched(dev(f), dev(g), desc, m, flags=nt.FLAG_PER_ITEM))
    assert np.array_equal(h, h1)
    for i in (0, count - 1):
        idx = np.unique(np.concatenate([[0, 1, N // 2, N - 1], rng.integers(0, N, 12)])).astype(np.uint64)
        ref = oracle.conv_entries(f[i * N:(i + 1) * N], g[i * N:(i + 1) * N], m, idx)
        assert np.array_equal(h[i * N + idx.astype(np.int64)], ref.astype(dt)), i
    # transforms: 64 rows (512-thread blocks from 2^15 on) against one row
    x = rng.integers(0, m, (64, N), dtype=dt)
    X = host(nt.ntt_forward(dev(x), m))
    X0 = host(nt.ntt_forward(dev(x[:1]), m))
    assert np.array_equal(X[:1], X0)
    assert np.array_equal(host(nt.ntt_inverse(dev(X0), m)), x[:1])
