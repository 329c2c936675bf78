"""GPU parity for 64-bit words: the 45-bit Rader prime 31065037602817
(59251857 * 2^19 + 1, a factor of F_17, order of 2 equal to 2^18), bit-exact
against the oracle (whose products are exact 128-bit integers)."""
import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from tests.gpu_util import dev, host, root_of_order

pytestmark = pytest.mark.gpu

M = si.M_U64
LOGNU = 18


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def u64(seed, n, hi=M):
    return np.random.default_rng(seed).integers(0, hi, size=n, dtype=np.uint64)


@pytest.mark.parametrize("n", list(range(0, 13)))
def test_conv_u64_small(nt, n):
    N = 1 << n
    w = root_of_order(M, LOGNU, n)
    f, g = u64(n, N), u64(n + 100, N)
    h = host(nt.conv_circular(dev(f), dev(g), M, w))
    assert np.array_equal(h, oracle.conv_direct(f, g, M))


@pytest.mark.parametrize("n", [0, 1, 4, 9, 12, 13, 14])
def test_ntt_u64_full(nt, n):
    N = 1 << n
    w = root_of_order(M, LOGNU, n, odd=3 if n > 1 else 1)
    x = u64(7 * n + 1, 2 * N).reshape(2, N)
    X = host(nt.ntt_forward(dev(x), M, w))
    for r in range(2):
        assert np.array_equal(X[r], oracle.ntt(x[r], M, w))
    assert np.array_equal(host(nt.ntt_inverse(dev(X), M, w)), x)


@pytest.mark.parametrize("n", [13, 15, 16, 18])
def test_conv_u64_large_sampled(nt, n):
    N = 1 << n
    w = root_of_order(M, LOGNU, n)
    f, g = u64(3 * n, N), u64(3 * n + 1, N)
    h = host(nt.conv_circular(dev(f), dev(g), M, w))
    rng = np.random.default_rng(n)
    idx = np.concatenate([[0, N - 1], rng.integers(0, N, 30)])
    assert np.array_equal(h[idx], oracle.conv_entries(f, g, M, idx))
    bins = rng.integers(0, N, 3)
    Fb, Gb, Hb = (oracle.ntt_bins(a, M, w, bins) for a in (f, g, h))
    assert [(int(a) * int(b)) % M for a, b in zip(Fb, Gb)] == [int(c) for c in Hb]


def test_u64_inputs_full_range(nt):
    """Any 64-bit value is read modulo m."""
    for n in (5, 11, 14):
        N = 1 << n
        f = np.random.default_rng(n).integers(0, 2 ** 64 - 1, size=N, dtype=np.uint64)
        g = np.random.default_rng(n + 1).integers(0, 2 ** 64 - 1, size=N, dtype=np.uint64)
        h = host(nt.conv_circular(dev(f), dev(g), M))
        idx = np.arange(0, N, max(1, N // 64))
        assert np.array_equal(h[idx], oracle.conv_entries(f, g, M, idx))


def test_u64_batched_uneven(nt):
    log2n = [8, 12, 9, 14, 8, 13, 16]
    offs = si.offsets(log2n)
    total = int(offs[-1]) + (1 << log2n[-1])
    f, g = u64(1, total), u64(2, total)
    desc = nt.BatchDesc(log2n, offs)
    h = host(nt.conv_batched(dev(f), dev(g), desc, M))
    h1 = host(nt.conv_batched(dev(f), dev(g), desc, M, flags=nt.FLAG_PER_ITEM))
    assert np.array_equal(h, h1)
    for n, o in zip(log2n, offs):
        N, o = 1 << n, int(o)
        idx = np.array([0, N // 2, N - 1])
        assert np.array_equal(h[o + idx], oracle.conv_entries(f[o:o + N], g[o:o + N], M, idx)), n


def test_u64_uniform_batch_fused(nt):
    n, count = 14, 40
    N = 1 << n
    f, g = u64(5, N * count), u64(6, N * count)
    desc = nt.BatchDesc([n] * count, si.offsets([n] * count))
    h = host(nt.conv_batched(dev(f), dev(g), desc, M))
    for i in (0, 17, count - 1):
        idx = np.array([0, 5, N - 1])
        assert np.array_equal(h[i * N + idx], oracle.conv_entries(f[i * N:(i + 1) * N], g[i * N:(i + 1) * N], M, idx))


def test_u64_single_launch_with_longer_class(nt):
    # 64-bit words with m = 13631489 (nu = 2^19): lengths up to 2^18 go into
    # the single persistent launch, 2^19 gets its own launch
    m = 13631489
    lengths = [19, 18, 5, 16, 12, 13, 9, 19, 1]
    offs = si.offsets(lengths)
    w = si.Workload("u64mix", m, tuple(lengths), 64, m, 41)
    f, g = si.operands(w)
    desc = nt.BatchDesc(lengths, offs)
    one = host(nt.conv_batched(dev(f), dev(g), desc, m))
    per_item = host(nt.conv_batched(dev(f), dev(g), desc, m, flags=nt.FLAG_PER_ITEM))
    assert np.array_equal(one, per_item)
    rng = np.random.default_rng(9)
    for n, o in zip(lengths, offs):
        N, o = 1 << n, int(o)
        idx = rng.integers(0, N, 4)
        ref = oracle.conv_entries(f[o:o + N], g[o:o + N], m, idx)
        assert np.array_equal(one[o + idx], ref.astype(np.uint64)), n
