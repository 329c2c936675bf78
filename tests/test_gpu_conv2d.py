"""GPU parity of the 2-D circular convolution (row transforms, transpose,
column transforms, product, inverses) against the oracle's direct 2-D sum:
full outputs for small arrays, sampled outputs for large ones, with the row
lengths on both the LDS (<= 2^12) and the four-step (> 2^12) paths."""
import numpy as np
import pytest
import torch

import oracle
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


@pytest.mark.parametrize("r,c", [(0, 0), (0, 5), (5, 0), (3, 3), (6, 5), (4, 9), (9, 4), (7, 7)])
def test_conv2d_full(nt, r, c):
    R, C = 1 << r, 1 << c
    rng = np.random.default_rng(r * 31 + c)
    f = rng.integers(0, M, (R, C), dtype=np.uint32)
    g = rng.integers(0, M, (R, C), dtype=np.uint32)
    h = host(nt.conv2d(dev(f), dev(g), M)).reshape(R, C)
    assert np.array_equal(h, oracle.conv2d_direct(f, g, M).astype(np.uint32))


@pytest.mark.parametrize("r,c", [(2, 14), (13, 3), (10, 10), (6, 13)])
def test_conv2d_sampled(nt, r, c):
    R, C = 1 << r, 1 << c
    rng = np.random.default_rng(r * 37 + c)
    f = rng.integers(0, M, (R, C), dtype=np.uint32)
    g = rng.integers(0, M, (R, C), dtype=np.uint32)
    h = host(nt.conv2d(dev(f), dev(g), M)).reshape(-1)
    idx = np.unique(np.r_[0, R * C - 1, rng.integers(0, R * C, 6)]).astype(np.uint64)
    assert np.array_equal(h[idx.astype(int)], oracle.conv2d_entries(f, g, M, idx).astype(np.uint32))


def test_conv2d_in_place_u64_and_euler(nt):
    rng = np.random.default_rng(5)
    f = rng.integers(0, M, (32, 64), dtype=np.uint32)
    g = rng.integers(0, M, (32, 64), dtype=np.uint32)
    fd = dev(f)
    nt.conv2d(fd, dev(g), M, out=fd)                       # h written over f
    assert np.array_equal(host(fd).reshape(32, 64), oracle.conv2d_direct(f, g, M).astype(np.uint32))
    m64 = si.M_U64
    a = rng.integers(0, m64, (16, 32), dtype=np.uint64)
    b = rng.integers(0, m64, (16, 32), dtype=np.uint64)
    assert np.array_equal(host(nt.conv2d(dev(a), dev(b), m64)).reshape(16, 32), oracle.conv2d_direct(a, b, m64))
    me = 7340033
    a = rng.integers(0, me, (64, 16), dtype=np.uint32)
    b = rng.integers(0, me, (64, 16), dtype=np.uint32)
    got = host(nt.conv2d(dev(a), dev(b), me, flags=nt.FLAG_EULER)).reshape(64, 16)
    assert np.array_equal(got, oracle.conv2d_direct(a, b, me).astype(np.uint32))


def test_conv2d_benched_size_by_2d_bins(nt):
    # the timed 2-D workload itself, 4096 x 4096 uniform in [0, m): the 2-D
    # convolution theorem H(u, v) = F(u, v) G(u, v) at 16 random bins, each
    # bin the oracle's O(R C) double sum of the 2-D transform (Eq. 2 along each
    # dimension), which involves every output; plus sampled direct sums
    R = C = 4096
    rng = np.random.default_rng(10)
    f = rng.integers(0, M, (R, C), dtype=np.uint32)
    g = rng.integers(0, M, (R, C), dtype=np.uint32)
    h = host(nt.conv2d(dev(f), dev(g), M)).reshape(R, C)
    w = pow(2, (1 << 19) // 4096, M)                     # exact order 4096
    bu = np.r_[0, 1, 2048, rng.integers(0, R, 13)].astype(np.uint64)
    bv = np.r_[0, 4095, 1, rng.integers(0, C, 13)].astype(np.uint64)
    F, G, H = (oracle.ntt2d_bins(x, M, w, w, bu, bv) for x in (f, g, h))
    assert [int(a) * int(b) % M for a, b in zip(F, G)] == [int(c) for c in H]
    idx = np.array([0, R * C - 1, 12345678], np.uint64)
    assert np.array_equal(h.reshape(-1)[idx.astype(int)], oracle.conv2d_entries(f, g, M, idx).astype(np.uint32))
