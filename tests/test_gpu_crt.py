"""GPU parity of the exact integer convolution by residue (CRT) arithmetic:
convolutions modulo 13631489 and 7340033 combined into the true integer
circular convolution (oracle: the direct integer sum, full up to 2^12 and on
sampled outputs above), including values far beyond either prime."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

M1, M2 = 13631489, 7340033


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def _bits_for(n):
    # operands below 2^b with N * 2^(2b) below m1 * m2: the result is exact
    return (46 - n) // 2


@pytest.mark.parametrize("n,rows", [(0, 3), (3, 5), (10, 2), (12, 1), (13, 2), (16, 1), (19, 1)])
def test_crt_matches_integer_oracle(nt, n, rows):
    N = 1 << n
    b = _bits_for(n)
    rng = np.random.default_rng(n + 40)
    f = rng.integers(0, 1 << b, (rows, N), dtype=np.uint32)
    g = rng.integers(0, 1 << b, (rows, N), dtype=np.uint32)
    h = host(nt.conv_crt(dev(f), dev(g))).reshape(rows, N)
    for r in range(rows):
        if n <= 12:
            assert np.array_equal(h[r], oracle.conv_integer(f[r], g[r])), (n, r)
        else:
            idx = np.unique(np.r_[0, N - 1, rng.integers(0, N, 10)]).astype(np.uint64)
            assert np.array_equal(h[r][idx.astype(int)], oracle.conv_integer_entries(f[r], g[r], idx)), (n, r)
    # the results really exceed both primes (the combination is doing work)
    assert n < 4 or h.max() > M1


def test_crt_extreme_values(nt):
    # every output at the top of the exact range: N = 2^10 and operands 2^18 - 1
    N = 1 << 10
    f = np.full(N, (1 << 18) - 1, np.uint32)
    g = np.full(N, (1 << 18) - 1, np.uint32)
    h = host(nt.conv_crt(dev(f), dev(g)))
    assert np.all(h == N * ((1 << 18) - 1) ** 2)
    assert N * ((1 << 18) - 1) ** 2 < M1 * M2
