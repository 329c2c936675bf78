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


def test_crt_benched_size_batch(nt):
    # the timed CRT workload itself: 4096 x N = 2^16 with 15-bit operands (every
    # true value below 2^46 < m1 m2, so h is the exact integer convolution).
    # Every item: the exact integer identity sum_j h(j) = (sum f)(sum g), and
    # the convolution theorem modulo each prime at two random bins (the
    # oracle's O(N) transform sums, Eq. 2, with a root of exact order 2^16
    # modulo m1 and modulo m2); sampled entries against the direct integer sum
    count, n = 4096, 16
    N = 1 << n
    rng = np.random.default_rng(9)
    f = rng.integers(0, 1 << 15, (count, N), dtype=np.uint32)
    g = rng.integers(0, 1 << 15, (count, N), dtype=np.uint32)
    h = host(nt.conv_crt(dev(f), dev(g))).reshape(count, N)
    sf = f.sum(axis=1, dtype=np.uint64)
    sg = g.sum(axis=1, dtype=np.uint64)
    assert np.array_equal(h.sum(axis=1, dtype=np.uint64), sf * sg)       # < 2^62, no wrap
    assert h.max() < M1 * M2
    bins = np.random.default_rng(91).integers(1, N, (count, 2)).astype(np.uint64)
    r1 = pow(2, (1 << 19) // N, M1)
    z = next(z for z in range(2, 100) if pow(z, (M2 - 1) // 2, M2) == M2 - 1)
    r2 = pow(z, (M2 - 1) // N, M2)
    assert pow(r2, N // 2, M2) == M2 - 1 and pow(r1, N // 2, M1) == M1 - 1
    for m, r in ((M1, r1), (M2, r2)):
        Fb = oracle.ntt_bins_rows(f, m, r, bins)
        Gb = oracle.ntt_bins_rows(g, m, r, bins)
        Hb = oracle.ntt_bins_rows(h % np.uint64(m), m, r, bins)
        prod = (Fb.astype(object) * Gb.astype(object)) % m
        assert np.array_equal(prod.astype(np.uint64), Hb), m
    for i in (0, 2048, count - 1):
        idx = np.array([0, 1, N - 1], np.uint64)
        assert np.array_equal(h[i][idx.astype(int)], oracle.conv_integer_entries(f[i], g[i], idx)), i
