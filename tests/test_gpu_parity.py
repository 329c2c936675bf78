"""GPU parity: every result of the HIP path equals the oracle bit for bit.

The oracle is the O(N^2) definition (Eq. 1 direct sum; Eqs. 2, 3 as sums).
Integers and exact residues only, so the bar is equality (tolerance 0)."""
import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from tests.gpu_util import dev, host, root_of_order

pytestmark = pytest.mark.gpu

TABLE1 = [(641, 6), (2424833, 10), (319489, 12), (13631489, 19)]
M = 13631489


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def _cases(max_logn):
    for m, lognu in TABLE1:
        for n in range(0, min(lognu, max_logn) + 1):
            yield m, lognu, n


@pytest.mark.parametrize("m,lognu,n", list(_cases(12)))
def test_conv_small_all_table1(nt, m, lognu, n):
    N = 1 << n
    w = root_of_order(m, lognu, n)
    for seed in (0, 1):
        f = si.uniform(100 * n + seed, N, m)
        g = si.uniform(100 * n + seed + 50, N, m)
        h = host(nt.conv_circular(dev(f), dev(g), m, w))
        assert np.array_equal(h, oracle.conv_direct(f, g, m).astype(np.uint32)), (m, n, seed)


@pytest.mark.parametrize("m,lognu,n", list(_cases(12)))
def test_ntt_forward_inverse_small(nt, m, lognu, n):
    N = 1 << n
    w = root_of_order(m, lognu, n, odd=3 if n > 1 else 1)
    x = si.uniform(7 + n, 3 * N, m).reshape(3, N)
    X = host(nt.ntt_forward(dev(x), m, w))
    for r in range(3):
        assert np.array_equal(X[r], oracle.ntt(x[r], m, w).astype(np.uint32)), (m, n, r)
    xb = host(nt.ntt_inverse(dev(X), m, w))
    assert np.array_equal(xb, x)
    # the inverse alone against Eq. 3
    assert np.array_equal(xb[0], oracle.ntt(X[0], m, w, inverse=True).astype(np.uint32))


@pytest.mark.parametrize("n", [13, 14])
def test_conv_fourstep_full(nt, n):
    N = 1 << n
    w = root_of_order(M, 19, n)
    f = si.uniform(n, N, M)
    g = si.uniform(n + 1, N, M)
    h = host(nt.conv_circular(dev(f), dev(g), M, w))
    assert np.array_equal(h, oracle.conv_direct(f, g, M).astype(np.uint32))


@pytest.mark.parametrize("n", [13, 14])
def test_ntt_fourstep_full(nt, n):
    N = 1 << n
    w = root_of_order(M, 19, n, odd=5)
    x = si.uniform(n + 3, 2 * N, M).reshape(2, N)
    X = host(nt.ntt_forward(dev(x), M, w))
    for r in range(2):
        assert np.array_equal(X[r], oracle.ntt(x[r], M, w).astype(np.uint32))
    assert np.array_equal(host(nt.ntt_inverse(dev(X), M, w)), x)


@pytest.mark.parametrize("n", [15, 16, 17, 18, 19])
def test_conv_fourstep_sampled(nt, n):
    """Large single convolutions: sampled outputs against the O(N) direct sums,
    and the convolution theorem at random bins for the whole output."""
    N = 1 << n
    w = root_of_order(M, 19, n)
    f = si.uniform(2 * n, N, M)
    g = si.uniform(2 * n + 1, N, M)
    h = host(nt.conv_circular(dev(f), dev(g), M, w))
    rng = np.random.default_rng(n)
    idx = np.concatenate([[0, 1, N // 2, N - 1], rng.integers(0, N, 60)])
    assert np.array_equal(h[idx], oracle.conv_entries(f, g, M, idx).astype(np.uint32))
    bins = rng.integers(0, N, 4)
    Fb, Gb, Hb = (oracle.ntt_bins(a, M, w, bins) for a in (f, g, h))
    assert [(int(a) * int(b)) % M for a, b in zip(Fb, Gb)] == [int(c) for c in Hb]


@pytest.mark.parametrize("n", [15, 16, 19])
def test_ntt_fourstep_sampled(nt, n):
    N = 1 << n
    w = root_of_order(M, 19, n, odd=3)
    x = si.uniform(3 * n, N, M)
    X = host(nt.ntt_forward(dev(x), M, w))
    bins = np.concatenate([[0, 1, N - 1], np.random.default_rng(n).integers(0, N, 29)])
    assert np.array_equal(X[bins], oracle.ntt_bins(x, M, w, bins).astype(np.uint32))
    assert np.array_equal(host(nt.ntt_inverse(dev(X), M, w)), x)


def test_single_n1024_full():
    """N = 1024, m = 13631489, root 2^512 (the single-convolution workload)."""
    import paper_1005_1497_amd as nt
    w = si.single_n1024()
    f, g = si.operands(w)
    h = host(nt.conv_circular(dev(f), dev(g), w.m, nt.default_root(w.m, 10)))
    assert nt.default_root(w.m, 10) == 10252398
    assert np.array_equal(h, oracle.conv_direct(f, g, w.m).astype(np.uint32))


def test_n524288_exact_integer_convolution(nt):
    """N = 2^19 with values in {0..3}: the residues equal the true integer
    circular convolution (max 9 N < m), computed here with numpy's FFT."""
    w = si.single_n524288_small()
    f, g = si.operands(w)
    h = host(nt.conv_circular(dev(f), dev(g), w.m, 2))
    N = 1 << 19
    ref = np.rint(np.fft.irfft(np.fft.rfft(f.astype(np.float64)) * np.fft.rfft(g.astype(np.float64)), N))
    assert np.array_equal(h.astype(np.int64), ref.astype(np.int64))
    idx = np.array([0, 1, 12345, N - 1])
    assert np.array_equal(h[idx], oracle.conv_entries(f, g, w.m, idx).astype(np.uint32))


@pytest.mark.slow
def test_n524288_whole_output_against_integer_oracle(nt):
    """The same N = 2^19 convolution: every output against the oracle's direct
    integer sum (Eq. 1 without the modulus; exact because 9 N < m), an O(N^2)
    sum of 2.7e11 products on the host."""
    w = si.single_n524288_small()
    f, g = si.operands(w)
    h = host(nt.conv_circular(dev(f), dev(g), w.m, 2))
    assert np.array_equal(h.astype(np.uint64), oracle.conv_integer(f, g))


def test_inputs_above_m_are_reduced(nt):
    for n in (4, 10, 16):
        N = 1 << n
        f = si.uniform(5, N, 2 ** 32)
        g = si.uniform(6, N, 2 ** 32)
        h = host(nt.conv_circular(dev(f), dev(g), M, nt.default_root(M, n)))
        if n <= 10:
            assert np.array_equal(h, oracle.conv_direct(f, g, M).astype(np.uint32))
        else:
            idx = np.arange(0, N, 997)
            assert np.array_equal(h[idx], oracle.conv_entries(f, g, M, idx).astype(np.uint32))
        x = si.uniform(9, N, 2 ** 32)
        X = host(nt.ntt_forward(dev(x), M))
        bins = np.arange(0, N, max(1, N // 16))
        assert np.array_equal(X[bins], oracle.ntt_bins(x, M, nt.default_root(M, n), bins).astype(np.uint32))


@pytest.mark.parametrize("n", [0, 1, 3, 10, 16])
def test_special_inputs(nt, n):
    N = 1 << n
    w = nt.default_root(M, n)
    d0 = np.zeros(N, np.uint32); d0[0] = 1
    ones = np.ones(N, np.uint32)
    assert np.array_equal(host(nt.ntt_forward(dev(d0), M)), ones)
    e = np.zeros(N, np.uint32); e[0] = N % M
    assert np.array_equal(host(nt.ntt_forward(dev(ones), M)), e)
    g = si.uniform(n, N, M)
    for s in sorted({0, 1 % N, N - 1}):
        d = np.zeros(N, np.uint32); d[s] = 1
        assert np.array_equal(host(nt.conv_circular(dev(d), dev(g), M, w)), np.roll(g, s))
    mx = np.full(N, M - 1, np.uint32)
    if n <= 10:
        assert np.array_equal(host(nt.conv_circular(dev(mx), dev(mx), M, w)),
                              oracle.conv_direct(mx, mx, M).astype(np.uint32))


def test_in_place(nt):
    for n in (6, 10, 14):
        N = 1 << n
        f = si.uniform(1, N, M)
        g = si.uniform(2, N, M)
        ref = host(nt.conv_circular(dev(f), dev(g), M))
        tf, tg = dev(f), dev(g)
        nt.conv_circular(tf, tg, M, out=tf)
        assert np.array_equal(host(tf), ref)
        x = dev(f)
        nt.ntt_forward(x, M, out=x)
        nt.ntt_inverse(x, M, out=x)
        assert np.array_equal(host(x), f)


def test_check_range_flag(nt):
    N = 256
    f = si.uniform(1, N, M)
    g = si.uniform(2, N, M)
    nt.conv_circular(dev(f), dev(g), M, flags=nt.FLAG_CHECK_RANGE)
    f[17] = M
    with pytest.raises(nt.NttError) as e:
        nt.conv_circular(dev(f), dev(g), M, flags=nt.FLAG_CHECK_RANGE)
    assert e.value.name == "NTT_E_RANGE"
