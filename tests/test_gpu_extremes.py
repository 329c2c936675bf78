"""GPU parity at extreme operand values through every long-length kernel.

Random operands keep the values inside a transform far from the bounds that
the kernels' exact fp64 arithmetic rests on (a radix-16 pass output reaches
16 (m/2 + 2) only when its sixteen inputs line up).  Constant operands near
m/2, and sequences that are pure tones c w^(-u0 t), reach those bounds in the
first passes, and their convolutions have closed forms that hold at any N
(Eq. 1 summed directly):
  constants a, b:              h(j) = N a b mod m
  tones a w^(-u0 t), b w^(-u0 t): h(j) = N a b w^(-u0 j) mod m
  tone (u0 != 0) with a constant: h = 0
Every output is compared with its closed form, and a few entries with the
oracle's direct sum.  The launch counters confirm which kernel ran: the
multi-launch four-step form (k_fs_*), the persistent fused kernel
(k_conv_fused), the multi-length kernel (k_conv_multi)."""
import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

M = 13631489
LOGNU = 19
M64 = si.M_U64          # 31065037602817, the 45-bit Rader prime (order of 2: 2^18)
LOGNU64 = 18


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def extremes(m, bits):
    """Word values whose residues sit at the ends of the centred range, and the
    all-ones word (read modulo m)."""
    return [(m - 1) // 2, (m + 1) // 2, m - 1, (1 << bits) - 1]


def tone(N, c, u0, w, m):
    """c w^(-u0 t) mod m for t < N (Python integers)."""
    z = pow(w, (N - u0) % N, m)          # w^(-u0)
    out, x = [], c % m
    for _ in range(N):
        out.append(x)
        x = x * z % m
    return out


def counts_delta(nt, before):
    after = nt.launch_counts()
    return {k: after[k] - before[k] for k in after}


def check_entries(h, f, g, m, idx):
    ref = oracle.conv_entries(f, g, m, idx)
    assert np.array_equal(h[idx].astype(np.uint64), ref), idx


@pytest.mark.parametrize("n", [13, 14, 15, 16, 17, 18, 19])
def test_single_convolution_extremes_fourstep(nt, n):
    N = 1 << n
    w = pow(2, 1 << (LOGNU - n), M)
    ext = extremes(M, 32)
    pairs = [(ext[0], ext[0]), (ext[1], ext[2]), (ext[3], ext[3]), (ext[2], ext[2])]
    for a, b in pairs:
        f = np.full(N, a, np.uint32)
        g = np.full(N, b, np.uint32)
        before = nt.launch_counts()
        h = host(nt.conv_circular(dev(f), dev(g), M, w))
        assert counts_delta(nt, before)["fourstep"] == 1
        assert np.all(h == (N * (a % M) * (b % M)) % M), (a, b)
        check_entries(h, f, g, M, np.array([0, N - 1]))
    # tones at the Nyquist bin (alternating signs) and at a random bin
    for u0 in (N // 2, 12345 % N):
        c = (M - 1) // 2
        f = np.array(tone(N, c, u0, w, M), np.uint32)
        g = np.array(tone(N, c, u0, w, M), np.uint32)
        h = host(nt.conv_circular(dev(f), dev(g), M, w))
        want = np.array(tone(N, N * c * c, u0, w, M), np.uint32)
        assert np.array_equal(h, want), u0
        const = np.full(N, (M + 1) // 2, np.uint32)
        h0 = host(nt.conv_circular(dev(f), dev(const), M, w))
        assert np.all(h0 == 0), u0


def _uniform_batch(nt, n, count, m, bits, lognu, expect):
    """count items of 2^n: item i holds the constants (ext[i % 4], ext[i // 4 % 4]),
    every 7th item a pair of tones; all outputs against the closed forms."""
    N = 1 << n
    w = pow(2, 1 << (lognu - n), m)
    ext = extremes(m, bits)
    dt = np.uint32 if bits == 32 else np.uint64
    f = np.empty(count * N, dt)
    g = np.empty(count * N, dt)
    want = np.empty(count * N, dt)
    c = (m - 1) // 2
    tf = np.array(tone(N, c, N // 2 + 3, w, m), dt)
    tw = np.array(tone(N, N * c * c, N // 2 + 3, w, m), dt)
    for i in range(count):
        s = slice(i * N, (i + 1) * N)
        if i % 7 == 3:
            f[s], g[s], want[s] = tf, tf, tw
        else:
            a, b = ext[i % 4], ext[(i // 4) % 4]
            f[s], g[s] = a, b
            want[s] = (N * (a % m) * (b % m)) % m
    desc = nt.BatchDesc([n] * count, si.offsets([n] * count))
    before = nt.launch_counts()
    h = host(nt.conv_batched(dev(f), dev(g), desc, m))
    d = counts_delta(nt, before)
    assert d[expect] == 1, (expect, d)
    bad = np.nonzero(h != want)[0]
    assert bad.size == 0, ("item", int(bad[0]) // N, "entry", int(bad[0]) % N)
    for i in (0, 3, count - 1):
        s = slice(i * N, (i + 1) * N)
        check_entries(h[s], f[s], g[s], m, np.array([0, N // 2 + 1]))


@pytest.mark.parametrize("n,count", [(13, 600), (14, 600), (15, 600), (16, 600), (17, 300), (18, 300), (19, 300)])
def test_batch_extremes_fused(nt, n, count):
    # enough items that the persistent fused kernel runs (fewer than two thirds
    # of its resident workgroups would take the four-step form)
    _uniform_batch(nt, n, count, M, 32, LOGNU, "fused")


def test_batch_extremes_multi_length(nt):
    # several lengths with scattered items of the long ones: the single
    # multi-length launch, its four-step items and its LDS tiles
    rng = np.random.default_rng(70)
    lengths = [int(x) for x in rng.integers(6, 20, 140)] + [19, 19, 18, 18, 13, 13]
    rng.shuffle(lengths)
    ext = extremes(M, 32)
    offs = si.offsets(lengths)
    total = int(offs[-1]) + (1 << lengths[-1])
    f = np.empty(total, np.uint32)
    g = np.empty(total, np.uint32)
    want = np.empty(total, np.uint32)
    c = (M - 1) // 2
    for i, (n, o) in enumerate(zip(lengths, offs)):
        N, o = 1 << n, int(o)
        s = slice(o, o + N)
        if i % 5 == 2 and n >= 2:
            w = pow(2, 1 << (LOGNU - n), M)
            t = np.array(tone(N, c, N // 2 + 1, w, M), np.uint32)
            f[s], g[s] = t, t
            want[s] = np.array(tone(N, N * c * c, N // 2 + 1, w, M), np.uint32)
        else:
            a, b = ext[i % 4], ext[(i // 3) % 4]
            f[s], g[s] = a, b
            want[s] = (N * (a % M) * (b % M)) % M
    desc = nt.BatchDesc(lengths, offs)
    before = nt.launch_counts()
    h = host(nt.conv_batched(dev(f), dev(g), desc, M))
    assert counts_delta(nt, before)["multi"] == 1
    bad = np.nonzero(h != want)[0]
    assert bad.size == 0, int(bad[0])


@pytest.mark.parametrize("n", [13, 16, 18])
def test_u64_extremes(nt, n):
    # the 45-bit prime with 64-bit words: constants at the ends of the range and
    # all-ones words, one convolution (four-step) and a batch (fused kernel)
    N = 1 << n
    w = pow(2, 1 << (LOGNU64 - n), M64)
    ext = extremes(M64, 64)
    for a, b in [(ext[0], ext[0]), (ext[1], ext[2]), (ext[3], ext[3])]:
        f = np.full(N, a, np.uint64)
        g = np.full(N, b, np.uint64)
        h = host(nt.conv_circular(dev(f), dev(g), M64, w))
        assert np.all(h == (N * (a % M64) * (b % M64)) % M64), (a, b)
        check_entries(h, f, g, M64, np.array([0, N - 1]))
    _uniform_batch(nt, n, 300 if n <= 16 else 200, M64, 64, LOGNU64, "fused")
