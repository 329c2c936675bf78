"""GPU parity of the Euler (Pollard) form of Sec. I, Eq. 6 (NTT_FLAG_EULER):
primes k*2^n + 1 of which 2 is not a lambda-root, roots of unity that are not
powers of two, and lengths beyond the order of 2 for a Rader prime.  Every
result is compared bit for bit with the oracle (whose root is passed in)."""
import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nt():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1005_1497_amd as nt
    return nt


def _draw(seed, n, m, bits):
    dtype = np.uint32 if bits == 32 else np.uint64
    rng = np.random.default_rng(seed)
    return rng.integers(0, m, 1 << n, dtype=dtype), rng.integers(0, m, 1 << n, dtype=dtype)


CASES = [
    (7340033, 32, [0, 1, 4, 10, 12, 13, 16, 19, 20]),     # 7 * 2^20 + 1
    (5767169, 32, [6, 11, 14, 17]),                       # 11 * 2^19 + 1
    (13631489, 32, [20]),                                 # Rader prime, root of order 2^20 (not a power of 2)
    (998244353, 64, [3, 9, 12, 15, 18, 22]),              # 119 * 2^23 + 1
]


@pytest.mark.parametrize("m,bits,n", [(m, b, n) for m, b, ns in CASES for n in ns])
def test_euler_conv_matches_oracle(nt, m, bits, n):
    w = nt.euler_root(m, n)
    f, g = _draw(100 + n, n, m, bits)
    h = host(nt.conv_circular(dev(f), dev(g), m, root=w, flags=nt.FLAG_EULER))
    N = 1 << n
    if n <= 12:
        assert np.array_equal(h, oracle.conv_direct(f, g, m).astype(h.dtype)), (m, n)
    else:
        idx = np.unique(np.r_[0, N - 1, np.random.default_rng(n).integers(0, N, 10)])
        assert np.array_equal(h[idx], oracle.conv_entries(f, g, m, idx).astype(h.dtype)), (m, n)


@pytest.mark.parametrize("m,bits,n", [(7340033, 32, 9), (7340033, 32, 14), (998244353, 64, 11),
                                      (998244353, 64, 16)])
def test_euler_transforms_match_oracle(nt, m, bits, n):
    w = nt.euler_root(m, n)
    x, _ = _draw(200 + n, n, m, bits)
    X = nt.ntt_forward(dev(x), m, root=w, flags=nt.FLAG_EULER)
    Xh = host(X)
    N = 1 << n
    if n <= 12:
        assert np.array_equal(Xh, oracle.ntt(x, m, w).astype(Xh.dtype))
    else:
        bins = np.unique(np.r_[0, 1, N - 1, np.random.default_rng(n).integers(0, N, 12)])
        assert np.array_equal(Xh[bins], oracle.ntt_bins(x, m, w, bins).astype(Xh.dtype))
    back = host(nt.ntt_inverse(X, m, root=w, flags=nt.FLAG_EULER))
    assert np.array_equal(back, x)


def test_euler_batched_uneven(nt):
    m, v = 7340033, 20
    root = nt.euler_root(m, v)
    lengths = [20, 3, 12, 13, 16, 19, 7, 7, 0, 15]
    offs = si.offsets(lengths)
    w = si.Workload("euler", m, tuple(lengths), 32, m, 61)
    f, g = si.operands(w)
    desc = nt.BatchDesc(lengths, offs)
    one = host(nt.conv_batched(dev(f), dev(g), desc, m, root=root, root_log2order=v, flags=nt.FLAG_EULER))
    per_item = host(nt.conv_batched(dev(f), dev(g), desc, m, root=root, root_log2order=v,
                                    flags=nt.FLAG_EULER | nt.FLAG_PER_ITEM))
    assert np.array_equal(one, per_item)
    for n, o in zip(lengths, offs):
        N, o = 1 << n, int(o)
        idx = np.unique(np.r_[0, N - 1, np.random.default_rng(n + 1).integers(0, N, 4)])
        assert np.array_equal(one[o + idx], oracle.conv_entries(f[o:o + N], g[o:o + N], m, idx).astype(np.uint32)), n


def test_rader_prime_unchanged_without_flag(nt):
    # without the flag a prime of which 2 is not a lambda-root is refused
    x = dev(np.zeros(16, np.uint32))
    with pytest.raises(nt.NttError) as e:
        nt.ntt_forward(x, 7340033, root=nt.euler_root(7340033, 4))
    assert e.value.name == "NTT_E_MODULUS"
