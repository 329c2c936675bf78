"""Pins for the oracle, checked on the CPU against what the paper and the
mathematics fix, never against the oracle itself.

Each oracle routine is pinned by at least one check that a plausible mistake in
it (a dropped term, a wrong sign or index, a transposed operand, a wrong
normalisation, an overflow) would fail:

  powers / order   Fig. 1 sequences and N_Max; Table 1 N_Max; Sec. II (341, nu=10);
                   Prop. 1 (Fermat moduli); Prop. 2 proof (F_5 factors).
  is_prime         Table 1 primes; 341 composite; F_5 = 641 * 6700417; the printed
                   factorisations of 2^n - 1; a sieve of Eratosthenes.
  inverse          closed form N^-1 = 2^(nu - n) for the Rader primes; b*b^-1 = 1
                   checked with Python integers.
  ntt (Eq. 2, 3)   closed forms: delta_0 -> all ones, ones -> N*delta_0,
                   delta_1 -> root^u (fixes order and sign), linearity, round trip,
                   inverse of delta_1 -> N^-1 root^-t.
  conv_direct      numpy integer convolution folded mod N (exact small values);
                   shift by a delta; commutativity; Python big integers for the
                   45-bit prime.
  conv_via_ntt     equals conv_direct (convolution theorem) for every Table 1
                   prime and every N up to min(N_Max, 1024); independent of which
                   primitive N-th root is used.
  deconv_via_ntt   recovers g from f and conv_direct(f, g); brute force over all
                   g for tiny N; a shift by a delta undone; the all-ones
                   divisor (spectrum N*delta_0) reported singular.
  conv_integer     numpy integer circular convolution (np.convolve folded mod N)
                   and Python big integers; overflow past 2^64 reported.
  conv2d_direct    numpy 2-D circular convolution by shifted sums; a 1 x C
                   array reduces to conv_direct; separable operands give the
                   outer product of the 1-D convolutions.
  ntt_bins /       equal the matching entries of the full O(N^2) outputs.
  conv_entries
"""
import json
import os
import random

import numpy as np
import pytest

import oracle
import seeded_inputs as si

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


TABLE1 = gold("table1_rader_primes.json")["rows"]


def root_of_order(m, nu, N, odd=1):
    """2^k with k = (nu / N) * odd: an element of exact order N (Python pow)."""
    return pow(2, (nu // N) * odd, m)


# ---------------------------------------------------------------- digital circles
@pytest.mark.parametrize("c", gold("fig1_digital_circles.json")["circles"], ids=lambda c: c["panel"])
def test_fig1_digital_circles(c):
    seq = oracle.powers(c["a"], c["m"], len(c["sequence"]))
    assert seq.tolist() == c["sequence"]
    assert oracle.order(c["a"], c["m"]) == c["n_max"]


@pytest.mark.parametrize("row", TABLE1, ids=lambda r: str(r["m"]))
def test_table1_primes_and_orders(row):
    m = row["m"]
    assert oracle.is_prime(m)
    assert oracle.order(2, m) == row["n_max"]
    # m divides F_k = 2^(2^k) + 1, i.e. 2^(N_Max/2) = -1 (mod m), N_Max = 2^(k+1)
    assert row["n_max"] == 2 ** (row["fermat_index"] + 1)
    assert pow(2, row["n_max"] // 2, m) == m - 1
    # Euler form of Fermat factors, k * 2^(n+2) + 1 (Sec. III-A)
    assert (m - 1) % 2 ** (row["fermat_index"] + 2) == 0


def test_341_poulet():
    g = gold("carmichael_341.json")
    assert not oracle.is_prime(g["m"])
    assert int(np.prod(g["factors"])) == g["m"]
    assert all(oracle.is_prime(p) for p in g["factors"])
    assert oracle.order(2, g["m"]) == g["order_of_2"]
    assert int(np.prod(g["mersenne_2_10_minus_1_factors"])) == 2 ** 10 - 1
    assert pow(2, 340, 341) == 1


def test_prop2_fermat_f5_factors():
    g = gold("fermat_f5_factors.json")
    p, q = g["factors"]
    assert p * q == 2 ** 32 + 1
    assert oracle.is_prime(p) and oracle.is_prime(q)
    assert not oracle.is_prime(2 ** 32 + 1)
    assert oracle.order(2, p) == g["n_max"] and oracle.order(2, q) == g["n_max"]


@pytest.mark.parametrize("c", gold("fermat_moduli_prop1.json")["cases"], ids=lambda c: str(c["m"]))
def test_prop1_fermat_moduli(c):
    m = 2 ** (2 ** c["fermat_index"]) + 1
    assert m == c["m"]
    assert oracle.is_prime(m)
    assert oracle.order(2, m) == c["nu"]


def test_mersenne_factorisations():
    for n, facs in gold("mersenne_factorisations.json")["factorisations"].items():
        assert int(np.prod(facs)) == 2 ** int(n) - 1
        assert all(oracle.is_prime(p) for p in facs)


def test_is_prime_matches_sieve():
    lim = 20000
    sieve = np.ones(lim, dtype=bool)
    sieve[:2] = False
    for i in range(2, int(lim ** 0.5) + 1):
        if sieve[i]:
            sieve[i * i::i] = False
    got = np.array([oracle.is_prime(i) for i in range(lim)])
    assert np.array_equal(got, sieve)


def test_u64_rader_prime():
    """The 64-bit-word prime: prime, 2 of order 2^18, a factor of F_17."""
    m = si.M_U64
    assert m == 59251857 * 2 ** 19 + 1
    assert oracle.is_prime(m)
    assert oracle.order(2, m, limit=1 << 20) == si.M_U64_NMAX
    assert pow(2, 2 ** 17, m) == m - 1


def test_order_not_found_returns_zero():
    # 2 is not invertible mod 16: the walk never returns to 1
    assert oracle.order(2, 16, limit=1000) == 0


# ---------------------------------------------------------------- inverse
@pytest.mark.parametrize("row", TABLE1, ids=lambda r: str(r["m"]))
def test_inverse_closed_form(row):
    m, nu = row["m"], row["n_max"]
    n = 0
    while (1 << n) <= nu:
        # N^-1 = 2^-n = 2^(nu - n) because 2^nu = 1
        assert oracle.inverse(1 << n, m) == pow(2, nu - n, m)
        n += 1
    rng = random.Random(7)
    for _ in range(200):
        b = rng.randrange(1, m)
        assert (oracle.inverse(b, m) * b) % m == 1
    assert oracle.inverse(0, m) == 0


def test_inverse_no_inverse():
    assert oracle.inverse(11, 341) == 0
    assert oracle.inverse(6, 9) == 0


# ---------------------------------------------------------------- transform
def _cases(max_n=256):
    for row in TABLE1 + [{"m": si.M_U64, "n_max": si.M_U64_NMAX}]:
        N = 1
        while N <= min(row["n_max"], max_n):
            yield row["m"], row["n_max"], N
            N *= 2


@pytest.mark.parametrize("m,nu,N", list(_cases()))
def test_ntt_closed_forms(m, nu, N):
    w = root_of_order(m, nu, N)
    d0 = np.zeros(N, dtype=np.uint64); d0[0] = 1
    assert oracle.ntt(d0, m, w).tolist() == [1] * N
    ones = np.ones(N, dtype=np.uint64)
    exp = [0] * N; exp[0] = N % m
    assert oracle.ntt(ones, m, w).tolist() == exp
    if N > 1:
        d1 = np.zeros(N, dtype=np.uint64); d1[1] = 1
        # X(u) = root^(+u): pins the order of the outputs and the sign of Eq. 2
        assert oracle.ntt(d1, m, w).tolist() == [pow(w, u, m) for u in range(N)]
        # inverse of delta_1: N^-1 * root^(-t) (Eq. 3)
        ninv = pow(N, -1, m)
        winv = pow(w, -1, m)
        assert oracle.ntt(d1, m, w, inverse=True).tolist() == [ninv * pow(winv, t, m) % m for t in range(N)]
    rng = np.random.default_rng(N)
    x = rng.integers(0, m, N, dtype=np.uint64)
    y = rng.integers(0, m, N, dtype=np.uint64)
    X, Y = oracle.ntt(x, m, w), oracle.ntt(y, m, w)
    s = np.array([(int(a) + int(b)) % m for a, b in zip(x, y)], dtype=np.uint64)
    assert oracle.ntt(s, m, w).tolist() == [(int(a) + int(b)) % m for a, b in zip(X, Y)]
    assert oracle.ntt(X, m, w, inverse=True).tolist() == x.tolist()


def test_ntt_python_bigint_small():
    """Eq. 2 for a 45-bit modulus, where products need 90 bits: Python integers."""
    m, nu = si.M_U64, si.M_U64_NMAX
    for N in (2, 8, 32):
        w = root_of_order(m, nu, N, odd=3)
        x = [random.Random(N).randrange(m) for _ in range(N)]
        exp = [sum(x[t] * pow(w, u * t, m) for t in range(N)) % m for u in range(N)]
        assert oracle.ntt(x, m, w).tolist() == exp


def test_ntt_rejects_wrong_root():
    with pytest.raises(ValueError):
        oracle.ntt(np.arange(8), 13631489, 3)


def test_ntt_bins_match_full():
    m, nu, N = 13631489, 1 << 19, 512
    w = root_of_order(m, nu, N, odd=5)
    x = np.random.default_rng(3).integers(0, m, N, dtype=np.uint64)
    full = oracle.ntt(x, m, w)
    bins = np.array([0, 1, 2, 255, 256, 511, 77])
    assert oracle.ntt_bins(x, m, w, bins).tolist() == full[bins].tolist()


# ---------------------------------------------------------------- convolution
def _circular_int(f, g):
    """Exact integer circular convolution via numpy's linear convolution."""
    N = len(f)
    lin = np.convolve(np.asarray(f, dtype=np.int64), np.asarray(g, dtype=np.int64))
    out = lin[:N].copy()
    out[:N - 1] += lin[N:]
    return out


@pytest.mark.parametrize("N", [1, 2, 3, 8, 64, 1000])
def test_conv_direct_vs_numpy(N):
    m = 13631489
    rng = np.random.default_rng(N)
    f = rng.integers(0, 60, N)
    g = rng.integers(0, 60, N)
    assert oracle.conv_direct(f, g, m).tolist() == (_circular_int(f, g) % m).tolist()


def test_conv_direct_reduces_large_inputs():
    """Inputs are residues: values >= m behave like their remainders."""
    m, N = 641, 16
    rng = np.random.default_rng(1)
    f = rng.integers(0, 2 ** 63, N, dtype=np.uint64)
    g = rng.integers(0, 2 ** 63, N, dtype=np.uint64)
    fr = [int(v) % m for v in f]
    gr = [int(v) % m for v in g]
    assert oracle.conv_direct(f, g, m).tolist() == (_circular_int(fr, gr) % m).tolist()


def test_conv_direct_shift_and_commute():
    m, N = 13631489, 128
    rng = np.random.default_rng(2)
    g = rng.integers(0, m, N, dtype=np.uint64)
    f = rng.integers(0, m, N, dtype=np.uint64)
    for s in (0, 1, 5, 127):
        d = np.zeros(N, dtype=np.uint64); d[s] = 1
        assert oracle.conv_direct(d, g, m).tolist() == np.roll(g, s).tolist()
    assert oracle.conv_direct(f, g, m).tolist() == oracle.conv_direct(g, f, m).tolist()


def test_conv_direct_u64_bigint():
    m = si.M_U64
    for N in (4, 16, 64):
        r = random.Random(N)
        f = [r.randrange(m) for _ in range(N)]
        g = [r.randrange(m) for _ in range(N)]
        exp = [sum(f[k] * g[(j - k) % N] for k in range(N)) % m for j in range(N)]
        assert oracle.conv_direct(f, g, m).tolist() == exp


def _conv_cases():
    for row in TABLE1:
        N = 1
        while N <= min(row["n_max"], 1024):
            yield row["m"], row["n_max"], N
            N *= 2


@pytest.mark.parametrize("m,nu,N", list(_conv_cases()))
def test_convolution_theorem(m, nu, N):
    rng = np.random.default_rng(1000 + N)
    f = rng.integers(0, m, N, dtype=np.uint64)
    g = rng.integers(0, m, N, dtype=np.uint64)
    direct = oracle.conv_direct(f, g, m)
    assert oracle.conv_via_ntt(f, g, m, root_of_order(m, nu, N)).tolist() == direct.tolist()
    if N > 2:
        # any primitive N-th root gives the same convolution
        assert oracle.conv_via_ntt(f, g, m, root_of_order(m, nu, N, odd=3)).tolist() == direct.tolist()


def test_conv_entries_match_full():
    m, N = 13631489, 300
    rng = np.random.default_rng(9)
    f = rng.integers(0, m, N, dtype=np.uint64)
    g = rng.integers(0, m, N, dtype=np.uint64)
    full = oracle.conv_direct(f, g, m)
    idx = np.array([0, 1, 150, 299, 42])
    assert oracle.conv_entries(f, g, m, idx).tolist() == full[idx].tolist()


def test_worked_example_f17():
    """m = F_2 = 17 (Prop. 1), N = 8, root 2: the integer product of the
    polynomials 1+2x+3x^2+4x^3 and 5+6x+7x^2 reduced mod 17."""
    f = [1, 2, 3, 4, 0, 0, 0, 0]
    g = [5, 6, 7, 0, 0, 0, 0, 0]
    lin = np.convolve([1, 2, 3, 4], [5, 6, 7]).tolist()
    exp = [(lin[j] if j < len(lin) else 0) % 17 for j in range(8)]
    assert oracle.conv_via_ntt(f, g, 17, 2).tolist() == exp
    assert oracle.conv_direct(f, g, 17).tolist() == exp


# ---------------------------------------------------------------- Euler form
# Sec. I, Eq. 6 (Pollard's form by Euler's theorem): primes k*2^n + 1 whose
# roots of unity are not powers of two.  The root below is built here with
# Python integers (the smallest quadratic non-residue z, raised to (p-1)/N), and
# its order is checked against the definition before the oracle is trusted.
EULER_PRIMES = [(7340033, 20), (5767169, 19), (998244353, 23), (469762049, 26)]


def _euler_root(p, n):
    z = 2
    while pow(z, (p - 1) // 2, p) != p - 1:
        z += 1
    return pow(z, (p - 1) >> n, p)


@pytest.mark.parametrize("p,v2", EULER_PRIMES)
def test_euler_primes_and_root_order(p, v2):
    assert oracle.is_prime(p)
    assert (p - 1) % (1 << v2) == 0 and ((p - 1) >> v2) % 2 == 1
    w = _euler_root(p, 10)
    assert pow(w, 512, p) == p - 1 and pow(w, 1024, p) == 1
    assert oracle.order(w, p, 4096) == 1024
    # 2 itself is not a lambda-root of order 2^k for these primes
    o2 = oracle.order(2, p, 1 << 22)
    assert o2 == 0 or o2 & (o2 - 1) != 0


@pytest.mark.parametrize("p,v2", EULER_PRIMES)
@pytest.mark.parametrize("N", [1, 2, 8, 64])
def test_euler_convolution_theorem_and_closed_forms(p, v2, N):
    n = N.bit_length() - 1
    w = _euler_root(p, n)
    rng = np.random.default_rng(N + p % 97)
    dtype = np.uint64
    f = rng.integers(0, p, N, dtype=dtype)
    g = rng.integers(0, p, N, dtype=dtype)
    assert np.array_equal(oracle.conv_via_ntt(f, g, p, w), oracle.conv_direct(f, g, p))
    d1 = np.zeros(N, dtype)
    if N > 1:
        d1[1] = 1
        assert [int(v) for v in oracle.ntt(d1, p, w)] == [pow(w, u, p) for u in range(N)]
    x = rng.integers(0, p, N, dtype=dtype)
    assert np.array_equal(oracle.ntt(oracle.ntt(x, p, w), p, w, inverse=True), x)
    # the inverse includes N^-1: checked with Python integers
    X = oracle.ntt(x, p, w)
    t = N // 3
    ref = sum(int(X[u]) * pow(w, (-u * t) % N, p) for u in range(N)) * pow(N, p - 2, p) % p
    assert int(oracle.ntt(X, p, w, inverse=True)[t]) == ref



# ---------------------------------------------------------------- deconvolution
# Division filtering (Sec. III-A: the prime modulus makes every nonzero
# coefficient invertible).  Pinned by conv_direct (itself pinned above), by
# brute force, and by closed forms.
@pytest.mark.parametrize("m,nu", [(17, 8), (257, 16), (641, 64), (13631489, 524288)])
@pytest.mark.parametrize("N", [1, 2, 8, 32])
def test_deconv_recovers_g(m, nu, N):
    if N > nu:
        pytest.skip("N must divide nu")
    root = pow(2, nu // N, m)
    rng = np.random.default_rng(m % 1000 + N)
    g = rng.integers(0, m, N, dtype=np.uint64)
    for _ in range(50):
        f = rng.integers(0, m, N, dtype=np.uint64)
        try:
            out = oracle.deconv_via_ntt(f, oracle.conv_direct(f, g, m), m, root)
        except oracle.Singular:
            continue
        assert np.array_equal(out, g)
        return
    pytest.fail("no invertible divisor drawn")


def test_deconv_brute_force_tiny():
    # m = 17, N = 4, root 2^(8/4) = 4: the unique g with f * g = h among all 17^4
    m, N, root = 17, 4, 4
    f = [3, 1, 0, 5]
    h = [int(v) for v in oracle.conv_direct(np.array(f, np.uint64), np.array([2, 7, 11, 0], np.uint64), m)]
    sols = []
    for a in range(m):
        for b in range(m):
            for c in range(m):
                for d in range(m):
                    gg = (a, b, c, d)
                    if all(sum(f[k] * gg[(j - k) % N] for k in range(N)) % m == h[j] for j in range(N)):
                        sols.append(gg)
    assert sols == [(2, 7, 11, 0)]
    out = oracle.deconv_via_ntt(np.array(f, np.uint64), np.array(h, np.uint64), m, root)
    assert tuple(int(v) for v in out) == sols[0]


def test_deconv_shift_and_singular():
    m, nu, N = 13631489, 524288, 64
    root = pow(2, nu // N, m)
    h = np.random.default_rng(3).integers(0, m, N, dtype=np.uint64)
    d = np.zeros(N, np.uint64)
    d[5] = 1                                   # f = delta_5: g is h shifted back by 5
    assert np.array_equal(oracle.deconv_via_ntt(d, h, m, root), np.roll(h, -5))
    with pytest.raises(oracle.Singular):       # all ones: spectrum N * delta_0
        oracle.deconv_via_ntt(np.ones(N, np.uint64), h, m, root)



# ---------------------------------------------------------------- exact integers
@pytest.mark.parametrize("N,bits", [(1, 31), (8, 20), (64, 15), (256, 12)])
def test_conv_integer_vs_numpy(N, bits):
    rng = np.random.default_rng(N + bits)
    f = rng.integers(0, 1 << bits, N, dtype=np.uint64)
    g = rng.integers(0, 1 << bits, N, dtype=np.uint64)
    lin = np.convolve(f.astype(object), g.astype(object))
    ref = [0] * N
    for i, v in enumerate(lin):
        ref[i % N] += int(v)
    assert [int(v) for v in oracle.conv_integer(f, g)] == ref


def test_conv_integer_big_and_overflow():
    N = 16
    f = np.full(N, (1 << 32) - 1, np.uint64)
    g = np.full(N, (1 << 27) - 1, np.uint64)
    ref = N * ((1 << 32) - 1) * ((1 << 27) - 1)          # below 2^64
    assert all(int(v) == ref for v in oracle.conv_integer(f, g))
    with pytest.raises(ValueError):
        oracle.conv_integer(np.full(N, 1 << 62, np.uint64), np.full(N, 4, np.uint64))



def test_conv_integer_entries_match_full():
    rng = np.random.default_rng(77)
    N = 512
    f = rng.integers(0, 1 << 20, N, dtype=np.uint64)
    g = rng.integers(0, 1 << 20, N, dtype=np.uint64)
    idx = np.array([0, 1, 200, 511], np.uint64)
    assert np.array_equal(oracle.conv_integer_entries(f, g, idx), oracle.conv_integer(f, g)[idx.astype(int)])



# ---------------------------------------------------------------- 2-D convolution
def test_conv2d_vs_numpy_rolls():
    m = 13631489
    rng = np.random.default_rng(12)
    R, C = 4, 8
    f = rng.integers(0, 50, (R, C), dtype=np.uint64)
    g = rng.integers(0, 50, (R, C), dtype=np.uint64)
    ref = np.zeros((R, C), dtype=np.int64)
    for k in range(R):
        for l in range(C):
            ref += int(f[k, l]) * np.roll(np.roll(g.astype(np.int64), k, axis=0), l, axis=1)
    assert np.array_equal(oracle.conv2d_direct(f, g, m), (ref % m).astype(np.uint64))


def test_conv2d_reduces_to_1d_and_separates():
    m = 13631489
    rng = np.random.default_rng(13)
    a = rng.integers(0, m, 16, dtype=np.uint64)
    b = rng.integers(0, m, 16, dtype=np.uint64)
    assert np.array_equal(oracle.conv2d_direct(a[None, :], b[None, :], m)[0], oracle.conv_direct(a, b, m))
    assert np.array_equal(oracle.conv2d_direct(a[:, None], b[:, None], m)[:, 0], oracle.conv_direct(a, b, m))
    # separable: (p x q) conv (r x s) = conv(p, r) x conv(q, s), products mod m
    p, q = rng.integers(0, m, 8, dtype=np.uint64), rng.integers(0, m, 4, dtype=np.uint64)
    r, s = rng.integers(0, m, 8, dtype=np.uint64), rng.integers(0, m, 4, dtype=np.uint64)
    outer = lambda x, y: np.array([[int(u) * int(v) % m for v in y] for u in x], dtype=np.uint64)
    lhs = oracle.conv2d_direct(outer(p, q), outer(r, s), m)
    assert np.array_equal(lhs, outer(oracle.conv_direct(p, r, m), oracle.conv_direct(q, s, m)))
    idx = np.array([0, 5, 31], np.uint64)
    assert np.array_equal(oracle.conv2d_entries(outer(p, q), outer(r, s), m, idx), lhs.ravel()[idx.astype(int)])


# ---------------------------------------------------------------- batched and 2-D bins
def test_ntt_bins_rows_match_single_rows_and_deltas():
    # every row's bins equal ntt_bins of that row (pinned above against the full
    # O(N^2) transform); a delta at s gives X(u) = root^(u s) (Eq. 2)
    m, nu, N, rows = 13631489, 1 << 19, 256, 5
    w = root_of_order(m, nu, N, odd=3)
    rng = np.random.default_rng(8)
    x = rng.integers(0, m, (rows, N), dtype=np.uint64)
    bins = rng.integers(0, N, (rows, 4)).astype(np.uint64)
    got = oracle.ntt_bins_rows(x, m, w, bins)
    for r in range(rows):
        assert got[r].tolist() == oracle.ntt_bins(x[r], m, w, bins[r]).tolist()
    d = np.zeros((rows, N), np.uint64)
    for r in range(rows):
        d[r, 7 * r + 1] = 1
    got = oracle.ntt_bins_rows(d, m, w, bins)
    for r in range(rows):
        assert got[r].tolist() == [pow(w, int(u) * (7 * r + 1), m) for u in bins[r]]


def test_ntt2d_bins_closed_forms():
    m, nu = 13631489, 1 << 19
    R, C = 8, 16
    wr, wc = root_of_order(m, nu, R), root_of_order(m, nu, C, odd=5)
    rng = np.random.default_rng(9)
    bu = rng.integers(0, R, 12).astype(np.uint64)
    bv = rng.integers(0, C, 12).astype(np.uint64)
    # a delta at (k0, l0): X(u, v) = wr^(u k0) wc^(v l0)
    d = np.zeros((R, C), np.uint64)
    d[3, 11] = 1
    assert oracle.ntt2d_bins(d, m, wr, wc, bu, bv).tolist() == \
        [pow(wr, 3 * int(u), m) * pow(wc, 11 * int(v), m) % m for u, v in zip(bu, bv)]
    # separable: outer(a, b) -> A(u) B(v), with the 1-D transforms of Eq. 2
    a = rng.integers(0, m, R, dtype=np.uint64)
    b = rng.integers(0, m, C, dtype=np.uint64)
    outer = np.array([[int(p) * int(q) % m for q in b] for p in a], dtype=np.uint64)
    A, B = oracle.ntt(a, m, wr), oracle.ntt(b, m, wc)
    assert oracle.ntt2d_bins(outer, m, wr, wc, bu, bv).tolist() == \
        [int(A[int(u)]) * int(B[int(v)]) % m for u, v in zip(bu, bv)]
    # the 2-D convolution theorem against the direct 2-D sum
    f = rng.integers(0, m, (R, C), dtype=np.uint64)
    g = rng.integers(0, m, (R, C), dtype=np.uint64)
    h = oracle.conv2d_direct(f, g, m)
    F, G, H = (oracle.ntt2d_bins(x, m, wr, wc, bu, bv) for x in (f, g, h))
    assert [int(p) * int(q) % m for p, q in zip(F, G)] == [int(z) for z in H]


def test_conv_integer_full_matches_entries_at_wrap():
    # the index of g read modulo N, at the split between k <= j and k > j
    rng = np.random.default_rng(78)
    N = 64
    f = rng.integers(0, 1 << 28, N, dtype=np.uint64)
    g = rng.integers(0, 1 << 28, N, dtype=np.uint64)
    full = oracle.conv_integer(f, g)
    for j in (0, 1, N // 2, N - 1):
        assert int(full[j]) == sum(int(f[k]) * int(g[(j - k) % N]) for k in range(N))
