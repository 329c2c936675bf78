"""CPU records of the readings of the paper that decide what is built.

Sec. III-B, Eq. 13: an odd a satisfies a^(2^(alpha - 2)) = 1 modulo 2^alpha,
and the paper proposes transforms modulo 2^alpha with such roots ("modulus
free", overflow as the reduction) that would preserve the circular
convolution property.  Brute force shows that they do not: for every root of
exact order N = 4 or 8 modulo 2^alpha, alpha in {4, 8, 16, 32}, the sums
sum_t a^(k t) for 0 < k < N are not 0 modulo 2^alpha, and the transform-based
product differs from N times the circular convolution (Eq. 1) for delta inputs.
The build therefore does not implement that transform (the other transforms
use a prime modulus, where these sums vanish)."""
import itertools

import pytest


def _roots_of_exact_order(N, alpha):
    """Every a modulo 2^alpha with a^N = 1 and a^(N/2) != 1 (brute force over the
    odd residues for alpha <= 16; for alpha = 32 over the group structure
    {+-1} x <5>, in which these are +-5^(2^(alpha-2)/N * odd))."""
    mod = 1 << alpha
    if alpha <= 16:
        return [a for a in range(1, mod, 2) if pow(a, N, mod) == 1 and pow(a, N // 2, mod) != 1]
    step = (1 << (alpha - 2)) // N
    out = set()
    for j in range(1, N, 2):
        r = pow(5, step * j, mod)
        out.update({r, mod - r})
    return sorted(a for a in out if pow(a, N, mod) == 1 and pow(a, N // 2, mod) != 1)


def _transform(x, a, N, mod):
    return [sum(x[t] * pow(a, u * t, mod) for t in range(N)) % mod for u in range(N)]


@pytest.mark.parametrize("alpha", [4, 8, 16, 32])
@pytest.mark.parametrize("N", [4, 8])
def test_modulus_free_transform_breaks_the_convolution_property(alpha, N):
    mod = 1 << alpha
    if N > 1 << (alpha - 2):
        pytest.skip("no element of order N modulo 2^alpha")
    roots = _roots_of_exact_order(N, alpha)
    assert roots, (N, alpha)
    # Eq. 13 itself holds for every odd a
    assert all(pow(a, 1 << (alpha - 2), mod) == 1 for a in roots)
    for a in roots:
        # orthogonality fails: some sum_t a^(k t), 0 < k < N, is nonzero mod 2^alpha
        sums = [sum(pow(a, k * t, mod) for t in range(N)) % mod for k in range(1, N)]
        assert any(s != 0 for s in sums), (a, alpha, N)
        # and the convolution theorem (unnormalised inverse = N * (f * g)) fails
        # for some pair of deltas
        broken = False
        for i, j in itertools.product(range(N), repeat=2):
            f = [1 if t == i else 0 for t in range(N)]
            g = [1 if t == j else 0 for t in range(N)]
            F, G = _transform(f, a, N, mod), _transform(g, a, N, mod)
            inv = pow(a, N - 1, mod)                       # a^-1 (a has order N)
            H = [F[u] * G[u] % mod for u in range(N)]
            h = [sum(H[u] * pow(inv, u * t, mod) for u in range(N)) % mod for t in range(N)]
            want = [N if t == (i + j) % N else 0 for t in range(N)]
            if h != want:
                broken = True
                break
        assert broken, (a, alpha, N)


def test_prime_modulus_keeps_the_convolution_property():
    # the same check with the Rader prime 17 = F_2 (2 has order 8): the sums
    # vanish and the theorem holds for every pair of deltas
    m, N, a = 17, 8, 2
    assert all(sum(pow(a, k * t, m) for t in range(N)) % m == 0 for k in range(1, N))
    inv = pow(a, N - 1, m)
    for i, j in itertools.product(range(N), repeat=2):
        f = [1 if t == i else 0 for t in range(N)]
        g = [1 if t == j else 0 for t in range(N)]
        F, G = _transform(f, a, N, m), _transform(g, a, N, m)
        H = [F[u] * G[u] % m for u in range(N)]
        h = [sum(H[u] * pow(inv, u * t, m) for u in range(N)) % m for t in range(N)]
        assert h == [N if t == (i + j) % N else 0 for t in range(N)]
