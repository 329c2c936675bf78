/*
 * Oracle for exact digital circular convolution modulo m.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It is deliberately plain and slow: every routine is the
 * textbook definition written out, in exact integer arithmetic (products in
 * unsigned 128-bit, reduced with the % operator), with no blocking, fusion or
 * reordering beyond what the definition states.
 *
 * Paper: S. S. Chandra, "Fast Digital Convolutions using Bit-Shifts"
 * (arXiv:1005.1497).  Each routine cites the passage it follows.
 *
 * Conventions
 *   - All arrays are uint64_t.  Input elements may be any 64-bit value; they are
 *     interpreted modulo m (the % in every product does this).
 *   - Outputs are canonical residues in [0, m) (Appendix A, Sino notation).
 *   - Routines that can fail return a nonzero int; they never abort.
 *   - OpenMP parallelises the outer loop over output indices only; every output
 *     is still the plain sum in index order.
 */
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* <a*b>_m, exact (Appendix A). */
static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)(((u128)a * (u128)b) % m);
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of OpenMP threads for the parallel loops that follow (timing the
 * oracle on one core and on all of them). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Primality by trial division with every odd d <= sqrt(m).  The method picks
 * m prime so that every nonzero residue has a multiplicative inverse
 * (Sec. III-A). */
int oracle_is_prime(uint64_t m) {
    if (m < 2) return 0;
    if (m % 2 == 0) return m == 2;
    for (uint64_t d = 3; d <= m / d; d += 2)
        if (m % d == 0) return 0;
    return 1;
}

/* The digital circle of a modulo m (Eq. 5 and Fig. 1): out[i] = a^i mod m for
 * i < count, each term obtained from the previous one by one more factor a
 * (for a = 2 this is doubling). */
void oracle_powers(uint64_t a, uint64_t m, uint64_t count, uint64_t *out) {
    uint64_t x = 1 % m;
    for (uint64_t i = 0; i < count; ++i) {
        out[i] = x;
        x = mulmod(x, a, m);
    }
}

/* Order nu of a modulo m: the smallest nu >= 1 with a^nu = 1 (mod m)
 * (Eq. 7, Sec. II).  Walks the circle of Eq. 5 until it returns to 1.
 * Returns 0 when the walk has not returned within `limit` steps (for example
 * when gcd(a, m) != 1, where it never does). */
uint64_t oracle_order(uint64_t a, uint64_t m, uint64_t limit) {
    if (m == 1) return 1;
    uint64_t x = 1;
    for (uint64_t k = 1; k <= limit; ++k) {
        x = mulmod(x, a, m);
        if (x == 1) return k;
    }
    return 0;
}

/* Multiplicative inverse b^-1 modulo m by the extended Euclidean algorithm
 * (Appendix A).  Returns 0 when gcd(b, m) != 1 (no inverse). */
uint64_t oracle_inverse(uint64_t b, uint64_t m) {
    __int128 r0 = (__int128)m, r1 = (__int128)(b % m);
    __int128 s0 = 0, s1 = 1;
    while (r1 != 0) {
        __int128 q = r0 / r1;
        __int128 t = r0 - q * r1; r0 = r1; r1 = t;
        t = s0 - q * s1; s0 = s1; s1 = t;
    }
    if (r0 != 1) return 0;
    s0 %= (__int128)m;
    if (s0 < 0) s0 += (__int128)m;
    return (uint64_t)s0;
}

/* Transform of Eq. 2 (inverse = 0) or Eq. 3 (inverse = 1), evaluated as the
 * O(N^2) sum, with `root` as the N-th root of unity in place of 2 (Eq. 2 is
 * the case N = N_Max, root = 2):
 *     forward  X(u) = < sum_t x(t) * root^(u t) >_m
 *     inverse  x(t) = < N^-1 * sum_u X(u) * root^(-u t) >_m
 * root^(-e) is root^(N - e mod N) (the exponent is read modulo N, Sec. I), and
 * N^-1 comes from the extended Euclidean algorithm (Appendix A).
 * Returns 1 if root is not an N-th root of unity, 2 if N has no inverse,
 * 3 on allocation failure. */
int oracle_ntt(const uint64_t *x, uint64_t *X, uint64_t N, uint64_t m,
               uint64_t root, int inverse) {
    if (N == 0) return 0;
    uint64_t *P = (uint64_t *)malloc((size_t)(N + 1) * sizeof(uint64_t));
    if (!P) return 3;
    oracle_powers(root, m, N + 1, P);
    if (P[N] != 1 % m) { free(P); return 1; }
    uint64_t ninv = 1 % m;
    if (inverse) {
        ninv = oracle_inverse(N % m, m);
        if (ninv == 0) { free(P); return 2; }
    }
    long long n = (long long)N;
#pragma omp parallel for schedule(dynamic, 16)
    for (long long u = 0; u < n; ++u) {
        u128 acc = 0;
        for (uint64_t t = 0; t < N; ++t) {
            uint64_t e = ((uint64_t)u * t) % N;
            if (inverse) e = (N - e) % N;
            acc += (u128)mulmod(x[t], P[e], m);
        }
        uint64_t s = (uint64_t)(acc % m);
        X[u] = inverse ? mulmod(s, ninv, m) : s;
    }
    free(P);
    return 0;
}

/* Selected outputs of the forward transform of Eq. 2: out[i] = X(bins[i]).
 * Each is the O(N) sum over t with root^(u t) built up one factor at a time.
 * Used to check single outputs of very long transforms. */
int oracle_ntt_bins(const uint64_t *x, uint64_t N, uint64_t m, uint64_t root,
                    const uint64_t *bins, uint64_t nbins, uint64_t *out) {
    long long nb = (long long)nbins;
#pragma omp parallel for schedule(dynamic, 1)
    for (long long i = 0; i < nb; ++i) {
        /* z = root^u by repeated multiplication, then sum_t x(t) z^t */
        uint64_t u = bins[i] % (N ? N : 1), z = 1 % m;
        for (uint64_t k = 0; k < u; ++k) z = mulmod(z, root, m);
        u128 acc = 0;
        uint64_t zt = 1 % m;
        for (uint64_t t = 0; t < N; ++t) {
            acc += (u128)mulmod(x[t], zt, m);
            zt = mulmod(zt, z, m);
        }
        out[i] = (uint64_t)(acc % m);
    }
    return 0;
}

/* Selected outputs of the forward transform of Eq. 2 for each of `rows`
 * contiguous length-N sequences: out[r * nbins + i] = X_r(bins[r * nbins + i]),
 * each the O(N) sum of oracle_ntt_bins (the same root for every row). */
int oracle_ntt_bins_rows(const uint64_t *x, uint64_t rows, uint64_t N, uint64_t m, uint64_t root,
                         const uint64_t *bins, uint64_t nbins, uint64_t *out) {
    long long total = (long long)(rows * nbins);
#pragma omp parallel for schedule(dynamic, 4)
    for (long long q = 0; q < total; ++q) {
        const uint64_t r = (uint64_t)q / nbins;
        const uint64_t *xr = x + r * N;
        uint64_t u = bins[q] % (N ? N : 1), z = 1 % m;
        for (uint64_t k = 0; k < u; ++k) z = mulmod(z, root, m);
        u128 acc = 0;
        uint64_t zt = 1 % m;
        for (uint64_t t = 0; t < N; ++t) {
            acc += (u128)mulmod(xr[t], zt, m);
            zt = mulmod(zt, z, m);
        }
        out[q] = (uint64_t)(acc % m);
    }
    return 0;
}

/* Selected outputs of the two-dimensional transform of an R x C array
 * (row-major): Eq. 2 applied along each dimension with its own root,
 *     X(u, v) = < sum_{k<R} sum_{l<C} x(k, l) root_r^(u k) root_c^(v l) >_m,
 * out[i] = X(bu[i], bv[i]), each the O(R C) double sum (inner sum over l). */
int oracle_ntt2d_bins(const uint64_t *x, uint64_t R, uint64_t C, uint64_t m, uint64_t root_r,
                      uint64_t root_c, const uint64_t *bu, const uint64_t *bv, uint64_t nbins, uint64_t *out) {
    for (uint64_t i = 0; i < nbins; ++i) {
        uint64_t u = bu[i] % (R ? R : 1), v = bv[i] % (C ? C : 1);
        uint64_t zr = 1 % m, zc = 1 % m;
        for (uint64_t k = 0; k < u; ++k) zr = mulmod(zr, root_r, m);
        for (uint64_t k = 0; k < v; ++k) zc = mulmod(zc, root_c, m);
        /* zc^l for l < C, and the row sums S_k = sum_l x(k, l) zc^l */
        uint64_t *pc = (uint64_t *)malloc((size_t)(C ? C : 1) * sizeof(uint64_t));
        uint64_t *S = (uint64_t *)malloc((size_t)(R ? R : 1) * sizeof(uint64_t));
        if (!pc || !S) { free(pc); free(S); return 3; }
        oracle_powers(zc, m, C, pc);
        long long rr = (long long)R;
#pragma omp parallel for schedule(dynamic, 16)
        for (long long k = 0; k < rr; ++k) {
            u128 acc = 0;
            for (uint64_t l = 0; l < C; ++l) acc += (u128)mulmod(x[(uint64_t)k * C + l], pc[l], m);
            S[k] = (uint64_t)(acc % m);
        }
        u128 acc = 0;
        uint64_t zk = 1 % m;
        for (uint64_t k = 0; k < R; ++k) {
            acc += (u128)mulmod(S[k], zk, m);
            zk = mulmod(zk, zr, m);
        }
        out[i] = (uint64_t)(acc % m);
        free(pc); free(S);
    }
    return 0;
}

/* Circular convolution of Eq. 1, the O(N^2) direct sum:
 *     h(j) = < sum_{k<N} f(k) * g((j - k) mod N) >_m
 * (the index of g is read modulo N: the sequences are periodic, Sec. I). */
void oracle_conv_direct(const uint64_t *f, const uint64_t *g, uint64_t *h,
                        uint64_t N, uint64_t m) {
    long long n = (long long)N;
#pragma omp parallel for schedule(dynamic, 16)
    for (long long j = 0; j < n; ++j) {
        u128 acc = 0;
        for (uint64_t k = 0; k < N; ++k) {
            uint64_t idx = ((uint64_t)j + N - k) % N;
            acc += (u128)mulmod(f[k], g[idx], m);
        }
        h[j] = (uint64_t)(acc % m);
    }
}

/* Selected outputs of Eq. 1: out[i] = h(idx[i]), each the O(N) direct sum. */
void oracle_conv_entries(const uint64_t *f, const uint64_t *g, uint64_t N,
                         uint64_t m, const uint64_t *idx, uint64_t nidx,
                         uint64_t *out) {
    long long ni = (long long)nidx;
#pragma omp parallel for schedule(dynamic, 1)
    for (long long i = 0; i < ni; ++i) {
        uint64_t j = idx[i] % N;
        u128 acc = 0;
        for (uint64_t k = 0; k < N; ++k)
            acc += (u128)mulmod(f[k], g[(j + N - k) % N], m);
        out[i] = (uint64_t)(acc % m);
    }
}

/* Circular convolution through the convolution theorem (Sec. I): transform f
 * and g with Eq. 2, multiply the coefficients, invert with Eq. 3.  Every step
 * is the O(N^2) sum of oracle_ntt.  Returns oracle_ntt's error codes. */
int oracle_conv_via_ntt(const uint64_t *f, const uint64_t *g, uint64_t *h,
                        uint64_t N, uint64_t m, uint64_t root) {
    if (N == 0) return 0;
    uint64_t *F = (uint64_t *)malloc((size_t)N * sizeof(uint64_t));
    uint64_t *G = (uint64_t *)malloc((size_t)N * sizeof(uint64_t));
    if (!F || !G) { free(F); free(G); return 3; }
    int rc = oracle_ntt(f, F, N, m, root, 0);
    if (!rc) rc = oracle_ntt(g, G, N, m, root, 0);
    if (!rc) {
        for (uint64_t u = 0; u < N; ++u) F[u] = mulmod(F[u], G[u], m);
        rc = oracle_ntt(F, h, N, m, root, 1);
    }
    free(F); free(G);
    return rc;
}

/* Exact deconvolution (division filtering): the prime modulus lets every
 * nonzero coefficient be divided (Sec. III-A), so f * g = h is solved for g by
 * the convolution theorem read backwards (Sec. I):
 *     g = inverse( forward(h) / forward(f) ),
 * each spectral quotient H(u) F(u)^-1 with F(u)^-1 from the extended Euclidean
 * algorithm (Appendix A).  Returns 4 (and leaves g unspecified) when some
 * F(u) = 0, where no unique g exists; otherwise as oracle_ntt. */
int oracle_deconv_via_ntt(const uint64_t *f, const uint64_t *h, uint64_t *g,
                          uint64_t N, uint64_t m, uint64_t root) {
    if (N == 0) return 0;
    uint64_t *F = (uint64_t *)malloc((size_t)N * sizeof(uint64_t));
    uint64_t *H = (uint64_t *)malloc((size_t)N * sizeof(uint64_t));
    if (!F || !H) { free(F); free(H); return 3; }
    int rc = oracle_ntt(f, F, N, m, root, 0);
    if (!rc) rc = oracle_ntt(h, H, N, m, root, 0);
    for (uint64_t u = 0; !rc && u < N; ++u) {
        if (F[u] == 0) { rc = 4; break; }
        H[u] = mulmod(H[u], oracle_inverse(F[u], m), m);
    }
    if (!rc) rc = oracle_ntt(H, g, N, m, root, 1);
    free(F); free(H);
    return rc;
}

/* The true integer circular convolution, Eq. 1 without the reduction modulo m:
 *     h(j) = sum_{k<N} f(k) g(j - k mod N),
 * f and g read as non-negative integers.  This is what the convolution modulo
 * m equals when every h(j) < m (Sec. I: "impervious to overflow" only inside
 * the modulus), and what a residue-number (CRT) combination of convolutions
 * modulo several primes reconstructs.  Returns 5 if some h(j) >= 2^64. */
int oracle_conv_integer(const uint64_t *f, const uint64_t *g, uint64_t *h, uint64_t N) {
    long long n = (long long)N;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (long long j = 0; j < n; ++j) {
        u128 acc = 0;
        /* k = 0..N-1 in order; (j - k) mod N is j - k for k <= j and
         * j + N - k above (no division in the inner loop) */
        for (uint64_t k = 0; k < N; ++k) {
            uint64_t idx = k <= (uint64_t)j ? (uint64_t)j - k : (uint64_t)j + N - k;
            u128 p = (u128)f[k] * g[idx];
            if (acc + p < acc) bad = 1;
            acc += p;
        }
        if (acc >> 64) bad = 1;
        h[j] = (uint64_t)acc;
    }
    return bad ? 5 : 0;
}

/* Selected outputs of the integer circular convolution: out[i] = h(idx[i]),
 * each the O(N) direct sum.  Returns 5 if one reaches 2^64. */
int oracle_conv_integer_entries(const uint64_t *f, const uint64_t *g, uint64_t N,
                                const uint64_t *idx, uint64_t nidx, uint64_t *out) {
    long long ni = (long long)nidx;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (long long i = 0; i < ni; ++i) {
        uint64_t j = idx[i] % N;
        u128 acc = 0;
        for (uint64_t k = 0; k < N; ++k) acc += (u128)f[k] * g[(j + N - k) % N];
        if (acc >> 64) bad = 1;
        out[i] = (uint64_t)acc;
    }
    return bad ? 5 : 0;
}

/* Two-dimensional circular convolution of R x C arrays (row-major), the
 * multi-dimensional form of Eq. 1 (Sec. I mentions multi-dimensional
 * techniques; the transform applies to each dimension in turn):
 *     h(i, j) = < sum_{k<R} sum_{l<C} f(k, l) g((i - k) mod R, (j - l) mod C) >_m,
 * as the O(R^2 C^2) direct sum. */
void oracle_conv2d_direct(const uint64_t *f, const uint64_t *g, uint64_t *h,
                          uint64_t R, uint64_t C, uint64_t m) {
    long long n = (long long)(R * C);
#pragma omp parallel for schedule(dynamic, 16)
    for (long long o = 0; o < n; ++o) {
        uint64_t i = (uint64_t)o / C, j = (uint64_t)o % C;
        u128 acc = 0;
        for (uint64_t k = 0; k < R; ++k)
            for (uint64_t l = 0; l < C; ++l) {
                uint64_t a = (i + R - k) % R, b = (j + C - l) % C;
                acc += (u128)mulmod(f[k * C + l], g[a * C + b], m);
            }
        h[o] = (uint64_t)(acc % m);
    }
}

/* Selected outputs of the 2-D convolution: out[q] = h(idx[q] / C, idx[q] % C). */
void oracle_conv2d_entries(const uint64_t *f, const uint64_t *g, uint64_t R, uint64_t C,
                           uint64_t m, const uint64_t *idx, uint64_t nidx, uint64_t *out) {
    long long ni = (long long)nidx;
#pragma omp parallel for schedule(dynamic, 1)
    for (long long q = 0; q < ni; ++q) {
        uint64_t o = idx[q] % (R * C), i = o / C, j = o % C;
        u128 acc = 0;
        for (uint64_t k = 0; k < R; ++k)
            for (uint64_t l = 0; l < C; ++l)
                acc += (u128)mulmod(f[k * C + l], g[((i + R - k) % R) * C + (j + C - l) % C], m);
        out[q] = (uint64_t)(acc % m);
    }
}
