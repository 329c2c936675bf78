// CPU sweep of the library's exact fp64 residue arithmetic (csrc/arith.hpp,
// compiled here for the host) against exact integer arithmetic.
//
// The kernels carry residues modulo m as doubles and form every product modulo
// m with fused multiply-adds (the <.>_m of Appendix A applied to the products
// of Eqs. 2 and 3).  The claims checked here are the ones the kernels' range
// bookkeeping rests on, each at the operand ranges the kernels can produce:
//
//   32-bit words (m < 2^24)
//     mulmod(b, w, w/m)   |b| m < 2^53 - m, 0 <= w < m  ->  r = b w mod m, |r| <= m/2 + 2
//                         (|b| up to 48 m for m = 13631489, 32 m near 2^24;
//                         the kernels' products have |b| <= 16 m: a first-pass
//                         output of canonical words; later passes' <= 8 m + 32)
//     mulmod_var(a, b)    |a b| < 2^53 - m          ->  r = a b mod m, |r| <= m/2 + 2
//     reduce(y)           |y| < 2^51                ->  r = y mod m,   |r| <= m/2 + 2
//     canon_u32(y)        as reduce                 ->  the canonical residue
//   64-bit words (m < 2^46)
//     mulmod_dd(b, w)     |b| <= 12 m, |w| < m      ->  r = b w mod m, |r| <= 0.69 m
//     reduce_dd(y)        |y| < 2^52                ->  r = y mod m,   |r| <= m/2 + 2
//     W64::load_reduce(x) any 64-bit word           ->  r = x mod m,   |r| <= 0.69 m
//     W64::canon(y)       |y| <= 12 m               ->  the canonical residue
//
// "r = ... mod m" is checked as an exact congruence in 128-bit integers, and
// r must be an integer-valued double.  Besides uniform draws, every product
// family takes adversarial operands whose exact quotient b w / m lies within
// 1/(2m) of a half-integer (b w = (m +- 1)/2 mod m and neighbours), where the
// rounded quotient may be off by one, and operands at the ends of their range.
//
// Usage: fp64_sweep [cases_per_family]   (exit status 0 when every case holds)
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>

#include "../paper_1005_1497_amd/csrc/arith.hpp"

using namespace nttmi;
typedef __int128 i128;

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {   // splitmix64
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// uniform integer in [lo, hi]
static int64_t uni(int64_t lo, int64_t hi) {
    const uint64_t span = (uint64_t)(hi - lo) + 1;
    return lo + (int64_t)(next_u64() % span);
}

static int64_t modp(i128 x, int64_t m) {
    i128 r = x % m;
    if (r < 0) r += m;
    return (int64_t)r;
}
static int64_t powm(int64_t b, int64_t e, int64_t m) {
    i128 r = 1, x = modp(b, m);
    while (e) {
        if (e & 1) r = r * x % m;
        x = x * x % m;
        e >>= 1;
    }
    return (int64_t)r;
}
static int64_t invm(int64_t b, int64_t m) { return powm(b, m - 2, m); }   // m prime

static long failures = 0, checked = 0;

// r must be an integer-valued double with r = want (mod m) and |r| <= bound
static void check(const char* what, int64_t m, double r, i128 want, double bound, double a, double b) {
    ++checked;
    const bool integral = std::isfinite(r) && r == std::floor(r) && std::fabs(r) < 9.007199254740992e15;
    const bool ok = integral && modp((i128)(int64_t)r - want, m) == 0 && std::fabs(r) <= bound;
    if (!ok && failures++ < 20)
        std::printf("FAIL %s m=%lld a=%.17g b=%.17g -> r=%.17g (want %lld mod m, |r| <= %.17g)\n", what,
                    (long long)m, a, b, r, (long long)modp(want, m), bound);
}

// operand b (nonzero mod m) and a twiddle w with b w = t (mod m) for t near m/2
static int64_t adversarial_w(int64_t b, int64_t m, int k) {
    const int64_t half = (m - 1) / 2;
    const int64_t t = half + (k % 6) - 2;   // (m-5)/2 .. (m+5)/2
    return (int64_t)modp((i128)t * invm(modp(b, m), m), m);
}

static void sweep32(int64_t m, long cases) {
    const ModC M = make_modc((uint64_t)m);
    const double rb = (double)m / 2 + 2;
    const int64_t bfit = (int64_t)((((int64_t)1 << 53) - 2 * m) / m);   // |b| m < 2^53 - m
    const int64_t bmax = 48 * m - 1 < bfit ? 48 * m - 1 : bfit, fmax = 16 * m;
    for (long i = 0; i < cases; ++i) {
        // twiddle product, uniform and adversarial
        int64_t b = uni(-bmax, bmax);
        int64_t w = uni(0, m - 1);
        if (i % 4 == 1 && modp(b, m) != 0) w = adversarial_w(b, m, (int)i);
        if (i % 64 == 2) b = (i & 128) ? bmax : -bmax;
        if (i % 64 == 3) w = m - 1;
        const double2 tw = tw_pair((uint64_t)w, (uint64_t)m);
        check("mulmod", m, mulmod((double)b, tw.x, tw.y, M), (i128)b * w, rb, (double)b, (double)w);
        // variable product: a pass output (up to a first pass's 16 m) times a
        // reduced value, or a twiddle
        int64_t a = uni(-fmax, fmax);
        int64_t c = (i & 1) ? uni(-(m / 2 + 2), m / 2 + 2) : uni(0, m - 1);
        if (i % 4 == 3 && modp(a, m) != 0) c = adversarial_w(a, m, (int)i) - ((i & 1) ? m : 0);
        if (i % 64 == 5) { a = (i & 128) ? fmax : -fmax; c = (i & 256) ? m - 1 : -(m / 2 + 2); }
        if (std::fabs((double)a * (double)c) >= 9.007199254740992e15 - m) c = c / 2;   // |a c| < 2^53 - m
        check("mulmod_var", m, mulmod_var((double)a, (double)c, M), (i128)a * c, rb, (double)a, (double)c);
        // reductions: a 32-bit word on load, a pass output, a wide value
        const int64_t y1 = (int64_t)(next_u64() & 0xFFFFFFFFull);
        check("reduce(word)", m, reduce((double)y1, M), y1, rb, (double)y1, 0);
        const int64_t y2 = (i % 3 == 0) ? uni(-(1ll << 51) + 1, (1ll << 51) - 1) : uni(-fmax, fmax);
        check("reduce", m, reduce((double)y2, M), y2, rb, (double)y2, 0);
        const double cu = (double)canon_u32((double)y2, M);
        check("canon_u32", m, cu, y2, (double)m - 1, (double)y2, 0);
        if (!(cu >= 0 && cu < (double)m)) check("canon_u32 range", m, NAN, 0, 0, (double)y2, 0);
    }
}

static void sweep64(int64_t m, long cases) {
    const ModC M = make_modc((uint64_t)m);
    const double r69 = 0.69 * (double)m, rh = (double)m / 2 + 2;
    const int64_t bmax = 12 * m;
    for (long i = 0; i < cases; ++i) {
        int64_t b = uni(-bmax, bmax);
        int64_t w = (i & 1) ? uni(0, m - 1) : uni(-(m - 1), m - 1);
        if (i % 4 == 1 && modp(b, m) != 0) w = adversarial_w(b, m, (int)i);
        if (i % 64 == 2) b = (i & 128) ? bmax : -bmax;
        if (i % 64 == 3) w = (i & 128) ? m - 1 : -(m - 1);
        check("mulmod_dd", m, mulmod_dd((double)b, (double)w, M), (i128)b * w, r69, (double)b, (double)w);
        const int64_t y = (i % 3 == 0) ? uni(-(1ll << 52) + 1, (1ll << 52) - 1) : uni(-bmax, bmax);
        check("reduce_dd", m, reduce_dd((double)y, M), y, rh, (double)y, 0);
        uint64_t x = next_u64();
        if (i % 64 == 4) x = ~0ull;
        if (i % 64 == 5) x = (uint64_t)m - 1 + ((uint64_t)(i & 7) << 46);
        check("W64::load_reduce", m, W64::load_reduce(x, M), (i128)x, r69, (double)x, 0);
        const int64_t z = uni(-bmax, bmax);
        const uint64_t cz = W64::canon((double)z, M);
        ++checked;
        if (cz != (uint64_t)modp(z, m) && failures++ < 20)
            std::printf("FAIL W64::canon m=%lld y=%lld -> %llu\n", (long long)m, (long long)z, (unsigned long long)cz);
    }
}

int main(int argc, char** argv) {
    const long cases = argc > 1 ? std::atol(argv[1]) : 2000000;
    // 32-bit words: the Table 1 primes, the Euler-form primes the tests use and
    // the largest prime below 2^24
    const int64_t m32[] = {641, 319489, 2424833, 13631489, 7340033, 5767169, 16777213};
    // 64-bit words: the 45-bit Rader prime of the served workload, an Euler
    // prime, and the largest prime k 2^20 + 1 below 2^46
    const int64_t m64[] = {31065037602817ll, 998244353ll, 70368714817537ll};
    for (int64_t m : m32) sweep32(m, cases);
    for (int64_t m : m64) sweep64(m, cases);
    std::printf("%ld cases, %ld failures\n", checked, failures);
    return failures ? 1 : 0;
}
