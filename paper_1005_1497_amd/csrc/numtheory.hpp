// Host number theory for plan validation (independent of the test oracle).
//
// Validation follows the paper's conditions: m prime (Sec. III-A), the order
// nu of 2 modulo m a power of two so that 2 is a lambda-root of m (Sec. II,
// Eq. 7; Prop. 2), N = 2^n dividing nu (Sec. I), and a root of exact order N.
#pragma once
#include <stdint.h>

namespace nttmi {

typedef unsigned __int128 u128;

inline uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

inline uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod64(r, a, m);
        a = mulmod64(a, a, m);
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin for 64-bit integers (the first twelve primes as
// bases are a proven witness set below 3.3e24).
inline bool is_prime64(uint64_t n) {
    if (n < 2) return false;
    static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (uint64_t p : small) {
        if (n % p == 0) return n == p;
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; ++s; }
    for (uint64_t a : small) {
        uint64_t x = powmod64(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; ++r) {
            x = mulmod64(x, x, n);
            if (x == n - 1) { comp = false; break; }
        }
        if (comp) return false;
    }
    return true;
}

// log2 of the order of 2 modulo an odd m when that order is a power of two,
// else -1.  2^(2^k) is built by repeated squaring; the order is 2^k for the
// first k with 2^(2^k) = 1 (the order divides 2^k and no smaller power of two).
inline int log2_order_of_two(uint64_t m) {
    if (m < 3 || (m & 1) == 0) return -1;
    uint64_t x = 2 % m;
    for (int k = 0; k < 64; ++k) {
        if (x == 1) return k;
        x = mulmod64(x, x, m);
    }
    return -1;
}

}  // namespace nttmi
