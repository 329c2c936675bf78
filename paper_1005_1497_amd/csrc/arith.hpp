// Exact modular arithmetic on residues held in fp64 registers (device side).
//
// Residues modulo m < 2^24 are carried as exactly representable doubles.  A
// product b*w is at most 53 bits when |b| < 48 m, and the fused multiply-add
// keeps every intermediate exact, so a twiddle product modulo m costs three
// FMAs and no integer multiply:
//   q' = fma(b, w/m, C)        C = 1.5*2^52: q' - C = round(b*w/m)
//   x  = fma(q', -m, C*m)      = -round(b*w/m)*m, exact (|x| < 2^53)
//   r  = fma(b, w, x)          = b*w - q*m, exact, |r| <= m/2 + 2
// The quotient may be off by one only when b*w/m lies within ~1e-7 of a
// half-integer, so the remainder stays within m/2 + 2 in every case.
//
// Every routine here is also compiled for the host, so that a CPU test can
// sweep them against exact integer arithmetic.
//
// This is the word-level form of the paper's twiddle product (Eq. 2): the
// coefficients are the powers 2^e mod m of the digital circle (Eq. 5) and the
// reduction is the <.>_m of Appendix A; see the design notes for why literal
// bit shifts of up to 2^18 bits are not used on 64-lane vector units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttmi {

// Per-modulus constants, uniform across a launch.
struct ModC {
    double m;      // the modulus
    double minv;   // fl(1/m)
    double C;      // 1.5 * 2^52 (round-to-integer shifter)
    double Cm;     // C * m (exact for 32-bit words: 3m < 2^26; unused for 64-bit words)
    double c32;    // 2^32 mod m (64-bit words: reduction of the high half on load)
};

// The constants of modulus m (host side; kernels receive them by value).
inline ModC make_modc(uint64_t m) {
    ModC M;
    M.m = (double)m;
    M.minv = 1.0 / (double)m;
    M.C = 6755399441055744.0;  // 1.5 * 2^52
    M.Cm = M.C * (double)m;    // exact for m < 2^26 (3m fits the significand)
    M.c32 = (double)((1ull << 32) % m);
    return M;
}

// A twiddle w as the pair (w, w/m) that mulmod takes (host side).
inline double2 tw_pair(uint64_t w, uint64_t m) {
    double2 t;
    t.x = (double)w;
    t.y = (double)w / (double)m;
    return t;
}

__host__ __device__ __forceinline__ double mulmod(double b, double w, double wq, const ModC& M) {
    double q = __builtin_fma(b, wq, M.C);
    double x = __builtin_fma(q, -M.m, M.Cm);
    return __builtin_fma(b, w, x);
}

// a*b mod m for two variable operands with |a*b| < 2^53 - m; result in
// [-m/2 - 2, m/2 + 2].
__host__ __device__ __forceinline__ double mulmod_var(double a, double b, const ModC& M) {
    double bq = b * M.minv;
    double q = __builtin_fma(a, bq, M.C);
    double x = __builtin_fma(q, -M.m, M.Cm);
    return __builtin_fma(a, b, x);
}

// y mod m into [-m/2 - 2, m/2 + 2] for |y| < 2^51.
__host__ __device__ __forceinline__ double reduce(double y, const ModC& M) {
    double q = __builtin_fma(y, M.minv, M.C);
    double x = __builtin_fma(q, -M.m, M.Cm);
    return y + x;
}

// Canonical residue in [0, m) (Appendix A) as an unsigned word.
__host__ __device__ __forceinline__ uint32_t canon_u32(double y, const ModC& M) {
    double r = reduce(y, M);
    r = (r < 0.0) ? r + M.m : r;
    return (uint32_t)r;
}

// Scratch words hold reduced residues as signed 32-bit integers.
__host__ __device__ __forceinline__ int32_t to_i32(double y) { return (int32_t)y; }
__host__ __device__ __forceinline__ double from_i32(int32_t v) { return (double)v; }

}  // namespace nttmi

namespace nttmi {

// ---------------------------------------------------------------------------
// Word policies: how residues are loaded, multiplied and stored for each word
// width.  Both carry residues as exact fp64 values.
//
// W32: 32-bit words, m < 2^24.  Twiddle products use the three-FMA form above
//      with a precomputed w/m.  Scratch words are int32.
// W64: 64-bit words, m < 2^46 (the 45-bit Rader prime of the serving
//      workload).  A product b*w (up to ~2^96) is split exactly into
//      hi = fl(b w) and lo = fma(b, w, -hi); the quotient q = round(hi/m) comes
//      from an fp64 multiply-add, |q - b w / m| <= 1/2 + |b| 2^-52;
//      r = fma(-q, m, hi) + lo is exact because hi - q m is an integer below
//      2^53.  |r| <= m/2 + |b| m 2^-52 <= 0.69 m for |b| <= 12 m and m < 2^46,
//      so a radix-16 pass output is at most 16 * 0.69 m < 12 m: the bounds
//      close, and every value stays below 2^53.
//      Scratch words are the fp64 values themselves.
// ---------------------------------------------------------------------------
struct W32 {
    using word = uint32_t;
    using sword = int32_t;
    static constexpr int WB = 4;   // bytes per word
    static constexpr int SB = 4;   // bytes per scratch word
    __host__ __device__ static __forceinline__ double mul_tw(double b, const double2& w, const ModC& M) {
        return mulmod(b, w.x, w.y, M);
    }
    __host__ __device__ static __forceinline__ double mul_w(double b, double w, const ModC& M) { return mulmod_var(b, w, M); }
    __host__ __device__ static __forceinline__ double mul_var(double a, double b, const ModC& M) { return mulmod_var(a, b, M); }
    __host__ __device__ static __forceinline__ double load_reduce(word x, const ModC& M) { return reduce((double)x, M); }
    __host__ __device__ static __forceinline__ word canon(double y, const ModC& M) { return canon_u32(y, M); }
    __host__ __device__ static __forceinline__ sword to_s(double y) { return (int32_t)y; }
    __host__ __device__ static __forceinline__ double from_s(sword v) { return (double)v; }
    __host__ __device__ static __forceinline__ double reduce_s(double y, const ModC& M) { return reduce(y, M); }
};

__host__ __device__ __forceinline__ double mulmod_dd(double b, double w, const ModC& M) {
    const double hi = b * w;
    const double lo = __builtin_fma(b, w, -hi);
    const double q = __builtin_fma(hi, M.minv, M.C) - M.C;
    const double r1 = __builtin_fma(q, -M.m, hi);
    return r1 + lo;
}

// y mod m into about [-m/2, m/2] for |y| < 2^52 (64-bit words).
__host__ __device__ __forceinline__ double reduce_dd(double y, const ModC& M) {
    const double q = __builtin_fma(y, M.minv, M.C) - M.C;
    return __builtin_fma(q, -M.m, y);
}

struct W64 {
    using word = uint64_t;
    using sword = double;
    static constexpr int WB = 8;
    static constexpr int SB = 8;
    __host__ __device__ static __forceinline__ double mul_tw(double b, const double2& w, const ModC& M) {
        return mulmod_dd(b, w.x, M);
    }
    __host__ __device__ static __forceinline__ double mul_w(double b, double w, const ModC& M) { return mulmod_dd(b, w, M); }
    __host__ __device__ static __forceinline__ double mul_var(double a, double b, const ModC& M) { return mulmod_dd(a, b, M); }
    // x = xh 2^32 + xl; (xh * (2^32 mod m) mod m) + xl, then reduced
    __host__ __device__ static __forceinline__ double load_reduce(word x, const ModC& M) {
        const double h = mulmod_dd((double)(uint32_t)(x >> 32), M.c32, M);
        return reduce_dd(h + (double)(uint32_t)x, M);
    }
    __host__ __device__ static __forceinline__ word canon(double y, const ModC& M) {
        double r = reduce_dd(y, M);
        r = (r < 0.0) ? r + M.m : r;
        r = (r >= M.m) ? r - M.m : r;
        const double hi = __builtin_floor(r * 2.3283064365386963e-10);   // 2^-32
        const double lo = __builtin_fma(hi, -4294967296.0, r);
        return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
    }
    __host__ __device__ static __forceinline__ sword to_s(double y) { return y; }
    __host__ __device__ static __forceinline__ double from_s(sword v) { return v; }
    __host__ __device__ static __forceinline__ double reduce_s(double y, const ModC& M) { return reduce_dd(y, M); }
};

// x^e mod m by left-to-right square and multiply over the bits of e (bit
// `top` is the highest set bit; e and top are uniform across the wave, so the
// branch is too).  x reduced; result reduced.  With e = m - 2 this is the
// inverse of x for a prime m (Fermat's little theorem), 0 for x = 0.
template <class W>
__host__ __device__ __forceinline__ double pow_mod(double x, uint64_t e, int top, const ModC& M) {
    double r = x;
    for (int b = top - 1; b >= 0; --b) {
        r = W::mul_var(r, r, M);
        if ((e >> b) & 1) r = W::mul_var(r, x, M);
    }
    return r;
}

}  // namespace nttmi
