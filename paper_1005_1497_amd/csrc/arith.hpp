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
    double Cm;     // C * m, exact because 3m < 2^26
};

__device__ __forceinline__ double mulmod(double b, double w, double wq, const ModC& M) {
    double q = __builtin_fma(b, wq, M.C);
    double x = __builtin_fma(q, -M.m, M.Cm);
    return __builtin_fma(b, w, x);
}

// a*b mod m for two variable operands with |a*b| < 2^53 - m; result in
// [-m/2 - 2, m/2 + 2].
__device__ __forceinline__ double mulmod_var(double a, double b, const ModC& M) {
    double bq = b * M.minv;
    double q = __builtin_fma(a, bq, M.C);
    double x = __builtin_fma(q, -M.m, M.Cm);
    return __builtin_fma(a, b, x);
}

// y mod m into [-m/2 - 2, m/2 + 2] for |y| < 2^51.
__device__ __forceinline__ double reduce(double y, const ModC& M) {
    double q = __builtin_fma(y, M.minv, M.C);
    double x = __builtin_fma(q, -M.m, M.Cm);
    return y + x;
}

// Canonical residue in [0, m) (Appendix A) as an unsigned word.
__device__ __forceinline__ uint32_t canon_u32(double y, const ModC& M) {
    double r = reduce(y, M);
    r = (r < 0.0) ? r + M.m : r;
    return (uint32_t)r;
}

// Scratch words hold reduced residues as signed 32-bit integers.
__device__ __forceinline__ int32_t to_i32(double y) { return (int32_t)y; }
__device__ __forceinline__ double from_i32(int32_t v) { return (double)v; }

}  // namespace nttmi
